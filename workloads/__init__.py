"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests, the bench and the smoke check.  It holds
no Shifted-Fresnel arithmetic: it draws scatterer positions, builds in-line
(Gabor) holograms from paraxial point-source waves, resizes, and lists view
parameters.  The paper's optical holograms (USAF target, mosquito, fly) are
not available; these synthetic holograms stand in for them.

Recipe (all draws from ``numpy.random.default_rng`` / ``SeedSequence``):

* wavelength 632.8 nm (the He-Ne laser of Section 2), hologram pitch 4.65 um
  (the CCD of Section 2);
* object wave O = sum_j (a_j / sqrt(J)) w_j(x) w_j(y) with
  w_j(x) = exp(i pi (x - x_j)^2 / (lambda z_j)) exp(-(x - x_j)^2 / (2 s_j^2)):
  a paraxial point-source wave limited, by a Gaussian envelope of width
  s_j = lambda z_j / (4 p), to the region where its fringes stay below the
  sampling limit of the sensor;
* hologram H = |1 + O|^2 + N(0, 0.01^2), float32 (unit plane reference wave).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

WAVELENGTH = 632.8e-9
CCD_PITCH = 4.65e-6


@dataclass(frozen=True)
class GridSpec:
    nx: int
    ny: int
    px: float
    py: float
    ox: float = 0.0
    oy: float = 0.0


@dataclass(frozen=True)
class ViewSpec:
    grid: GridSpec
    z: float
    holo: int = 0


@dataclass
class Workload:
    name: str
    wavelength: float
    holo_grid: GridSpec
    holograms: np.ndarray  # [n_holo, ny, nx], float32 or complex64
    views: list = field(default_factory=list)
    extra: dict = field(default_factory=dict)


def _axis(n: int, p: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - n // 2) * p


def gabor_hologram(rng: np.random.Generator, nx: int, ny: int, p: float,
                   n_scat: int, z_choice, amp=(0.2, 1.0), noise=0.01,
                   wavelength: float = WAVELENGTH) -> np.ndarray:
    """In-line hologram of ``n_scat`` point scatterers, float32 [ny, nx].

    ``z_choice(rng, n)`` draws the scatterer depths.  Scatterer (x, y) are
    uniform over the field.
    """
    x = _axis(nx, p)
    y = _axis(ny, p)
    xj = rng.uniform(x[0], x[-1], n_scat)
    yj = rng.uniform(y[0], y[-1], n_scat)
    zj = np.asarray(z_choice(rng, n_scat), dtype=np.float64)
    aj = rng.uniform(amp[0], amp[1], n_scat) / np.sqrt(n_scat)
    sj = wavelength * zj / (4.0 * p)
    dx = x[:, None] - xj[None, :]
    dy = y[:, None] - yj[None, :]
    wx = np.exp(1j * np.pi * dx * dx / (wavelength * zj)) * np.exp(-dx * dx / (2 * sj * sj))
    wy = np.exp(1j * np.pi * dy * dy / (wavelength * zj)) * np.exp(-dy * dy / (2 * sj * sj))
    obj = (wy * aj[None, :]) @ wx.T  # [ny, nx]
    holo = np.abs(1.0 + obj) ** 2 + rng.normal(0.0, noise, (ny, nx))
    return holo.astype(np.float32)


def bilinear_resize_x(img: np.ndarray, nx_out: int) -> np.ndarray:
    """Bilinear resize along x with half-pixel centres (y unchanged)."""
    ny, nx = img.shape
    s = (np.arange(nx_out) + 0.5) * (nx / nx_out) - 0.5
    s = np.clip(s, 0.0, nx - 1.0)
    i0 = np.floor(s).astype(np.int64)
    i1 = np.minimum(i0 + 1, nx - 1)
    w = (s - i0)[None, :]
    out = img[:, i0] * (1.0 - w) + img[:, i1] * w
    return out.astype(img.dtype)


def _spawn(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def config1() -> Workload:
    """Single view: 256^2 hologram (8 scatterers, z_j = 5 cm) -> 256^2 view at
    z = 5 cm, pitch 2.325 um (half the CCD pitch), shift (+100, -50) um."""
    rng = _spawn(1, 1)[0]
    n = 256
    holo = gabor_hologram(rng, n, n, CCD_PITCH, 8, lambda r, k: np.full(k, 0.05))
    hg = GridSpec(n, n, CCD_PITCH, CCD_PITCH)
    view = ViewSpec(GridSpec(n, n, CCD_PITCH / 2, CCD_PITCH / 2, 100e-6, -50e-6), 0.05, 0)
    return Workload("config1-single-256", WAVELENGTH, hg, holo[None], [view])


def config2() -> Workload:
    """Paper-shaped: a 1360 x 1024 CCD field of 64 scatterers (z_j drawn from
    {3, 6, 10} cm), bilinearly resized along x to 1024^2, and four 1024^2 views.
    ``extra["ccd"]`` keeps the unresized frame (1 x 1024 x 1360)."""
    rng = _spawn(2, 1)[0]
    ccd = gabor_hologram(rng, 1360, 1024, CCD_PITCH, 64,
                         lambda r, k: r.choice([0.03, 0.06, 0.10], k))
    holo = bilinear_resize_x(ccd, 1024)
    px0 = 1360 * CCD_PITCH / 1024
    hg = GridSpec(1024, 1024, px0, CCD_PITCH)
    n = 1024
    views = [
        ViewSpec(GridSpec(n, n, 8e-6, 8e-6), 0.03, 0),
        ViewSpec(GridSpec(n, n, 1.5e-6, 1.5e-6, 400e-6, -400e-6), 0.03, 0),
        ViewSpec(GridSpec(n, n, 4.65e-6, 4.65e-6), 0.06, 0),
        ViewSpec(GridSpec(n, n, 2e-6, 2e-6, 200e-6, 200e-6), 0.10, 0),
    ]
    return Workload("config2-paper-4view-1024", WAVELENGTH, hg, holo[None], views,
                    extra={"ccd": ccd[None].astype(np.float32)})


def config3(n_holo: int = 8, views_per_holo: int = 8, n: int = 1024) -> Workload:
    """Batched uneven: 8 holograms of 1024^2 (64 scatterers each, z_j in
    U[2, 12] cm) x 8 views: N1 from {256, 512, 768, 1024}, z in U[2, 12] cm,
    pitch log-uniform in [1, 10] um, shifts U[-1, 1] mm."""
    rngs = _spawn(3, n_holo + 1)
    holos = np.stack([
        gabor_hologram(rngs[h], n, n, CCD_PITCH, 64, lambda r, k: r.uniform(0.02, 0.12, k))
        for h in range(n_holo)])
    hg = GridSpec(n, n, CCD_PITCH, CCD_PITCH)
    r = rngs[-1]
    views = []
    for h in range(n_holo):
        for _ in range(views_per_holo):
            n1 = int(r.choice([256, 512, 768, 1024]))
            z = float(r.uniform(0.02, 0.12))
            p1 = float(np.exp(r.uniform(np.log(1e-6), np.log(10e-6))))
            ox, oy = (float(v) for v in r.uniform(-1e-3, 1e-3, 2))
            views.append(ViewSpec(GridSpec(n1, n1, p1, p1, ox, oy), z, h))
    return Workload("config3-batched-uneven-64view", WAVELENGTH, hg, holos, views)


def smooth_phase_screen(rng: np.random.Generator, n: int, sigma_px: float = 8.0) -> np.ndarray:
    """exp(i phi), phi = pi x (white noise smoothed by a periodic Gaussian of
    sigma_px pixels, normalised to unit standard deviation), complex64."""
    w = rng.normal(size=(n, n))
    f = np.fft.fftfreq(n)
    g = np.exp(-2.0 * (np.pi * sigma_px) ** 2 * (f[:, None] ** 2 + f[None, :] ** 2))
    s = np.real(np.fft.ifft2(np.fft.fft2(w) * g))
    s = (s - s.mean()) / s.std()
    return np.exp(1j * np.pi * s).astype(np.complex64)


def config4(batch: int = 16, n: int = 1024) -> Workload:
    """Differentiation: ``batch`` complex object fields (smoothed random phase
    screens) at pitch 2.325 um, each propagated to a hologram plane at pitch
    4.65 um and its own z in U[3, 8] cm.  ``extra`` carries the target
    screens w_b and the offsets delta_b in U[-2, 2] mm that define the
    targets T_b = |A(z_b + delta_b) w_b|^2."""
    rngs = _spawn(4, 2 * batch + 1)
    fields = np.stack([smooth_phase_screen(rngs[b], n) for b in range(batch)])
    targets_w = np.stack([smooth_phase_screen(rngs[batch + b], n) for b in range(batch)])
    r = rngs[-1]
    zs = r.uniform(0.03, 0.08, batch)
    deltas = r.uniform(-2e-3, 2e-3, batch)
    hg = GridSpec(n, n, CCD_PITCH / 2, CCD_PITCH / 2)
    views = [ViewSpec(GridSpec(n, n, CCD_PITCH, CCD_PITCH), float(zs[b]), b) for b in range(batch)]
    return Workload("config4-diff-16x1024", WAVELENGTH, hg, fields, views,
                    extra={"target_fields": targets_w, "deltas": deltas})


def config5(n: int = 4096) -> Workload:
    """Large/precision: a 4096^2 hologram of 256 scatterers (z_j in U[10, 20] cm),
    eight 4096^2 views with the (z, pitch) pairs below and shifts U[-1, 1] mm."""
    rngs = _spawn(5, 2)
    holo = gabor_hologram(rngs[0], n, n, CCD_PITCH, 256, lambda r, k: r.uniform(0.10, 0.20, k))
    hg = GridSpec(n, n, CCD_PITCH, CCD_PITCH)
    pairs = [(0.02, 0.5e-6), (0.02, 4.65e-6), (0.05, 1e-6), (0.05, 4.65e-6),
             (0.10, 0.5e-6), (0.10, 2e-6), (0.20, 0.5e-6), (0.20, 4.65e-6)]
    r = rngs[1]
    views = []
    for z, p in pairs:
        ox, oy = (float(v) for v in r.uniform(-1e-3, 1e-3, 2))
        views.append(ViewSpec(GridSpec(n, n, p, p, ox, oy), z, 0))
    return Workload("config5-large-4096-8view", WAVELENGTH, hg, holo[None], views)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def random_case(seed: int, n0=(5, 40), n1=(5, 40), complex_input=True):
    """A small random problem (rectangular grids, anisotropic pitches, shifts,
    signed z) for property tests.  Returns (u0, holo GridSpec, view GridSpec, z)."""
    r = np.random.default_rng(seed)
    nx0, ny0 = (int(v) for v in r.integers(n0[0], n0[1] + 1, 2))
    nx1, ny1 = (int(v) for v in r.integers(n1[0], n1[1] + 1, 2))
    px0, py0 = (float(v) for v in r.uniform(2e-6, 8e-6, 2))
    px1, py1 = (float(v) for v in r.uniform(1e-6, 10e-6, 2))
    o0 = (float(v) for v in r.uniform(-100e-6, 100e-6, 2))
    o1 = (float(v) for v in r.uniform(-300e-6, 300e-6, 2))
    z = float(r.uniform(0.005, 0.05) * r.choice([-1.0, 1.0]))
    if complex_input:
        u0 = (r.normal(size=(ny0, nx0)) + 1j * r.normal(size=(ny0, nx0))).astype(np.complex64)
    else:
        u0 = r.uniform(0.0, 2.0, size=(ny0, nx0)).astype(np.float32)
    g0 = GridSpec(nx0, ny0, px0, py0, *o0)
    g1 = GridSpec(nx1, ny1, px1, py1, *o1)
    return u0, g0, g1, z
