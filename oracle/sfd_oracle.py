"""Plain FP64 oracle for Shifted-Fresnel diffraction (Section 2.1, Eqs. 1-5).

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import this module.

Notation follows Section 2.1: hologram u0 on plane 0 with pitches (px0, py0)
and shifts (Ox0, Oy0); reconstruction u1 on plane 1 with (px1, py1) and
(Ox1, Oy1); wavelength lambda, distance z, k = 2 pi / lambda,
S = p0 p1 / (lambda z).  Arrays are indexed [row, column] = [n, m], i.e. y
first, x second.

Readings taken where the paper is silent, ambiguous or garbled
--------------------------------------------------------------
R1 (grids, shift units).  The symbol list after Eq. (4) places the samples at
   x0 = m0 px0 + Ox0, while Eqs. (2)-(3) contain (-N/2 + O) p, i.e. a centred
   grid with the shift in pixels.  We take centred grids with shifts in
   metres: x[m] = (m - floor(N/2)) p + O.  Inside Eqs. (2)-(3) the shift then
   enters as O/p.
R2 (which N).  Eqs. (2)-(3) use one N for both planes (the paper has
   N0 = N1 = 1024).  The factorisation is exact only with the hologram size N0
   in Eq. (2) and the output size N1 in Eq. (3), per axis.
R3 (odd N).  floor(N/2), the FFT-shift centre.
R4 (padding, crop).  Steps 2 and 9 of Section 2.2 double the grid and "reduce
   the area".  Any padded length L >= N0 + N1 - 1 evaluates the same linear
   convolution: u0' occupies [0, N0), h[k] sits at k mod L for
   k in [-(N0-1), N1-1] (zero elsewhere), and [0, N1) is kept.
R5 (C1 and the area element).  The reported intensity keeps the full
   prefactor c(z) = exp(i k z) px0 py0 / (i lambda z): Eq. (2)'s constant
   times the hologram's area element, so that the sum approximates the
   Fresnel integral (the Gaussian-beam pin needs it).  Eq. (5) is |u1|^2 of
   that field.
R6 (FFT convention).  Forward FFT with exp(-2 pi i jk/L), inverse scaled by
   1/L per axis (numpy's convention).  The result does not depend on it.
R7 (sign of z).  z is the signed distance from plane 0 to plane 1; z < 0 is
   allowed and means back-propagation.  For a real hologram I(z) = I(-z).
R8 (the CCD resize, Section 3).  The 1360 x 1024 camera frame is resized to
   1024 x 1024 before reconstruction; the method is not named.  We take
   bilinear interpolation along x only (rows unchanged) with half-pixel
   centres: output sample c reads the frame at s = (c + 1/2) n_in / n_out - 1/2,
   clamped to [0, n_in - 1], so the output pitch is n_in / n_out times the
   camera's.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    """A sampled plane: nx x ny samples at pitch (px, py), shifted by (ox, oy).

    Units are metres.  Sample m along x sits at (m - floor(nx/2)) px + ox
    (reading R1 of the module docstring).
    """

    nx: int
    ny: int
    px: float
    py: float
    ox: float = 0.0
    oy: float = 0.0


def coords(n: int, p: float, o: float) -> np.ndarray:
    """Sample positions of one axis, Section 2.1 symbol list with reading R1."""
    m = np.arange(n, dtype=np.float64)
    return (m - (n // 2)) * p + o


def prefactor(src: Grid, wavelength: float, z: float) -> complex:
    """c(z) = exp(i k z) px0 py0 / (i lambda z): Eq. (2)'s constant with the
    hologram's area element (reading R5)."""
    k = 2.0 * np.pi / wavelength
    return complex(np.exp(1j * k * z) * src.px * src.py / (1j * wavelength * z))


def fresnel_matrix(n_out: int, p_out: float, o_out: float,
                   n_in: int, p_in: float, o_in: float,
                   wavelength: float, z: float) -> np.ndarray:
    """One axis of the Fresnel kernel, K[m1, m0] = exp(i pi (x1 - x0)^2 / (lambda z)).

    This is the plain definition behind Eq. (1): the convolution of the
    pre-chirped hologram with h (Eq. 4), times the chirps of Eqs. (2)-(3),
    recombines into this single quadratic phase of the sample separation.
    """
    x1 = coords(n_out, p_out, o_out)
    x0 = coords(n_in, p_in, o_in)
    d = x1[:, None] - x0[None, :]
    return np.exp(1j * np.pi * d * d / (wavelength * z))


def _kernels(src: Grid, dst: Grid, wavelength: float, z: float,
             rows=None, cols=None):
    kx = fresnel_matrix(dst.nx, dst.px, dst.ox, src.nx, src.px, src.ox, wavelength, z)
    ky = fresnel_matrix(dst.ny, dst.py, dst.oy, src.ny, src.py, src.oy, wavelength, z)
    if cols is not None:
        kx = kx[np.asarray(cols)]
    if rows is not None:
        ky = ky[np.asarray(rows)]
    return kx, ky


def direct(u0: np.ndarray, src: Grid, dst: Grid, wavelength: float, z: float,
           rows=None, cols=None) -> np.ndarray:
    """Reconstructed field u1 on ``dst`` (Eq. 1 evaluated as the sum it stands for).

    u1[n1, m1] = c(z) sum_{n0, m0} u0[n0, m0] exp(i pi ((x1-x0)^2 + (y1-y0)^2) / (lambda z)).
    The quadratic phase splits into an x factor and a y factor, so the double
    sum is the matrix product c Ky u0 Kx^T.  ``rows``/``cols`` restrict the
    output to a subset of (n1, m1) indices.
    """
    u0 = np.asarray(u0)
    assert u0.shape == (src.ny, src.nx), (u0.shape, src)
    kx, ky = _kernels(src, dst, wavelength, z, rows, cols)
    return prefactor(src, wavelength, z) * (ky @ u0.astype(np.complex128) @ kx.T)


def intensity(u1: np.ndarray) -> np.ndarray:
    """Eq. (5): I = |u1|^2."""
    return np.abs(u1) ** 2


def brute_force(u0: np.ndarray, src: Grid, dst: Grid, wavelength: float, z: float) -> np.ndarray:
    """The same sum as ``direct`` with one full 2D phase per (output, input)
    pair and no separation of axes.  For tiny grids only."""
    x0 = coords(src.nx, src.px, src.ox)
    y0 = coords(src.ny, src.py, src.oy)
    x1 = coords(dst.nx, dst.px, dst.ox)
    y1 = coords(dst.ny, dst.py, dst.oy)
    c = prefactor(src, wavelength, z)
    out = np.zeros((dst.ny, dst.nx), dtype=np.complex128)
    for n1 in range(dst.ny):
        for m1 in range(dst.nx):
            acc = 0.0 + 0.0j
            for n0 in range(src.ny):
                for m0 in range(src.nx):
                    r2 = (x1[m1] - x0[m0]) ** 2 + (y1[n1] - y0[n0]) ** 2
                    acc += u0[n0, m0] * np.exp(1j * np.pi * r2 / (wavelength * z))
            out[n1, m1] = c * acc
    return out


def fft_path(u0: np.ndarray, src: Grid, dst: Grid, wavelength: float, z: float,
             lx: int | None = None, ly: int | None = None) -> np.ndarray:
    """Steps 2-10 of Section 2.2 on an Lx x Ly zero-padded grid, FP64.

    Step 2: zero-pad to the padded grid (default: double the larger size, as
    the paper does).  Step 3: multiply u0 by the three exponentials of
    Eq. (3).  Step 4: forward FFT.  Step 5: sample h of Eq. (4) on the padded
    grid.  Step 6: its FFT.  Step 7: multiply.  Step 8: inverse FFT.  Step 9:
    keep the N1 region.  The constant C1 of Eq. (2) is applied last so that
    the field, not only the intensity, can be compared (step 10 is
    ``intensity`` of the result).  Readings R1, R2 and R4 fix the shift
    units, which N enters where, and where h and the crop sit.
    """
    lam = wavelength
    if lx is None:
        lx = 2 * max(src.nx, dst.nx)
    if ly is None:
        ly = 2 * max(src.ny, dst.ny)
    if lx < src.nx + dst.nx - 1 or ly < src.ny + dst.ny - 1:
        raise ValueError("padded size too small for a linear convolution")
    sx = src.px * dst.px / (lam * z)
    sy = src.py * dst.py / (lam * z)
    # Shifts in pixel units inside Eqs. (2)-(3) (reading R1), N0 in Eq. (2)
    # and N1 in Eq. (3) (reading R2).
    m0 = np.arange(src.nx, dtype=np.float64)
    n0 = np.arange(src.ny, dtype=np.float64)
    m1 = np.arange(dst.nx, dtype=np.float64)
    n1 = np.arange(dst.ny, dtype=np.float64)
    x0 = coords(src.nx, src.px, src.ox)
    y0 = coords(src.ny, src.py, src.oy)
    x1 = coords(dst.nx, dst.px, dst.ox)
    y1 = coords(dst.ny, dst.py, dst.oy)
    cx1 = -(dst.nx // 2) + dst.ox / dst.px  # (-N/2 + O_x1) of Eq. (3)
    cy1 = -(dst.ny // 2) + dst.oy / dst.py
    cx0 = -(src.nx // 2) + src.ox / src.px  # (-N/2 + O_x0) of Eq. (2)
    cy0 = -(src.ny // 2) + src.oy / src.py

    # Step 3: u0' of Eq. (3).
    e1 = np.exp(1j * np.pi / (lam * z) * (x0[None, :] ** 2 + y0[:, None] ** 2))
    e2 = np.exp(-2j * np.pi * (m0[None, :] * sx * cx1 + n0[:, None] * sy * cy1))
    e3 = np.exp(-1j * np.pi * (sx * m0[None, :] ** 2 + sy * n0[:, None] ** 2))
    u0p = np.asarray(u0, dtype=np.complex128) * e1 * e2 * e3

    # Step 2: zero padding, u0' at [0, N0).
    pad = np.zeros((ly, lx), dtype=np.complex128)
    pad[: src.ny, : src.nx] = u0p

    # Step 5: h of Eq. (4) at lags k in [-(N0-1), N1-1], stored at k mod L.
    kx = np.arange(-(src.nx - 1), dst.nx, dtype=np.int64)
    ky = np.arange(-(src.ny - 1), dst.ny, dtype=np.int64)
    hx = np.zeros(lx, dtype=np.complex128)
    hy = np.zeros(ly, dtype=np.complex128)
    hx[kx % lx] = np.exp(1j * np.pi * sx * kx.astype(np.float64) ** 2)
    hy[ky % ly] = np.exp(1j * np.pi * sy * ky.astype(np.float64) ** 2)
    h = hy[:, None] * hx[None, :]  # exp(i pi (Sx k^2 + Sy l^2)) on the padded grid

    # Steps 4, 6, 7, 8.
    conv = np.fft.ifft2(np.fft.fft2(pad) * np.fft.fft2(h))
    # Step 9: keep [0, N1).
    crop = conv[: dst.ny, : dst.nx]

    # C1 of Eq. (2), with the area element (reading R5).
    k = 2.0 * np.pi / lam
    c1 = (np.exp(1j * k * z) / (1j * lam * z)) * src.px * src.py
    c1 = c1 * np.exp(1j * np.pi / (lam * z) * (x1[None, :] ** 2 + y1[:, None] ** 2))
    c1 = c1 * np.exp(-2j * np.pi / (lam * z) * (cx0 * src.px * x1[None, :] + cy0 * src.py * y1[:, None]))
    c1 = c1 * np.exp(-1j * np.pi * (sx * m1[None, :] ** 2 + sy * n1[:, None] ** 2))
    return c1 * crop


def adjoint(g: np.ndarray, src: Grid, dst: Grid, wavelength: float, z: float) -> np.ndarray:
    """A^H g for the linear map u0 -> u1 of ``direct``: conj(c) Ky^H g conj(Kx).

    Returns an array on ``src``.  This is the conjugate transpose of the
    explicit matrices, with no reuse of the forward's factorisation.
    """
    g = np.asarray(g, dtype=np.complex128)
    assert g.shape == (dst.ny, dst.nx)
    kx, ky = _kernels(src, dst, wavelength, z)
    c = prefactor(src, wavelength, z)
    return np.conj(c) * (ky.conj().T @ g @ kx.conj())


def dfield_dz(u0: np.ndarray, src: Grid, dst: Grid, wavelength: float, z: float) -> np.ndarray:
    """d u1 / d z at fixed pitches and shifts, by the product rule on ``direct``.

    d/dz [c(z) exp(i pi r^2 / (lambda z))] = c exp(...) (i k - 1/z - i pi r^2 / (lambda z^2)),
    with r^2 = (x1 - x0)^2 + (y1 - y0)^2 split into its x and y parts.
    """
    lam = wavelength
    k = 2.0 * np.pi / lam
    u0c = np.asarray(u0, dtype=np.complex128)
    kx, ky = _kernels(src, dst, lam, z)
    dx2 = (coords(dst.nx, dst.px, dst.ox)[:, None] - coords(src.nx, src.px, src.ox)[None, :]) ** 2
    dy2 = (coords(dst.ny, dst.py, dst.oy)[:, None] - coords(src.ny, src.py, src.oy)[None, :]) ** 2
    c = prefactor(src, lam, z)
    u1 = c * (ky @ u0c @ kx.T)
    r2_term = c * (ky @ u0c @ (kx * dx2).T + (ky * dy2) @ u0c @ kx.T)
    return (1j * k - 1.0 / z) * u1 - (1j * np.pi / (lam * z * z)) * r2_term


def grads(u0: np.ndarray, src: Grid, dst: Grid, wavelength: float, z: float,
          grad_i: np.ndarray):
    """Gradients of a real loss L(I), I = |u1|^2, given grad_i = dL/dI.

    Returns (grad_u0, grad_z) in PyTorch's convention for complex tensors:
    grad = dL/dRe + i dL/dIm = 2 dL/d(conj u).  With g = 2 grad_i u1 (the
    gradient with respect to u1), grad_u0 = A^H g and
    dL/dz = Re sum conj(g) du1/dz.  For a real u0 PyTorch keeps Re(A^H g).
    """
    u1 = direct(u0, src, dst, wavelength, z)
    g = 2.0 * np.asarray(grad_i, dtype=np.float64) * u1
    gu = adjoint(g, src, dst, wavelength, z)
    if not np.iscomplexobj(u0):
        gu = gu.real
    gz = float(np.real(np.sum(np.conj(g) * dfield_dz(u0, src, dst, wavelength, z))))
    return gu, gz


def resize_x(frame: np.ndarray, n_out: int) -> np.ndarray:
    """The camera frame resized along x to n_out samples per row (Section 3's
    1360 -> 1024 resize; reading R8), in FP64: each output sample is the
    linear blend of the two input samples around its source position."""
    f = np.asarray(frame, dtype=np.float64)
    n_in = f.shape[-1]
    out = np.empty(f.shape[:-1] + (n_out,), dtype=np.float64)
    for c in range(n_out):
        s = (c + 0.5) * n_in / n_out - 0.5
        s = min(max(s, 0.0), n_in - 1.0)
        i0 = int(np.floor(s))
        i1 = min(i0 + 1, n_in - 1)
        t = s - i0
        out[..., c] = (1.0 - t) * f[..., i0] + t * f[..., i1]
    return out
