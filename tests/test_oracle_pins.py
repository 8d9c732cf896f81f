"""Pins of the FP64 oracle against facts other than itself (CPU only).

Each test states what it fixes.  Expected values are computed here from the
mathematics (closed forms, library convolution, invariants) with test-local
code, never by re-calling the oracle routine under test for its expectation.
"""

import json
import os

import numpy as np
import pytest
import scipy.signal

import oracle
from oracle import Grid

LAM = 632.8e-9
HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def axis(n, p, o=0.0):
    # Test-local copy of the grid reading: centred samples, shift in metres.
    return (np.arange(n) - n // 2) * p + o


TINY = [
    # (src grid, dst grid, z)
    (Grid(7, 5, 4.0e-6, 5.5e-6, 10e-6, -20e-6), Grid(6, 9, 2.0e-6, 7.0e-6, 50e-6, 30e-6), 0.004),
    (Grid(8, 6, 4.65e-6, 4.65e-6), Grid(7, 9, 1.5e-6, 3.0e-6, -80e-6, 40e-6), -0.006),
    (Grid(5, 5, 6e-6, 3e-6, 0.0, 0.0), Grid(5, 5, 6e-6, 3e-6, 0.0, 0.0), 0.003),
    (Grid(9, 4, 3e-6, 9e-6, -5e-6, 15e-6), Grid(3, 8, 11e-6, 2e-6, 0.0, -60e-6), 0.01),
]


@pytest.mark.parametrize("case", range(len(TINY)))
def test_p1_brute_force_direct_and_fft_path_agree(case):
    """P1: the separable sum, the unseparated 4-fold sum and the paper's
    padded-FFT steps 2-10 give the same field on tiny rectangular,
    anisotropic, shifted grids with N0 != N1 and either sign of z."""
    src, dst, z = TINY[case]
    rng = np.random.default_rng(case)
    u0 = rng.normal(size=(src.ny, src.nx)) + 1j * rng.normal(size=(src.ny, src.nx))
    bf = oracle.brute_force(u0, src, dst, LAM, z)
    d = oracle.direct(u0, src, dst, LAM, z)
    assert rel(d, bf) < 1e-12
    f = oracle.fft_path(u0, src, dst, LAM, z)
    assert rel(f, bf) < 1e-11
    # Any padded length >= N0 + N1 - 1 gives the same result (reading R4).
    lmin_x, lmin_y = src.nx + dst.nx - 1, src.ny + dst.ny - 1
    f2 = oracle.fft_path(u0, src, dst, LAM, z, lx=lmin_x, ly=lmin_y)
    f3 = oracle.fft_path(u0, src, dst, LAM, z, lx=lmin_x + 7, ly=3 * lmin_y)
    assert rel(f2, bf) < 1e-11 and rel(f3, bf) < 1e-11
    with pytest.raises(ValueError):
        oracle.fft_path(u0, src, dst, LAM, z, lx=lmin_x - 1, ly=lmin_y)


def test_p2_equal_pitch_is_textbook_impulse_response_convolution():
    """P2 (a): with equal pitches on both planes the sum is the discrete linear
    convolution of u0 with the sampled Fresnel impulse response
    c exp(i pi (x^2 + y^2) / (lambda z)), computed here by scipy's direct
    2D convolution."""
    p = 4.65e-6
    src = Grid(11, 8, p, p)
    dst = Grid(9, 13, p, p)
    z = 0.002
    rng = np.random.default_rng(7)
    u0 = rng.normal(size=(src.ny, src.nx)) + 1j * rng.normal(size=(src.ny, src.nx))
    dx = src.nx // 2 - dst.nx // 2
    dy = src.ny // 2 - dst.ny // 2
    sx = (np.arange(src.nx + dst.nx - 1) - (src.nx - 1) + dx) * p
    sy = (np.arange(src.ny + dst.ny - 1) - (src.ny - 1) + dy) * p
    k = np.exp(1j * np.pi * (sx[None, :] ** 2 + sy[:, None] ** 2) / (LAM * z))
    full = scipy.signal.convolve2d(u0, k, mode="full")
    c = np.exp(2j * np.pi * z / LAM) * p * p / (1j * LAM * z)
    expect = c * full[src.ny - 1: src.ny - 1 + dst.ny, src.nx - 1: src.nx - 1 + dst.nx]
    assert rel(oracle.direct(u0, src, dst, LAM, z), expect) < 1e-12


@pytest.mark.parametrize("zfac", [1.0, 1.5, 2.0])
def test_p2_matches_transfer_function_method_beyond_critical_distance(zfac):
    """P2 (b): for equal pitches and no shift, a compact Gaussian propagated by
    the ordinary Fresnel transfer-function method
    (H = exp(ikz) exp(-i pi lambda z (fx^2 + fy^2)) on a 2N padded grid)
    agrees with the impulse-response sum when z >= z_c = L p^2 / lambda (and
    the propagated beam still fits the padded window, so that the transfer
    function's periodic wrap-around stays negligible)."""
    n, p, w0 = 64, 4.65e-6, 20e-6
    lpad = 2 * n
    zc = lpad * p * p / LAM
    z = zfac * zc
    g = Grid(n, n, p, p)
    x = axis(n, p)
    u0 = np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / w0 ** 2)
    pad = np.zeros((lpad, lpad), complex)
    off = (lpad - n) // 2
    pad[off:off + n, off:off + n] = u0
    f = np.fft.fftfreq(lpad, p)
    h = np.exp(2j * np.pi * z / LAM) * np.exp(-1j * np.pi * LAM * z * (f[None, :] ** 2 + f[:, None] ** 2))
    tf = np.fft.ifft2(np.fft.fft2(pad) * h)[off:off + n, off:off + n]
    assert rel(oracle.direct(u0, g, g, LAM, z), tf) < 1e-9


@pytest.mark.parametrize("nx,ny", [(24, 24), (25, 18)])
def test_p3_natural_sampling_energy_and_round_trip(nx, ny):
    """P3: with S = 1/N on both axes (p1 = lambda z / (N p0)) the map is
    chirp x DFT x chirp: energy sum |u|^2 px py is conserved exactly and
    propagating back by -z onto the original grid is the identity, for any
    shifts."""
    z = 0.01
    src = Grid(nx, ny, 5e-6, 3e-6, 40e-6, -25e-6)
    dst = Grid(nx, ny, LAM * z / (nx * 5e-6), LAM * z / (ny * 3e-6), -300e-6, 120e-6)
    rng = np.random.default_rng(3)
    u0 = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    u1 = oracle.direct(u0, src, dst, LAM, z)
    e0 = np.sum(np.abs(u0) ** 2) * src.px * src.py
    e1 = np.sum(np.abs(u1) ** 2) * dst.px * dst.py
    assert abs(e1 / e0 - 1) < 1e-12
    back = oracle.direct(u1, dst, src, LAM, -z)
    assert rel(back, u0) < 1e-12


@pytest.mark.parametrize("n0,n1", [(256, 64), (255, 63)])
def test_p4_gaussian_beam_closed_form(n0, n1):
    """P4: u0 = exp(-(x^2 + y^2)/w0^2) propagates to
    u1 = exp(ikz)/(i lambda z) * pi/(a - ib) * exp(i a b (x1^2 + y1^2)/(a - ib)),
    a = 1/w0^2, b = pi/(lambda z): the continuous Fresnel integral of a
    Gaussian, evaluated on a rescaled, shifted output grid (odd sizes
    check the centring)."""
    p0, w0, z = 4.65e-6, 100e-6, 0.05
    src = Grid(n0, n0, p0, p0)
    dst = Grid(n1, n1, 8e-6, 8e-6, 300e-6, -150e-6)
    x0 = axis(n0, p0)
    u0 = np.exp(-(x0[None, :] ** 2 + x0[:, None] ** 2) / w0 ** 2)
    x1 = axis(n1, 8e-6, 300e-6)
    y1 = axis(n1, 8e-6, -150e-6)
    a, b = 1.0 / w0 ** 2, np.pi / (LAM * z)
    expect = (np.exp(2j * np.pi * z / LAM) / (1j * LAM * z) * np.pi / (a - 1j * b)
              * np.exp(1j * a * b * (x1[None, :] ** 2 + y1[:, None] ** 2) / (a - 1j * b)))
    got = oracle.direct(u0, src, dst, LAM, z)
    assert rel(got, expect) < 1e-12
    # The padded-FFT route reaches the same field at a smaller size.
    src_s = Grid(128, 128, p0, p0)
    xs = axis(128, p0)
    us = np.exp(-(xs[None, :] ** 2 + xs[:, None] ** 2) / (50e-6) ** 2)
    a2 = 1.0 / (50e-6) ** 2
    x1s = axis(32, 8e-6, 100e-6)
    y1s = axis(32, 8e-6, -60e-6)
    exp2 = (np.exp(2j * np.pi * z / LAM) / (1j * LAM * z) * np.pi / (a2 - 1j * b)
            * np.exp(1j * a2 * b * (x1s[None, :] ** 2 + y1s[:, None] ** 2) / (a2 - 1j * b)))
    fp = oracle.fft_path(us, src_s, Grid(32, 32, 8e-6, 8e-6, 100e-6, -60e-6), LAM, z)
    assert rel(fp, exp2) < 1e-11


def test_p5_common_shift_of_both_planes_changes_nothing():
    """P5: the kernel depends only on x1 - x0, so shifting both planes by the
    same distance leaves the field unchanged; the large, cancelling chirps of
    Eqs. (2)-(3) in the padded-FFT route must honour this."""
    src = Grid(10, 12, 4e-6, 6e-6, 10e-6, -30e-6)
    dst = Grid(14, 9, 2e-6, 3e-6, 50e-6, 70e-6)
    d = (1.3e-3, -0.7e-3)
    src2 = Grid(10, 12, 4e-6, 6e-6, 10e-6 + d[0], -30e-6 + d[1])
    dst2 = Grid(14, 9, 2e-6, 3e-6, 50e-6 + d[0], 70e-6 + d[1])
    rng = np.random.default_rng(5)
    u0 = rng.normal(size=(12, 10)) + 1j * rng.normal(size=(12, 10))
    z = 0.008
    ref = oracle.brute_force(u0, src, dst, LAM, z)
    assert rel(oracle.fft_path(u0, src2, dst2, LAM, z), ref) < 1e-9
    assert rel(oracle.direct(u0, src2, dst2, LAM, z), ref) < 1e-10


def test_p6_real_hologram_intensity_is_even_in_z():
    """P6: for a real hologram A(-z) u0 = conj(A(z) u0), so I(z) = I(-z)."""
    src = Grid(16, 12, 4.65e-6, 4.65e-6)
    dst = Grid(10, 14, 3e-6, 2e-6, 60e-6, -20e-6)
    u0 = np.random.default_rng(11).uniform(0, 2, (12, 16))
    up = oracle.direct(u0, src, dst, LAM, 0.02)
    um = oracle.direct(u0, src, dst, LAM, -0.02)
    assert rel(um, np.conj(up)) < 1e-12
    assert rel(oracle.intensity(um), oracle.intensity(up)) < 1e-12


def test_p7_adjoint_dot_test_and_reverse_propagation_identity():
    """P7: <A u, v> = <u, A^H v>, and A(z)^H = (px0 py0)/(px1 py1) A(-z) with
    the two planes swapped."""
    src = Grid(13, 11, 4e-6, 5e-6, 20e-6, 0.0)
    dst = Grid(9, 15, 2.5e-6, 6e-6, -40e-6, 90e-6)
    z = 0.012
    rng = np.random.default_rng(9)
    u = rng.normal(size=(11, 13)) + 1j * rng.normal(size=(11, 13))
    v = rng.normal(size=(15, 9)) + 1j * rng.normal(size=(15, 9))
    lhs = np.vdot(oracle.direct(u, src, dst, LAM, z), v)
    rhs = np.vdot(u, oracle.adjoint(v, src, dst, LAM, z))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12
    rev = oracle.direct(v, dst, src, LAM, -z) * (src.px * src.py) / (dst.px * dst.py)
    assert rel(oracle.adjoint(v, src, dst, LAM, z), rev) < 1e-12


def _loss(u0, src, dst, z, target):
    return float(np.sum((oracle.intensity(oracle.direct(u0, src, dst, LAM, z)) - target) ** 2))


@pytest.mark.parametrize("cplx", [True, False])
def test_p8_gradients_match_central_differences(cplx):
    """P8: dL/dz and the field gradient of L = sum (I - T)^2 agree with central
    finite differences (z step 1 um, field step 1e-3 along a random unit-RMS
    direction, each with Richardson extrapolation from half the step)."""
    src = Grid(12, 10, 4.65e-6, 4.65e-6)
    dst = Grid(11, 9, 3e-6, 4e-6, 30e-6, -10e-6)
    z = 0.004
    rng = np.random.default_rng(21)
    if cplx:
        u0 = np.exp(1j * rng.uniform(0, 2 * np.pi, (10, 12)))
    else:
        u0 = rng.uniform(0.5, 1.5, (10, 12))
    target = oracle.intensity(oracle.direct(u0 * 1.1, src, dst, LAM, z * 1.05))
    i0 = oracle.intensity(oracle.direct(u0, src, dst, LAM, z))
    gu, gz = oracle.grads(u0, src, dst, LAM, z, 2.0 * (i0 - target))

    def fd_z(h):
        return (_loss(u0, src, dst, z + h, target) - _loss(u0, src, dst, z - h, target)) / (2 * h)

    f1, f2 = fd_z(1e-6), fd_z(0.5e-6)
    rich = (4 * f2 - f1) / 3
    assert abs(gz - rich) / abs(rich) < 1e-5
    assert abs(f1 - f2) / abs(rich) < 1e-2  # the step is in the asymptotic range

    if cplx:
        d = rng.normal(size=u0.shape) + 1j * rng.normal(size=u0.shape)
    else:
        d = rng.normal(size=u0.shape)
    d /= np.sqrt(np.mean(np.abs(d) ** 2))
    def fd_u(h):
        return (_loss(u0 + h * d, src, dst, z, target) - _loss(u0 - h * d, src, dst, z, target)) / (2 * h)

    g1, g2 = fd_u(1e-3), fd_u(0.5e-3)
    fd = (4 * g2 - g1) / 3
    an = float(np.sum(np.real(np.conj(gu) * d)))
    assert abs(an - fd) / abs(fd) < 1e-7


def test_p9_paper_geometry():
    """P9: the wide view of Section 3 spans about 4.8 mm with 1024 samples at
    the CCD pitch, and the doubled grid of step 2 holds the linear
    convolution of two 1024-sample rows."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
    n = g["grid"]["value"]
    p = g["ccd_pitch_m"]["value"]
    x = oracle.coords(n, p, 0.0)
    side = x[-1] - x[0] + p
    assert round(side * 1e3, 1) == g["wide_view_side_m"]["value"] * 1e3
    assert g["padded_grid"]["value"] >= 2 * n - 1
    src = Grid(n, 8, p, p)
    assert src.nx == n
    # The Fig. 3 pitches are the CCD pitch over 1, 2 and 4.
    assert np.allclose(g["fig3_output_pitches_m"]["value"], [p, p / 2, p / 4])


def test_prefactor_and_intensity_definitions():
    """c(z) has modulus px0 py0 / (lambda |z|); Eq. (5) is |u1|^2."""
    src = Grid(4, 4, 3e-6, 7e-6)
    for z in (0.01, -0.03):
        c = oracle.prefactor(src, LAM, z)
        assert abs(abs(c) - 3e-6 * 7e-6 / (LAM * abs(z))) < 1e-18
    u = np.array([[3 + 4j]])
    assert oracle.intensity(u)[0, 0] == 25.0


# P10: the camera-frame resize (Section 3, reading R8) against a library
# routine with the same definition (bilinear, half-pixel centres), and its
# invariants: constants stay constant, a ramp stays a ramp away from the
# clamped ends, equal sizes are the identity.
@pytest.mark.parametrize("n_in,n_out", [(1360, 1024), (17, 40), (40, 17), (8, 8)])
def test_p10_resize_matches_library_bilinear(n_in, n_out):
    import torch
    r = np.random.default_rng(n_in + n_out)
    f = r.normal(size=(5, n_in))
    got = oracle.resize_x(f, n_out)
    ref = torch.nn.functional.interpolate(torch.from_numpy(f)[None, None], size=(5, n_out), mode="bilinear",
                                          align_corners=False)[0, 0].numpy()
    assert np.max(np.abs(got - ref)) < 1e-12
    assert np.allclose(oracle.resize_x(np.full((3, n_in), 2.5), n_out), 2.5, rtol=0, atol=1e-14)
    if n_in == n_out:
        assert np.array_equal(oracle.resize_x(f, n_out), f)


def test_p10_resize_keeps_ramps_inside():
    n_in, n_out = 1360, 1024
    ramp = 3.0 + 0.25 * np.arange(n_in)[None, :]
    got = oracle.resize_x(ramp, n_out)[0]
    s = (np.arange(n_out) + 0.5) * n_in / n_out - 0.5
    inside = (s >= 0) & (s <= n_in - 1)
    assert np.max(np.abs(got[inside] - (3.0 + 0.25 * s[inside]))) < 1e-10
