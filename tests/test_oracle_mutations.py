"""Planted mistakes in the oracle must trip at least one pin (CPU only).

Each mutation replaces one oracle function with a plausible slip (a dropped
term, a wrong sign or index, a transposed operand) and runs the pins; the
test passes only if some pin fails under the mutation.
"""

import numpy as np
import pytest

import oracle
import oracle.sfd_oracle as so
import tests.test_oracle_pins as pins

LAM = pins.LAM

ALL_PINS = [
    lambda: [pins.test_p1_brute_force_direct_and_fft_path_agree(i) for i in range(len(pins.TINY))],
    pins.test_p2_equal_pitch_is_textbook_impulse_response_convolution,
    lambda: [pins.test_p2_matches_transfer_function_method_beyond_critical_distance(f) for f in (1.0, 2.0)],
    lambda: [pins.test_p3_natural_sampling_energy_and_round_trip(*s) for s in ((24, 24), (25, 18))],
    lambda: [pins.test_p4_gaussian_beam_closed_form(*s) for s in ((256, 64), (255, 63))],
    pins.test_p5_common_shift_of_both_planes_changes_nothing,
    pins.test_p6_real_hologram_intensity_is_even_in_z,
    pins.test_p7_adjoint_dot_test_and_reverse_propagation_identity,
    lambda: [pins.test_p8_gradients_match_central_differences(c) for c in (True, False)],
    pins.test_prefactor_and_intensity_definitions,
]


def _some_pin_fails():
    failed = []
    for i, pin in enumerate(ALL_PINS):
        try:
            pin()
        except (AssertionError, ValueError):
            failed.append(i)
    return failed


def _orig(name):
    return getattr(so, name)


def m_phase_sign(n_out, p_out, o_out, n_in, p_in, o_in, wavelength, z):
    return np.conj(_ORIG["fresnel_matrix"](n_out, p_out, o_out, n_in, p_in, o_in, wavelength, z))


def m_no_area_element(src, wavelength, z):
    return _ORIG["prefactor"](src, wavelength, z) / (src.px * src.py)


def m_wrong_kz_sign(src, wavelength, z):
    k = 2 * np.pi / wavelength
    return complex(np.exp(-1j * k * z) * src.px * src.py / (1j * wavelength * z))


def m_ceil_centre(n, p, o):
    return (np.arange(n, dtype=np.float64) - (n + 1) // 2) * p + o


def m_transposed_operand(u0, src, dst, wavelength, z, rows=None, cols=None):
    kx, ky = so._kernels(src, dst, wavelength, z, rows, cols)
    u = np.asarray(u0, dtype=np.complex128)
    return so.prefactor(src, wavelength, z) * (ky @ u @ kx.T).T.reshape(dst.ny, dst.nx)


def m_pitch_swap(n_out, p_out, o_out, n_in, p_in, o_in, wavelength, z):
    return _ORIG["fresnel_matrix"](n_out, p_in, o_out, n_in, p_out, o_in, wavelength, z)


def m_adjoint_no_conj_c(g, src, dst, wavelength, z):
    kx, ky = so._kernels(src, dst, wavelength, z)
    return so.prefactor(src, wavelength, z) * (ky.conj().T @ np.asarray(g, complex) @ kx.conj())


def m_dz_drop_inv_z(u0, src, dst, wavelength, z):
    u1 = so.direct(u0, src, dst, wavelength, z)
    return _ORIG["dfield_dz"](u0, src, dst, wavelength, z) + u1 / z


def m_fft_path_wrong_n(u0, src, dst, wavelength, z, lx=None, ly=None):
    # Eq. (2)'s linear term built with the output size N1 where the
    # hologram size N0 belongs: (-N1/2 + O0/p0) p0 instead of
    # (-N0/2 + O0/p0) p0.  The constant C1 multiplies the cropped result, so
    # the slip is the correct result times
    # exp(-2 pi i (N0/2 - N1/2) p0 x1 / (lambda z)) per axis.
    good = _ORIG["fft_path"](u0, src, dst, wavelength, z, lx, ly)
    x1 = so.coords(dst.nx, dst.px, dst.ox)
    y1 = so.coords(dst.ny, dst.py, dst.oy)
    dx = (src.nx // 2 - dst.nx // 2) * src.px
    dy = (src.ny // 2 - dst.ny // 2) * src.py
    lz = wavelength * z
    return good * np.exp(-2j * np.pi / lz * (dx * x1[None, :] + dy * y1[:, None]))


_ORIG = {n: getattr(so, n) for n in ("fresnel_matrix", "prefactor", "coords", "direct",
                                      "adjoint", "dfield_dz", "fft_path")}

MUTATIONS = {
    "phase_sign": ("fresnel_matrix", m_phase_sign),
    "no_area_element": ("prefactor", m_no_area_element),
    "wrong_kz_sign": ("prefactor", m_wrong_kz_sign),
    "ceil_centre": ("coords", m_ceil_centre),
    "transposed_operand": ("direct", m_transposed_operand),
    "pitch_swap": ("fresnel_matrix", m_pitch_swap),
    "adjoint_no_conj_c": ("adjoint", m_adjoint_no_conj_c),
    "dz_drop_inv_z": ("dfield_dz", m_dz_drop_inv_z),
    "fft_path_wrong_n": ("fft_path", m_fft_path_wrong_n),
}


def test_unmutated_oracle_passes_every_pin():
    assert _some_pin_fails() == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(so, attr, fn)
    if hasattr(oracle, attr):
        monkeypatch.setattr(oracle, attr, fn)
    assert _some_pin_fails(), f"mutation {name} escaped every pin"
