"""FP64 CPU oracle for Shifted-Fresnel multi-view reconstruction.

TEST INFRASTRUCTURE ONLY.  This package is imported, called or executed only by
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py``.  The product path (``paper_1001_4309_amd`` and its HIP library)
never imports it, and it shares no code, table or constant with that path.

What it computes is fixed by Section 2.1 of the paper (Shimobaba, Masuda,
Ichihashi, Ito, "Real-time digital holographic microscopy observable in
multi-view and multi-resolution"): Eqs. (1)-(4) evaluate, by a chirp
factorisation, the discrete Fresnel sum of the hologram onto a scaled and
shifted output grid, and Eq. (5) takes its intensity.  The oracle writes that
sum out directly (``direct``, ``brute_force``) and, separately, follows the
paper's steps 2-10 of Section 2.2 on a zero-padded grid (``fft_path``).

Every function states the passage it follows; the readings taken where the
paper is silent or garbled are listed in ``sfd_oracle``'s module docstring.
Pins (``tests/test_oracle_pins.py``) tie the oracle to facts other than itself:
brute force, textbook special cases, a closed-form Gaussian beam, energy and
round-trip invariants, the adjoint identity and finite differences.
"""

from .sfd_oracle import (  # noqa: F401
    Grid,
    coords,
    prefactor,
    fresnel_matrix,
    direct,
    intensity,
    brute_force,
    fft_path,
    adjoint,
    dfield_dz,
    grads,
    resize_x,
)
