"""Shared test helpers: oracle evaluation of workload views and error metrics."""

import numpy as np

import oracle


def ogrid(g):
    return oracle.Grid(int(g.nx), int(g.ny), float(g.px), float(g.py), float(g.ox), float(g.oy))


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def max_rel(a, b) -> float:
    """Element-wise bound: max |a - b| over max |b|.  Unlike the relative L2
    it does not average a local mistake (a wrong crop edge, one bad row) over
    the whole view."""
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def oracle_field(w, v, z=None, rows=None, cols=None):
    view = w.views[v]
    return oracle.direct(w.holograms[view.holo], ogrid(w.holo_grid), ogrid(view.grid), w.wavelength,
                         view.z if z is None else z, rows=rows, cols=cols)


# Relative L2 bound for FP32 results against the FP64 oracle (the stated
# parity target of the method's single-precision path).
TOL = 1e-4

# Element-wise bound, max |gpu - oracle| / max |oracle|.  FP32 rounding of
# the chirp tables (2^-24 relative) and of the 4 log2 L butterfly levels of
# a view's transforms gives an absolute error of about
# sqrt(4 log2 L) 2^-24 times the rms of the field at every sample
# (~4e-7 rms at L = 2048); the largest sample of a view is at least its
# rms, so the bar leaves more than an order of magnitude for the tails of
# the error distribution.
ELEM_TOL = 1e-5


def check(got, ref, label, tol=TOL, elem_tol=ELEM_TOL):
    """Relative L2 and element-wise error of one result against the oracle;
    prints both and asserts the bars.  Returns (relative L2, element-wise)."""
    e = rel_l2(got, ref)
    m = max_rel(got, ref)
    print(f"{label}: rel L2 {e:.3e}, max elem {m:.3e}", flush=True)
    assert e <= tol and m <= elem_tol, (label, e, m)
    return e, m
