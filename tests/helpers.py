"""Shared test helpers: oracle evaluation of workload views and error metrics."""

import numpy as np

import oracle


def ogrid(g):
    return oracle.Grid(int(g.nx), int(g.ny), float(g.px), float(g.py), float(g.ox), float(g.oy))


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def oracle_field(w, v, z=None, rows=None, cols=None):
    view = w.views[v]
    return oracle.direct(w.holograms[view.holo], ogrid(w.holo_grid), ogrid(view.grid), w.wavelength,
                         view.z if z is None else z, rows=rows, cols=cols)


# Relative L2 bound for FP32 results against the FP64 oracle (the stated
# parity target of the method's single-precision path).
TOL = 1e-4
