"""Long transforms and the large workloads vs the FP64 oracle (GPU).

* padded lengths 4096 and 8192 on rectangular grids, where the x and y
  transforms of one view have different lengths, compared in full;
* the batched uneven workload (8 holograms of 1024^2, 64 views with
  N1 in {256, 512, 768, 1024}): every view from one batched call, a seeded
  sample of two views per size class against the oracle, and all 64 views
  bitwise against one launch sequence per view;
* the large workload (4096^2 hologram, eight 4096^2 views, L = 8192): two
  512^2 crops per view (centre and a seeded corner) against the oracle, for
  the FP64-reduced default and, reported only, the all-FP32 phase variant.

Bar: relative L2 <= 1e-4 per view (per crop) for the default path.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.helpers import TOL, oracle_field, rel_l2

pytestmark = pytest.mark.gpu

sfd = pytest.importorskip("paper_1001_4309_amd")
DEV = "cuda:0"


def _holo(w):
    return torch.from_numpy(np.ascontiguousarray(w.holograms)).to(DEV)


@pytest.mark.parametrize("shape,lengths", [
    ((1500, 300, 700, 200), (4096, 512)),
    ((300, 2500, 200, 3000), (512, 8192)),
    ((4000, 40, 4100, 30), (8192, 128)),
])
def test_long_transforms_rectangular(shape, lengths):
    n0x, n0y, n1x, n1y = shape
    r = np.random.default_rng(n0x + 3 * n0y)
    g0 = workloads.GridSpec(n0x, n0y, 4.65e-6, 3.5e-6, 30e-6, -20e-6)
    g1 = workloads.GridSpec(n1x, n1y, 3.0e-6, 5.0e-6, -200e-6, 120e-6)
    holo = r.uniform(0, 2, (n0y, n0x)).astype(np.float32)
    w = workloads.Workload("long", workloads.WAVELENGTH, g0, holo[None], [workloads.ViewSpec(g1, 0.04, 0)])
    p = sfd.Plan(w.wavelength, g0, 1, w.views, outputs="both", device=DEV)
    assert p.lengths(0) == lengths
    res = p.reconstruct(_holo(w))
    torch.cuda.synchronize()
    ref = oracle_field(w, 0)
    ei = rel_l2(res[0].cpu().numpy(), oracle.intensity(ref))
    ef = rel_l2(res[1].cpu().numpy(), ref)
    print(f"L={lengths}: intensity rel L2 {ei:.3e}, field rel L2 {ef:.3e}", flush=True)
    assert ei <= TOL and ef <= TOL


def _sample_views(w, per_class=2, seed=3):
    """Two views per output size class, seeded."""
    r = np.random.default_rng(seed)
    by_size = {}
    for v, view in enumerate(w.views):
        by_size.setdefault(view.grid.nx, []).append(v)
    picked = []
    for n in sorted(by_size):
        picked += sorted(r.choice(by_size[n], size=min(per_class, len(by_size[n])), replace=False).tolist())
    return picked


def test_config3_batched_uneven_views():
    w = workloads.config3()
    assert len(w.views) == 64 and len(w.holograms) == 8
    holo = _holo(w)
    a = sfd.Plan(w.wavelength, w.holo_grid, 8, w.views, device=DEV).reconstruct(holo)
    b = sfd.Plan(w.wavelength, w.holo_grid, 8, w.views, device=DEV, per_view_launch=True).reconstruct(holo)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    worst = 0.0
    for v in _sample_views(w):
        e = rel_l2(a[v].cpu().numpy(), oracle.intensity(oracle_field(w, v)))
        print(f"config3 view {v} (N1 {w.views[v].grid.nx}, holo {w.views[v].holo}): intensity rel L2 {e:.3e}",
              flush=True)
        worst = max(worst, e)
        assert e <= TOL
    print(f"config3 worst sampled rel L2 {worst:.3e}", flush=True)


def test_config5_large_crops_and_fp32_phase_report():
    w = workloads.config5()
    holo = _holo(w)
    n = w.holo_grid.nx
    c = 512
    r = np.random.default_rng(55)
    base = sfd.Plan(w.wavelength, w.holo_grid, 1, w.views, outputs="field", device=DEV)
    assert all(base.lengths(v) == (8192, 8192) for v in range(len(w.views)))
    u_a = base.reconstruct(holo)
    torch.cuda.synchronize()
    crops = []
    for v in range(len(w.views)):
        corner = [(0, 0), (0, n - c), (n - c, 0), (n - c, n - c)][int(r.integers(4))]
        crops.append([((n - c) // 2, (n - c) // 2), corner])
    refs = {}
    for v in range(len(w.views)):
        for (r0, c0) in crops[v]:
            rows, cols = np.arange(r0, r0 + c), np.arange(c0, c0 + c)
            ref = oracle_field(w, v, rows=rows, cols=cols)
            refs[(v, r0, c0)] = ref
            got = u_a[v][r0:r0 + c, c0:c0 + c].cpu().numpy()
            ef = rel_l2(got, ref)
            ei = rel_l2(np.abs(got) ** 2, oracle.intensity(ref))
            print(f"config5 view {v} crop ({r0},{c0}): field {ef:.3e} intensity {ei:.3e}", flush=True)
            assert ef <= TOL and ei <= TOL
    del u_a
    torch.cuda.empty_cache()
    fp32 = sfd.Plan(w.wavelength, w.holo_grid, 1, w.views, outputs="field", phase_fp32=True, device=DEV)
    u_b = fp32.reconstruct(holo)
    torch.cuda.synchronize()
    for v in range(len(w.views)):
        for (r0, c0) in crops[v]:
            got = u_b[v][r0:r0 + c, c0:c0 + c].cpu().numpy()
            eb = rel_l2(got, refs[(v, r0, c0)])
            print(f"config5 view {v} crop ({r0},{c0}): all-FP32 phases field {eb:.3e}", flush=True)
            assert np.isfinite(eb)
