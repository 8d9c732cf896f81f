"""HIP path vs the FP64 oracle, element by element, through the C-ABI (GPU).

Bar per view, for the intensity and, in field mode, for the complex field:
relative L2 <= 1e-4 and max |error| / max |oracle| <= 1e-5.  Sizes span several row tiles, ragged tails, odd and
rectangular grids, anisotropic pitches, shifts on both planes, N0 != N1 and
either sign of z; the paper-shaped 1024^2 views are compared in full.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.helpers import check, ogrid, oracle_field, rel_l2

pytestmark = pytest.mark.gpu

sfd = pytest.importorskip("paper_1001_4309_amd")
DEV = "cuda:0"


def _plan(w, **kw):
    return sfd.Plan(w.wavelength, w.holo_grid, len(w.holograms), w.views, device=DEV, **kw)


def _holo(w):
    return torch.from_numpy(np.ascontiguousarray(w.holograms)).to(DEV)


def _random_workload(seed, n0=(5, 90), n1=(5, 90), complex_input=False, n_views=3):
    r = np.random.default_rng(1000 + seed)
    u0, g0, g1, z = workloads.random_case(seed, n0, n1, complex_input)
    views = [workloads.ViewSpec(g1, z, 0)]
    for _ in range(n_views - 1):
        _, _, gv, zv = workloads.random_case(int(r.integers(1 << 30)), n0, n1, complex_input)
        views.append(workloads.ViewSpec(gv, zv, 0))
    return workloads.Workload(f"random{seed}", workloads.WAVELENGTH, g0, u0[None], views)


def _check(w, outputs, res, label):
    """Every view against the oracle: relative L2 and the element-wise bound,
    for the intensity and, in field mode, the complex field."""
    nv = len(w.views)
    worst = 0.0
    for v in range(nv):
        ref = oracle_field(w, v)
        if outputs in ("intensity", "both"):
            e, _ = check(res[v].cpu().numpy(), oracle.intensity(ref), f"{label} view {v} intensity")
            worst = max(worst, e)
        if outputs in ("field", "both"):
            k = v if outputs == "field" else nv + v
            e, _ = check(res[k].cpu().numpy(), ref, f"{label} view {v} field")
            worst = max(worst, e)
    return worst


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("outputs", ["intensity", "field", "both"])
def test_small_random_grids(seed, outputs):
    w = _random_workload(seed, complex_input=seed % 2 == 1)
    p = _plan(w, outputs=outputs, complex_input=seed % 2 == 1)
    res = p.reconstruct(_holo(w))
    torch.cuda.synchronize()
    _check(w, outputs, res, f"random{seed}")


@pytest.mark.parametrize("n0,n1", [(300, 200), (257, 511), (640, 130), (1, 1), (1, 63), (2, 3)])
def test_ragged_and_degenerate_sizes(n0, n1):
    r = np.random.default_rng(n0 * 7 + n1)
    g0 = workloads.GridSpec(n0, max(1, n0 // 2 + 1), 4.65e-6, 3.1e-6, 20e-6, -10e-6)
    g1 = workloads.GridSpec(n1, max(1, (n1 * 3) // 4), 2.5e-6, 6e-6, -150e-6, 75e-6)
    holo = r.uniform(0, 2, (g0.ny, g0.nx)).astype(np.float32)
    w = workloads.Workload("ragged", workloads.WAVELENGTH, g0, holo[None],
                           [workloads.ViewSpec(g1, 0.012, 0), workloads.ViewSpec(g1, -0.02, 0)])
    p = _plan(w, outputs="both")
    res = p.reconstruct(_holo(w))
    torch.cuda.synchronize()
    _check(w, "both", res, f"ragged{n0}x{n1}")


def test_config1_single_view():
    w = workloads.config1()
    for outputs in ("intensity", "field"):
        p = _plan(w, outputs=outputs)
        assert p.lengths(0) == (512, 512)
        res = p.reconstruct(_holo(w))
        torch.cuda.synchronize()
        _check(w, outputs, res, "config1")


def test_config2_paper_shaped_four_views():
    w = workloads.config2()
    p = _plan(w, outputs="both")
    assert all(p.lengths(v) == (2048, 2048) for v in range(4))
    res = p.reconstruct(_holo(w))
    torch.cuda.synchronize()
    worst = _check(w, "both", res, "config2")
    print(f"config2 worst rel L2 {worst:.3e}")


def test_batched_equals_per_view_launch():
    w = workloads.config2()
    holo = _holo(w)
    a = _plan(w).reconstruct(holo)
    b = _plan(w, per_view_launch=True).reconstruct(holo)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_z_override_and_repeated_calls():
    w = workloads.config1()
    p = _plan(w, outputs="field")
    holo = _holo(w)
    first = p.reconstruct(holo)[0].clone()
    z2 = 0.037
    second = p.reconstruct(holo, z=[z2])[0]
    third = p.reconstruct(holo)[0]
    torch.cuda.synchronize()
    ref2 = oracle_field(w, 0, z=z2)
    check(second.cpu().numpy(), ref2, "config1 z override")
    # Plan z again: bitwise identical to the first call.
    assert torch.equal(first, third)


@pytest.mark.parametrize("persistent", [False, True])
def test_alternating_inputs_keep_their_descriptors(persistent):
    """Calls that cycle over several input buffers (two descriptor slots, a
    recorded graph per slot): every call's result equals that of a fresh
    plan on the same input, bit for bit, and the oracle's."""
    w = workloads.config2()
    r = np.random.default_rng(41)
    base = np.ascontiguousarray(w.holograms).astype(np.float32)
    holos = [torch.from_numpy((base * r.uniform(0.8, 1.2, base.shape)).astype(np.float32)).to(DEV)
             for _ in range(3)]
    ref_plan = _plan(w)
    refs = [ref_plan.reconstruct(hh)[0].clone() for hh in holos]
    p = _plan(w)
    if persistent:
        p.set_launch(True)
    else:
        p.set_launch(False)
    for k in (0, 1, 0, 1, 2, 0, 2, 2, 1):
        got = p.reconstruct(holos[k])[0]
        torch.cuda.synchronize()
        assert torch.equal(got, refs[k]), (persistent, k)
    ref = oracle.intensity(oracle_field(workloads.Workload(w.name, w.wavelength, w.holo_grid,
                                                          holos[2].cpu().numpy(), w.views), 0))
    check(refs[2].cpu().numpy(), ref, "third input, view 0")


def test_fp32_phase_variant_runs_and_is_reported():
    """The all-FP32 phase variant is a comparison path: its error is printed,
    and it must stay finite; the FP64-reduced default must meet the bar."""
    w = workloads.config2()
    holo = _holo(w)
    a = _plan(w, outputs="field").reconstruct(holo)
    b = _plan(w, outputs="field", phase_fp32=True).reconstruct(holo)
    torch.cuda.synchronize()
    for v in range(len(w.views)):
        ref = oracle_field(w, v)
        check(a[v].cpu().numpy(), ref, f"config2 view {v} FP64-reduced phases")
        eb = rel_l2(b[v].cpu().numpy(), ref)
        print(f"config2 view {v}: all-FP32 phases rel L2 {eb:.3e}", flush=True)
        assert np.isfinite(eb)


def test_multiple_holograms_and_shared_views():
    w = workloads.config3(n_holo=3, views_per_holo=2, n=256)
    p = _plan(w, outputs="intensity")
    res = p.reconstruct(_holo(w))
    torch.cuda.synchronize()
    _check(w, "intensity", res, "multi-holo")


def test_graph_replays_equal_eager_launches():
    """Batched plans replay a recorded HIP graph; every replay, with eager
    device work and synchronisations between them, changed distances and new
    output buffers, must equal the directly launched kernels bit for bit."""
    w = workloads.config2()
    holo = _holo(w)
    eager = _plan(w, outputs="both", eager=True)
    graph = _plan(w, outputs="both")
    ref = [t.clone() for t in eager.reconstruct(holo)]
    z2 = [v.z * 1.1 for v in w.views]
    ref_z2 = [t.clone() for t in eager.reconstruct(holo, z=z2)]
    torch.cuda.synchronize()
    outs = graph.new_outputs()
    for rep in range(4):
        got = graph.reconstruct(holo, outs=outs)
        junk = torch.randn(1 << 20, device=DEV)
        _ = float(junk.sum())  # eager library work between replays
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), rep
    got = graph.reconstruct(holo, z=z2, outs=outs)
    torch.cuda.synchronize()
    for a, b in zip(got, ref_z2):
        assert torch.equal(a, b)
    fresh = graph.reconstruct(holo)  # new output buffers
    torch.cuda.synchronize()
    for a, b in zip(fresh, ref):
        assert torch.equal(a, b)


def _ragged(kind):
    """Padded length 2048 with a ragged side: ``out`` maps a 1024^2 hologram to
    a 1000^2 view (half-padded input, 1000 output rows: a partial last tile
    for every tile width); ``in`` maps a 1000^2 hologram to a 1024^2 view (no
    half-padded input, so the general kernels run, with several transforms
    per slot where the width has them)."""
    n0, n1 = (1024, 1000) if kind == "out" else (1000, 1024)
    r = np.random.default_rng(n0 + 7 * n1)
    g0 = workloads.GridSpec(n0, n0, 4.65e-6, 4.65e-6, 20e-6, -10e-6)
    g1 = workloads.GridSpec(n1, n1, 5.0e-6, 4.0e-6, 100e-6, -50e-6)
    holo = r.uniform(0, 2, (1, n0, n0)).astype(np.float32)
    return workloads.Workload(f"ragged-{kind}", workloads.WAVELENGTH, g0, holo, [workloads.ViewSpec(g1, 0.03, 0)])


@pytest.mark.parametrize("outputs", ["both", "intensity"])
@pytest.mark.parametrize("cfg", ["config1", "config2", "ragged-out", "ragged-in"])
def test_every_tile_width_gives_identical_results(cfg, outputs):
    """Each transform is computed the same way whichever workgroup holds it
    (and whichever slot of it, in whichever turn), so every schedule must
    reproduce the default bit for bit; the default is checked against the
    oracle for the ragged shapes."""
    w = _ragged(cfg.split("-")[1]) if cfg.startswith("ragged") else getattr(workloads, cfg)()
    holo = _holo(w)
    p = _plan(w, outputs=outputs)
    if p.launch_mode()[1]:
        p.set_launch(False)  # tile widths belong to the pass schedule
    ref = [t.clone() for t in p.reconstruct(holo)]
    torch.cuda.synchronize()
    lx, ly = p.lengths(0)
    if cfg.startswith("ragged"):
        assert (lx, ly) == (2048, 2048)
        _check(w, outputs, ref, cfg)
    for col, L in ((True, ly), (False, lx)):
        default = p.schedule()[("col" if col else "row", L)]
        shapes = sfd.sfd_tile_widths(L, col)
        assert shapes and shapes[0][0] == default
        for g, per_slot in shapes:
            p.set_schedule(L, col, g)
            got = p.reconstruct(holo)
            torch.cuda.synchronize()
            for a, b in zip(got, ref):
                assert torch.equal(a, b), (col, L, g, per_slot)
        p.set_schedule(L, col, default)


def test_autotune_keeps_results_and_seeds_new_plans():
    w = workloads.config2()
    holo = _holo(w)
    p = _plan(w)
    ref = [t.clone() for t in p.reconstruct(holo)]
    sched = p.autotune(holo, reps=3)
    print("tuned schedule", sched, flush=True)
    got = p.reconstruct(holo)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    assert _plan(w).schedule() == sched


def test_autotune_writes_the_schedule_cache(tmp_path, monkeypatch):
    """With SFD_TUNE_CACHE set, a tuned schedule is written to the JSON file
    under the plan's key (architecture, schedule version, shapes, flags),
    with the tile widths, launch mode and length policy the plan now uses."""
    import json

    path = tmp_path / "schedule.json"
    monkeypatch.setenv("SFD_TUNE_CACHE", str(path))
    w = workloads.config1()
    p = _plan(w)
    sched = p.autotune(_holo(w), reps=2)
    d = json.loads(path.read_text())
    assert d["format"] == "sfd-schedule-cache"
    entries = [e for k, e in d["entries"].items() if k.startswith("gfx950|") and "256x256/1/" in k]
    assert len(entries) == 1, d["entries"].keys()
    e = entries[0]
    for (kind, L), g in sched.items():
        assert e[kind][str(L)] == g
    assert e["persist"] == (1 if p.launch_mode()[0] == "persistent" else 0)
    assert e["smooth"] == sfd.sfd_length_policy(p.handle)


def test_caller_captured_graph_replays():
    """A caller that captures a reconstruction into its own graph (the
    library then launches into the capture): every replay, with eager work
    and synchronisations between replays, equals the eager result.  The
    eager calls between replays use the same arguments (the captured kernels
    read the descriptors those calls leave in the workspace)."""
    w = workloads.config1()
    holo = _holo(w)
    p = _plan(w, outputs="both")
    outs = p.new_outputs()
    ref = [t.clone() for t in p.reconstruct(holo, outs=outs)]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.reconstruct(holo, outs=outs)
    torch.cuda.synchronize()
    junk = torch.randn(1 << 16, device=DEV)
    for rep in range(4):
        for t in outs:
            t.zero_()
        _ = float(junk.sum())
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), rep
        for t in outs:
            t.zero_()
        p.reconstruct(holo, outs=outs)
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), rep
