"""The persistent launch (Section 2.2's steps 2-10 for every view of every
hologram in one kernel) against the FP64 oracle and, bit for bit, against
the three-launch schedule of the same plan (GPU).

Both schedules run the same transform bodies, the same spectrum transform
shape and the same chirp arithmetic, so they must agree exactly; the
persistent launch adds only the order in which workgroups take the items and
the completion counters between them.  Every test also checks that no
dependency wait gave up (the counters' error word stays zero).
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.helpers import check, oracle_field

pytestmark = pytest.mark.gpu

sfd = pytest.importorskip("paper_1001_4309_amd")
DEV = "cuda:0"


def _plan(w, **kw):
    return sfd.Plan(w.wavelength, w.holo_grid, len(w.holograms), w.views, device=DEV, **kw)


def _holo(w):
    return torch.from_numpy(np.ascontiguousarray(w.holograms)).to(DEV)


def _both_modes(p, holo, **kw):
    """(persistent results, pass-schedule results) of one plan, cloned."""
    assert p.launch_mode()[1]
    p.set_launch(True)
    a = [t.clone() for t in p.reconstruct(holo, **kw)]
    torch.cuda.synchronize()
    assert p.sync_faults() == 0
    p.set_launch(False)
    b = [t.clone() for t in p.reconstruct(holo, **kw)]
    torch.cuda.synchronize()
    p.set_launch(True)
    return a, b


def _small_1024():
    """A 512^2 hologram and views whose padded lengths are 1024 on both axes
    (the persistent launch's other length), rectangular and ragged."""
    r = np.random.default_rng(77)
    g0 = workloads.GridSpec(512, 512, 4.65e-6, 4.65e-6, 15e-6, -25e-6)
    views = [workloads.ViewSpec(workloads.GridSpec(512, 512, 3.0e-6, 3.0e-6), 0.02, 0),
             workloads.ViewSpec(workloads.GridSpec(384, 256, 6.0e-6, 2.5e-6, 300e-6, -120e-6), -0.035, 0),
             workloads.ViewSpec(workloads.GridSpec(7, 100, 9.0e-6, 4.0e-6, -50e-6, 80e-6), 0.05, 0)]
    holo = r.uniform(0, 2, (1, 512, 512)).astype(np.float32)
    return workloads.Workload("persist-1024", workloads.WAVELENGTH, g0, holo, views)


def test_availability():
    """Available for the paper's doubled grid at L = 2048 (new plans start
    persistent unless an autotune of the same shapes chose the passes)."""
    w2 = workloads.config2()
    assert _plan(w2).launch_mode()[1]
    assert _plan(w2, per_view_launch=True).launch_mode() == ("passes", False)
    w1 = workloads.config1()  # padded length 512: the pass schedule only
    p1 = _plan(w1)
    assert p1.launch_mode() == ("passes", False)
    with pytest.raises(sfd.SfdError):
        p1.set_launch(True)


@pytest.mark.parametrize("outputs", ["intensity", "field", "both"])
def test_config2_persistent_equals_passes_and_oracle(outputs):
    w = workloads.config2()
    p = _plan(w, outputs=outputs)
    a, b = _both_modes(p, _holo(w))
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    nv = len(w.views)
    for v in range(nv):
        ref = oracle_field(w, v)
        if outputs in ("intensity", "both"):
            check(a[v].cpu().numpy(), oracle.intensity(ref), f"persistent config2 view {v} intensity")
        if outputs in ("field", "both"):
            check(a[v if outputs == "field" else nv + v].cpu().numpy(), ref, f"persistent config2 view {v} field")


def test_length_1024_rectangular_views():
    w = _small_1024()
    p = _plan(w, outputs="both")
    assert all(p.lengths(v) == (1024, 1024) for v in range(len(w.views)))
    a, b = _both_modes(p, _holo(w))
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    nv = len(w.views)
    for v in range(nv):
        ref = oracle_field(w, v)
        check(a[v].cpu().numpy(), oracle.intensity(ref), f"L=1024 view {v} intensity")
        check(a[nv + v].cpu().numpy(), ref, f"L=1024 view {v} field")


def test_complex_input_and_several_holograms():
    """Complex holograms (the column pass's complex strips) on three
    holograms with two views each."""
    r = np.random.default_rng(5)
    w0 = _small_1024()
    fields = np.exp(1j * r.uniform(0, 2 * np.pi, (3, 512, 512))).astype(np.complex64)
    views = [workloads.ViewSpec(v.grid, v.z * (1 + 0.1 * h), h) for h in range(3) for v in w0.views[:2]]
    w = workloads.Workload("persist-complex", w0.wavelength, w0.holo_grid, fields, views)
    p = _plan(w, outputs="both", complex_input=True)
    a, b = _both_modes(p, _holo(w))
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    nv = len(w.views)
    for v in range(nv):
        check(a[nv + v].cpu().numpy(), oracle_field(w, v), f"complex holo {w.views[v].holo} view {v} field")


def test_graph_replays_eager_and_profiled_launches_agree():
    """The recorded graph replayed with eager device work and
    synchronisations between replays, with changed distances and new output
    buffers; the eager (unrecorded) persistent launch; and the profiled one
    (one launch of kind "persist" per call): all bit for bit equal."""
    w = workloads.config2()
    holo = _holo(w)
    eager = _plan(w, outputs="both", eager=True)
    graph = _plan(w, outputs="both")
    eager.set_launch(True)
    graph.set_launch(True)
    ref = [t.clone() for t in eager.reconstruct(holo)]
    z2 = [v.z * 1.1 for v in w.views]
    ref_z2 = [t.clone() for t in eager.reconstruct(holo, z=z2)]
    torch.cuda.synchronize()
    outs = graph.new_outputs()
    for rep in range(4):
        got = graph.reconstruct(holo, outs=outs)
        junk = torch.randn(1 << 20, device=DEV)
        _ = float(junk.sum())
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), rep
    got = graph.reconstruct(holo, z=z2, outs=outs)
    torch.cuda.synchronize()
    for a, b in zip(got, ref_z2):
        assert torch.equal(a, b)
    graph.profile(True)
    for _ in range(3):
        got = graph.reconstruct(holo)
    rep = graph.profile_report()
    graph.profile(False)
    assert rep["persist"][0] == 3 and rep["pass_x"][0] == 0 and rep["pass_y"][0] == 0
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    assert graph.sync_faults() == 0 and eager.sync_faults() == 0


def test_reused_tables_skip_setup_items():
    """A reuse_tables plan's second call runs no setup items (the columns do
    not wait for them) and still equals the plain plan bit for bit."""
    w = workloads.config2()
    holo = _holo(w)
    plain = [t.clone() for t in _plan(w).reconstruct(holo)]
    p = _plan(w, reuse_tables=True)
    p.set_launch(True)
    for _ in range(3):
        got = p.reconstruct(holo)
        torch.cuda.synchronize()
        for a, b in zip(got, plain):
            assert torch.equal(a, b)
    assert p.sync_faults() == 0


def test_raw_camera_frames_persistent():
    """8-bit 1360 x 1024 camera frames resized in the strip items equal the
    pass schedule's resize (in its hologram copy) bit for bit."""
    w = workloads.config2()
    ccd = w.extra["ccd"]
    q = np.clip(np.rint(ccd / ccd.max() * 255.0), 0, 255).astype(np.uint8)
    p = _plan(w, raw_width=1360, raw_bits=8)
    a, b = _both_modes(p, torch.from_numpy(q).to(DEV))
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_caller_captured_persistent_graph():
    w = workloads.config2()
    holo = _holo(w)
    p = _plan(w, outputs="both")
    p.set_launch(True)
    outs = p.new_outputs()
    ref = [t.clone() for t in p.reconstruct(holo, outs=outs)]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.reconstruct(holo, outs=outs)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs:
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), rep
    assert p.sync_faults() == 0


def test_many_consecutive_launches_stay_exact():
    """200 persistent launches in a row on one workspace, cycling over three
    hologram buffers and three sets of distances (so that column tiles find
    their spectra both ready and not yet ready, and the counters are reset
    by every launch's last workgroup): each result is bit-equal to the pass
    schedule's for the same input, and no dependency wait gives up."""
    w = workloads.config2()
    r = np.random.default_rng(9)
    base = np.ascontiguousarray(w.holograms).astype(np.float32)
    holos = [torch.from_numpy((base * r.uniform(0.8, 1.2, base.shape)).astype(np.float32)).to(DEV)
             for _ in range(3)]
    zs = [[v.z for v in w.views], [v.z * 1.1 for v in w.views], [-v.z for v in w.views]]
    p = _plan(w)
    p.set_launch(False)
    refs = {}
    for i in range(3):
        for j in range(3):
            refs[i, j] = [t.clone() for t in p.reconstruct(holos[i], z=zs[j])]
    torch.cuda.synchronize()
    p.set_launch(True)
    for k in range(200):
        i, j = k % 3, (k // 3) % 3
        got = p.reconstruct(holos[i], z=zs[j])
        for a, b in zip(got, refs[i, j]):
            assert torch.equal(a, b), (k, i, j)
    torch.cuda.synchronize()
    assert p.sync_faults() == 0
