"""Raw camera frames (Section 3: the 1360 x 1024 CCD frame resized to the
1024^2 hologram grid) resized on the GPU as they are copied for the column
pass, against the oracle's resize (reading R8, pinned to a library bilinear
routine) followed by its direct sum; and the same path through the streaming
entry point."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.helpers import TOL, ogrid, rel_l2

pytestmark = pytest.mark.gpu

sfd = pytest.importorskip("paper_1001_4309_amd")
DEV = "cuda:0"


def _oracle_views(w, frame):
    held = oracle.resize_x(frame[0], w.holo_grid.nx)
    src = ogrid(w.holo_grid)
    return [oracle.direct(held, src, ogrid(v.grid), w.wavelength, v.z) for v in w.views]


def test_config2_raw_ccd_frame():
    w = workloads.config2()
    ccd = w.extra["ccd"]
    assert ccd.shape == (1, 1024, 1360)
    p = sfd.Plan(w.wavelength, w.holo_grid, 1, w.views, outputs="both", raw_width=1360, device=DEV)
    res = p.reconstruct(torch.from_numpy(ccd).to(DEV))
    torch.cuda.synchronize()
    refs = _oracle_views(w, ccd)
    nv = len(w.views)
    for v in range(nv):
        ei = rel_l2(res[v].cpu().numpy(), oracle.intensity(refs[v]))
        ef = rel_l2(res[nv + v].cpu().numpy(), refs[v])
        print(f"raw frame view {v}: intensity rel L2 {ei:.3e}, field rel L2 {ef:.3e}", flush=True)
        assert ei <= TOL and ef <= TOL
    # The plain plan on the host-resized hologram agrees to rounding.
    q = sfd.Plan(w.wavelength, w.holo_grid, 1, w.views, outputs="both", device=DEV)
    held = torch.from_numpy(oracle.resize_x(ccd[0], 1024)[None].astype(np.float32)).to(DEV)
    res2 = q.reconstruct(held)
    torch.cuda.synchronize()
    for a, b in zip(res, res2):
        assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-5


def test_raw_frames_streamed():
    w = workloads.config2()
    ccd = w.extra["ccd"]
    p = sfd.Plan(w.wavelength, w.holo_grid, 1, w.views, raw_width=1360, reuse_tables=True, device=DEV)
    fs = sfd.FrameStream(p)
    r = np.random.default_rng(4)
    for k in range(3):
        frame = (ccd * r.uniform(0.9, 1.1, ccd.shape)).astype(np.float32)
        got = [t.clone() for t in fs.push(torch.from_numpy(frame).pin_memory())]
        torch.cuda.synchronize()
        ref = p.reconstruct(torch.from_numpy(frame).to(DEV))
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
    e = rel_l2(got[2].cpu().numpy(), oracle.intensity(_oracle_views(w, frame)[2]))
    print(f"streamed raw frame view 2 intensity rel L2 {e:.3e}", flush=True)
    assert e <= TOL


@pytest.mark.parametrize("n_in", [1000, 1100, 2000])
def test_raw_widths_rectangular(n_in):
    """Down- and up-sampling along x onto a 1024 x 300 hologram grid."""
    r = np.random.default_rng(n_in)
    g0 = workloads.GridSpec(1024, 300, 4.65e-6 * n_in / 1024, 4.65e-6)
    g1 = workloads.GridSpec(700, 200, 3e-6, 4e-6, 50e-6, -30e-6)
    frame = r.uniform(0, 2, (1, 300, n_in)).astype(np.float32)
    w = workloads.Workload("raw", workloads.WAVELENGTH, g0, frame, [workloads.ViewSpec(g1, 0.04, 0)])
    p = sfd.Plan(w.wavelength, g0, 1, w.views, raw_width=n_in, device=DEV)
    res = p.reconstruct(torch.from_numpy(frame).to(DEV))
    torch.cuda.synchronize()
    e = rel_l2(res[0].cpu().numpy(), oracle.intensity(_oracle_views(w, frame)[0]))
    print(f"raw width {n_in}: intensity rel L2 {e:.3e}", flush=True)
    assert e <= TOL


@pytest.mark.parametrize("bits", [8, 16])
def test_integer_camera_samples(bits):
    """8- and 16-bit camera frames (the samples taken at their value),
    converted and resized on the GPU, against the oracle on the same samples;
    and through the streaming entry point, whose copies then move 1 or 2
    bytes per sample."""
    w = workloads.config2()
    ccd = w.extra["ccd"]
    top = 255.0 if bits == 8 else 4095.0  # a 12-bit sensor in 16-bit words
    dt = np.uint8 if bits == 8 else np.uint16
    frame = np.clip(np.rint(ccd / ccd.max() * top), 0, top).astype(dt)
    p = sfd.Plan(w.wavelength, w.holo_grid, 1, w.views, raw_width=1360, raw_bits=bits, reuse_tables=True,
                 device=DEV)
    res = [t.clone() for t in p.reconstruct(torch.from_numpy(frame).to(DEV))]
    torch.cuda.synchronize()
    refs = _oracle_views(w, frame.astype(np.float64))
    for v in range(len(w.views)):
        e = rel_l2(res[v].cpu().numpy(), oracle.intensity(refs[v]))
        print(f"{bits}-bit frame view {v}: intensity rel L2 {e:.3e}", flush=True)
        assert e <= TOL
    fs = sfd.FrameStream(p)
    got = fs.push(torch.from_numpy(frame).pin_memory())
    torch.cuda.synchronize()
    for a, b in zip(got, res):
        assert torch.equal(a, b)
