"""Adjoint and z-derivative on the GPU vs the FP64 oracle (GPU).

Checks, through the C-ABI: A^H g for a complex g against the oracle's
explicit conjugate-transpose product; the dot test <A u, g> = <u, A^H g>
between the GPU forward and backward; and the gradients of the intensity
loss L = sum (I - T)^2 with respect to the complex input field and to z,
against the oracle's product-rule derivative (itself pinned to finite
differences on the CPU).  Bar: relative L2 <= 1e-4 and max |error| /
max |oracle| <= 1e-4 for the adjoint and the field gradient (the gradient
of an intensity loss is formed from differences I - T of nearly equal
values, which raises the relative error of its small samples), relative
error <= 1e-4 for dL/dz.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.helpers import TOL, check, ogrid

pytestmark = pytest.mark.gpu

sfd = pytest.importorskip("paper_1001_4309_amd")
DEV = "cuda:0"
LAM = workloads.WAVELENGTH


def _case(seed, n_holo=2, views_per=2, n0=(20, 70), n1=(10, 60)):
    r = np.random.default_rng(500 + seed)
    _, g0, _, _ = workloads.random_case(seed, n0, n1, True)
    fields = np.stack([np.exp(1j * r.uniform(0, 2 * np.pi, (g0.ny, g0.nx))).astype(np.complex64)
                       for _ in range(n_holo)])
    views = []
    for h in range(n_holo):
        for _ in range(views_per):
            _, _, g1, z = workloads.random_case(int(r.integers(1 << 30)), n0, n1, True)
            views.append(workloads.ViewSpec(g1, z, h))
    return workloads.Workload(f"bwd{seed}", LAM, g0, fields, views)


def _plan(w, outputs="both"):
    return sfd.Plan(w.wavelength, w.holo_grid, len(w.holograms), w.views, outputs=outputs, complex_input=True,
                    device=DEV)


@pytest.mark.parametrize("seed", range(4))
def test_adjoint_of_complex_gradient_matches_oracle(seed):
    w = _case(seed)
    p = _plan(w, "field")
    r = np.random.default_rng(seed)
    gs = [(r.normal(size=(v.grid.ny, v.grid.nx)) + 1j * r.normal(size=(v.grid.ny, v.grid.nx))).astype(np.complex64)
          for v in w.views]
    holo = torch.from_numpy(w.holograms).to(DEV)
    grad_in, gz = p.backward([torch.from_numpy(g).to(DEV) for g in gs], holo, grad_z=False)
    torch.cuda.synchronize()
    assert gz is None
    src = ogrid(w.holo_grid)
    for h in range(len(w.holograms)):
        ref = sum(oracle.adjoint(gs[v], src, ogrid(view.grid), LAM, view.z)
                  for v, view in enumerate(w.views) if view.holo == h)
        check(grad_in[h].cpu().numpy(), ref, f"seed {seed} holo {h}: adjoint", elem_tol=TOL)


def test_dot_product_between_gpu_forward_and_backward():
    w = _case(7, n_holo=1, views_per=3, n0=(60, 120), n1=(40, 100))
    p = _plan(w, "field")
    r = np.random.default_rng(1)
    holo = torch.from_numpy(w.holograms).to(DEV)
    u1 = p.reconstruct(holo)
    gs = [torch.from_numpy((r.normal(size=(v.grid.ny, v.grid.nx)) + 1j * r.normal(size=(v.grid.ny, v.grid.nx)))
                           .astype(np.complex64)).to(DEV) for v in w.views]
    grad_in, _ = p.backward(gs, holo, grad_z=False)
    torch.cuda.synchronize()
    lhs = sum(np.vdot(u.cpu().numpy().astype(np.complex128), g.cpu().numpy()) for u, g in zip(u1, gs))
    rhs = np.vdot(holo.cpu().numpy()[0].astype(np.complex128), grad_in[0].cpu().numpy())
    # <A u, g> = <u, A^H g>, conjugated on both sides by vdot's convention.
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


def _intensity_loss_grads(w, targets, z=None):
    """Oracle field and z gradients of L = sum_v sum (|A_v u|^2 - T_v)^2."""
    src = ogrid(w.holo_grid)
    gu = np.zeros(w.holograms.shape, np.complex128)
    gz = []
    for v, view in enumerate(w.views):
        zz = view.z if z is None else z[v]
        u1 = oracle.direct(w.holograms[view.holo], src, ogrid(view.grid), LAM, zz)
        gi = 2.0 * (np.abs(u1) ** 2 - targets[v])
        a, b = oracle.grads(w.holograms[view.holo], src, ogrid(view.grid), LAM, zz, gi)
        gu[view.holo] += a
        gz.append(b)
    return gu, np.array(gz)


@pytest.mark.parametrize("seed", range(3))
def test_intensity_loss_gradients_match_oracle(seed):
    w = _case(20 + seed, n_holo=2, views_per=2)
    src = ogrid(w.holo_grid)
    r = np.random.default_rng(seed)
    targets = [np.abs(oracle.direct(w.holograms[v.holo] * 1.05, src, ogrid(v.grid), LAM, v.z * 1.02)) ** 2
               for v in w.views]
    ref_gu, ref_gz = _intensity_loss_grads(w, targets)
    p = _plan(w, "both")
    holo = torch.from_numpy(w.holograms).to(DEV)
    res = p.reconstruct(holo)
    nv = len(w.views)
    inten, u1 = res[:nv], res[nv:]
    gi = [2.0 * (inten[v] - torch.from_numpy(targets[v].astype(np.float32)).to(DEV)) for v in range(nv)]
    grad_in, gz = p.backward(gi, holo, field_out=u1)
    torch.cuda.synchronize()
    check(grad_in.cpu().numpy(), ref_gu, f"seed {seed}: field gradient", elem_tol=TOL)
    gz = gz.cpu().numpy()
    for v in range(nv):
        ez = abs(gz[v] - ref_gz[v]) / abs(ref_gz[v])
        print(f"seed {seed} view {v}: dL/dz {gz[v]:.6e} oracle {ref_gz[v]:.6e} rel {ez:.2e}", flush=True)
        assert ez <= TOL


def test_complex_gradient_mode_z_derivative():
    """dL/dz for a general complex g (no saved field): L = Re sum conj(q) u1 for a fixed q,
    so g = q and dL/dz = Re sum conj(q) du1/dz."""
    w = _case(40, n_holo=1, views_per=2)
    src = ogrid(w.holo_grid)
    r = np.random.default_rng(3)
    qs = [(r.normal(size=(v.grid.ny, v.grid.nx)) + 1j * r.normal(size=(v.grid.ny, v.grid.nx))) for v in w.views]
    p = _plan(w, "field")
    holo = torch.from_numpy(w.holograms).to(DEV)
    _, gz = p.backward([torch.from_numpy(q.astype(np.complex64)).to(DEV) for q in qs], holo)
    torch.cuda.synchronize()
    for v, view in enumerate(w.views):
        ref = float(np.real(np.sum(np.conj(qs[v]) * oracle.dfield_dz(w.holograms[0], src, ogrid(view.grid), LAM,
                                                                      view.z))))
        got = float(gz[v].cpu())
        print(f"view {v}: dL/dz {got:.6e} oracle {ref:.6e}", flush=True)
        assert abs(got - ref) / abs(ref) <= TOL


def test_autograd_function_config4():
    """The autograd path on the differentiation workload (sixteen 1024^2
    complex object fields, pitch 2.325 um -> 4.65 um, z in [3, 8] cm, the
    batch the bench times) against the oracle, field by field: the
    intensities, the field gradients and dL/dz."""
    w = workloads.config4()
    assert len(w.views) == 16
    src = ogrid(w.holo_grid)
    targets = []
    for b, view in enumerate(w.views):
        t = oracle.direct(w.extra["target_fields"][b], src, ogrid(view.grid), LAM, view.z + w.extra["deltas"][b])
        targets.append((np.abs(t) ** 2).astype(np.float32))
    p = _plan(w, "both")
    fields = torch.from_numpy(w.holograms).to(DEV).requires_grad_(True)
    z = torch.tensor([v.z for v in w.views], dtype=torch.float64, requires_grad=True)
    inten = sfd.SFDFunction.apply(fields, z, p)
    loss = sum(((i.double() - torch.from_numpy(t).to(DEV).double()) ** 2).sum() for i, t in zip(inten, targets))
    loss.backward()
    torch.cuda.synchronize()
    ref_gu, ref_gz = _intensity_loss_grads(w, targets)
    for b, view in enumerate(w.views):
        u1 = oracle.direct(w.holograms[view.holo], src, ogrid(view.grid), LAM, view.z)
        check(inten[b].detach().cpu().numpy(), oracle.intensity(u1), f"field {b}: intensity")
        check(fields.grad[b].cpu().numpy(), ref_gu[b], f"field {b}: field gradient", elem_tol=TOL)
        ez = abs(float(z.grad[b]) - ref_gz[b]) / abs(ref_gz[b])
        print(f"field {b}: dL/dz {float(z.grad[b]):.6e} oracle {ref_gz[b]:.6e} rel {ez:.2e}", flush=True)
        assert ez <= TOL


def test_backward_every_tile_width():
    """Forward and backward at the differentiation workload's shape (1024^2
    complex fields, L = 2048) under every tile width of both passes: the
    forward outputs and the field gradient bit for bit equal to the default
    schedule's; dL/dz, whose FP64 partial sums are grouped by tile, to 1e-12
    relative."""
    w = workloads.config4(batch=2)
    p = _plan(w, "both")
    holo = torch.from_numpy(w.holograms).to(DEV)
    r = np.random.default_rng(9)
    nv = len(w.views)
    targets = [torch.from_numpy(r.uniform(0, 1e-9, (v.grid.ny, v.grid.nx)).astype(np.float32)).to(DEV)
               for v in w.views]

    def run():
        res = p.reconstruct(holo)
        gi = [2.0 * (res[v] - targets[v]) for v in range(nv)]
        gin, gz = p.backward(gi, holo, field_out=res[nv:])
        torch.cuda.synchronize()
        return [t.clone() for t in res], gin.clone(), gz.clone()

    ref_res, ref_gin, ref_gz = run()
    lx, ly = p.lengths(0)
    assert (lx, ly) == (2048, 2048)
    for col, L in ((True, ly), (False, lx)):
        default = p.schedule()[("col" if col else "row", L)]
        for g, per_slot in sfd.sfd_tile_widths(L, col):
            p.set_schedule(L, col, g)
            res, gin, gz = run()
            for a, b in zip(res, ref_res):
                assert torch.equal(a, b), (col, g, per_slot)
            assert torch.equal(gin, ref_gin), (col, g, per_slot)
            rel = (gz - ref_gz).abs() / ref_gz.abs()
            print(f"col={col} width {g} ({per_slot} per slot): dL/dz max rel change {float(rel.max()):.2e}",
                  flush=True)
            assert float(rel.max()) <= 1e-12, (col, g, per_slot)
        p.set_schedule(L, col, default)


@pytest.mark.parametrize("n_holo,views_per", [(1, 1), (2, 2)])
def test_real_hologram_gradients(n_holo, views_per):
    """Real holograms (SFD_WITH_BACKWARD): the gradient of an intensity loss
    with respect to a real input is Re(A^H g), and dL/dz as for complex
    input; both against the oracle, through the autograd function."""
    r = np.random.default_rng(60 + n_holo)
    w0 = _case(70 + n_holo, n_holo=n_holo, views_per=views_per)
    holos = r.uniform(0.5, 1.5, w0.holograms.shape).astype(np.float32)
    w = workloads.Workload("bwd-real", LAM, w0.holo_grid, holos, w0.views)
    src = ogrid(w.holo_grid)
    targets = [(np.abs(oracle.direct(holos[v.holo] * 1.05, src, ogrid(v.grid), LAM, v.z * 1.02)) ** 2)
               .astype(np.float32) for v in w.views]
    p = sfd.Plan(LAM, w.holo_grid, n_holo, w.views, outputs="both", backward=True, device=DEV)
    fields = torch.from_numpy(holos).to(DEV).requires_grad_(True)
    z = torch.tensor([v.z for v in w.views], dtype=torch.float64, requires_grad=True)
    inten = sfd.SFDFunction.apply(fields, z, p)
    loss = sum(((i.double() - torch.from_numpy(t).to(DEV).double()) ** 2).sum() for i, t in zip(inten, targets))
    loss.backward()
    torch.cuda.synchronize()
    assert fields.grad.dtype == torch.float32
    ref_gu, ref_gz = _intensity_loss_grads(w, targets)
    assert not np.iscomplexobj(ref_gu) or np.allclose(ref_gu.imag, 0)
    for h in range(n_holo):
        check(fields.grad[h].cpu().numpy(), np.real(ref_gu[h]), f"real hologram {h}: field gradient", elem_tol=TOL)
    for v in range(len(w.views)):
        ez = abs(float(z.grad[v]) - ref_gz[v]) / abs(ref_gz[v])
        print(f"real view {v}: dL/dz {float(z.grad[v]):.6e} oracle {ref_gz[v]:.6e} rel {ez:.2e}", flush=True)
        assert ez <= TOL
