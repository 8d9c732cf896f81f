"""Batched Shifted-Fresnel reconstruction on AMD MI355X (gfx950).

Python binding of the C-ABI declared in ``include/sfd.h``.  The functions
``sfd_plan``, ``sfd_workspace_size``, ``sfd_view_lengths``, ``sfd_reconstruct``,
``sfd_backward`` and ``sfd_destroy`` marshal their arguments (torch tensors
become device pointers, the current torch stream becomes the HIP stream) and
call the library; every step of the computation runs in the library's HIP
kernels.  ``Plan`` bundles a plan handle with its workspace tensor, and
``SFDFunction`` exposes forward and backward to ``torch.autograd``.

The method: Shimobaba, Masuda, Ichihashi, Ito, "Real-time digital holographic
microscopy observable in multi-view and multi-resolution", Section 2
(Eqs. 1-5 and the per-view steps 2-10).
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import (SFD_EAGER, SFD_IN_C64, SFD_IN_REAL_F32, SFD_OUT_FIELD, SFD_OUT_INTENSITY,  # noqa: F401
                   SFD_PER_VIEW_LAUNCH, SFD_PHASE_FP32, SFD_REUSE_TABLES, SFD_SMOOTH_1280, SFD_SMOOTH_1536,
                   SFD_SMOOTH_1792, SFD_SMOOTH_ALL, SFD_WITH_BACKWARD, SfdError, SfdGrid, SfdView)

__all__ = ["Plan", "SFDFunction", "sfd_plan", "sfd_workspace_size", "sfd_view_lengths", "sfd_reconstruct",
           "sfd_backward", "sfd_autotune", "sfd_schedule", "sfd_set_schedule", "sfd_tile_widths",
           "sfd_stream_frame", "sfd_set_raw_input", "sfd_profile_enable", "sfd_profile_report", "sfd_destroy",
           "sfd_set_launch", "sfd_launch_mode", "sfd_sync_faults", "sfd_set_length_policy", "sfd_length_policy",
           "sfd_reconstruct_noalloc", "SfdError", "FrameStream"]


def _grid(g) -> SfdGrid:
    return SfdGrid(int(g.nx), int(g.ny), float(g.px), float(g.py), float(getattr(g, "ox", 0.0)),
                   float(getattr(g, "oy", 0.0)))


def _views(views) -> "ctypes.Array":
    arr = (SfdView * len(views))()
    for i, v in enumerate(views):
        arr[i] = SfdView(_grid(v.grid), float(v.z), int(getattr(v, "holo", 0)))
    return arr


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _ptr_array(ts) -> "ctypes.Array":
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


def _z_array(z):
    if z is None:
        return None
    z = [float(v) for v in z]
    return (ctypes.c_double * len(z))(*z)


# ---- C-ABI mirrors -------------------------------------------------------

def sfd_plan(wavelength: float, holo_grid, n_holo: int, views: Sequence, flags: int) -> ctypes.c_void_p:
    lib = _lib.load()
    h = ctypes.c_void_p()
    g = _grid(holo_grid)
    va = _views(views)
    _lib.check(lib.sfd_plan(ctypes.byref(h), float(wavelength), ctypes.byref(g), int(n_holo), va, len(views),
                            int(flags)))
    return h


def sfd_workspace_size(plan: ctypes.c_void_p) -> int:
    n = ctypes.c_size_t()
    _lib.check(_lib.load().sfd_workspace_size(plan, ctypes.byref(n)))
    return int(n.value)


def sfd_view_lengths(plan: ctypes.c_void_p, v: int):
    lx, ly = ctypes.c_int32(), ctypes.c_int32()
    _lib.check(_lib.load().sfd_view_lengths(plan, int(v), ctypes.byref(lx), ctypes.byref(ly)))
    return int(lx.value), int(ly.value)


def sfd_reconstruct(plan, holo: torch.Tensor, z, outs: Sequence[torch.Tensor], workspace: torch.Tensor) -> None:
    za = _z_array(z)
    _lib.check(_lib.load().sfd_reconstruct(plan, _ptr(holo), za, _ptr_array(outs), _ptr(workspace),
                                           workspace.numel() * workspace.element_size(),
                                           _stream_handle(holo.device)))


def sfd_reconstruct_noalloc(plan, holo: torch.Tensor, z, outs: Sequence[torch.Tensor]) -> None:
    """sfd_reconstruct on the library's static scratch array (no workspace,
    no allocation)."""
    za = _z_array(z)
    _lib.check(_lib.load().sfd_reconstruct_noalloc(plan, _ptr(holo), za, _ptr_array(outs),
                                                   _stream_handle(holo.device)))


def sfd_stream_frame(plan, host_frame: torch.Tensor, dev_holo: Sequence[torch.Tensor], outs: Sequence[torch.Tensor],
                     workspace: torch.Tensor) -> None:
    arr = (ctypes.c_void_p * 2)(_ptr(dev_holo[0]), _ptr(dev_holo[1]))
    _lib.check(_lib.load().sfd_stream_frame(plan, ctypes.c_void_p(host_frame.data_ptr()), arr, _ptr_array(outs),
                                            _ptr(workspace), workspace.numel() * workspace.element_size(),
                                            _stream_handle(dev_holo[0].device)))


def sfd_set_raw_input(plan, nx_raw: int, sample_bits: int = 32) -> None:
    _lib.check(_lib.load().sfd_set_raw_input(plan, int(nx_raw), int(sample_bits)))


_RAW_DTYPES = {32: torch.float32, 16: torch.uint16, 8: torch.uint8}


def sfd_backward(plan, grad_out: Sequence[torch.Tensor], field_out: Optional[Sequence[torch.Tensor]],
                 holo: torch.Tensor, z, grad_in: torch.Tensor, grad_z: Optional[torch.Tensor],
                 workspace: torch.Tensor) -> None:
    za = _z_array(z)
    fo = _ptr_array(field_out) if field_out is not None else None
    _lib.check(_lib.load().sfd_backward(plan, _ptr_array(grad_out), fo, _ptr(holo), za, _ptr(grad_in),
                                        _ptr(grad_z), _ptr(workspace),
                                        workspace.numel() * workspace.element_size(),
                                        _stream_handle(holo.device)))


def sfd_autotune(plan, holo: torch.Tensor, outs: Sequence[torch.Tensor], workspace: torch.Tensor,
                 reps: int = 5) -> None:
    _lib.check(_lib.load().sfd_autotune(plan, _ptr(holo), _ptr_array(outs), _ptr(workspace),
                                        workspace.numel() * workspace.element_size(), int(reps),
                                        _stream_handle(holo.device)))


def sfd_schedule(plan, L: int, col: bool) -> int:
    g = ctypes.c_int32()
    _lib.check(_lib.load().sfd_schedule(plan, int(L), 1 if col else 0, ctypes.byref(g)))
    return int(g.value)


def sfd_tile_widths(L: int, col: bool) -> list:
    """[(tile width, transforms per slot), ...] of the column (col) or row
    pass at transform length L, the default first (empty if L is not
    supported)."""
    return _lib.tile_widths(L, col)


def sfd_set_schedule(plan, L: int, col: bool, tile_width: int) -> None:
    _lib.check(_lib.load().sfd_set_schedule(plan, int(L), 1 if col else 0, int(tile_width)))


def sfd_profile_enable(plan, enable: bool) -> None:
    _lib.check(_lib.load().sfd_profile_enable(plan, 1 if enable else 0))


def sfd_profile_report(plan, kind: int):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _lib.check(_lib.load().sfd_profile_report(plan, int(kind), ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def sfd_set_launch(plan, mode: int) -> None:
    _lib.check(_lib.load().sfd_set_launch(plan, int(mode)))


def sfd_launch_mode(plan):
    """(mode, persistent launch available) with mode SFD_LAUNCH_PASSES (0) or
    SFD_LAUNCH_PERSISTENT (1)."""
    m, a = ctypes.c_int32(), ctypes.c_int32()
    _lib.check(_lib.load().sfd_launch_mode(plan, ctypes.byref(m), ctypes.byref(a)))
    return int(m.value), bool(a.value)


def sfd_set_length_policy(plan, smooth: int) -> None:
    """smooth: mask of SFD_SMOOTH_1280 | SFD_SMOOTH_1536 | SFD_SMOOTH_1792
    (0: powers of two only)."""
    _lib.check(_lib.load().sfd_set_length_policy(plan, int(smooth)))


def sfd_length_policy(plan) -> int:
    """Mask of the smooth lengths (1280, 1536, 1792) the plan may use where
    they are shorter than the next power of two."""
    v = ctypes.c_int32()
    _lib.check(_lib.load().sfd_length_policy(plan, ctypes.byref(v)))
    return int(v.value)


def sfd_sync_faults(plan, workspace: torch.Tensor, clear: bool = False) -> int:
    f = ctypes.c_uint32()
    _lib.check(_lib.load().sfd_sync_faults(plan, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                           1 if clear else 0, ctypes.byref(f), _stream_handle(workspace.device)))
    return int(f.value)


def sfd_destroy(plan) -> None:
    if plan:
        _lib.check(_lib.load().sfd_destroy(plan))


# ---- convenience wrapper ---------------------------------------------------

class Plan:
    """A plan plus its device workspace.

    ``views`` are objects with ``grid`` (nx, ny, px, py, ox, oy in metres),
    ``z`` (metres) and ``holo`` (hologram index) attributes.
    """

    def __init__(self, wavelength: float, holo_grid, n_holo: int, views: Sequence, *,
                 outputs: str = "intensity", complex_input: bool = False, phase_fp32: bool = False,
                 per_view_launch: bool = False, eager: bool = False, reuse_tables: bool = False,
                 raw_width: Optional[int] = None, raw_bits: int = 32, backward: bool = False, device=None):
        if outputs not in ("intensity", "field", "both"):
            raise ValueError("outputs must be 'intensity', 'field' or 'both'")
        self.device = torch.device(device if device is not None else "cuda")
        self.wavelength = float(wavelength)
        self.holo_grid = holo_grid
        self.n_holo = int(n_holo)
        self.views = list(views)
        self.outputs = outputs
        self.complex_input = complex_input
        out_flags = {"intensity": SFD_OUT_INTENSITY, "field": SFD_OUT_FIELD,
                     "both": SFD_OUT_INTENSITY | SFD_OUT_FIELD}[outputs]
        flags = (SFD_IN_C64 if complex_input else SFD_IN_REAL_F32) | out_flags
        if phase_fp32:
            flags |= SFD_PHASE_FP32
        if per_view_launch:
            flags |= SFD_PER_VIEW_LAUNCH
        if eager:
            flags |= SFD_EAGER
        if reuse_tables:
            flags |= SFD_REUSE_TABLES
        if backward and not complex_input:
            flags |= SFD_WITH_BACKWARD
        self.flags = flags
        self.handle = None
        self.handle = sfd_plan(wavelength, holo_grid, n_holo, self.views, flags)
        # Raw camera frames: rows of raw_width samples of raw_bits bits (float32,
        # or uint16 / uint8), converted and resized along x on the GPU.
        if raw_bits not in _RAW_DTYPES:
            raise ValueError("raw_bits must be 8, 16 or 32")
        self.raw_width = int(raw_width) if raw_width else holo_grid.nx
        self.input_dtype = torch.complex64 if complex_input else torch.float32
        if raw_width or raw_bits != 32:
            sfd_set_raw_input(self.handle, self.raw_width, raw_bits)
            self.input_dtype = _RAW_DTYPES[raw_bits]
        self.ws_bytes = sfd_workspace_size(self.handle)
        self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)

    def lengths(self, v: int):
        return sfd_view_lengths(self.handle, v)

    def autotune(self, holo: torch.Tensor, reps: int = 5, outs=None):
        """Time every tile width of every pass on this data and keep the
        fastest (see ``sfd_autotune``); returns the schedule."""
        holo = self._check_holo(holo)
        outs = self.new_outputs() if outs is None else outs
        sfd_autotune(self.handle, holo, outs, self.workspace, reps)
        return self.schedule()

    def set_schedule(self, L: int, col: bool, tile_width: int) -> None:
        sfd_set_schedule(self.handle, L, col, tile_width)

    def set_launch(self, persistent: bool) -> None:
        """One persistent launch per call, or the three pass launches."""
        sfd_set_launch(self.handle, _lib.SFD_LAUNCH_PERSISTENT if persistent else _lib.SFD_LAUNCH_PASSES)

    def launch_mode(self):
        """("persistent" | "passes", persistent launch available)."""
        m, avail = sfd_launch_mode(self.handle)
        return ("persistent" if m == _lib.SFD_LAUNCH_PERSISTENT else "passes"), avail

    def set_lengths(self, smooth) -> None:
        """Length policy: a mask of SFD_SMOOTH_* (True: all three smooth
        lengths, False: powers of two only); the workspace stays valid."""
        if isinstance(smooth, bool):
            smooth = _lib.SFD_SMOOTH_ALL if smooth else 0
        sfd_set_length_policy(self.handle, smooth)

    def length_policy(self) -> str:
        """"pow2", or "smooth:" and the smooth lengths allowed."""
        m = sfd_length_policy(self.handle)
        on = [str(L) for b, L in ((1, 1280), (2, 1536), (4, 1792)) if m & b]
        return "smooth:" + ",".join(on) if on else "pow2"

    def sync_faults(self, clear: bool = False) -> int:
        """Dependency waits of persistent launches that gave up on this
        workspace (0 in a correct run); synchronises."""
        return sfd_sync_faults(self.handle, self.workspace, clear)

    def schedule(self):
        """{(pass, L): tile width} with pass "col" (y transforms) or "row" (x transforms)."""
        out = {}
        for v in range(len(self.views)):
            lx, ly = self.lengths(v)
            out[("col", ly)] = sfd_schedule(self.handle, ly, True)
            out[("row", lx)] = sfd_schedule(self.handle, lx, False)
        return out

    def new_outputs(self):
        """Output tensors for one call: intensities, fields, or both (intensities first)."""
        def make(dt):
            return [torch.empty((v.grid.ny, v.grid.nx), dtype=dt, device=self.device) for v in self.views]
        if self.outputs == "intensity":
            return make(torch.float32)
        if self.outputs == "field":
            return make(torch.complex64)
        return make(torch.float32) + make(torch.complex64)

    def _check_holo(self, holo: torch.Tensor) -> torch.Tensor:
        g = self.holo_grid
        want = self.input_dtype
        if holo.dtype != want:
            raise TypeError(f"holograms must be {want}, got {holo.dtype}")
        if holo.device != self.device and not (holo.is_cuda and self.device.index is None):
            raise ValueError("holograms must be on the plan's device")
        nx = self.raw_width
        if tuple(holo.shape[-2:]) != (g.ny, nx) or holo.numel() != self.n_holo * g.ny * nx:
            raise ValueError(f"holograms must be [{self.n_holo}, {g.ny}, {nx}], got {tuple(holo.shape)}")
        return holo.contiguous()

    def _check_z(self, z):
        if z is not None and len(z) != len(self.views):
            raise ValueError(f"expected {len(self.views)} distances, got {len(z)}")

    def reconstruct(self, holo: torch.Tensor, z=None, outs=None):
        holo = self._check_holo(holo)
        self._check_z(z)
        if outs is None:
            outs = self.new_outputs()
        sfd_reconstruct(self.handle, holo, z, outs, self.workspace)
        return outs

    def reconstruct_noalloc(self, holo: torch.Tensor, z=None, outs=None):
        """As reconstruct, on the library's static scratch array instead of
        the plan's workspace (sfd_reconstruct_noalloc); ``outs`` must be
        given by callers that cannot allocate."""
        holo = self._check_holo(holo)
        self._check_z(z)
        if outs is None:
            outs = self.new_outputs()
        sfd_reconstruct_noalloc(self.handle, holo, z, outs)
        return outs

    def stream_frame(self, host_frame: torch.Tensor, dev_holo: Sequence[torch.Tensor], outs) -> None:
        """One frame of the real-time loop (``sfd_stream_frame``): copy
        ``host_frame`` (pinned CPU) into the next of ``dev_holo`` (two device
        buffers shaped like the holograms) and reconstruct it on the current
        stream into ``outs``; returns before either is done."""
        g = self.holo_grid
        want = self.input_dtype
        shape = (self.n_holo, g.ny, self.raw_width)
        if host_frame.dtype != want or host_frame.device.type != "cpu" or not host_frame.is_contiguous() \
                or host_frame.numel() != self.n_holo * g.ny * self.raw_width:
            raise ValueError(f"host_frame must be a contiguous CPU {want} tensor of shape {shape}")
        for d in dev_holo:
            self._check_holo(d)
            if not d.is_contiguous():
                raise ValueError("dev_holo buffers must be contiguous")
        sfd_stream_frame(self.handle, host_frame, dev_holo, outs, self.workspace)

    def backward(self, grad_out, holo, z=None, field_out=None, grad_z: bool = True):
        holo = self._check_holo(holo)
        self._check_z(z)
        g = self.holo_grid
        # Complex holograms get the complex gradient; real ones its real part.
        grad_in = torch.empty((self.n_holo, g.ny, g.nx), dtype=self.input_dtype, device=self.device)
        gz = torch.empty(len(self.views), dtype=torch.float64, device=self.device) if grad_z else None
        sfd_backward(self.handle, [t.contiguous() for t in grad_out],
                     None if field_out is None else [t.contiguous() for t in field_out],
                     holo, z, grad_in, gz, self.workspace)
        return grad_in, gz

    def profile(self, enable: bool = True) -> None:
        """Start (clearing earlier records) or stop event timing of the plan's kernels."""
        sfd_profile_enable(self.handle, enable)

    def profile_report(self):
        """{kind name: (launches, total ms)} since profiling was enabled."""
        return {name: sfd_profile_report(self.handle, k) for k, name in _lib.KERNEL_KIND_NAMES.items()}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                sfd_destroy(h)
            except Exception:
                pass
            self.handle = None


class SFDFunction(torch.autograd.Function):
    """I_v = |A_v(z_v) u_{holo(v)}|^2 for every view, differentiable in the
    input fields (complex, or real holograms) and in z.  ``plan`` must have
    ``outputs="both"`` (the library writes each intensity and keeps the field
    for the backward pass) and, for real input, ``backward=True``.  Returns
    one intensity tensor per view."""

    @staticmethod
    def forward(ctx, fields: torch.Tensor, z: torch.Tensor, plan: "Plan"):
        if plan.outputs != "both" or not (plan.complex_input or plan.flags & SFD_WITH_BACKWARD):
            raise ValueError("SFDFunction needs a plan with outputs='both' and complex_input=True or backward=True")
        zl = z.detach().to("cpu", torch.float64).tolist()
        res = plan.reconstruct(fields, zl)
        nv = len(plan.views)
        ctx.plan = plan
        ctx.zl = zl
        ctx.z_meta = (z.device, z.dtype)
        ctx.save_for_backward(fields)
        ctx.u1 = res[nv:]
        return tuple(res[:nv])

    @staticmethod
    def backward(ctx, *grad_i):
        (fields,) = ctx.saved_tensors
        plan = ctx.plan
        gi = [g if g is not None else torch.zeros_like(u, dtype=torch.float32) for g, u in zip(grad_i, ctx.u1)]
        grad_in, gz = plan.backward([g.to(torch.float32) for g in gi], fields, ctx.zl, field_out=ctx.u1)
        zdev, zdtype = ctx.z_meta
        return grad_in.view_as(fields), gz.to(zdev, zdtype), None


class FrameStream:
    """The real-time loop (Section 2.2, steps 1-11 for every captured frame):
    a plan made with ``reuse_tables=True`` (tables and spectra computed for
    the first frame only), two device hologram buffers and two sets of output
    buffers.  ``push(host_frame)`` enqueues one frame (its copy overlaps the
    previous frame's reconstruction) and returns the outputs it will write,
    valid once the current stream reaches them and until the frame after next
    is pushed."""

    def __init__(self, plan: "Plan"):
        if not plan.flags & SFD_REUSE_TABLES:
            raise ValueError("FrameStream needs a plan made with reuse_tables=True")
        self.plan = plan
        g = plan.holo_grid
        self.dev = [torch.empty((plan.n_holo, g.ny, plan.raw_width), dtype=plan.input_dtype, device=plan.device)
                    for _ in range(2)]
        self.outs = [plan.new_outputs() for _ in range(2)]
        self.count = 0

    def push(self, host_frame: torch.Tensor):
        outs = self.outs[self.count & 1]
        self.plan.stream_frame(host_frame, self.dev, outs)
        self.count += 1
        return outs
