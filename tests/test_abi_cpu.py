"""The C-ABI library loads, exports every declared entry point, and validates
its arguments before touching the GPU (CPU only: no compute call is made)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfd.h")

lib_mod = pytest.importorskip("paper_1001_4309_amd._lib")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lib_mod.LIB_PATH):
        pytest.fail("libsfd.so is not built: run `python -m paper_1001_4309_amd.build`")
    return lib_mod.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:sfd_status|const char\*|int32_t|size_t)\s+(sfd_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sfd_plan", "sfd_workspace_size", "sfd_reconstruct", "sfd_backward", "sfd_destroy",
              "sfd_last_error"):
        assert n in names


def test_binding_flag_values_match_the_header():
    text = open(HEADER).read()
    flags = dict(re.findall(r"^\s*(SFD_[A-Z0-9_]+)\s*=\s*1u\s*<<\s*(\d+)", text, re.M))
    assert {"SFD_IN_REAL_F32", "SFD_IN_C64", "SFD_OUT_INTENSITY", "SFD_OUT_FIELD", "SFD_PHASE_FP32",
            "SFD_PER_VIEW_LAUNCH", "SFD_EAGER"} <= set(flags)
    for name, shift in flags.items():
        assert getattr(lib_mod, name) == 1 << int(shift), name
    kinds = dict(re.findall(r"^\s*(SFD_KERNEL_[A-Z_]+)\s*=\s*(\d+)", text, re.M))
    for name, value in kinds.items():
        assert getattr(lib_mod, name) == int(value), name
    smooth = dict(re.findall(r"(SFD_SMOOTH_[A-Z0-9]+)\s*=\s*(\d+)", text))
    assert len(smooth) == 4
    for name, value in smooth.items():
        assert getattr(lib_mod, name) == int(value), name


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), f"{n} declared in include/sfd.h but not exported"
    assert sorted(declared_functions()) == sorted(lib_mod.EXPORTED)


def test_tile_width_query(lib):
    """Every supported length has kernels for both passes, the default first;
    widths are distinct; transforms per slot divide the width; the argument
    checks and the unsupported-length answer."""
    for L in (64, 128, 256, 512, 1024, 1280, 1536, 1792, 2048, 4096, 8192):
        for col in (0, 1):
            w = (ctypes.c_int32 * 64)()
            p = (ctypes.c_int32 * 64)()
            n = lib.sfd_tile_widths(L, col, w, p, 64)
            assert n >= 1
            widths, per_slot = list(w[:n]), list(p[:n])
            assert len(set(widths)) == n
            assert all(g % q == 0 and q >= 1 for g, q in zip(widths, per_slot))
            one = (ctypes.c_int32 * 1)()
            assert lib.sfd_tile_widths(L, col, one, None, 1) == n and one[0] == widths[0]
            assert lib.sfd_tile_widths(L, col, None, None, 0) == n
    assert lib.sfd_tile_widths(1000, 0, None, None, 0) == 0
    assert lib.sfd_tile_widths(2048, 0, None, None, 4) == -1
    assert lib.sfd_tile_widths(2048, 0, None, None, -1) == -1
    # Several transforms per slot exist at the paper's padded length.
    assert any(q > 1 for _, q in lib_mod.tile_widths(2048, True))
    assert any(q > 1 for _, q in lib_mod.tile_widths(2048, False))


def _grid(nx=64, ny=48, px=4.65e-6, py=4.65e-6, ox=0.0, oy=0.0):
    return lib_mod.SfdGrid(nx, ny, px, py, ox, oy)


def _plan(lib, lam=632.8e-9, holo=None, n_holo=1, views=None, flags=None):
    holo = holo or _grid()
    if views is None:
        views = [lib_mod.SfdView(_grid(40, 30, 2e-6, 3e-6, 1e-4, -2e-4), 0.05, 0)]
    arr = (lib_mod.SfdView * len(views))(*views)
    if flags is None:
        flags = lib_mod.SFD_IN_REAL_F32 | lib_mod.SFD_OUT_INTENSITY
    h = ctypes.c_void_p()
    st = lib.sfd_plan(ctypes.byref(h), lam, ctypes.byref(holo), n_holo, arr, len(views), flags)
    return st, h


def test_valid_plan_sizes_and_lengths(lib):
    st, h = _plan(lib)
    assert st == lib_mod.SFD_OK
    n = ctypes.c_size_t()
    assert lib.sfd_workspace_size(h, ctypes.byref(n)) == lib_mod.SFD_OK
    assert n.value > 0 and n.value % 256 == 0
    lx, ly = ctypes.c_int32(), ctypes.c_int32()
    assert lib.sfd_view_lengths(h, 0, ctypes.byref(lx), ctypes.byref(ly)) == lib_mod.SFD_OK
    # Smallest supported padded length >= N0 + N1 - 1 on each axis.
    assert lx.value == 128 and ly.value == 128
    assert lib.sfd_view_lengths(h, 1, ctypes.byref(lx), ctypes.byref(ly)) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_destroy(h) == lib_mod.SFD_OK
    assert lib.sfd_destroy(None) == lib_mod.SFD_OK


def test_paper_size_uses_doubled_grid(lib):
    views = [lib_mod.SfdView(_grid(1024, 1024, 8e-6, 8e-6), 0.03, 0)]
    st, h = _plan(lib, holo=_grid(1024, 1024), views=views)
    assert st == lib_mod.SFD_OK
    lx, ly = ctypes.c_int32(), ctypes.c_int32()
    lib.sfd_view_lengths(h, 0, ctypes.byref(lx), ctypes.byref(ly))
    assert (lx.value, ly.value) == (2048, 2048)
    lib.sfd_destroy(h)


@pytest.mark.parametrize("mask,want", [(0, (2048, 2048)), (1, (1280, 2048)), (2, (1536, 1536)),
                                       (3, (1280, 1536)), (4, (1792, 1792)), (7, (1280, 1536))])
def test_length_policy_mask_picks_the_smallest_allowed_length(lib, mask, want):
    """Each axis takes the smallest length >= N0 + N1 - 1 that the mask
    allows (x: 1024 + 200 - 1 = 1223, y: 1024 + 500 - 1 = 1523)."""
    views = [lib_mod.SfdView(_grid(200, 500, 8e-6, 8e-6), 0.03, 0)]
    st, h = _plan(lib, holo=_grid(1024, 1024), views=views)
    assert st == lib_mod.SFD_OK
    lx, ly, m = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.sfd_length_policy(h, ctypes.byref(m)) == lib_mod.SFD_OK
    assert m.value == lib_mod.SFD_SMOOTH_1280
    assert lib.sfd_set_length_policy(h, mask) == lib_mod.SFD_OK
    lib.sfd_view_lengths(h, 0, ctypes.byref(lx), ctypes.byref(ly))
    assert (lx.value, ly.value) == want
    assert lib.sfd_set_length_policy(h, 8) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_set_length_policy(h, -1) == lib_mod.SFD_ERR_INVALID_ARG
    lib.sfd_destroy(h)


BAD = [
    ("wavelength zero", dict(lam=0.0)),
    ("wavelength nan", dict(lam=float("nan"))),
    ("holo pitch negative", dict(holo=_grid(px=-1e-6))),
    ("holo size zero", dict(holo=_grid(nx=0))),
    ("holo shift inf", dict(holo=_grid(ox=float("inf")))),
    ("n_holo zero", dict(n_holo=0)),
    ("z zero", dict(views=[lib_mod.SfdView(_grid(), 0.0, 0)])),
    ("z nan", dict(views=[lib_mod.SfdView(_grid(), float("nan"), 0)])),
    ("holo index", dict(views=[lib_mod.SfdView(_grid(), 0.01, 1)])),
    ("view pitch zero", dict(views=[lib_mod.SfdView(_grid(py=0.0), 0.01, 0)])),
    ("no input flag", dict(flags=lib_mod.SFD_OUT_INTENSITY)),
    ("two input flags", dict(flags=lib_mod.SFD_IN_REAL_F32 | lib_mod.SFD_IN_C64 | lib_mod.SFD_OUT_FIELD)),
    ("no output flag", dict(flags=lib_mod.SFD_IN_REAL_F32)),
    ("unknown flag", dict(flags=lib_mod.SFD_IN_REAL_F32 | lib_mod.SFD_OUT_FIELD | (1 << 20))),
]


@pytest.mark.parametrize("name,kw", BAD, ids=[b[0] for b in BAD])
def test_invalid_plans_are_rejected(lib, name, kw):
    st, h = _plan(lib, **kw)
    assert st == lib_mod.SFD_ERR_INVALID_ARG, name
    assert not h.value
    assert lib.sfd_last_error().decode()


def test_too_large_is_unsupported(lib):
    views = [lib_mod.SfdView(_grid(8000, 16, 1e-6, 1e-6), 0.01, 0)]
    st, h = _plan(lib, holo=_grid(1000, 16), views=views)
    assert st == lib_mod.SFD_ERR_UNSUPPORTED
    assert "8192" in lib.sfd_last_error().decode()


def test_reconstruct_validates_before_any_hip_call(lib):
    st, h = _plan(lib)
    assert st == lib_mod.SFD_OK
    n = ctypes.c_size_t()
    lib.sfd_workspace_size(h, ctypes.byref(n))
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails validation
    outs = (ctypes.c_void_p * 1)(1 << 21)
    null_outs = (ctypes.c_void_p * 1)(0)
    assert lib.sfd_reconstruct(None, fake, None, outs, fake, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_reconstruct(h, None, None, outs, fake, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_reconstruct(h, fake, None, null_outs, fake, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_reconstruct(h, fake, None, outs, None, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_reconstruct(h, fake, None, outs, ctypes.c_void_p((1 << 20) + 8), n.value,
                               None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_reconstruct(h, ctypes.c_void_p((1 << 20) + 4), None, outs, fake, n.value,
                               None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_reconstruct(h, fake, None, outs, fake, n.value - 1, None) == lib_mod.SFD_ERR_WORKSPACE
    zbad = (ctypes.c_double * 1)(0.0)
    assert lib.sfd_reconstruct(h, fake, zbad, outs, fake, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    lib.sfd_destroy(h)


def test_backward_validates_before_any_hip_call(lib):
    st, h = _plan(lib, flags=lib_mod.SFD_IN_C64 | lib_mod.SFD_OUT_FIELD)
    assert st == lib_mod.SFD_OK
    n = ctypes.c_size_t()
    lib.sfd_workspace_size(h, ctypes.byref(n))
    fake = ctypes.c_void_p(1 << 20)
    g = (ctypes.c_void_p * 1)(1 << 21)
    assert lib.sfd_backward(h, g, None, fake, None, fake, None, fake, n.value - 1,
                            None) == lib_mod.SFD_ERR_WORKSPACE
    assert lib.sfd_backward(h, None, None, fake, None, fake, None, fake, n.value,
                            None) == lib_mod.SFD_ERR_INVALID_ARG
    lib.sfd_destroy(h)


def test_last_error_is_cleared_on_success(lib):
    _plan(lib, lam=-1.0)
    assert lib.sfd_last_error().decode()
    st, h = _plan(lib)
    assert st == lib_mod.SFD_OK and lib.sfd_last_error().decode() == ""
    lib.sfd_destroy(h)


def test_schedule_queries_and_manual_setting(lib):
    """Tile widths: defaults, the allowed set per length, rejection of others,
    and a workspace size that does not depend on the schedule."""
    views = [lib_mod.SfdView(_grid(1024, 1024, 8e-6, 8e-6), 0.03, 0)]
    st, h = _plan(lib, holo=_grid(1024, 1024), views=views)
    assert st == 0
    g = ctypes.c_int32()
    assert lib.sfd_schedule(h, 2048, 1, ctypes.byref(g)) == 0 and g.value == 8
    assert lib.sfd_schedule(h, 2048, 0, ctypes.byref(g)) == 0 and g.value == 2
    assert lib.sfd_schedule(h, 1024, 1, ctypes.byref(g)) == lib_mod.SFD_ERR_INVALID_ARG
    n0 = ctypes.c_size_t()
    assert lib.sfd_workspace_size(h, ctypes.byref(n0)) == 0
    for col, width in ((1, 4), (1, 2), (1, 16), (0, 1), (0, 4), (0, 8), (0, 16)):
        assert lib.sfd_set_schedule(h, 2048, col, width) == 0
        assert lib.sfd_schedule(h, 2048, col, ctypes.byref(g)) == 0 and g.value == width
        n = ctypes.c_size_t()
        assert lib.sfd_workspace_size(h, ctypes.byref(n)) == 0 and n.value == n0.value
    assert lib.sfd_set_schedule(h, 2048, 1, 3) == lib_mod.SFD_ERR_INVALID_ARG
    assert b"tile width 3" in lib.sfd_last_error()
    assert lib.sfd_set_schedule(h, 2048, 0, 32) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_set_schedule(h, 4096, 1, 2) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_destroy(h) == 0


def test_autotune_validates_before_any_hip_call(lib):
    st, h = _plan(lib)
    assert st == 0
    n = ctypes.c_size_t()
    lib.sfd_workspace_size(h, ctypes.byref(n))
    out = (ctypes.c_void_p * 1)(4096)
    assert lib.sfd_autotune(h, ctypes.c_void_p(4096), out, ctypes.c_void_p(0), n.value, 3, None) == \
        lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_autotune(h, ctypes.c_void_p(4096), out, ctypes.c_void_p(256), n.value, 0, None) == \
        lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_autotune(h, ctypes.c_void_p(4096), out, ctypes.c_void_p(256), 0, 3, None) == \
        lib_mod.SFD_ERR_WORKSPACE
    assert lib.sfd_destroy(h) == 0


def test_stream_frame_validates_before_any_hip_call(lib):
    flags = lib_mod.SFD_IN_REAL_F32 | lib_mod.SFD_OUT_INTENSITY | lib_mod.SFD_REUSE_TABLES
    st, h = _plan(lib, flags=flags)
    assert st == 0
    n = ctypes.c_size_t()
    lib.sfd_workspace_size(h, ctypes.byref(n))
    out = (ctypes.c_void_p * 1)(4096)
    ws = ctypes.c_void_p(256)
    two = (ctypes.c_void_p * 2)(4096, 8192)
    same = (ctypes.c_void_p * 2)(4096, 4096)
    host = ctypes.c_void_p(4096)
    assert lib.sfd_stream_frame(h, None, two, out, ws, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_stream_frame(h, host, None, out, ws, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_stream_frame(h, host, same, out, ws, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    assert b"two distinct" in lib.sfd_last_error()
    assert lib.sfd_stream_frame(h, host, two, out, ws, 0, None) == lib_mod.SFD_ERR_WORKSPACE
    assert lib.sfd_destroy(h) == 0
    st, h = _plan(lib, flags=flags | lib_mod.SFD_PER_VIEW_LAUNCH)
    assert st == 0
    lib.sfd_workspace_size(h, ctypes.byref(n))
    assert lib.sfd_stream_frame(h, host, two, out, ws, n.value, None) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_destroy(h) == 0
    # Unknown flag bits are still refused.
    st, _ = _plan(lib, flags=lib_mod.SFD_IN_REAL_F32 | lib_mod.SFD_OUT_INTENSITY | (1 << 9))
    assert st == lib_mod.SFD_ERR_INVALID_ARG


def test_raw_input_validation(lib):
    st, h = _plan(lib)
    assert st == 0
    assert lib.sfd_set_raw_input(h, -1, 32) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_set_raw_input(h, 70000, 32) == lib_mod.SFD_ERR_INVALID_ARG
    assert lib.sfd_set_raw_input(h, 85, 12) == lib_mod.SFD_ERR_INVALID_ARG
    assert b"sample_bits" in lib.sfd_last_error()
    for bits in (8, 16, 32):
        assert lib.sfd_set_raw_input(h, 85, bits) == 0
    assert lib.sfd_set_raw_input(h, 0, 32) == 0
    assert lib.sfd_destroy(h) == 0
    st, h = _plan(lib, flags=lib_mod.SFD_IN_C64 | lib_mod.SFD_OUT_FIELD)
    assert st == 0
    assert lib.sfd_set_raw_input(h, 85, 32) == lib_mod.SFD_ERR_INVALID_ARG
    assert b"real-input" in lib.sfd_last_error()
    assert lib.sfd_destroy(h) == 0


def test_noalloc_rejects_plans_larger_than_its_scratch(lib):
    """The no-allocation entry point checks the plan's workspace against its
    static array before any HIP call: the 64-view batch (370 MiB) does not
    fit the 64 MiB array."""
    import workloads
    import paper_1001_4309_amd as sfd

    assert lib.sfd_noalloc_capacity() == 64 << 20
    w = workloads.config3()
    h = sfd.sfd_plan(w.wavelength, w.holo_grid, len(w.holograms), w.views,
                     lib_mod.SFD_IN_REAL_F32 | lib_mod.SFD_OUT_INTENSITY)
    try:
        assert sfd.sfd_workspace_size(h) > lib.sfd_noalloc_capacity()
        outs = (ctypes.c_void_p * len(w.views))(*([16] * len(w.views)))
        st = lib.sfd_reconstruct_noalloc(h, ctypes.c_void_p(16), None, outs, None)
        assert st == lib_mod.SFD_ERR_WORKSPACE
        assert b"scratch" in lib.sfd_last_error()
        assert lib.sfd_reconstruct_noalloc(None, ctypes.c_void_p(16), None, outs, None) == lib_mod.SFD_ERR_INVALID_ARG
    finally:
        sfd.sfd_destroy(h)


def test_schedule_cache_file_seeds_plans_and_corrupt_files_are_ignored(lib, tmp_path, monkeypatch):
    """SFD_TUNE_CACHE: a plan whose key (architecture, schedule version,
    hologram grid and count, flags, view sizes) is in the file starts from
    its schedule; an unreadable file is ignored (defaults)."""
    import json

    import workloads
    import paper_1001_4309_amd as sfd

    flags = lib_mod.SFD_IN_REAL_F32 | lib_mod.SFD_OUT_INTENSITY
    w = workloads.config2()
    g = w.holo_grid
    sig = f"{g.nx}x{g.ny}/1/{flags}" + "".join(f";{v.grid.nx}x{v.grid.ny}@{v.holo}" for v in w.views)
    path = tmp_path / "schedule.json"
    path.write_text(json.dumps({"format": "sfd-schedule-cache", "version": 2, "entries": {
        "gfx950|v2|" + sig: {"col": {"2048": 4}, "row": {"2048": 16}, "persist": 0, "smooth": 1}}}))
    monkeypatch.setenv("SFD_TUNE_CACHE", str(path))
    h = sfd.sfd_plan(w.wavelength, g, 1, w.views, flags)
    try:
        assert sfd.sfd_schedule(h, 2048, True) == 4
        assert sfd.sfd_schedule(h, 2048, False) == 16
        assert sfd.sfd_launch_mode(h) == (lib_mod.SFD_LAUNCH_PASSES, True)
    finally:
        sfd.sfd_destroy(h)
    # Another shape, unreadable file: the defaults.
    path.write_text("{\"format\": \"sfd-schedule-cache\", \"entries\": {oops")
    w1 = workloads.config1()
    h = sfd.sfd_plan(w1.wavelength, w1.holo_grid, 1, w1.views, flags)
    try:
        for col in (True, False):
            assert sfd.sfd_schedule(h, 512, col) == sfd.sfd_tile_widths(512, col)[0][0]
    finally:
        sfd.sfd_destroy(h)
