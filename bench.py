#!/usr/bin/env python3
"""Throughput of batched Shifted-Fresnel reconstruction on one MI355X.

One step = one pass of the whole reconstruction path over one batch: chirp
tables (Eqs. 2-4), kernel spectra, the fused x and y row passes, crop and
intensity, for every view of the batch.  The default workload is the
paper-shaped one: a 1024 x 1024 synthetic in-line hologram (1360 x 1024
CCD-like field of 64 point scatterers, bilinearly resized), four 1024 x 1024
views with their own depth, pitch and shift, padded length 2048.

Prints ONE JSON line on stdout; everything else goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "views/s (1024² hologram→1024² view) + % HBM peak; batched vs per-view launch"
HBM_PEAK_GBPS = 8000.0
# FP32 vector peak available to these kernels: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops (FMA) x 2.4 GHz.  Packed dual-FP32 instructions are disabled at
# compile time, so the 157.3 TFLOP/s packed figure is out of reach by design.
FP32_VECTOR_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def row_flops(L: int) -> float:
    """Algorithmic flops of one padded row transform: forward and inverse FFT
    (5 L log2 L each, the usual nominal count) plus the spectrum multiply (6 L)."""
    return 2 * 5 * L * math.log2(L) + 6 * L


def pass_costs(w, plan):
    """Per-batch algorithmic bytes and flops of the two passes.

    pass_y (column pass): read the hologram, write the N1y x N0x intermediate,
    one length-Ly transform per hologram column.  pass_x (row pass): read the
    intermediate, write the N1y x N1x image, one length-Lx transform per row.
    """
    g = w.holo_grid
    in_elem = 8 if w.holograms.dtype.kind == "c" else 4
    cost = {"pass_x": [0.0, 0.0], "pass_y": [0.0, 0.0]}
    for v, view in enumerate(w.views):
        lx, ly = plan.lengths(v)
        n1x, n1y = view.grid.nx, view.grid.ny
        cost["pass_y"][0] += g.nx * g.ny * in_elem + n1y * g.nx * 8
        cost["pass_y"][1] += g.nx * row_flops(ly)
        cost["pass_x"][0] += n1y * g.nx * 8 + n1x * n1y * 4
        cost["pass_x"][1] += n1y * row_flops(lx)
    return cost


KERNEL_SOURCES = ("paper_1001_4309_amd/csrc/sfd_kernels.hip", "paper_1001_4309_amd/csrc/sfd_rows.hip",
                  "paper_1001_4309_amd/csrc/sfd_cols.hip", "paper_1001_4309_amd/csrc/sfd_persist.hip",
                  "paper_1001_4309_amd/csrc/sfd_device.h", "paper_1001_4309_amd/csrc/fft_core.h",
                  "paper_1001_4309_amd/csrc/sfd_internal.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_name(kind: str, L: int, g: int, var: int) -> str:
    """The kernel's name as rocprofv3 reports it: template arguments length,
    tile width, specialisation and transforms per slot."""
    import paper_1001_4309_amd as sfd

    col = kind == "pass_y"
    per_slot = dict(sfd.sfd_tile_widths(L, col)).get(g, 1)
    return f"{'col' if col else 'row'}_kernel<{L}, {g}, {var}, {per_slot}>"


def pass_variant(w, plan, kind: str) -> int:
    """The kernel specialisation the library picks for a pass of this
    workload (the rule of the library's pass launcher).  Row pass: 2
    (half-padded input, cropped output, intensity only), 1 (half-padded and
    cropped) or 0 (general).  Column pass: 1 (half-padded and cropped,
    complex input), 2 (the same with a real input and no post-chirp), 3 (real
    input with post-chirp) or 0."""
    g = w.holo_grid

    def fast_input(L):  # the library's fast_input: half the row at powers of two, else 1024
        return L // 2 if (L & (L - 1)) == 0 else 1024

    fast = True
    for v, view in enumerate(w.views):
        lx, ly = plan.lengths(v)
        if kind == "pass_x":
            fast = fast and g.nx == fast_input(lx) and view.grid.nx <= fast_input(lx)
        else:
            fast = fast and g.ny == fast_input(ly) and view.grid.ny <= fast_input(ly)
    if not fast:
        return 0
    if kind == "pass_x":
        return 2 if plan.outputs == "intensity" else 1
    if plan.complex_input:
        return 1
    return 2 if plan.outputs == "intensity" else 3


def traffic_file(config: int, tag: str) -> str:
    return os.path.join(ROOT, "profiles", f"{tag}_traffic_config{config}.txt")


def _summaries(kind: str, config: int):
    """(header fields, {kernel: fields}) of every committed summary of this
    kind and workload whose kernel sources match the current ones."""
    import glob

    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"*_{kind}_config{config}.txt"))):
        fields, kernels = {}, {}
        for line in open(path):
            line = line.strip()
            if line.startswith("kernel:"):
                k, _, rest = line[len("kernel:"):].partition("|")
                kernels[k.strip()] = dict(kv.split("=") for kv in rest.split())
            elif ":" in line and not line.startswith("#"):
                a, _, b = line.partition(":")
                fields[a.strip()] = b.strip()
        if fields.get("source-sha256") == kernel_source_hash():
            out.append((fields, kernels))
    return out


def read_traffic(config: int, name: str):
    """HBM bytes per launch of kernel ``name`` from the committed counter
    summaries, or None when there is none or the kernel sources have changed
    since the counters were taken."""
    for fields, kernels in _summaries("traffic", config):
        if name in kernels:
            k = kernels[name]
            return (float(k["fetch_kib"]) * float(fields["fetch-factor"]) +
                    float(k["write_kib"]) * float(fields["write-factor"])) * 1024.0
    return None


def summarize_pmc(fetch_dir: str, write_dir: str, config: int, copy_mib: int, command: str, tag: str) -> None:
    """Write the per-kernel traffic summary from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  The factors scale the
    counters to bytes: a plain device copy of ``copy_mib`` MiB per run reads
    and writes that much."""
    import csv
    import glob

    def per_kernel(d, counter):
        acc = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                if row["Counter_Name"] != counter:
                    continue
                name = row["Kernel_Name"].replace("void ", "").replace("sfd::", "")
                name = name.split("(")[0]
                key = row.get("Dispatch_Id") or row.get("Correlation_Id")
                acc.setdefault(name, {}).setdefault(key, 0.0)
                acc[name][key] += float(row["Counter_Value"])
        return {k: (sum(v.values()) / len(v), len(v)) for k, v in acc.items()}

    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    # The calibration copy is split into equal dispatches: total KiB / copied KiB.
    f_copy = sum(v * n for v, n in [fetch[k] for k in copy])
    w_copy = sum(v * n for v, n in [write[k] for k in copy if k in write])
    ff = copy_mib * 1024.0 / f_copy
    wf = copy_mib * 1024.0 / w_copy
    lines = [f"# rocprofv3 FETCH_SIZE / WRITE_SIZE per dispatch (KiB), workload config {config}",
             f"# command: {command}",
             f"source-sha256: {kernel_source_hash()}",
             f"fetch-factor: {ff:.4f}",
             f"write-factor: {wf:.4f}",
             f"# calibration: a {copy_mib} MiB device copy read {f_copy:.0f} KiB on FETCH_SIZE and wrote "
             f"{w_copy:.0f} KiB on WRITE_SIZE"]
    for k in sorted(fetch):
        if "copyBuffer" in k or k not in write or "elementwise" in k:
            continue
        (fk, n), (wk, _) = fetch[k], write[k]
        lines.append(f"kernel: {k} | fetch_kib={fk:.1f} write_kib={wk:.1f} dispatches={n} "
                     f"hbm_mib={(fk * ff + wk * wf) / 1024:.2f}")
    with open(traffic_file(config, tag), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cpu_info():
    """Host cores this process may use and the CPU model."""
    cores = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cores, model


def cpu_baseline(w, seconds: float):
    """The FP64 oracle as it stands, timed on the host cores (BLAS threads set
    to the cores this process may use): the separable direct sum over all
    views until ``seconds`` have passed, then the paper-literal FFT path
    (steps 2-10 on the padded 2D grid) over all views once."""
    import numpy as np
    import threadpoolctl

    import oracle
    from tests.helpers import ogrid

    cores, model = cpu_info()
    with threadpoolctl.threadpool_limits(limits=cores):
        info = threadpoolctl.threadpool_info()
        blas = max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
        src = ogrid(w.holo_grid)
        n = 0
        t0 = time.perf_counter()
        while True:
            for view in w.views:
                u = oracle.direct(w.holograms[view.holo], src, ogrid(view.grid), w.wavelength, view.z)
                _ = np.abs(u) ** 2
                n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
        t1 = time.perf_counter()
        for view in w.views:
            oracle.fft_path(w.holograms[view.holo], src, ogrid(view.grid), w.wavelength, view.z)
        dt_fft = time.perf_counter() - t1
    nv = len(w.views)
    return {"value": n / dt, "unit": "views/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": model, "blas_threads": int(blas),
            "sample": f"{n} views ({n // nv} passes over the {nv} views of the workload), "
                      f"FP64 separable direct sum (zgemm) plus |u|^2, {dt:.1f} s",
            "fft_path_views_per_s": nv / dt_fft,
            "fft_path_sample": f"all {nv} views through the FP64 steps 2-10 on the padded 2D grid "
                               f"(numpy FFT, one thread), {dt_fft:.2f} s"}


def apply_schedule(plan, schedule: str) -> None:
    """A --schedule string (launch=..., lengths=..., col<L>=G, row<L>=G) onto a plan."""
    for item in schedule.split(","):
        key, g = item.split("=")
        if key == "launch":
            plan.set_launch(g == "persistent")
        elif key == "lengths":
            plan.set_lengths(0 if g == "pow2" else
                             sum({"1280": 1, "1536": 2, "1792": 4}[x] for x in g.split(":")[1].split("+")))
        else:
            plan.set_schedule(int(key[3:]), key.startswith("col"), int(g))


def bench_backward(dev, steps: int, warmup: int, schedule: str = ""):
    """Forward (intensity and field) plus backward (field gradient and dL/dz)
    of the differentiation workload: 16 complex 1024^2 fields, one view each,
    L = 2048.  The loss gradient dL/dI = 2 (I - T) is formed once, outside the
    timed region; the timed step is the two library calls.  schedule: tile
    widths to use instead of autotuning (as --schedule)."""
    import numpy as np
    import torch

    import paper_1001_4309_amd as sfd
    import workloads

    w = workloads.config4()
    plan = sfd.Plan(w.wavelength, w.holo_grid, len(w.holograms), w.views, outputs="both", complex_input=True,
                    device=dev)
    fields = torch.from_numpy(w.holograms).to(dev)
    outs = plan.new_outputs()
    nv = len(w.views)
    if schedule:
        apply_schedule(plan, schedule)
    else:
        plan.autotune(fields, reps=5, outs=outs)  # the backward's passes use the same tile widths
    res = plan.reconstruct(fields, outs=outs)
    gi = [2.0 * (res[v] - 0.5 * res[v].mean()) for v in range(nv)]
    torch.cuda.synchronize()

    def step():
        r = plan.reconstruct(fields, outs=outs)
        plan.backward(gi, fields, field_out=r[nv:])

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.reconstruct(fields, outs=outs)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / steps
    # Algorithmic work: the forward is two passes of transforms, the backward
    # six (the adjoint's two, and four for the z-moment fields of dL/dz).
    fwd_fl = bwd_fl = 0.0
    g = w.holo_grid
    for v, view in enumerate(w.views):
        lx, ly = plan.lengths(v)
        fwd_fl += g.nx * row_flops(ly) + view.grid.ny * row_flops(lx)
        bwd_fl += (view.grid.nx + 2 * g.nx) * row_flops(ly) + (g.ny + 2 * view.grid.ny) * row_flops(lx)
    bwd_s = sec - fwd
    extra = {"forward_TFLOPs": fwd_fl / fwd / 1e12, "backward_TFLOPs": bwd_fl / bwd_s / 1e12,
             "backward_frac_of_fp32_vector_peak": bwd_fl / bwd_s / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
             "algorithmic_gflop_forward": fwd_fl / 1e9, "algorithmic_gflop_backward": bwd_fl / 1e9}
    return {**extra, "workload": w.name, "fields_per_step": nv, "ms_per_step": sec * 1e3,
            "schedule": {f"{k[0]}{k[1]}": g for k, g in sorted(plan.schedule().items())},
            "backward_over_forward": (sec - fwd) / fwd,
            "fields_per_s": nv / sec, "forward_ms": fwd * 1e3, "backward_ms": (sec - fwd) * 1e3,
            "what": "forward (intensity + field) and backward (field gradient + dL/dz), per 16-field batch"}


def time_steps(plan, holo, outs, steps: int) -> float:
    """Seconds per step over exactly ``steps`` calls, bracketed by device
    synchronisations (the contract's timed region)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.reconstruct(holo, outs=outs)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def event_stats(plan, holo, outs, n: int):
    """Per-call durations from HIP events recorded around each call on the
    stream the library launches on (torch's current stream): median, p10 and
    p90 over n calls."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        plan.reconstruct(holo, outs=outs)
        b.record()
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
    return {"calls": n, "median_us": t[n // 2], "p10_us": t[n // 10], "p90_us": t[(9 * n) // 10],
            "how": "hipEvent pair around each call on the launch stream (one direct launch of the persistent "
                   "kernel, or one graph replay of the pass schedule)"}


def counters_file(config: int, tag: str) -> str:
    return os.path.join(ROOT, "profiles", f"{tag}_counters_config{config}.txt")


def _pmc_per_kernel(d: str):
    """{kernel: {counter: mean per dispatch}} from rocprofv3 --pmc CSV output
    (each dispatch's counter summed over its instances)."""
    import csv
    import glob

    acc = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            name = row["Kernel_Name"].replace("void ", "").replace("sfd::", "").split("(")[0]
            key = row.get("Dispatch_Id") or row.get("Correlation_Id")
            per = acc.setdefault(name, {}).setdefault(row["Counter_Name"], {})
            per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    return {k: {c: sum(v.values()) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def summarize_counters(dirs, config: int, command: str, tag: str) -> None:
    """Write the VALU / LDS counter summary of rocprofv3 --pmc runs (one
    directory per counter pass) for every kernel they saw."""
    per = {}
    for d in dirs:
        for k, cs in _pmc_per_kernel(d).items():
            per.setdefault(k, {}).update(cs)
    lines = [f"# rocprofv3 --pmc counters per dispatch (mean over dispatches), workload config {config}",
             f"# command: {command}",
             "# valu_busy = SQ_INSTS_VALU * 4 / (1024 SIMDs * GRBM_GUI_ACTIVE / 8 XCDs): the share of the",
             "#   kernel's cycles the 1024 SIMDs spend issuing VALU instructions (a wave64 instruction",
             "#   occupies a 16-lane SIMD for 4 cycles); GRBM_GUI_ACTIVE counts busy cycles summed over the 8 XCDs",
             f"source-sha256: {kernel_source_hash()}"]
    for k in sorted(per):
        cs = per[k]
        if "copyBuffer" in k or "elementwise" in k or "SQ_INSTS_VALU" not in cs:
            continue
        if cs.get("GRBM_GUI_ACTIVE"):
            cs["valu_busy"] = cs["SQ_INSTS_VALU"] * 4.0 / (1024.0 * cs["GRBM_GUI_ACTIVE"] / 8.0)
        lines.append(f"kernel: {k} | " + " ".join(f"{c}={v:.4g}" for c, v in sorted(cs.items())))
    with open(counters_file(config, tag), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_counters(config: int, name: str):
    """VALU and LDS counter figures of kernel ``name`` from the committed
    summaries (see profiles/), or None when absent or stale."""
    for _, kernels in _summaries("counters", config):
        if name in kernels:
            return {a: float(b) for a, b in kernels[name].items()}
    return None


def measure(w, dev, args, steps: int, warmup: int, config: int, tune: bool = True, schedule: str = ""):
    """One workload: plan, schedule (autotuned unless told otherwise), the
    contract's timed steps, per-call event statistics, and the kernels'
    event-measured durations with the dominant kernel's roofline."""
    import numpy as np
    import torch

    import paper_1001_4309_amd as sfd

    holo = torch.from_numpy(np.ascontiguousarray(w.holograms)).to(dev)
    plan = sfd.Plan(w.wavelength, w.holo_grid, len(w.holograms), w.views, device=dev)
    outs = plan.new_outputs()
    nv = len(w.views)
    if schedule:
        apply_schedule(plan, schedule)
    elif tune:
        plan.autotune(holo, reps=10, outs=outs)
    sched = {f"{k[0]}{k[1]}": g for k, g in sorted(plan.schedule().items())}
    mode = plan.launch_mode()[0]
    log(f"{w.name}: launch {mode}, lengths {plan.length_policy()}, tile widths {sched}")
    for _ in range(warmup):
        plan.reconstruct(holo, outs=outs)
    sec = time_steps(plan, holo, outs, steps)
    stats = event_stats(plan, holo, outs, max(100, steps))
    log(f"{w.name}: {sec * 1e6:.1f} us/step over {steps} steps, {nv / sec:.0f} views/s; per call median "
        f"{stats['median_us']:.1f} us (p10 {stats['p10_us']:.1f}, p90 {stats['p90_us']:.1f})")

    prof_steps = max(1, min(steps, 100))
    plan.profile(True)
    for _ in range(prof_steps):
        plan.reconstruct(holo, outs=outs)
    torch.cuda.synchronize()
    rep = plan.profile_report()
    plan.profile(False)
    costs = pass_costs(w, plan)
    costs["persist"] = [costs["pass_x"][0] + costs["pass_y"][0], costs["pass_x"][1] + costs["pass_y"][1]]
    kern = {k: {"launches": n, "avg_us": (ms / n * 1e3) if n else 0.0} for k, (n, ms) in rep.items() if n}
    if rep.get("persist", (0, 0.0))[0] > 0:
        dom = "persist"  # one launch per step holds every pass
    else:
        dom = max(("pass_x", "pass_y"), key=lambda k: rep[k][1])
    n_launch, tot_ms = rep[dom]
    avg_s = tot_ms / n_launch / 1e3
    per_step = n_launch / prof_steps
    flops, nbytes = costs[dom][1] / per_step, costs[dom][0] / per_step
    if dom == "persist":
        dom_name = f"persist_kernel<{'true' if plan.complex_input else 'false'}>"
    else:
        lx0, ly0 = plan.lengths(0)
        dom_L = lx0 if dom == "pass_x" else ly0
        dom_name = kernel_name(dom, dom_L, plan.schedule()[("row" if dom == "pass_x" else "col", dom_L)],
                               pass_variant(w, plan, dom))
    alu = flops / avg_s / 1e12
    hbm = nbytes / avg_s / 1e9
    frac_alu, frac_hbm = alu / FP32_VECTOR_PEAK_TFLOPS, hbm / HBM_PEAK_GBPS
    # The bound: the roofline the kernel's algorithmic work sits closer to
    # (its flop/byte ratio against the ridge of the two peaks).
    bound = "alu" if flops / nbytes > FP32_VECTOR_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBPS * 1e9) else "hbm"
    roofline = {"bound": bound,
                "achieved": alu if bound == "alu" else hbm,
                "peak": FP32_VECTOR_PEAK_TFLOPS if bound == "alu" else HBM_PEAK_GBPS,
                "unit": "TFLOP/s" if bound == "alu" else "GB/s",
                "frac": frac_alu if bound == "alu" else frac_hbm,
                "traffic": read_traffic(config, dom_name),
                "kernel": dom_name, "avg_launch_us": avg_s * 1e6,
                "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes,
                "frac_of_fp32_vector_peak": frac_alu, "frac_of_hbm_peak": frac_hbm,
                "hbm_GBps": hbm, "fp32_TFLOPs": alu,
                "counters": read_counters(config, dom_name)}
    cnt = roofline["counters"]
    if cnt and "SQ_INSTS_VALU" in cnt:
        # Measured evidence for the bound: the share of cycles the SIMDs
        # spent issuing VALU instructions (counters) against the share of the
        # HBM peak the kernel's measured traffic reached.
        roofline["valu_insts_per_nominal_flop"] = cnt["SQ_INSTS_VALU"] * 64.0 / flops
        if "valu_busy" in cnt:
            hbm_meas = (roofline["traffic"] or nbytes) / avg_s / 1e9 / HBM_PEAK_GBPS
            roofline["valu_busy"] = cnt["valu_busy"]
            roofline["hbm_busy"] = hbm_meas
            roofline["bound_from_counters"] = "alu" if cnt["valu_busy"] >= hbm_meas else "hbm"
    step_bytes = costs["pass_x"][0] + costs["pass_y"][0]
    res = {"workload": w.name, "views_per_step": nv, "views_per_s": nv / sec, "ms_per_step": sec * 1e3,
           "per_call": stats, "launch_mode": mode, "length_policy": plan.length_policy(), "schedule": sched,
           "lengths": sorted({plan.lengths(v) for v in range(nv)}),
           "kernels": kern, "roofline": roofline,
           "hbm": {"algorithmic_bytes_per_step": step_bytes, "achieved_GBps": step_bytes / sec / 1e9,
                   "frac_of_8TBps": step_bytes / sec / 1e9 / HBM_PEAK_GBPS}}
    return plan, holo, outs, res


def per_view_baseline(w, dev, holo, steps: int, warmup: int, tune: bool, batched_sec: float):
    """The same views with one launch sequence per view (setup, column pass,
    row pass for each view in turn), with its own tuned tile widths."""
    import paper_1001_4309_amd as sfd

    nv = len(w.views)
    pv = sfd.Plan(w.wavelength, w.holo_grid, len(w.holograms), w.views, device=dev, per_view_launch=True)
    pouts = pv.new_outputs()
    if tune:
        pv.autotune(holo, reps=10, outs=pouts)
    for _ in range(warmup):
        pv.reconstruct(holo, outs=pouts)
    psec = time_steps(pv, holo, pouts, steps)
    log(f"{w.name} per-view launch: {psec * 1e6:.1f} us/step, {nv / psec:.0f} views/s")
    return {"views_per_s": nv / psec, "ms_per_step": psec * 1e3, "batched_speedup": psec / batched_sec,
            "schedule": {f"{k[0]}{k[1]}": g for k, g in pv.schedule().items()}}


def bench_streaming(w, plan, steps: int, warmup: int):
    """The real-time loop on the same workload: frames arrive in pinned host
    memory, each is copied to the device on the plan's copy stream while the
    previous one is reconstructed, and the tables and spectra are computed for
    the first frame only (a plan made with reuse_tables, on the batched
    plan's tile widths).  Reports frames/s of the overlapped loop, and beside
    it the host-to-device copy alone and the reconstruction alone."""
    import numpy as np
    import torch

    import paper_1001_4309_amd as sfd

    dev = torch.device("cuda:0")
    sp = sfd.Plan(w.wavelength, w.holo_grid, len(w.holograms), w.views, device=dev, reuse_tables=True)
    r = np.random.default_rng(5)
    base = np.ascontiguousarray(w.holograms).astype(np.float32)
    frames = [torch.from_numpy((base * r.uniform(0.9, 1.1, base.shape)).astype(np.float32)).pin_memory()
              for _ in range(8)]
    fs = sfd.FrameStream(sp)
    # The loop's own schedule (tables kept between frames changes what is fastest).
    fs.dev[0].copy_(frames[0])
    sp.autotune(fs.dev[0], reps=10)
    for k in range(warmup):
        fs.push(frames[k % len(frames)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        fs.push(frames[k % len(frames)])
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    # The copy alone, on a side stream, and the reconstruction alone (tables kept).
    side = torch.cuda.Stream()
    dst = fs.dev[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(side):
        for k in range(steps):
            dst.copy_(frames[k % len(frames)], non_blocking=True)
    torch.cuda.synchronize()
    copy_sec = (time.perf_counter() - t0) / steps
    res_mode = sp.launch_mode()[0]
    outs = sp.new_outputs()
    sp.reconstruct(dst, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sp.reconstruct(dst, outs=outs)
    torch.cuda.synchronize()
    comp_sec = (time.perf_counter() - t0) / steps
    nbytes = frames[0].numel() * 4
    nv = len(w.views)
    res = {"frames_per_s": 1.0 / sec, "views_per_s": nv / sec, "ms_per_frame": sec * 1e3,
           "h2d_ms_per_frame": copy_sec * 1e3, "h2d_GBps": nbytes / copy_sec / 1e9,
           "reconstruct_ms_per_frame": comp_sec * 1e3, "launch_mode": res_mode,
           "what": f"{len(frames)} pinned host frames cycled; copy of frame k+1 overlapped with the "
                   f"reconstruction of frame k; tables and spectra from the first frame"}
    ccd = w.extra.get("ccd")
    if ccd is not None:
        # Raw 8-bit camera frames (unresized), converted and resized on the GPU.
        raw = sfd.Plan(w.wavelength, w.holo_grid, len(w.holograms), w.views, device=dev, reuse_tables=True,
                       raw_width=ccd.shape[-1], raw_bits=8)
        q = np.clip(np.rint(ccd / ccd.max() * 255.0), 0, 255)
        u8 = [torch.from_numpy(np.clip(q * r.uniform(0.9, 1.1, q.shape), 0, 255).astype(np.uint8)).pin_memory()
              for _ in range(8)]
        fr = sfd.FrameStream(raw)
        fr.dev[0].copy_(u8[0])
        raw.autotune(fr.dev[0], reps=10)
        for k in range(warmup):
            fr.push(u8[k % len(u8)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            fr.push(u8[k % len(u8)])
        torch.cuda.synchronize()
        rsec = (time.perf_counter() - t0) / steps
        # The same plan on a resident frame (no copies), for the loop's overhead.
        routs = raw.new_outputs()
        raw.reconstruct(fr.dev[0], outs=routs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            raw.reconstruct(fr.dev[0], outs=routs)
        torch.cuda.synchronize()
        rcomp = (time.perf_counter() - t0) / steps
        res["camera_u8"] = {"frames_per_s": 1.0 / rsec, "views_per_s": nv / rsec, "ms_per_frame": rsec * 1e3,
                            "reconstruct_ms_per_frame": rcomp * 1e3, "launch_mode": raw.launch_mode()[0],
                            "frame": list(ccd.shape[1:]), "bytes_per_frame": int(u8[0].numel()),
                            "what": "8-bit 1360 x 1024 camera frames, converted and resized to the 1024^2 "
                                    "hologram grid on the GPU, same loop"}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 5])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--legs", default="3,5",
                    help="other workloads to measure beside the main one (comma-separated config numbers; "
                         "'' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile widths")
    ap.add_argument("--no-backward", action="store_true", help="skip the forward + backward measurement")
    ap.add_argument("--no-streaming", action="store_true", help="skip the real-time loop measurement")
    ap.add_argument("--backward-only", action="store_true",
                    help="only the forward + backward measurement (config 4), printed as one JSON line; "
                         "--schedule then fixes its tile widths instead of autotuning")
    ap.add_argument("--schedule", default="",
                    help="tile widths to use instead of autotuning, e.g. col2048=4,row2048=4")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic summary of two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_DIR",
                    help="write the VALU / LDS counter summary of rocprofv3 --pmc runs and exit")
    ap.add_argument("--pmc-command", default="", help="command recorded in the traffic summary")
    ap.add_argument("--profile-tag", default="sfd_kernels", help="file name prefix of a written summary")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (calibrates traffic counters)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.config, args.calib_copy_mib,
                      args.pmc_command, args.profile_tag)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.config, args.pmc_command, args.profile_tag)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
                  "views are independent, so a multi-GPU run would split the view list without any exchange, "
                  "and that path is not built here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1001_4309_amd as sfd
    import workloads

    dev = torch.device("cuda:0")
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del a, b
    if args.backward_only:
        backward = bench_backward(dev, max(1, args.steps), max(1, args.warmup), args.schedule)
        log(f"forward + backward: {backward['ms_per_step']:.3f} ms per 16 fields "
            f"({backward['fields_per_s']:.0f} fields/s; forward {backward['forward_ms']:.3f} ms)")
        print(json.dumps({"backward": backward}), flush=True)
        return
    tune = not args.no_autotune
    w = workloads.CONFIGS[args.config]()
    nv = len(w.views)
    plan, holo, outs, main_res = measure(w, dev, args, args.steps, args.warmup, args.config, tune, args.schedule)
    sec = main_res["ms_per_step"] / 1e3
    value = main_res["views_per_s"]
    if args.calib_copy_mib <= 0:  # a counter run keeps its only copy the calibration one
        # Reference: a plain 1 GiB device-to-device copy on the same GPU.
        ca = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        cb = torch.empty_like(ca)
        cb.copy_(ca)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            cb.copy_(ca)
        e1.record()
        torch.cuda.synchronize()
        copy_gbps = 5 * 2 * ca.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del ca, cb
        main_res["hbm"]["device_copy_GBps"] = copy_gbps
        main_res["hbm"]["frac_of_device_copy"] = main_res["hbm"]["achieved_GBps"] / copy_gbps

    per_view = None
    if not args.no_per_view:
        per_view = per_view_baseline(w, dev, holo, args.steps, args.warmup, tune, sec)

    # Other workloads of the method: the batched uneven views (64 views of 8
    # holograms) and the large one (L = 8192), each with its own roofline.
    legs = {}
    for c in [int(x) for x in args.legs.split(",") if x.strip()]:
        if c == args.config:
            continue
        wl = workloads.CONFIGS[c]()
        lsteps = max(5, min(args.steps, 20 if c == 5 else 50))
        _, lholo, _, lres = measure(wl, dev, args, lsteps, max(2, min(args.warmup, 5)), c, tune)
        if c == 3 and not args.no_per_view:
            lres["per_view_launch"] = per_view_baseline(wl, dev, lholo, lsteps, 2, tune, lres["ms_per_step"] / 1e3)
        legs[f"config{c}"] = lres
        del lholo
        torch.cuda.empty_cache()

    streaming = None
    if not args.no_streaming:
        streaming = bench_streaming(w, plan, args.steps, args.warmup)
        log(f"streaming: {streaming['ms_per_frame'] * 1e3:.1f} us/frame, {streaming['frames_per_s']:.0f} frames/s "
            f"(copy alone {streaming['h2d_ms_per_frame'] * 1e3:.1f} us at {streaming['h2d_GBps']:.1f} GB/s, "
            f"reconstruction alone {streaming['reconstruct_ms_per_frame'] * 1e3:.1f} us)")
        if "camera_u8" in streaming:
            cu = streaming["camera_u8"]
            log(f"streaming 8-bit camera frames: {cu['ms_per_frame'] * 1e3:.1f} us/frame, "
                f"{cu['frames_per_s']:.0f} frames/s")

    backward = None
    if not args.no_backward:
        backward = bench_backward(dev, max(1, min(args.steps, 50)), max(1, min(args.warmup, 5)))
        log(f"forward + backward: {backward['ms_per_step']:.3f} ms per 16 fields "
            f"({backward['fields_per_s']:.0f} fields/s; forward {backward['forward_ms']:.3f} ms)")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.3f} views/s on {cpu['cores']} cores ({cpu['cpu_model']})")

    g = w.holo_grid
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "holograms": len(w.holograms), "views_per_step": nv,
                   "hologram": [g.ny, g.nx], "views": [[v.grid.ny, v.grid.nx] for v in w.views],
                   "padded_lengths": main_res["lengths"], "phase": "fp64-reduced", "output": "intensity",
                   "schedule": main_res["schedule"],
                   "launch": ("one persistent kernel, launched directly" if main_res["launch_mode"] == "persistent"
                              else "hip-graph replay of setup, column and row passes"),
                   "launch_mode": main_res["launch_mode"], "length_policy": main_res["length_policy"]},
        "roofline": main_res["roofline"],
        "per_call": main_res["per_call"],
        "hbm": main_res["hbm"],
        "per_view_launch": per_view,
        "legs": legs,
        "backward": backward,
        "streaming": streaming,
        "kernels": main_res["kernels"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
