"""Throughput of the Morse-Smale segmentation on one MI355X.

One step = one full segmentation of one field: order field (radix sort),
steepest neighbours, path compression, MS ids -- every step of the method,
with the input already resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c1|c3f64]

Single GPU only: ``--gpus`` above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mvertices/s full MS segmentation (bit-exact), batched vs plain; p99 ms"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per vertex of one launch of each kernel kind: every
# array the kernel is defined on is read once and written once (float32 field,
# int32 labels, 32-bit keys).
#   steepest      : read order or f (4), write up, dn (8)
#   jump          : read up, dn (8), write asc, desc (8).  Its other writes
#                   are overhead, not counted: each vertex's MS pair record
#                   index, kept in ms until the ids are known (4 B/vertex),
#                   and the listed pair records (12 B per listed pair, about
#                   7% of N)
#   ms_final      : read slot (4), write ms (4)
#   order_first   : read f (4), write key and id (8)
#   order_scatter : read key and id (8), write key and id (8)  (a middle pass)
#   order_last    : read key and id (8); write (id, position) grouped by id
#                   range (8) [order_invert = 1] or the sorted id (4) [>= 2]
#   order_invert  : read (id, position) (8), write order (4) [order_invert = 1];
#                   the fused last pass: read key and id (8), write order (4)
#                   [0]; read sorted ids (4), write order (4 / w) [w >= 2]
#   order_regroup : read (id, position) (8), write it regrouped by id chunk (8)
#   order_hist    : read key (4)
ALGO_BYTES = {"steepest": 12.0, "jump": 16.0, "ms_final": 8.0, "order_first": 12.0, "order_scatter": 16.0,
              "order_hist": 4.0, "order_regroup": 16.0}


def algo_bytes(kind: str, invert: int):
    if kind == "order_last":
        return 16.0 if invert == 1 else 12.0
    if kind == "order_invert":
        return 12.0 if invert in (0, 1) else 4.0 + 4.0 / invert
    return ALGO_BYTES.get(kind)


# Launch-shape knobs each kernel kind depends on (a traffic profile taken
# with other values of these does not describe the kernel that ran).
KIND_KNOBS = {"steepest": ("scan_depth", "scan_rounds", "packed_codes"), "jump": ("scan_depth", "scan_rounds"),
              "ms_final": ("scan_depth", "scan_rounds")}
for _k in ("order_first", "order_scatter", "order_last", "order_regroup", "order_invert", "order_hist"):
    KIND_KNOBS[_k] = ("order_workers", "order_invert", "order_packed", "order_concurrent")
for _k in ("radix_hist", "radix_scatter", "radix_digit_scan", "pair_rank"):
    KIND_KNOBS[_k] = ("sort_workers", "pair_stream")


def kernel_source_digest() -> str:
    """Digest of the kernel sources: a traffic profile holds only for the code it was taken on."""
    import glob
    import hashlib

    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2303_15491_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "include", "plmss.h"))
    for path in files:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


# The kernel (as rocprofv3 names it) each trace kind launches on the headline
# workload: one 3-D float32 field with its order field, default scan tiles.
HEADLINE_SYMBOLS = {
    "jump": "k_chase<JTile<32, 8, 8>, true, true, true>",
    "steepest": "k_steepest<RankOrderPacked, 8, 16, true, 512>",
    "ms_final": "k_ms_final<JTile<32, 8, 8>, true>",
    "order_scatter": "k_radix_scatter<PackedSrc, PackedDst>",
    "order_first": "k_radix_scatter<FieldSrc<float, unsigned int>, PackedDst>",
    "order_last": "k_rank_partition<PackedSrc>",
    "order_regroup": "k_chunk_partition",
    "order_invert": "k_invert_chunks",
}


def profile_entry(name: str, workload: str, kind: str, knobs: dict):
    """The committed rocprofv3 summary `profiles/<name>_<workload>.md` row of
    the kernel `kind` launches on this workload, or (None, reason).  A
    summary holds only for the kernel sources and launch-shape knobs it was
    taken with."""
    path = os.path.join(ROOT, "profiles", f"{name}_{workload}.md")
    try:
        with open(path) as fh:
            text = fh.read()
    except OSError:
        return None, f"no {name} profile for this workload"
    start = text.find("```json")
    end = text.find("```", start + 7)
    if start < 0 or end < 0:
        return None, f"{name} profile has no data block"
    data = json.loads(text[start + 7:end])
    if data.get("source_digest") != kernel_source_digest():
        return None, "kernels changed since the profile was taken"
    for k in KIND_KNOBS.get(kind, ()):
        if data.get("knobs", {}).get(k) != knobs.get(k):
            return None, f"profile was taken with {k}={data.get('knobs', {}).get(k)}, this run used {knobs.get(k)}"
    sym = HEADLINE_SYMBOLS.get(kind)
    entry = data.get("symbols", {}).get(sym) if sym else None
    if not entry:
        return None, f"no profile row for {kind}"
    return entry, os.path.relpath(path, ROOT)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name: str):
    from paper_2303_15491_amd import fields

    if name == "c1":
        return fields.workload_c1(), "2D 64x64 float32 sum of 8 Gaussians + U(-0.01,0.01) noise (seed 1)"
    if name == "c2":
        return fields.workload_c2(256), "3D 256^3 float32 N(0,1) smoothed sigma=3 + 0.1 z-ramp (seed 2)"
    if name == "c3":
        return fields.workload_c3(512), "3D 512^3 float32 N(0,1) smoothed sigma=1.5 (seed 3)"
    if name == "c3f64":
        return fields.workload_c3(512).astype(np.float64), "3D 512^3 float64 (widened float32) N(0,1) smoothed sigma=1.5 (seed 3)"
    raise SystemExit(f"unknown workload {name}")


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def step_stats(ms):
    """The paper's protocol over per-step times (drop the best and the worst
    run, average the rest) and the median."""
    a = sorted(ms)
    trimmed = a[1:-1] if len(a) > 2 else a
    return {"trimmed_mean_ms": sum(trimmed) / len(trimmed), "median_ms": float(np.median(a)),
            "min_ms": a[0], "max_ms": a[-1], "steps": len(a)}


def timed_region(step, steps, torch, lib=None, trace=None, max_launches=0, per_step=None):
    """Runs `steps` steps between two device synchronisations; returns the wall
    time in ms and (if traced) the per-launch (kind, ms) list.  per_step (a
    list) receives each step's time from events recorded on the current
    stream between the steps (the steps' work runs on that stream)."""
    torch.cuda.synchronize()
    if trace is not None:
        lib.plmss_trace_begin(trace)
    events = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if per_step is not None else None
    t0 = time.perf_counter()
    if events:
        events[0].record()
    for i in range(steps):
        step()
        if events:
            events[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if events:
        per_step.extend(events[i].elapsed_time(events[i + 1]) for i in range(steps))
    launches = []
    if trace is not None:
        lib.plmss_trace_end(trace)
        kinds = (ctypes.c_int32 * max_launches)()
        ms = (ctypes.c_float * max_launches)()
        m = lib.plmss_trace_read(trace, kinds, ms, max_launches)
        if m < 0:
            raise RuntimeError(f"trace read failed: {m}")
        launches = [(lib.plmss_kernel_name(kinds[i]).decode(), ms[i]) for i in range(m)]
    return (t1 - t0) * 1e3, launches


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Achieved device-to-device copy rate in GB/s (bytes read + written)."""
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (times[len(times) // 2] * 1e-3) / 1e9


def per_kernel(launches, steps):
    agg = {}
    for name, ms in launches:
        a = agg.setdefault(name, {"launches": 0, "total_ms": 0.0})
        a["launches"] += 1
        a["total_ms"] += ms
    for a in agg.values():
        a["ms_per_step"] = a["total_ms"] / steps
        a["avg_launch_ms"] = a["total_ms"] / a["launches"]
    return agg


def bench_float64_copy(torch, plmss, lib, field32, ref, steps: int, warmup: int):
    """The float64 copy of the same field (every value widened exactly): full
    and labels-only step times, the per-kernel times of the full step, and a
    check that every output equals the float32 run's."""
    field = field32.double()
    dims = plmss.dims_of(field.shape)
    outs = {k: torch.empty(field.shape, dtype=torch.int32, device=field.device)
            for k in ("asc", "desc", "ms", "order")}
    outs["info"] = torch.zeros(4, dtype=torch.int32, device=field.device)
    ws_bytes = lib.plmss_workspace_bytes(dims, plmss.F64, 1)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=field.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    jobs = [plmss.Job(field.data_ptr(), dims, plmss.F64, outs["asc"].data_ptr(), outs["desc"].data_ptr(),
                      outs["ms"].data_ptr(), outs["order"].data_ptr() if with_order else None,
                      outs["info"].data_ptr()) for with_order in (True, False)]

    def step(job):
        rc = lib.plmss_segment(ctypes.byref(job), ctypes.c_void_p(ws.data_ptr()), ws_bytes, stream)
        if rc:
            raise plmss.PlmssError(rc, "plmss_segment")

    for _ in range(warmup):
        step(jobs[0])
    torch.cuda.synchronize()
    identical = all(torch.equal(outs[k], ref[k]) for k in ("asc", "desc", "ms", "order", "info"))
    wall_full, _ = timed_region(lambda: step(jobs[0]), steps, torch)
    wall_labels, _ = timed_region(lambda: step(jobs[1]), steps, torch)
    max_launches = 128 * max(steps, 1)
    trace = lib.plmss_trace_create(max_launches)
    _, launches = timed_region(lambda: step(jobs[0]), steps, torch, lib, trace, max_launches)
    lib.plmss_trace_destroy(trace)
    n = field.numel()
    del ws, outs, field
    torch.cuda.empty_cache()
    return {"ms_per_step": wall_full / steps, "value": n / (wall_full / steps * 1e-3) / 1e6,
            "labels_only_ms_per_step": wall_labels / steps,
            "labels_only_value": n / (wall_labels / steps * 1e-3) / 1e6, "unit": "Mvertices/s",
            "identical_to_float32": identical,
            "kernels_ms_per_step": {k: round(v["ms_per_step"], 4)
                                    for k, v in sorted(per_kernel(launches, steps).items())}}


def bench_marching(torch, plmss, lib, labels, steps: int, warmup: int, cpu_planes: int):
    """The multi-label marching index over the MS labels of the field: time
    per call with and without per-cell codes (region separators), the
    per-launch time of the count kernel against the HBM roofline of its
    algorithmic bytes (labels read once, codes written once, one offset per
    row), and the oracle on a slab of the same labels."""
    dims = plmss.dims_of(labels.shape)
    rows = int(lib.plmss_marching_rows(dims))
    cubes = rows * (int(dims.nx) - 1)
    per = 6 if dims.nz > 1 else 2
    codes = torch.empty(max(cubes * per, 2), dtype=torch.uint8, device=labels.device)
    offs = torch.empty(rows + 1, dtype=torch.int64, device=labels.device)
    ws_bytes = lib.plmss_marching_workspace_bytes(dims)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=labels.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {"rows": rows, "cells": cubes * per}
    for with_codes in (True, False):
        cptr = ctypes.c_void_p(codes.data_ptr()) if with_codes else None

        def step():
            rc = lib.plmss_marching_index(ctypes.c_void_p(labels.data_ptr()), dims, plmss.MARCH_SEPARATORS, cptr,
                                          ctypes.c_void_p(offs.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                          ws_bytes, stream)
            if rc:
                raise plmss.PlmssError(rc, "plmss_marching_index")

        for _ in range(warmup):
            step()
        wall, _ = timed_region(step, steps, torch)
        max_launches = 8 * steps
        trace = lib.plmss_trace_create(max_launches)
        _, launches = timed_region(step, steps, torch, lib, trace, max_launches)
        lib.plmss_trace_destroy(trace)
        kern = per_kernel(launches, steps)
        avg = kern["march_count"]["avg_launch_ms"]
        nbytes = 4.0 * labels.numel() + (per * cubes if with_codes else 0) + 8.0 * rows
        key = "with_codes" if with_codes else "counts_only"
        res[key] = {"ms_per_call": wall / steps, "value": labels.numel() / (wall / steps * 1e-3) / 1e6,
                    "unit": "Mvertices/s", "count_kernel_avg_launch_ms": avg,
                    "algorithmic_bytes_per_launch": nbytes,
                    "basis": f"4 B/vertex labels read{f' + {per} B/cube codes written' if with_codes else ''}"
                             f" + 8 B/row offsets",
                    "achieved_gbs": nbytes / (avg * 1e-3) / 1e9,
                    "frac": nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "kernels_ms_per_call": {k: round(v["ms_per_step"], 4) for k, v in sorted(kern.items())}}
    res["total_separators"] = int(offs[-1].item())
    # the geometry pass: every primitive written (points and side labels)
    for mode, key in ((plmss.MARCH_SEPARATORS, "geometry_separators"), (plmss.MARCH_BOUNDARIES, "geometry_boundaries")):
        rc = lib.plmss_marching_index(ctypes.c_void_p(labels.data_ptr()), dims, mode, None,
                                      ctypes.c_void_p(offs.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws_bytes,
                                      stream)
        if rc:
            raise plmss.PlmssError(rc, "plmss_marching_index")
        total = int(offs[-1].item())
        pts = (3, 3) if dims.nz > 1 else (2, 2)
        xyz = torch.empty((max(total, 1),) + pts, dtype=torch.float32, device=labels.device)
        sides = torch.empty((max(total, 1), 2), dtype=torch.int32, device=labels.device)

        def gstep():
            rc = lib.plmss_marching_geometry(ctypes.c_void_p(labels.data_ptr()), dims, mode,
                                             ctypes.c_void_p(offs.data_ptr()), total,
                                             ctypes.c_void_p(xyz.data_ptr()), ctypes.c_void_p(sides.data_ptr()),
                                             stream)
            if rc:
                raise plmss.PlmssError(rc, "plmss_marching_geometry")

        gsteps = max(2, steps // 2)
        gstep()
        wall, _ = timed_region(gstep, gsteps, torch)
        trace = lib.plmss_trace_create(4 * gsteps)
        _, launches = timed_region(gstep, gsteps, torch, lib, trace, 4 * gsteps)
        lib.plmss_trace_destroy(trace)
        avg = per_kernel(launches, gsteps)["march_geometry"]["avg_launch_ms"]
        # the same output buffers written by a plain fill, in the same run: the
        # write rate this machine gives buffers of this size
        fills = []
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            xyz.fill_(1.0)
            sides.fill_(1)
            b.record()
            b.synchronize()
            fills.append(a.elapsed_time(b))
        fill_ms = sorted(fills)[1]
        per_prim = 4 * pts[0] * pts[1] + 8
        nbytes = 4.0 * labels.numel() + 8.0 * (rows + 1) + per_prim * total
        res[key] = {"primitives": total, "ms_per_call": wall / gsteps, "kernel_avg_launch_ms": avg,
                    "output_gb": per_prim * total / 1e9, "algorithmic_bytes_per_launch": nbytes,
                    "basis": f"4 B/vertex labels read + {per_prim} B/primitive written (points, side labels)",
                    "achieved_gbs": nbytes / (avg * 1e-3) / 1e9, "frac": nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "primitives_per_s": total / (avg * 1e-3),
                    "write_only_fill_ms": fill_ms,
                    "write_only_fill_gbs": (xyz.numel() + sides.numel()) * 4 / (fill_ms * 1e-3) / 1e9,
                    "kernel_vs_fill": fill_ms / avg}
        del xyz, sides
        torch.cuda.empty_cache()
    if cpu_planes > 0:
        import oracle

        sl = np.ascontiguousarray(labels[:cpu_planes].cpu().numpy())
        t0 = time.perf_counter()
        oracle.marching(sl, 0)
        t1 = time.perf_counter()
        res["cpu_baseline"] = {"value": sl.size / (t1 - t0) / 1e6, "unit": "Mvertices/s", "cores": 1,
                               "kind": "oracle", "sample": f"serial C oracle with codes on {tuple(sl.shape)}, "
                                                           f"{t1 - t0:.2f} s"}
        # the geometry oracle on a thinner slab (its output is ~44 B per primitive in host memory)
        gl = np.ascontiguousarray(labels[:min(cpu_planes, 8)].cpu().numpy())
        cap = oracle.marching(gl, 0, with_codes=False)["total"]
        t0 = time.perf_counter()
        g = oracle.marching_geometry(gl, 0, capacity=cap)
        t1 = time.perf_counter()
        res["geometry_cpu_baseline"] = {"value": g["count"] / (t1 - t0) / 1e6, "unit": "M primitives/s", "cores": 1,
                                        "kind": "oracle",
                                        "sample": f"serial C oracle, separators with points and sides, on "
                                                  f"{tuple(gl.shape)} ({g['count']} triangles), {t1 - t0:.2f} s"}
        del g
    del codes, offs, ws
    return res


def oracle_all_cores(host_fields):
    """The oracle on every field, one call per field in a pool of host threads
    (each call runs in C without the interpreter lock): the all-core CPU
    figure for a set of independent fields.  Returns (seconds, threads)."""
    import concurrent.futures

    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        for _ in ex.map(oracle.segment, host_fields):
            pass
    return time.perf_counter() - t0, threads


def bench_batched(torch, plmss, steps: int, warmup: int, cpu: bool = True):
    """The uneven batch (64 fields, sides 32..192): one plan launch (hipGraph)
    against a loop of plain per-field calls, timed two ways with the same
    synchronisation on both sides: launches only (one device synchronisation
    after the whole batch), and with K read back as a caller would (the plain
    loop reads each field's K after its call; the batch copies all of its
    info words to the host once).  Both include everything from resident
    inputs to labels."""
    from paper_2303_15491_amd import fields

    log("generating the uneven batch")
    host = fields.batch_fields(64, seed=4)
    dev = [torch.from_numpy(f).cuda() for f in host]
    nv = int(sum(f.size for f in host))
    ws = torch.empty(max(plmss.workspace_bytes(t.shape) for t in dev), dtype=torch.uint8, device="cuda")

    def outs_with_infos():
        infos = torch.zeros((len(dev), 4), dtype=torch.int32, device="cuda")
        outs = [{k: torch.empty(t.shape, dtype=torch.int32, device="cuda") for k in ("asc", "desc", "ms")}
                | {"info": infos[i]} for i, t in enumerate(dev)]
        return outs, infos

    outs_plain, _ = outs_with_infos()
    outs_b, infos_b = outs_with_infos()

    def plain_launches():
        for t, o in zip(dev, outs_plain):
            plmss.segment(t, workspace=ws, out=o)

    def plain_read_k():
        for t, o in zip(dev, outs_plain):
            plmss.segment(t, workspace=ws, out=o)
            int(o["info"][3].item())  # the caller reads K

    from paper_2303_15491_amd import autotune

    saved = plmss.tune_get()
    tuned = autotune.tune_batch(dev, use_cache=False, log=log)
    tuned.pop("trials", None)
    needs = plmss.batch_needs(dev)
    plan = plmss.Plan(*needs)
    plan.set(dev, outs=outs_b)
    plan.launch(graph=True)  # the graph keeps the tuned grids
    torch.cuda.synchronize()
    plmss.tune_set(**saved)  # the plain loop runs with the single-field settings

    def batched_launches():
        plan.set(dev, outs=outs_b)
        plan.launch(graph=True)

    def batched_read_k():
        batched_launches()
        infos_b.cpu()  # every field's K in one copy

    for _ in range(warmup):
        plain_read_k()
        batched_read_k()
    torch.cuda.synchronize()
    same = all(torch.equal(a[k], b[k]) for a, b in zip(outs_plain, outs_b) for k in ("asc", "desc", "ms", "info"))
    t_plain, _ = timed_region(plain_launches, steps, torch)
    t_batch, _ = timed_region(batched_launches, steps, torch)
    t_plain_k, _ = timed_region(plain_read_k, steps, torch)
    t_batch_k, _ = timed_region(batched_read_k, steps, torch)
    plan.close()
    t_plain, t_batch, t_plain_k, t_batch_k = (t / steps for t in (t_plain, t_batch, t_plain_k, t_batch_k))
    # the same pair with every field's order field built on both sides
    log("batched and plain loop with order fields")
    plmss.tune_set(**tuned["knobs"])
    plan_o = plmss.Plan(*needs, with_order=True)
    outs_bo = plmss._outs_for(dev, with_order=True)
    plan_o.set(dev, outs=outs_bo)
    plan_o.launch(graph=True)
    torch.cuda.synchronize()
    plmss.tune_set(**saved)
    ws_o = torch.empty(max(plmss.workspace_bytes(t.shape, with_order=True) for t in dev), dtype=torch.uint8,
                       device="cuda")
    outs_po = plmss._outs_for(dev, with_order=True)

    def plain_order():
        for t, o in zip(dev, outs_po):
            plmss.segment(t, with_order=True, workspace=ws_o, out=o)

    def batched_order():
        plan_o.set(dev, outs=outs_bo)
        plan_o.launch(graph=True)

    for _ in range(warmup):
        plain_order()
        batched_order()
    torch.cuda.synchronize()
    same_o = all(torch.equal(a[k], b[k]) for a, b in zip(outs_po, outs_bo)
                 for k in ("asc", "desc", "ms", "order", "info"))
    t_plain_o, _ = timed_region(plain_order, steps, torch)
    t_batch_o, _ = timed_region(batched_order, steps, torch)
    t_plain_o, t_batch_o = t_plain_o / steps, t_batch_o / steps
    plan_o.close()
    del ws_o, outs_po, outs_bo
    torch.cuda.empty_cache()
    cpu_all = None
    if cpu:
        log("oracle on every field of the batch, all host cores")
        secs, threads = oracle_all_cores(host)
        model, ncpu = cpu_info()
        cpu_all = {"value": nv / secs / 1e6, "unit": "Mvertices/s", "cores": threads, "kind": "oracle",
                   "sample": f"all 64 fields, one serial oracle call per field on {threads} host threads, "
                             f"{secs:.2f} s", "host_cpu": model, "host_nproc": ncpu}
    return {"workload": "64 fields, sides uniform in 32..192, sum of 16..256 Gaussians + N(0,0.02) (seeds 4+j)",
            "vertices": nv, "batched_ms": t_batch, "plain_loop_ms": t_plain,
            "batched_mvps": nv / t_batch / 1e3, "plain_loop_mvps": nv / t_plain / 1e3,
            "speedup": t_plain / t_batch,
            "timing": "launches only; one device synchronisation after all steps on each side",
            "with_k_read": {"batched_ms": t_batch_k, "plain_loop_ms": t_plain_k, "speedup": t_plain_k / t_batch_k,
                            "timing": "plain loop reads K after every field; the batch copies its info words "
                                      "once"},
            "with_order_fields": {"batched_ms": t_batch_o, "plain_loop_ms": t_plain_o,
                                  "batched_mvps": nv / t_batch_o / 1e3, "plain_loop_mvps": nv / t_plain_o / 1e3,
                                  "speedup": t_plain_o / t_batch_o, "identical": bool(same_o),
                                  "timing": "launches only, as above; every field's order field built"},
            "cpu_all_cores": cpu_all, "identical": bool(same), "tuned": tuned}


def bench_serving(torch, plmss, n_requests: int, rate: float, saturate_rate: float, cpu: bool = True):
    """Poisson arrivals of mixed 2-D (128^2..2048^2) and 3-D (64^3..384^3)
    requests through the continuous-batching server, in real time: at the
    workload's rate, and at a rate far above what the GPU sustains (its
    capacity).  Beside them the plain loop over the same requests in arrival
    order: upload, plmss_segment, wait, one request at a time."""
    from paper_2303_15491_amd import fields
    from paper_2303_15491_amd.serve import Server, run_trace

    log("generating the serving pool")
    pool_n = 64
    _, pool_np = fields.serving_pool(pool_n, seed=5)
    pool = [torch.from_numpy(f).pin_memory() for f in pool_np]
    sizes = [tuple(p.shape) for p in pool]

    def trace_at(r):
        tr = fields.serving_trace(n_requests, seed=5, rate=r)
        for i, req in enumerate(tr):  # every request is one of the pool's fields
            req["shape"] = sizes[i % pool_n]
        return tr

    def served(r):
        trace = trace_at(r)
        server = Server(budget_bytes=48 << 30, max_batch_vertices=64 << 20, max_batch_fields=32)
        # warm-up: compile the graphs on a few requests
        run_trace(server, trace[:16], lambda i, q: pool[i % pool_n], realtime=False)
        server.done.clear()
        server.batch_sizes.clear()
        log(f"serving {n_requests} requests at {r}/s")
        run_trace(server, trace, lambda i, q: pool[i % pool_n], realtime=True)
        st = server.stats()
        server.close()
        st.update({"rate_per_s": r,
                   "offered_mvps": sum(int(np.prod(q["shape"])) for q in trace) / trace[-1]["t"] / 1e6})
        return st

    res = served(rate)
    res["saturated"] = served(saturate_rate)
    # the plain loop: one request after the other
    log("plain per-request loop")
    ws = torch.empty(max(plmss.workspace_bytes(s) for s in sizes), dtype=torch.uint8, device="cuda")
    devbuf = [torch.empty(s, dtype=torch.float32, device="cuda") for s in sizes]
    outs = [{k: torch.empty(s, dtype=torch.int32, device="cuda") for k in ("asc", "desc", "ms")}
            | {"info": torch.empty(4, dtype=torch.int32, device="cuda")} for s in sizes]
    order = [i % pool_n for i in range(n_requests)]
    for i in order[:8]:
        devbuf[i].copy_(pool[i], non_blocking=True)
        plmss.segment(devbuf[i], workspace=ws, out=outs[i])
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i in order:
        t = time.perf_counter()
        devbuf[i].copy_(pool[i], non_blocking=True)
        plmss.segment(devbuf[i], workspace=ws, out=outs[i])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
    wall = time.perf_counter() - t0
    verts = sum(int(np.prod(sizes[i])) for i in order)
    res["plain_loop"] = {"requests": n_requests, "wall_s": wall, "throughput_mvps": verts / wall / 1e6,
                         "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                         "timing": "upload from page-locked memory, plmss_segment, device synchronisation, per "
                                   "request, back to back (no arrival gaps)"}
    res["saturated_vs_plain_loop"] = res["saturated"]["throughput_mvps"] / res["plain_loop"]["throughput_mvps"]
    if cpu:
        log("oracle on the serving pool's fields, all host cores")
        secs, threads = oracle_all_cores(pool_np)
        model, ncpu = cpu_info()
        pv = sum(int(f.size) for f in pool_np)
        res["cpu_all_cores"] = {"value": pv / secs / 1e6, "unit": "Mvertices/s", "cores": threads, "kind": "oracle",
                                "sample": f"the 64 distinct request fields of the mix ({pv} vertices), one serial "
                                          f"oracle call per field on {threads} host threads, {secs:.2f} s",
                                "host_cpu": model, "host_nproc": ncpu}
    res["workload"] = ("Poisson arrivals; half 2-D n^2 (n in 128..2048), half 3-D n^3 (n in 64..384), smoothed "
                       "N(0,1) noise, sigma 1.5..4 (seed 5)")
    del ws, devbuf, outs
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--cpu-slab", type=int, default=128,
                    help="planes of the field the CPU oracle segments for the baseline (0 = skip)")
    ap.add_argument("--no-batched", action="store_true", help="skip the uneven-batch measurement")
    ap.add_argument("--serve-requests", type=int, default=2000, help="serving requests (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-saturate-rate", type=float, default=5000.0,
                    help="arrival rate of the serving capacity run (far above what the GPU sustains)")
    ap.add_argument("--knobs", default=None,
                    help='launch-shape knobs as JSON (e.g. {"scan_depth": 8}); skips the autotuner')
    ap.add_argument("--no-float64", action="store_true", help="skip the float64 copy of the field")
    ap.add_argument("--no-marching", action="store_true", help="skip the marching index over the MS labels")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device three times (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the segmentation of one field runs on one device)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2303_15491_amd as plmss

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 4, "copy_probe_bytes_written": dst.numel() * 4,
                          "launches": 3}))
        return
    lib = plmss.library()
    log(f"generating workload {args.workload}")
    f_host, desc = workload(args.workload)
    n = int(f_host.size)
    dev = torch.device("cuda:0")
    field = torch.from_numpy(f_host).to(dev)
    dims = plmss.dims_of(field.shape)
    code = plmss.F64 if field.dtype == torch.float64 else plmss.F32
    outs = {k: torch.empty(field.shape, dtype=torch.int32, device=dev) for k in ("asc", "desc", "ms", "order")}
    outs["info"] = torch.zeros(4, dtype=torch.int32, device=dev)
    ws_bytes = lib.plmss_workspace_bytes(dims, code, 1)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def make_job(with_order):
        return plmss.Job(field.data_ptr(), dims, code, outs["asc"].data_ptr(), outs["desc"].data_ptr(),
                         outs["ms"].data_ptr(), outs["order"].data_ptr() if with_order else None,
                         outs["info"].data_ptr())

    job_full, job_labels = make_job(True), make_job(False)

    def step_full():
        rc = lib.plmss_segment(ctypes.byref(job_full), ctypes.c_void_p(ws.data_ptr()), ws_bytes, stream)
        if rc:
            raise plmss.PlmssError(rc, "plmss_segment")

    def step_labels():
        rc = lib.plmss_segment(ctypes.byref(job_labels), ctypes.c_void_p(ws.data_ptr()), ws_bytes, stream)
        if rc:
            raise plmss.PlmssError(rc, "plmss_segment")

    max_launches = 128 * max(args.steps, 1)
    trace = lib.plmss_trace_create(max_launches)
    if not trace:
        raise RuntimeError("plmss_trace_create failed")

    from paper_2303_15491_amd import autotune

    if args.knobs:
        plmss.tune_set(**json.loads(args.knobs))
        tuned = {"knobs": plmss.tune_get(), "given": True}
    else:
        log("autotuning launch shapes")
        t_tune = time.perf_counter()
        tuned = autotune.tune_segment(field, with_order=True, use_cache=False, log=log)
        tuned["seconds"] = time.perf_counter() - t_tune
        tuned.pop("trials", None)
    knobs = plmss.tune_get()
    log(f"tuned: {tuned}")
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step_full()
        step_labels()
    torch.cuda.synchronize()
    info = outs["info"].cpu().tolist()
    if info[0] != 0:
        raise RuntimeError(f"device status {info[0]}")

    # the throughput comes from untraced steps; the per-kernel times from the
    # same number of steps again with a HIP event pair around every launch
    # (the events add a little time of their own)
    log(f"timing {args.steps} full steps")
    steps_full, steps_labels = [], []
    wall_full, _ = timed_region(step_full, args.steps, torch, per_step=steps_full)
    log(f"timing {args.steps} label-only steps")
    wall_labels, _ = timed_region(step_labels, args.steps, torch, per_step=steps_labels)
    log(f"timing {args.steps} full and {args.steps} label-only steps with per-kernel events")
    wall_full_traced, launches = timed_region(step_full, args.steps, torch, lib, trace, max_launches)
    wall_labels_traced, launches_l = timed_region(step_labels, args.steps, torch, lib, trace, max_launches)
    lib.plmss_trace_destroy(trace)
    copy_gbs = copy_bandwidth(torch)

    ms_step = wall_full / args.steps
    value = n / (ms_step * 1e-3) / 1e6
    ms_step_l = wall_labels / args.steps
    kern = per_kernel(launches, args.steps)
    kern_l = per_kernel(launches_l, args.steps)

    # roofline of the dominant kernel of the full step
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    avg_ms = kern[dom]["avg_launch_ms"]
    bpv = algo_bytes(dom, knobs["order_invert"])
    if bpv is not None:
        per_launch_bytes = bpv * n
        basis = f"{bpv:g} B/vertex x {n} vertices per launch"
    else:
        per_launch_bytes = None
        basis = "n/a"
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9 if per_launch_bytes else None
    counters, traffic_src = profile_entry("hbm_traffic", args.workload, dom, knobs)
    traffic = counters["hbm_bytes_per_dispatch"] if counters else None
    stats, stats_src = profile_entry("kernel_stats", args.workload, dom, knobs)
    rocprof_ms = stats["avg_us"] * 1e-3 if stats else None
    roofline = {"bound": "hbm", "kernel": dom, "symbol": HEADLINE_SYMBOLS.get(dom), "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "traffic_source": traffic_src, "avg_launch_ms": avg_ms,
                "avg_launch_source": "HIP events around every launch of the kind, on its own stream, in this run",
                "rocprof_avg_launch_ms": rocprof_ms, "rocprof_source": stats_src,
                "frac_at_rocprof_time": (per_launch_bytes / (rocprof_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                         if rocprof_ms and per_launch_bytes else None),
                "algorithmic_bytes_per_launch": per_launch_bytes, "basis": basis,
                "kernel_source_digest": kernel_source_digest(),
                "copy_probe_gbs": copy_gbs,
                "copy_probe": "device-to-device copy of 1 GiB (read + write bytes / time), median of 5"}
    # the next kinds by time per step, each against its own algorithmic bytes
    # (at 512^3 the chase and the two middle radix scatters are within a few
    # percent of each other, so either can come out on top)
    top = []
    for k in sorted(kern, key=lambda k: -kern[k]["ms_per_step"])[:4]:
        b = algo_bytes(k, knobs["order_invert"])
        a = b * n / (kern[k]["avg_launch_ms"] * 1e-3) / 1e9 if b else None
        top.append({"kind": k, "symbol": HEADLINE_SYMBOLS.get(k), "ms_per_step": kern[k]["ms_per_step"],
                    "avg_launch_ms": kern[k]["avg_launch_ms"], "algorithmic_bytes_per_vertex": b,
                    "frac": a / HBM_PEAK_GBS if a else None})
    roofline["top_kinds"] = top

    # CPU baseline: the oracle on a bounded slab of the same field, one core
    cpu = None
    if args.cpu_slab > 0:
        import oracle

        sl = f_host[: args.cpu_slab] if f_host.ndim == 3 else f_host
        log(f"cpu baseline on {sl.shape}")
        t0 = time.perf_counter()
        oracle.segment(np.ascontiguousarray(sl))
        t1 = time.perf_counter()
        model, ncpu = cpu_info()
        cpu = {"value": sl.size / (t1 - t0) / 1e6, "unit": "Mvertices/s", "cores": 1, "kind": "oracle",
               "sample": f"serial C oracle (order field, steepest, labels, MS ids) on the first "
                         f"{sl.shape[0] if sl.ndim == 3 else 1} planes {tuple(sl.shape)} of the same field, "
                         f"{t1 - t0:.2f} s", "host_cpu": model, "host_nproc": ncpu}

    labels_value = n / (ms_step_l * 1e-3) / 1e6
    f64 = None
    if field.dtype == torch.float32 and not args.no_float64:
        log("float64 copy of the field")
        step_full()  # the outputs to compare against: the full path's
        torch.cuda.synchronize()
        f64 = bench_float64_copy(torch, plmss, lib, field, outs, steps=max(3, args.steps // 2), warmup=2)
    marching = None
    if not args.no_marching and field.ndim >= 2:
        log("marching index over the MS labels")
        step_full()
        torch.cuda.synchronize()
        marching = bench_marching(torch, plmss, lib, outs["ms"], steps=args.steps, warmup=2,
                                  cpu_planes=args.cpu_slab if field.ndim == 3 else 0)
    del ws, outs, field
    torch.cuda.empty_cache()
    if marching is not None and f_host.ndim == 3:
        # the triangle (2-D) kernels on a 4096^2 terrain-like field (smoothed
        # noise, sigma 1.5): its MS labels through the same index and geometry
        from paper_2303_15491_amd import fields as _fields

        log("marching index and geometry on a 4096^2 field")
        t2 = torch.from_numpy(_fields.smoothed_noise((4096, 4096), 1.5, seed=6)).to(dev)
        seg = plmss.segment(t2)
        torch.cuda.synchronize()
        marching["planar_4096sq"] = bench_marching(torch, plmss, lib, seg["ms"], steps=args.steps, warmup=2,
                                                   cpu_planes=0)
        del t2, seg
        torch.cuda.empty_cache()
    batched = (None if args.no_batched else
               bench_batched(torch, plmss, steps=max(3, args.steps // 2), warmup=2, cpu=args.cpu_slab > 0))
    serving = (bench_serving(torch, plmss, args.serve_requests, args.serve_rate, args.serve_saturate_rate,
                             cpu=args.cpu_slab > 0) if args.serve_requests else None)
    out = {
        "metric": METRIC, "value": value, "unit": "Mvertices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": desc, "n_vertices": n, "field_dtype": str(f_host.dtype), "order_field": True,
                   "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "tuned": tuned,
        "path_frac_of_hbm_roofline": n * 48.0 / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "step_times": step_stats(steps_full),
        "step_times_note": "per-step device times (events between steps): the mean of the middle runs "
                           "(best and worst dropped, the paper's protocol) and the median; value and "
                           "ms_per_step are the wall time over all timed steps",
        "labels_only": {"value": labels_value, "ms_per_step": ms_step_l, "step_times": step_stats(steps_labels),
                        "path_frac_of_hbm_roofline": n * 48.0 / (ms_step_l * 1e-3) / (HBM_PEAK_GBS * 1e9),
                        "note": "same labels, order field not materialised (vertex order compared in place)"},
        "ms_per_step_traced": wall_full_traced / args.steps,
        "ms_per_step_labels_only_traced": wall_labels_traced / args.steps,
        "kernels_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in sorted(kern.items())},
        "kernels_ms_per_step_labels_only": {k: round(v["ms_per_step"], 4) for k, v in sorted(kern_l.items())},
        "float64_copy": f64,
        "marching_index": marching,
        "batched": batched,
        "serving": serving,
        "paper_context": "PLMSS Asc/Desc+MS on Miranda 512^3 (a different, simplified field): 57.6 Mvertices/s "
                         "on 24 Xeon SP 6126 cores, 3.36 on 1 core (Table 2)",
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
