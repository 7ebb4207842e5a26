"""Autotuner for the library's launch shapes.

The library exposes a few knobs (``plmss_tune_set``): the blocks of each
order-field radix pass, how the order field is inverted, whether 32-bit keys
travel packed with their ids, the grid of the device-sized pair sort, the
z-depth of the 3-D neighbour-scan tiles and their in-tile compression sweeps,
and the grid of a plan's persistent launches.  None of them changes a result; they
trade occupancy, tile-local path compression and write locality against each
other, and the best values depend on the field's size and shape.

``tune_segment`` and ``tune_batch`` time candidate values on the actual
inputs (coordinate descent: one knob at a time, the others held, each
candidate timed with HIP events over a few repetitions, the median kept),
check that every candidate produces exactly the labels of the starting
configuration, keep a candidate only when it is at least 1% faster twice in a
row (the candidate and the current best are timed again before it replaces
the best), leave the winners set, and remember them in a JSON cache keyed
by GPU architecture, element type, workload kind, dimensionality and size
bucket (log2 of the vertex count).  ``apply`` sets cached values without
timing anything.
"""
from __future__ import annotations

import json
import math
import os
import threading

from . import KNOBS, Plan, PlmssError, batch_needs, segment, tune_get, tune_set

SPACE = {
    "order_workers": [0, 8192, 16384, 4096],
    "order_invert": [1, 0, 2, 4],
    "order_packed": [1, 0],
    "scan_rounds": [3, 2, 4],
    "order_concurrent": [0, 1],  # not tuned by default: overlapping streams blur per-kernel times
    "packed_codes": [1, 0],  # not tuned by default: the packed form is the faster one where it applies
    "sort_workers": [512, 256, 1024, 2048, 4096],
    "scan_depth": [8, 16, 32],
    "persist_blocks": [512, 1024, 2048, 4096, 8192, 16384],
    "pair_stream": [2, 0, 1],
}

SEGMENT_KNOBS = ("scan_depth", "scan_rounds", "sort_workers", "pair_stream")
ORDER_KNOBS = ("order_workers", "order_invert", "order_packed")
BATCH_KNOBS = ("persist_blocks", "scan_depth", "scan_rounds", "sort_workers", "pair_stream")

# a candidate replaces the current setting only when it is this much faster,
# so that timing noise does not flip settings from run to run
MIN_GAIN = 0.01

_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("PLMSS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "plmss", "tune.json"))


def _arch(torch) -> str:
    try:
        return str(torch.cuda.get_device_properties(0).gcnArchName).split(":")[0]
    except Exception:
        return "unknown"


def cache_key(arch: str, dtype: str, kind: str, ndim: int, nvertices: int) -> str:
    bucket = int(round(math.log2(max(int(nvertices), 1))))
    return f"{arch}|{dtype}|{kind}|{ndim}d|2^{bucket}"


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(key: str, values: dict):
    with _lock:
        data = _load()
        data[key] = values
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)


def lookup(key: str):
    v = _load().get(key)
    return {k: int(x) for k, x in v.items() if k in KNOBS} if isinstance(v, dict) else None


def apply(key: str) -> bool:
    """Sets the cached knob values of ``key``; False when there are none."""
    v = lookup(key)
    if not v:
        return False
    tune_set(**v)
    return True


def _time(torch, fn, reps: int) -> float:
    """Median milliseconds of ``fn`` on the current stream (one untimed run first)."""
    fn()
    times = []
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def _descend(torch, knobs, run, result, reps: int, log=None):
    """Coordinate descent over ``knobs``; ``run()`` executes the workload once
    (asynchronously) and ``result()`` copies its outputs; every candidate must
    reproduce the starting configuration's outputs exactly."""
    best = {k: tune_get()[k] for k in knobs}
    tune_set(**best)
    run()
    ref = result()
    base_ms = _time(torch, run, reps)
    trials = [{"knobs": dict(best), "ms": base_ms}]
    best_ms = base_ms
    for k in knobs:
        for v in SPACE[k]:
            if v == best[k]:
                continue
            cand = dict(best, **{k: v})
            tune_set(**cand)
            run()
            if not _same(ref, result()):
                tune_set(**best)
                raise RuntimeError(f"knobs {cand} changed the result")
            ms = _time(torch, run, reps)
            trials.append({"knobs": cand, "ms": ms})
            if log:
                log(f"tune {cand}: {ms:.3f} ms")
            if ms < best_ms * (1.0 - MIN_GAIN):
                # confirm: time the current best and the candidate once more
                tune_set(**best)
                again_best = _time(torch, run, reps)
                tune_set(**cand)
                again = _time(torch, run, reps)
                if log:
                    log(f"tune confirm {cand}: {again:.3f} ms against {again_best:.3f} ms")
                if again < again_best * (1.0 - MIN_GAIN):
                    best, best_ms = cand, min(ms, again)
                else:
                    best_ms = min(best_ms, again_best)
        tune_set(**best)
    return best, best_ms, base_ms, trials


def _same(a, b) -> bool:
    import torch

    if isinstance(a, dict):
        return all(torch.equal(a[k], b[k]) for k in a)
    return all(_same(x, y) for x, y in zip(a, b))


def tune_segment(field, with_order: bool = False, reps: int = 5, use_cache: bool = True, log=None) -> dict:
    """Tunes the single-field path on ``field`` (a device tensor); returns
    {"key", "knobs", "ms", "baseline_ms", "cached"}."""
    import torch

    dtype = "f64" if field.dtype == torch.float64 else "f32"
    kind = "segment+order" if with_order else "segment"
    key = cache_key(_arch(torch), dtype, kind, field.dim(), field.numel())
    if use_cache and apply(key):
        return {"key": key, "knobs": lookup(key), "cached": True}
    knobs = SEGMENT_KNOBS + (ORDER_KNOBS if with_order else ())
    if field.dim() < 3:
        knobs = tuple(k for k in knobs if k != "scan_depth")
    out = {k: torch.empty(field.shape, dtype=torch.int32, device=field.device) for k in ("asc", "desc", "ms")}
    if with_order:
        out["order"] = torch.empty(field.shape, dtype=torch.int32, device=field.device)
    out["info"] = torch.empty(4, dtype=torch.int32, device=field.device)
    ws = torch.empty(segment_workspace(field, with_order), dtype=torch.uint8, device=field.device)

    def run():
        segment(field, with_order=with_order, workspace=ws, out=out)

    def result():
        return {k: v.clone() for k, v in out.items()}

    best, ms, base, trials = _descend(torch, knobs, run, result, reps, log)
    _store(key, best)
    return {"key": key, "knobs": best, "ms": ms, "baseline_ms": base, "trials": len(trials), "cached": False}


def segment_workspace(field, with_order: bool) -> int:
    from . import workspace_bytes

    return workspace_bytes(field.shape, field.dtype, with_order)


def tune_batch(fields, reps: int = 5, use_cache: bool = True, log=None) -> dict:
    """Tunes capacity-plan launches (hipGraph replays) on a batch of device
    fields; a fresh plan is built per candidate, since a plan keeps the scan
    depth it was created with and its graph the grids it was captured with."""
    import torch

    nv = sum(int(f.numel()) for f in fields)
    dtype = "f64" if fields[0].dtype == torch.float64 else "f32"
    key = cache_key(_arch(torch), dtype, "batch", max(f.dim() for f in fields), nv)
    if use_cache and apply(key):
        return {"key": key, "knobs": lookup(key), "cached": True}
    state = {}

    def run():
        knobs = tuple(tune_get()[k] for k in BATCH_KNOBS)
        if state.get("knobs") != knobs:
            if state.get("plan") is not None:
                state["plan"].close()
            plan = Plan(*batch_needs(fields), dtype=fields[0].dtype)
            state.update(plan=plan, knobs=knobs, outs=None)
        plan = state["plan"]
        state["outs"] = plan.set(fields, outs=state["outs"])
        plan.launch(graph=True)

    def result():
        return [{k: v.clone() for k, v in o.items()} for o in state["outs"]]

    try:
        best, ms, base, trials = _descend(torch, BATCH_KNOBS, run, result, reps, log)
    finally:
        if state.get("plan") is not None:
            state["plan"].close()
    _store(key, best)
    return {"key": key, "knobs": best, "ms": ms, "baseline_ms": base, "trials": len(trials), "cached": False}


__all__ = ["SPACE", "tune_segment", "tune_batch", "apply", "lookup", "cache_key", "cache_path", "PlmssError"]
