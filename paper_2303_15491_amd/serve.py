"""Continuous-batching segmentation server.

Requests (a host field) arrive at any time.  The server admits a request when
its device footprint fits the HBM budget and a slot is free, uploads it on a
copy stream, and folds every uploaded request into the next batch.  Batches
run through capacity plans (one replayable hipGraph per plan, see
``Plan``); two plans on two compute streams alternate, so a batch's kernels
run while the next batch is being formed, uploaded and launched.  Labels stay
resident on the device until the caller takes them.  Each request records its
arrival, launch and completion times; ``stats()`` reports throughput and
latency percentiles.

Results are the same as ``segment`` of the request alone: a field's labels
never depend on the other fields of its batch.
"""
from __future__ import annotations

import collections
import threading
import time

import numpy as np

from . import Plan, PlmssError, batch_needs, dims_of  # noqa: F401


def _numel(r) -> int:
    return int(np.prod(r.shape))


ADMIT, WAIT, REJECT_BATCH, REJECT_BUDGET = "admit", "wait", "reject: batch", "reject: budget"


def admission(numel: int, nbytes: int, resident: int, queued: int, max_vertices: int, budget: int,
              max_queued: int) -> str:
    """What the server does with the request at the head of the queue: a
    request that can never run (more vertices than one batch holds, or a
    footprint above the whole budget) is rejected at once, so that it never
    blocks the queue; one that does not fit next to the requests already
    resident, or finds the upload queue full, waits; any other is admitted."""
    if numel > max_vertices:
        return REJECT_BATCH
    if nbytes > budget:
        return REJECT_BUDGET
    if resident + nbytes > budget or queued >= max_queued:
        return WAIT
    return ADMIT


class Request:
    __slots__ = ("rid", "host", "shape", "t_arrive", "t_admit", "t_launch", "t_done", "device", "out",
                 "event", "nbytes", "error", "staged")

    def __init__(self, rid, host, t_arrive):
        self.rid = rid
        self.host = host
        self.shape = host.shape
        self.t_arrive = t_arrive
        self.t_admit = self.t_launch = self.t_done = None
        self.device = self.out = self.event = self.staged = None
        self.error = None
        n = int(np.prod(host.shape))
        itemsize = host.element_size() if hasattr(host, "element_size") else host.itemsize
        # field + asc/desc/ms + info
        self.nbytes = n * itemsize + 3 * 4 * n + 16


class Server:
    """``budget_bytes``: device memory requests may hold at once (fields and
    labels).  ``max_batch_vertices`` / ``max_batch_fields``: capacity of one
    batch.  Requests larger than one batch are rejected."""

    def __init__(self, budget_bytes: int, max_batch_vertices: int, max_batch_fields: int = 64,
                 device="cuda", dtype=None, keep_results: bool = False):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.dtype = dtype or torch.float32
        self.budget = int(budget_bytes)
        self.max_v = int(max_batch_vertices)
        self.max_f = int(max_batch_fields)
        # scan and chase tiles: generous bounds for fields of at least 32^3 or
        # 128^2 vertices (tile padding)
        max_tiles = self.max_v // 1024 + 16 * self.max_f
        self.plans = [Plan(self.max_v, self.max_f, max_tiles, max_tiles, dtype=self.dtype, device=device)
                      for _ in range(2)]
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(2)]
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.keep_results = keep_results
        self.pending = collections.deque()  # arrived, not admitted
        self.admitted = collections.deque()  # uploaded (or uploading), not launched
        self.inflight = []  # (plan index, [requests], done event)
        self.done = []
        self.resident = 0
        self.next_plan = 0
        self.rejected = 0
        self.batch_sizes = collections.Counter()  # fields per launched batch -> launches
        self.lock = threading.Lock()

    # -- submission --------------------------------------------------------------------
    def submit(self, rid, host_field, t_arrive: float | None = None) -> Request:
        """host_field: a numpy array or a (preferably pinned) host tensor."""
        if not isinstance(host_field, self.torch.Tensor):
            host_field = np.ascontiguousarray(host_field)
        r = Request(rid, host_field, time.perf_counter() if t_arrive is None else t_arrive)
        with self.lock:
            self.pending.append(r)
        return r

    # -- one scheduling round ----------------------------------------------------------
    def _admit(self):
        torch = self.torch
        while self.pending:
            r = self.pending[0]
            decision = admission(_numel(r), r.nbytes, self.resident, len(self.admitted), self.max_v, self.budget,
                                4 * self.max_f)
            if decision == REJECT_BATCH or decision == REJECT_BUDGET:
                self.pending.popleft()
                r.error = "too large for one batch" if decision == REJECT_BATCH else "larger than the memory budget"
                self.rejected += 1
                continue
            if decision == WAIT:
                break
            self.pending.popleft()
            self.resident += r.nbytes
            r.t_admit = time.perf_counter()
            with torch.cuda.stream(self.copy_stream):
                # a host field already in page-locked memory is uploaded as is
                src = r.host if isinstance(r.host, torch.Tensor) else torch.from_numpy(r.host)
                if not src.is_pinned():
                    src = src.pin_memory()
                r.staged = src  # alive until the upload is done
                r.device = torch.empty(r.shape, dtype=self.dtype, device=self.device)
                r.device.copy_(src, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.copy_stream)
            r.event = ev
            self.admitted.append(r)

    def _retire(self, block: bool = False):
        still = []
        for pi, reqs, ev in self.inflight:
            if block:
                ev.synchronize()
            if ev.query():
                t = time.perf_counter()
                for r in reqs:
                    r.t_done = t
                    self.resident -= r.nbytes
                    r.device = None
                    r.staged = None  # its upload finished before the batch ran
                    if not self.keep_results:
                        r.out = None
                    self.done.append(r)
            else:
                still.append((pi, reqs, ev))
        self.inflight = still

    def _launch(self):
        torch = self.torch
        if not self.admitted:
            return False
        # a plan whose previous batch is still running cannot be refilled
        busy = {pi for pi, _, _ in self.inflight}
        pi = self.next_plan
        if pi in busy:
            pi = 1 - pi
            if pi in busy:
                return False
        batch, nv = [], 0
        while self.admitted and len(batch) < self.max_f and nv + _numel(self.admitted[0]) <= self.max_v:
            r = self.admitted.popleft()
            batch.append(r)
            nv += _numel(r)
        if not batch:
            return False
        stream = self.streams[pi]
        fields = [r.device for r in batch]
        plan = self.plans[pi]
        with torch.cuda.stream(stream):
            while True:
                try:
                    outs = plan.set(fields, stream=stream)
                    break
                except PlmssError:
                    # beyond the plan's tile capacity: send the tail back
                    if len(batch) == 1:
                        raise
                    half = len(batch) // 2
                    for r in reversed(batch[half:]):
                        self.admitted.appendleft(r)
                    batch, fields = batch[:half], fields[:half]
            for r in batch:
                stream.wait_event(r.event)
                if r.event.query():
                    r.staged = None  # the upload is done: drop the page-locked copy
            t = time.perf_counter()
            plan.launch(graph=True, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        for r, o in zip(batch, outs):
            r.out = o
            r.t_launch = t
        self.inflight.append((pi, batch, ev))
        self.batch_sizes[len(batch)] += 1
        self.next_plan = 1 - pi
        return True

    def step(self):
        """One round: retire finished batches, admit, launch what is ready."""
        with self.lock:
            self._retire()
            self._admit()
            self._launch()

    def drain(self):
        while True:
            with self.lock:
                self._retire()
                self._admit()
                launched = self._launch()
                idle = not self.pending and not self.admitted
            if idle and not launched:
                with self.lock:
                    self._retire(block=True)
                    if not self.inflight:
                        return
            elif not launched:
                with self.lock:
                    self._retire(block=True)

    # -- report ------------------------------------------------------------------------
    def stats(self):
        lat = np.array([r.t_done - r.t_arrive for r in self.done if r.t_done is not None])
        verts = sum(int(np.prod(r.shape)) for r in self.done)
        if len(lat) == 0:
            return {"requests": 0}
        t0 = min(r.t_arrive for r in self.done)
        t1 = max(r.t_done for r in self.done)
        return {"requests": len(self.done), "rejected": self.rejected, "vertices": verts,
                "wall_s": t1 - t0, "throughput_mvps": verts / (t1 - t0) / 1e6,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
                "batches": int(sum(self.batch_sizes.values())),
                "batch_size_histogram": {int(k): int(v) for k, v in sorted(self.batch_sizes.items())}}

    def close(self):
        for p in self.plans:
            p.close()


def run_trace(server: Server, trace, make_field, realtime: bool = True):
    """Feeds a list of {"t": arrival offset (s), ...} requests to the server
    (sleeping until each arrival when realtime), stepping the scheduler in
    between, then drains it.  make_field(i, req) returns the host field."""
    start = time.perf_counter()
    reqs = []
    i = 0
    while i < len(trace):
        now = time.perf_counter() - start
        while i < len(trace) and (not realtime or trace[i]["t"] <= now):
            arr = start + trace[i]["t"] if realtime else time.perf_counter()
            reqs.append(server.submit(i, make_field(i, trace[i]), t_arrive=arr))
            i += 1
        server.step()
        if realtime and i < len(trace):
            wait = start + trace[i]["t"] - time.perf_counter()
            if wait > 0:
                time.sleep(min(wait, 0.0005))
    server.drain()
    return reqs
