"""Batched counting: many independent jobs (streams, or hash-seed replicas of one stream) in
one persistent launch of the counting kernel, optionally captured in a HIP graph, with a
launch shape chosen by a small autotuner.

A job is one counting pass (all processors) of one built graph with its own REPT parameters
and output buffers; replicas of one stream share the built graph and differ only in the hash
seed.  The device work queue interleaves all jobs' apexes, so a batch of uneven jobs keeps
every compute unit busy until the last job finishes.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass, field

from . import rept


@dataclass
class Job:
    graph: "rept.Graph"
    params: "rept.Params"
    out: tuple = None            # (global int64[c], local int64[rows, n]) device tensors
    t0: int = 0
    t1: int = rept.UINT64_MAX
    unit0: int = 0
    unit1: int = rept.UINT32_MAX
    accumulate: bool = False
    workspace: object = None     # device slot table of (graph, params); allocated on demand
    table_ready: bool = False    # the workspace already holds it (written by an earlier launch)

    def ensure_outputs(self):
        if self.out is None:
            self.out = self.graph.outputs(self.params)
        return self.out

    def ensure_workspace(self):
        if self.workspace is None:
            self.workspace = self.graph.new_workspace(self.params)
        return self.workspace

    def c_job(self) -> "rept.rept_job":
        return rept.make_job(self.graph, self.params, self.ensure_outputs(), self.ensure_workspace(), t0=self.t0,
                             t1=self.t1, unit0=self.unit0, unit1=self.unit1, accumulate=self.accumulate,
                             table_ready=self.table_ready)


class Batch:
    """A prepared batch: job table written to a device workspace once; launch() replays it."""

    def __init__(self, jobs: list, tuning=None, stream=None):
        import torch
        if not jobs:
            raise ValueError("empty batch")
        self.jobs = list(jobs)
        self.device = self.jobs[0].graph.device
        self.tuning = tuning
        nbytes = rept.rept_batch_workspace_size(len(self.jobs))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._stream = stream
        self._graph = None
        rept.rept_batch_prepare([j.c_job() for j in self.jobs], tuning, self.workspace.data_ptr(),
                                self.workspace.numel(), rept._stream_ptr(stream))

    def launch(self, stream=None):
        """Enqueue the batch on `stream` (asynchronous)."""
        rept.rept_batch_launch(self.workspace.data_ptr(), rept._stream_ptr(stream or self._stream))

    def capture(self):
        """Capture one launch in a HIP graph; replay() then re-runs it with one graph launch.
        The launch clears its own queue counters and outputs with kernels (no memset nodes)."""
        import torch
        self.launch()  # make sure attributes and code objects are resident before capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            rept.rept_batch_launch(self.workspace.data_ptr(), torch.cuda.current_stream().cuda_stream)
        self._graph = g
        return self

    def replay(self):
        if self._graph is None:
            raise RuntimeError("capture() first")
        self._graph.replay()

    @property
    def stream_edges(self) -> int:
        return sum(j.graph.num_edges for j in self.jobs)


# ---------------------------------------------------------------------------------- autotuner

DEFAULT_CANDIDATES = [
    dict(),  # library defaults (wave_cap 64, b_chunk 128, 256 threads, grid from occupancy)
    dict(wave_cap=32),
    dict(wave_cap=128),
    dict(b_chunk=64),
    dict(b_chunk=256),
    dict(light_tile=2),
    dict(light_tile=32),
    dict(threads=512),
    dict(threads=512, b_chunk=256),  # R-MAT scale 24: 280 ms against 302 at the default shape
    dict(phase_launches=1),  # both phases in one launch (the 1M/20M power-law stream: 5.61 ms, 5.72 split)
]


def signature(jobs: list) -> str:
    """Bucketed description of a job set: the launch shape that wins depends on the amount of
    work, the longest apex list, the hash groups and processors, and the local layout."""
    work = sum(j.graph.info.oriented_work for j in jobs)
    max_out = max(j.graph.info.max_out_degree for j in jobs)
    G = max(j.params.groups for j in jobs)
    c = max(j.params.c for j in jobs)
    pp = any(j.params.per_proc for j in jobs)
    return (f"jobs{2 ** math.ceil(math.log2(len(jobs)))}-work{round(math.log2(work + 1))}"
            f"-maxout{2 ** math.ceil(math.log2(max_out + 1))}-G{G}-c{2 ** math.ceil(math.log2(c))}-pp{int(pp)}")


@dataclass
class Autotuner:
    """Times each candidate launch shape on the real job set (median of `reps` launches after
    one warm-up) and keeps the fastest per signature.  Every candidate computes the same
    integers; only time differs.  The cache can be kept in a JSON file."""
    candidates: list = field(default_factory=lambda: list(DEFAULT_CANDIDATES))
    reps: int = 3
    cache_path: str | None = None
    cache: dict = field(default_factory=dict)
    log: list = field(default_factory=list)

    def __post_init__(self):
        if self.cache_path and os.path.exists(self.cache_path):
            with open(self.cache_path) as f:
                self.cache = json.load(f)

    def best(self, jobs: list, stream=None) -> dict:
        import torch
        key = signature(jobs)
        if key in self.cache:
            return self.cache[key]
        timings = []
        for cand in self.candidates:
            try:
                b = Batch(jobs, rept.tuning(**cand), stream=stream)
            except rept.ReptError:
                continue  # shape does not fit this job set (LDS budget)
            b.launch()
            ts = []
            for _ in range(self.reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                b.launch()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ts.sort()
            timings.append((ts[len(ts) // 2], cand))
        timings.sort(key=lambda x: x[0])
        self.log.append({"signature": key, "timings_ms": [(t, c) for t, c in timings]})
        best = timings[0][1] if timings else {}
        self.cache[key] = best
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
        return best


def run_batched(jobs: list, tuner: Autotuner | None = None, capture: bool = False, stream=None) -> Batch:
    """Prepare (with the tuned shape if a tuner is given) and launch a batch."""
    shape = tuner.best(jobs, stream) if tuner else {}
    b = Batch(jobs, rept.tuning(**shape) if shape else None, stream=stream)
    if capture:
        b.capture()
        b.replay()
    else:
        b.launch()
    return b


def run_plain(jobs: list, stream=None):
    """The same jobs one by one through rept_count / rept_count_range (the single-job path)."""
    for j in jobs:
        out = j.ensure_outputs()
        full = j.t0 == 0 and j.t1 >= j.graph.num_edges and j.unit0 == 0 and j.unit1 >= j.graph.info.num_apex
        if full and not j.accumulate:
            j.graph.count(j.params, out, stream=stream, workspace=j.ensure_workspace())
        else:
            raise ValueError("plain path runs whole-stream, overwriting jobs only")


def time_call(fn, *a, **kw) -> float:
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    fn(*a, **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t
