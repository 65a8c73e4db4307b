"""Serving loop with continuous batching for REPT counting requests.

A request is one edge stream with its REPT parameters.  Requests are admitted in arrival
order while the HBM budget (a ledger of the bytes each admitted request holds) and the number
of slots allow.  An admitted request is uploaded and built on a side stream (a worker thread),
then joins the active set.  Each scheduler iteration launches ONE batched counting kernel that
covers the next chunk of apex units of every active request, so requests that finish their
builds while others are counting join at the next iteration and their work shares the device.
A request whose units are exhausted is finished: counters copied to the host, estimators
formed, memory returned to the budget, latency recorded.

The scheduler talks to an executor (the device one below, or a test double), so its admission,
chunking and failure isolation are testable without a GPU.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import math
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival_s: float
    edges: np.ndarray  # host uint32 [E, 2]
    n: int
    m: int
    c: int
    seed: int


@dataclass
class Result:
    rid: int
    arrival_s: float
    admitted_s: float = float("nan")
    built_s: float = float("nan")
    done_s: float = float("nan")
    status: str = "ok"
    glob: np.ndarray | None = None
    loc: np.ndarray | None = None
    tau_hat: float | None = None
    chunks: int = 0

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


# ------------------------------------------------------------------------------- executor

class DeviceExecutor:
    """GPU executor: uploads and builds on a side stream, counts with batched launches."""

    def __init__(self, device="cuda", tuning=None):
        import torch
        from . import rept
        self.torch = torch
        self.rept = rept
        self.device = torch.device(device)
        self.build_stream = torch.cuda.Stream(device=self.device)
        self.count_stream = torch.cuda.Stream(device=self.device)
        self.tuning = tuning
        self._ws = None
        self._ws_jobs = 0

    def bytes_needed(self, req: Request) -> int:
        """Stream + adjacency + build scratch + slot table + counters (the table's size follows
        rept_count_workspace_size: 16 bits per group per edge, groups padded to a power of two)."""
        p, s = self.rept.rept_query_sizes(req.n, len(req.edges))
        G = -(-req.c // req.m)
        gs = 1 if G <= 1 else (2 if G <= 2 else (4 if G <= 4 else 8))
        table = max(256, -(-2 * gs * len(req.edges) // 256) * 256)
        return 8 * len(req.edges) + p + s + table + 8 * (req.c + G * req.n)

    def build(self, req: Request):
        """Upload + build (blocking this worker thread; rept_build synchronises its stream)."""
        torch, rept = self.torch, self.rept
        with torch.cuda.stream(self.build_stream):
            d = rept.to_device_edges(req.edges, self.device)
            g = rept.Graph(d, req.n, stream=self.build_stream)
            params = rept.Params(req.m, req.c, req.seed)
            out = g.outputs(params)
            out[0].zero_()
            out[1].zero_()
            ws = g.new_workspace(params)
        self.build_stream.synchronize()
        return {"graph": g, "params": params, "out": out, "ws": ws, "table_ready": False,
                "units": g.info.num_apex, "cursor": 0}

    def units(self, state) -> int:
        return state["units"]

    def launch(self, chunks):
        """One batched launch over [(state, unit0, unit1)]; returns when it completed."""
        torch, rept = self.torch, self.rept
        # a request's first launch writes its slot table; its later chunks reuse it
        jobs = [rept.make_job(st["graph"], st["params"], st["out"], st["ws"], unit0=u0, unit1=u1, accumulate=True,
                              table_ready=st["table_ready"])
                for st, u0, u1 in chunks]
        nb = rept.rept_batch_workspace_size(len(jobs))
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(max(nb, 1 << 16), dtype=torch.uint8, device=self.device)
        sp = self.count_stream.cuda_stream
        rept.rept_batch_prepare(jobs, self.tuning, self._ws.data_ptr(), self._ws.numel(), sp)
        rept.rept_batch_launch(self._ws.data_ptr(), sp)
        self.count_stream.synchronize()
        for st, _, _ in chunks:
            st["table_ready"] = True

    def finish(self, state):
        g, params, out = state["graph"], state["params"], state["out"]
        glob, loc = out[0].cpu().numpy(), out[1].cpu().numpy()
        try:
            tau_hat = self.rept.rept_estimate(g.n, params, glob, None)[0]
        except self.rept.ReptError:
            tau_hat = None  # c > m with c % m != 0: counts only
        g.close()
        state.clear()
        return glob, loc, tau_hat


# ------------------------------------------------------------------------------- scheduler

@dataclass
class Server:
    executor: object
    budget_bytes: int
    max_active: int = 64
    chunk_units: int = 1 << 17
    build_workers: int = 2
    results: dict = field(default_factory=dict)
    trace: list = field(default_factory=list)

    def run(self, requests: list, clock=time.monotonic, sleep=time.sleep) -> list:
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        pending = collections.deque(reqs)
        waiting = collections.deque()          # arrived, not admitted
        building = {}                          # future -> (req, bytes)
        active = []                            # [req, state, bytes]
        used = 0
        t_start = clock()
        now = lambda: clock() - t_start
        lock = threading.Lock()
        pool = cf.ThreadPoolExecutor(max_workers=self.build_workers)
        try:
            while pending or waiting or building or active:
                t = now()
                while pending and pending[0].arrival_s <= t:
                    r = pending.popleft()
                    self.results[r.rid] = Result(r.rid, r.arrival_s)
                    waiting.append(r)
                # builds that completed join the active set (before admission, so the budget a
                # failed or empty build returns is seen by the admission below)
                for fut in [f for f in building if f.done()]:
                    r, need = building.pop(fut)
                    res = self.results[r.rid]
                    try:
                        state = fut.result()
                    except Exception as ex:  # a bad request fails alone
                        res.status, res.done_s = f"failed: {ex}", now()
                        used -= need
                        continue
                    res.built_s = now()
                    if self.executor.units(state) == 0:
                        self._finish(r, state, res, now)
                        used -= need
                    else:
                        active.append([r, state, need])
                # admission: FIFO, by budget and slots; a request larger than the whole budget
                # is refused (it can never fit) without blocking the ones behind it
                while waiting and len(active) + len(building) < self.max_active:
                    r = waiting[0]
                    need = self.executor.bytes_needed(r)
                    if need > self.budget_bytes:
                        waiting.popleft()
                        res = self.results[r.rid]
                        res.status, res.done_s = "rejected: over budget", now()
                        continue
                    if used + need > self.budget_bytes:
                        break
                    waiting.popleft()
                    used += need
                    self.results[r.rid].admitted_s = now()
                    building[pool.submit(self.executor.build, r)] = (r, need)
                if active:
                    chunks = []
                    for r, state, _ in active:
                        u0 = state["cursor"]
                        u1 = min(u0 + self.chunk_units, self.executor.units(state))
                        chunks.append((state, u0, u1))
                    self.executor.launch(chunks)
                    self.trace.append((now(), [r.rid for r, _, _ in active]))
                    still = []
                    for (r, state, need), (_, u0, u1) in zip(active, chunks):
                        state["cursor"] = u1
                        self.results[r.rid].chunks += 1
                        if u1 >= self.executor.units(state):
                            self._finish(r, state, self.results[r.rid], now)
                            used -= need
                        else:
                            still.append([r, state, need])
                    active = still
                elif building:
                    cf.wait(list(building), timeout=0.002, return_when=cf.FIRST_COMPLETED)
                elif pending and not waiting:
                    sleep(max(0.0, min(0.05, pending[0].arrival_s - now())))
                elif waiting:
                    # nothing holds budget or a slot, yet the head request was not admitted
                    raise RuntimeError(f"scheduler stalled: {len(waiting)} waiting, {used} bytes held")
        finally:
            pool.shutdown(wait=True)
        return [self.results[r.rid] for r in reqs]

    def _finish(self, r, state, res, now):
        res.glob, res.loc, res.tau_hat = self.executor.finish(state)
        res.done_s = now()


def run_fifo_plain(executor, requests: list, clock=time.monotonic, sleep=time.sleep) -> list:
    """Baseline: one request at a time in arrival order, each built and counted alone."""
    out = []
    t_start = clock()
    now = lambda: clock() - t_start
    for r in sorted(requests, key=lambda r: r.arrival_s):
        while now() < r.arrival_s:
            sleep(min(0.05, r.arrival_s - now()))
        res = Result(r.rid, r.arrival_s, admitted_s=now())
        try:
            state = executor.build(r)
            res.built_s = now()
            if executor.units(state):
                executor.launch([(state, 0, executor.units(state))])
            res.glob, res.loc, res.tau_hat = executor.finish(state)
        except Exception as ex:
            res.status = f"failed: {ex}"
        res.done_s = now()
        out.append(res)
    return out


def summarize(results: list, requests: list) -> dict:
    """Latency percentiles of the completed requests and their stream edges per second over
    the makespan (first arrival to last completion)."""
    size = {r.rid: len(r.edges) for r in requests}
    ok = [r for r in results if r.status == "ok"]
    if not ok:
        return {"requests": len(results), "ok": 0}
    lat = np.array([r.latency_s for r in ok])
    span = max(r.done_s for r in ok) - min(r.arrival_s for r in ok)
    edges = sum(size[r.rid] for r in ok)
    return {"requests": len(results), "ok": len(ok), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()), "makespan_s": float(span),
            "edges_per_s": edges / span if span > 0 else float("nan")}
