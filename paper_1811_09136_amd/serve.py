"""Serving loop with continuous batching for REPT counting requests.

A request is one edge stream with its REPT parameters.  Requests are admitted in arrival
order while the HBM budget (a ledger of the bytes each admitted request holds) and the number
of slots allow.  An admitted request is uploaded and built by a worker thread on a stream of its
own, then joins the active set.  Each scheduler iteration enqueues ONE batched counting launch
that covers the next chunk of apex units of every active request, so requests that finish their
builds while others are counting join at the next launch and their work shares the device.
Launches are asynchronous: the scheduler keeps at most `max_inflight` of them queued on the
device and never waits for one while there is other work.  A request whose last chunk has been
enqueued is retired once that launch's event has completed: a worker copies its counters to the
host, forms the estimators and frees its memory, which returns to the budget.

The scheduler talks to an executor (the device one below, or a test double), so its admission,
chunking and failure isolation are testable without a GPU.  An executor's launch may return a
token that `ready(token)` polls and `wait(token)` blocks on; a launch that returns None has
completed when it returns.
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

class Arena:
    """First-fit sub-allocator over one device buffer reserved up front (offsets 256-byte
    aligned, free ranges coalesced).  Requests take their buffers from it, so serving makes no
    device allocation per request and is not slowed by allocator pools that differ per stream."""

    ALIGN = 256

    def __init__(self, nbytes: int, device):
        import torch
        self.size = int(nbytes) // self.ALIGN * self.ALIGN
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]  # sorted, disjoint (offset, length)
        self.lock = threading.Lock()

    def alloc(self, nbytes: int):
        n = max(self.ALIGN, -(-int(nbytes) // self.ALIGN) * self.ALIGN)
        with self.lock:
            for i, (off, ln) in enumerate(self.free):
                if ln >= n:
                    if ln == n:
                        self.free.pop(i)
                    else:
                        self.free[i] = (off + n, ln - n)
                    return off, n
        return None

    def release(self, off: int, n: int):
        with self.lock:
            f = self.free
            i = 0
            while i < len(f) and f[i][0] < off:
                i += 1
            f.insert(i, (off, n))
            # coalesce with the neighbours
            if i + 1 < len(f) and f[i][0] + f[i][1] == f[i + 1][0]:
                f[i] = (f[i][0], f[i][1] + f[i + 1][1])
                f.pop(i + 1)
            if i > 0 and f[i - 1][0] + f[i - 1][1] == f[i][0]:
                f[i - 1] = (f[i - 1][0], f[i - 1][1] + f[i][1])
                f.pop(i)

    def view(self, off: int, nbytes: int):
        return self.buf[off:off + nbytes]


class _Built:
    """The parts of a built graph a count launch needs (rept.make_job reads .handle)."""

    def __init__(self, handle, n, info):
        self.handle = handle
        self.n = n
        self.info = info


class DeviceExecutor:
    """GPU executor: builds on per-thread streams into buffers from an HBM arena reserved up front,
    counts with asynchronous batched launches on one count stream (each returns an event).  A
    request the arena cannot place (fragmentation) uses torch allocations instead."""

    def __init__(self, device="cuda", tuning=None, arena_bytes: int = 0):
        import torch
        from . import rept
        self.torch = torch
        self.rept = rept
        self.device = torch.device(device)
        self.count_stream = torch.cuda.Stream(device=self.device)
        self.tuning = tuning
        self._ws = None
        self._local = threading.local()
        self.arena = Arena(arena_bytes, self.device) if arena_bytes else None

    def _build_stream(self):
        s = getattr(self._local, "stream", None)
        if s is None:
            s = self._local.stream = self.torch.cuda.Stream(device=self.device)
        return s

    def bytes_needed(self, req: Request) -> int:
        """Stream + adjacency + build scratch + slot table + counters (the table's size follows
        rept_count_workspace_size: 16 bits per group per edge, groups padded to a power of two)."""
        p, s = self.rept.rept_query_sizes(req.n, len(req.edges))
        G = -(-req.c // req.m)
        gs = 1 if G <= 1 else (2 if G <= 2 else (4 if G <= 4 else 8))
        table = max(256, -(-2 * gs * len(req.edges) // 256) * 256)
        return 8 * len(req.edges) + p + s + table + 8 * (req.c + G * req.n)

    def _take(self, nbytes, held):
        """A device byte tensor of nbytes from the arena (recorded in `held`), or from torch."""
        if self.arena is not None:
            got = self.arena.alloc(nbytes)
            if got is not None:
                held.append(got)
                return self.arena.view(got[0], got[1])
        return self.torch.empty(max(int(nbytes), 1), dtype=self.torch.uint8, device=self.device)

    def build(self, req: Request):
        """Copy the host stream in and build on this thread's stream (rept_build_host synchronises
        that stream once, so the graph is complete when this returns)."""
        torch, rept = self.torch, self.rept
        bs = self._build_stream()
        held, scr_held = [], []
        E = len(req.edges)
        params = rept.Params(req.m, req.c, req.seed)
        try:
            pb, sb = rept.rept_query_sizes(req.n, E)
            pers = self._take(pb, held)
            scr = self._take(sb, scr_held)
            edges = np.ascontiguousarray(req.edges, dtype=np.uint32)
            h = rept.rept_build_host(req.n, edges, pers.data_ptr(), pb, scr.data_ptr(), sb, bs.cuda_stream)
            while scr_held:  # the build's scratch is free once it returned
                self.arena.release(*scr_held.pop())
            del scr
            g = _Built(h, req.n, rept.rept_graph_get_info(h))
            G = params.groups
            rows = params.rows
            outb = self._take(8 * (req.c + rows * req.n), held)
            glob = outb[:8 * req.c].view(torch.int64)
            loc = outb[8 * req.c:8 * (req.c + rows * req.n)].view(torch.int64).view(rows, req.n)
            with torch.cuda.stream(bs):
                outb.zero_()
            ws = self._take(rept.rept_count_workspace_size(h, params), held)
            bs.synchronize()
        except Exception:
            for off, n in held + scr_held:
                self.arena.release(off, n)
            raise
        return {"graph": g, "params": params, "out": (glob, loc), "ws": ws, "table_ready": False,
                "units": g.info.num_apex, "cursor": 0, "held": held, "keep": (pers, outb)}

    def units(self, state) -> int:
        return state["units"]

    def launch(self, chunks):
        """Enqueue one batched launch over [(state, unit0, unit1)] on the count stream; returns
        an event recorded after it.  The job table is copied on the same stream (stream-ordered
        after the previous launch), so one workspace serves every launch."""
        torch, rept = self.torch, self.rept
        # a request's first launch writes its slot table; its later chunks reuse it
        jobs = [rept.make_job(st["graph"], st["params"], st["out"], st["ws"], unit0=u0, unit1=u1, accumulate=True,
                              table_ready=st["table_ready"])
                for st, u0, u1 in chunks]
        nb = rept.rept_batch_workspace_size(len(jobs))
        if self._ws is None or self._ws.numel() < nb:
            self.count_stream.synchronize()  # the old table may still be read
            self._ws = torch.empty(max(nb, 1 << 16), dtype=torch.uint8, device=self.device)
        sp = self.count_stream.cuda_stream
        rept.rept_batch_prepare(jobs, self.tuning, self._ws.data_ptr(), self._ws.numel(), sp)
        rept.rept_batch_launch(self._ws.data_ptr(), sp)
        ev = torch.cuda.Event()
        ev.record(self.count_stream)
        for st, _, _ in chunks:
            st["table_ready"] = True
        return ev

    def ready(self, token) -> bool:
        return token is None or token.query()

    def wait(self, token):
        if token is not None:
            token.synchronize()

    def finish(self, state):
        g, params, out = state["graph"], state["params"], state["out"]
        glob, loc = out[0].cpu().numpy(), out[1].cpu().numpy()
        try:
            tau_hat = self.rept.rept_estimate(g.n, params, glob, None)[0]
        except self.rept.ReptError:
            tau_hat = None  # c > m with c % m != 0: counts only
        self.rept.rept_destroy(g.handle)
        for off, n in state["held"]:
            self.arena.release(off, n)
        state.clear()
        return glob, loc, tau_hat


# ------------------------------------------------------------------------------- scheduler

def _nap(now, sleep, t_target: float):
    """One step of a wait until t_target: a coarse sleep while far from it, then yields, so the
    wake-up is not late by the OS timer's slack (tens of microseconds).  Callers loop on it."""
    left = t_target - now()
    if left > 3e-4:
        sleep(min(0.05, left - 2e-4))
    elif left > 0:
        sleep(0)


@dataclass
class Server:
    executor: object
    budget_bytes: int
    max_active: int = 64
    chunk_units: int = 1 << 17
    build_workers: int = 2
    max_inflight: int = 2       # batched launches queued on the device at once
    finish_workers: int = 2     # threads that copy results back and free requests
    hold_lone_newcomer: bool = True  # see the admission below
    results: dict = field(default_factory=dict)
    trace: list = field(default_factory=list)

    def run(self, requests: list, clock=time.monotonic, sleep=time.sleep) -> list:
        ex = self.executor
        ready = getattr(ex, "ready", lambda tok: True)
        wait = getattr(ex, "wait", lambda tok: None)
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        pending = collections.deque(reqs)
        waiting = collections.deque()          # arrived, not admitted
        building = {}                          # future -> (req, bytes)
        active = []                            # [req, state, bytes]: units left to enqueue
        draining = []                          # [req, state, bytes, token]: all enqueued
        finishing = {}                         # future -> (req, bytes)
        inflight = collections.deque()         # tokens of launches not known to be complete
        used = 0
        t_start = clock()
        now = lambda: clock() - t_start
        pool = cf.ThreadPoolExecutor(max_workers=self.build_workers)
        fpool = cf.ThreadPoolExecutor(max_workers=self.finish_workers)

        # the workers stamp their own completion times, so a result is not made later by the
        # scheduler being busy elsewhere when the worker ends
        def build_job(r):
            state = ex.build(r)
            self.results[r.rid].built_s = now()
            return state

        def retire(r, state):
            res = self.results[r.rid]
            try:
                res.glob, res.loc, res.tau_hat = ex.finish(state)
            except Exception as exc:  # pragma: no cover - a device error while copying back
                res.status = f"failed: {exc}"
            res.done_s = now()

        def done_finishing():
            nonlocal used
            for fut in [f for f in finishing if f.done()]:
                _, need = finishing.pop(fut)
                used -= need

        try:
            while pending or waiting or building or active or draining or finishing:
                progressed = False
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
                    progressed = True
                    try:
                        state = fut.result()
                    except Exception as exc:  # a bad request fails alone
                        res.status, res.done_s = f"failed: {exc}", now()
                        used -= need
                        continue
                    if ex.units(state) == 0:
                        finishing[fpool.submit(retire, r, state)] = (r, need)
                    else:
                        active.append([r, state, need])
                # requests whose last launch completed are retired by the finish workers, or here
                # when nothing else needs the scheduler but at most one newcomer (held back by the
                # admission below): no hand-off to add to the latency, and the newcomer's build
                # does not share the host with this copy-back
                still = []
                for r, state, need, tok in draining:
                    if ready(tok):
                        progressed = True
                        if not (active or building) and len(waiting) <= 1 and len(draining) == 1:
                            retire(r, state)
                            used -= need
                        else:
                            finishing[fpool.submit(retire, r, state)] = (r, need)
                    else:
                        still.append([r, state, need, tok])
                draining = still
                if finishing:
                    before = len(finishing)
                    done_finishing()
                    progressed = progressed or len(finishing) < before
                # admission: FIFO, by budget and slots; a request larger than the whole budget
                # is refused (it can never fit) without blocking the ones behind it
                while waiting and len(active) + len(building) < self.max_active:
                    r = waiting[0]
                    need = ex.bytes_needed(r)
                    if need > self.budget_bytes:
                        waiting.popleft()
                        res = self.results[r.rid]
                        res.status, res.done_s = "rejected: over budget", now()
                        continue
                    if used + need > self.budget_bytes:
                        break
                    if self.hold_lone_newcomer and len(waiting) == 1 and not building and (
                            (len(draining) == 1 and not active and inflight)
                            or (len(active) == 1 and not draining
                                and ex.units(active[0][1]) - active[0][1]["cursor"] <= self.chunk_units)):
                        # the one request in service has all its remaining work in one launch
                        # (enqueued, or about to be): a newcomer alone behind it would gain nothing
                        # from building now (its build kernels would only compete with that launch
                        # for the compute units and slow both), so it is admitted when that
                        # launch completes
                        break
                    waiting.popleft()
                    used += need
                    res = self.results[r.rid]
                    res.admitted_s = now()
                    progressed = True
                    if not (active or building or draining or waiting):
                        # alone in the system: build here, without a hand-off to a worker
                        try:
                            state = ex.build(r)
                        except Exception as exc:  # a bad request fails alone
                            res.status, res.done_s = f"failed: {exc}", now()
                            used -= need
                            continue
                        res.built_s = now()
                        if ex.units(state) == 0:
                            retire(r, state)
                            used -= need
                        else:
                            active.append([r, state, need])
                    else:
                        building[pool.submit(build_job, r)] = (r, need)
                while inflight and ready(inflight[0]):
                    inflight.popleft()
                if active and len(inflight) < self.max_inflight:
                    chunks = []
                    for r, state, _ in active:
                        u0 = state["cursor"]
                        u1 = min(u0 + self.chunk_units, ex.units(state))
                        chunks.append((state, u0, u1))
                    tok = ex.launch(chunks)
                    inflight.append(tok)
                    self.trace.append((now(), [r.rid for r, _, _ in active]))
                    still = []
                    for (r, state, need), (_, u0, u1) in zip(active, chunks):
                        state["cursor"] = u1
                        self.results[r.rid].chunks += 1
                        if u1 >= ex.units(state):
                            draining.append([r, state, need, tok])
                        else:
                            still.append([r, state, need])
                    active = still
                    progressed = True
                if progressed:
                    continue
                # nothing moved: wait for the event that comes first
                if inflight and (active or draining):
                    tok = inflight[0]
                    # the last launch of the one request in service: a newcomer arriving meanwhile
                    # would be held until it completes, so block on it as the plain loop does
                    lone = self.hold_lone_newcomer and len(draining) == 1 and not (active or building or waiting)
                    if pending and not lone:
                        # the oldest launch, or the next arrival if it comes first
                        while not ready(tok) and now() < pending[0].arrival_s:
                            sleep(0)
                    else:
                        wait(tok)
                elif building:
                    cf.wait(list(building), timeout=0.002, return_when=cf.FIRST_COMPLETED)
                elif finishing:
                    cf.wait(list(finishing), timeout=0.002, return_when=cf.FIRST_COMPLETED)
                elif draining:
                    wait(draining[0][3])
                elif pending and not waiting:
                    _nap(now, sleep, pending[0].arrival_s)
                elif waiting:
                    # nothing holds budget or a slot, yet the head request was not admitted
                    raise RuntimeError(f"scheduler stalled: {len(waiting)} waiting, {used} bytes held")
        finally:
            pool.shutdown(wait=True)
            fpool.shutdown(wait=True)
        return [self.results[r.rid] for r in reqs]


def run_fifo_plain(executor, requests: list, clock=time.monotonic, sleep=time.sleep) -> list:
    """Baseline: one request at a time in arrival order, each built and counted alone."""
    out = []
    t_start = clock()
    now = lambda: clock() - t_start
    for r in sorted(requests, key=lambda r: r.arrival_s):
        while now() < r.arrival_s:
            _nap(now, sleep, r.arrival_s)
        res = Result(r.rid, r.arrival_s, admitted_s=now())
        try:
            state = executor.build(r)
            res.built_s = now()
            if executor.units(state):
                tok = executor.launch([(state, 0, executor.units(state))])
                getattr(executor, "wait", lambda tok: None)(tok)
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
    wait = np.array([r.admitted_s - r.arrival_s for r in ok])
    build = np.array([r.built_s - r.admitted_s for r in ok])
    count = np.array([r.done_s - r.built_s for r in ok])
    return {"requests": len(results), "ok": len(ok), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()), "makespan_s": float(span),
            "edges_per_s": edges / span if span > 0 else float("nan"),
            # medians of the phases: arrival to admission, the build, then counting and copy-back
            "p50_admit_wait_s": float(np.median(wait)), "p50_build_s": float(np.median(build)),
            "p50_count_finish_s": float(np.median(count))}
