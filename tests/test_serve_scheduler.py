"""Serving scheduler on the CPU with a test double of the executor (CPU only).

The double computes each request's counters with the CPU oracle when the request finishes and
simulates device time on a fake clock, so admission by budget, slot limits, continuous
batching (requests joining a running batch) and failure isolation are checked without a GPU.
"""
import threading

import numpy as np

import oracle
import synth
from paper_1811_09136_amd.serve import Request, Server, run_fifo_plain, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0
        self.lock = threading.Lock()

    def __call__(self):
        with self.lock:
            return self.t

    def advance(self, dt):
        with self.lock:
            self.t += dt

    def sleep(self, dt):
        self.advance(max(dt, 1e-4))


class FakeExecutor:
    """Units = ceil(E / 50); a launch costs 1 ms of fake time per job in it."""

    def __init__(self, clock, bad=()):
        self.clock = clock
        self.bad = set(bad)
        self.launches = []

    def bytes_needed(self, r):
        return 100 * len(r.edges)

    def build(self, r):
        if r.rid in self.bad:
            raise ValueError("duplicate edge in stream")
        return {"req": r, "units": -(-len(r.edges) // 50), "cursor": 0}

    def units(self, st):
        return st["units"]

    def launch(self, chunks):
        self.launches.append([(st["req"].rid, u0, u1) for st, u0, u1 in chunks])
        self.clock.advance(1e-3 * len(chunks))

    def finish(self, st):
        r = st["req"]
        g, l = oracle.rept(r.edges, r.n, r.m, r.c, r.seed)
        return g, l, oracle.estimate(r.n, r.m, r.c, g)[0]


def _requests(k=12, rate=400.0):
    rng = np.random.default_rng(3)
    reqs, t = [], 0.0
    for i in range(k):
        t += rng.exponential(1 / rate)
        E = int(rng.integers(300, 3000))
        n = max(40, E // 10)
        e = synth.er(n, E, 100 + i, 200 + i)
        m = int(rng.choice([2, 3, 5]))
        reqs.append(Request(i, t, e, n, m, m * int(rng.choice([1, 2])), 1000 + i))
    return reqs


def test_all_requests_served_exactly():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _requests()
    srv = Server(ex, budget_bytes=10**9, max_active=4, chunk_units=7, build_workers=1)
    res = srv.run(reqs, clock=clk, sleep=clk.sleep)
    assert [r.status for r in res] == ["ok"] * len(reqs)
    for r, q in zip(res, reqs):
        g, l = oracle.rept(q.edges, q.n, q.m, q.c, q.seed)
        assert np.array_equal(r.glob, g) and np.array_equal(r.loc, l)
        assert r.done_s >= r.arrival_s and r.chunks >= 1
    # no launch holds more than max_active jobs, and every job's chunks tile its units
    assert max(len(L) for L in ex.launches) <= 4
    per_job = {}
    for L in ex.launches:
        for rid, u0, u1 in L:
            per_job.setdefault(rid, []).append((u0, u1))
    for q in reqs:
        spans = per_job[q.rid]
        assert spans[0][0] == 0 and spans[-1][1] == -(-len(q.edges) // 50)
        assert all(a[1] == b[0] for a, b in zip(spans[:-1], spans[1:]))
    s = summarize(res, reqs)
    assert s["ok"] == len(reqs) and s["p99_s"] >= s["p50_s"] > 0


def test_continuous_batching_joins_running_batches():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _requests(k=10, rate=2000.0)
    srv = Server(ex, budget_bytes=10**9, max_active=8, chunk_units=3, build_workers=1)
    srv.run(reqs, clock=clk, sleep=clk.sleep)
    # some request entered a launch after another request's first launch and before its last
    first, last = {}, {}
    for i, L in enumerate(ex.launches):
        for rid, _, _ in L:
            first.setdefault(rid, i)
            last[rid] = i
    joined = any(first[b] > first[a] and first[b] <= last[a] for a in first for b in first if a != b)
    assert joined


def test_budget_rejects_oversized_and_serves_the_rest():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _requests(k=6)
    budget = 100 * 2500
    srv = Server(ex, budget_bytes=budget, max_active=8, chunk_units=5, build_workers=1)
    res = srv.run(reqs, clock=clk, sleep=clk.sleep)
    for r, q in zip(res, reqs):
        if 100 * len(q.edges) > budget:
            assert r.status.startswith("rejected")
        else:
            assert r.status == "ok"
    # at no time did admitted requests exceed the budget
    assert any(r.status.startswith("rejected") for r in res) or all(100 * len(q.edges) <= budget for q in reqs)


def test_failed_build_is_isolated():
    clk = FakeClock()
    ex = FakeExecutor(clk, bad={2, 5})
    reqs = _requests(k=8)
    srv = Server(ex, budget_bytes=10**9, max_active=3, chunk_units=9, build_workers=1)
    res = srv.run(reqs, clock=clk, sleep=clk.sleep)
    for r, q in zip(res, reqs):
        if q.rid in (2, 5):
            assert r.status.startswith("failed")
        else:
            g, l = oracle.rept(q.edges, q.n, q.m, q.c, q.seed)
            assert r.status == "ok" and np.array_equal(r.glob, g)


def test_fifo_plain_baseline():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _requests(k=5)
    res = run_fifo_plain(ex, reqs, clock=clk, sleep=clk.sleep)
    assert all(r.status == "ok" for r in res)
    assert all(a.done_s <= b.done_s for a, b in zip(res[:-1], res[1:]))


def test_failed_build_frees_budget_for_waiting_requests():
    """A build that fails while it alone holds the budget returns that budget to the requests
    waiting behind it; none is dropped, and the ones not yet arrived are still served."""
    clk = FakeClock()
    reqs = _requests(k=6, rate=1e6)
    reqs.append(Request(6, reqs[-1].arrival_s + 1.0, reqs[0].edges, reqs[0].n, 2, 2, 77))
    ex = FakeExecutor(clk, bad={0})
    budget = max(100 * len(q.edges) for q in reqs)  # no two of the larger requests fit together
    srv = Server(ex, budget_bytes=budget, max_active=8, chunk_units=4, build_workers=1)
    res = srv.run(reqs, clock=clk, sleep=clk.sleep)
    assert res[0].status.startswith("failed")
    assert [r.status for r in res[1:]] == ["ok"] * (len(reqs) - 1)


def test_arena_first_fit_and_coalescing():
    """The serving executor's arena (CPU part: offsets only) hands out aligned, disjoint ranges
    and merges freed neighbours back into one range."""
    from paper_1811_09136_amd import serve
    a = serve.Arena.__new__(serve.Arena)
    a.size, a.free, a.lock = 4096, [(0, 4096)], threading.Lock()
    x = a.alloc(100)
    y = a.alloc(300)
    z = a.alloc(256)
    assert x == (0, 256) and y == (256, 512) and z == (768, 256)
    assert a.alloc(4096) is None
    a.release(*y)
    assert a.alloc(512) == (256, 512)  # first fit reuses the hole
    a.release(256, 512)
    a.release(*x)
    a.release(*z)
    assert a.free == [(0, 4096)]


def test_lone_newcomer_is_held_until_the_last_launch_completes():
    """One request in service with its remaining units in one launch, and one newcomer: with the
    hold rule the newcomer is admitted only when that launch has completed and the request is
    retired; without it, at once.  Results are exact either way."""
    def run(hold):
        clk = FakeClock()
        ex = FakeExecutor(clk)
        a = Request(0, 0.0, synth.er(200, 1250, 5, 6), 200, 3, 3, 11)  # 25 units: launches of 10, 10, 5
        b = Request(1, 0.0015, synth.er(150, 600, 7, 8), 150, 2, 4, 12)  # arrives after A's second launch
        srv = Server(ex, budget_bytes=10**9, max_active=4, chunk_units=10, build_workers=1,
                     hold_lone_newcomer=hold)
        res = srv.run([a, b], clock=clk, sleep=clk.sleep)
        for r, q in zip(res, [a, b]):
            g, l = oracle.rept(q.edges, q.n, q.m, q.c, q.seed)
            assert r.status == "ok" and np.array_equal(r.glob, g) and np.array_equal(r.loc, l)
        spans_a = [(u0, u1) for L in ex.launches for rid, u0, u1 in L if rid == 0]
        assert spans_a == [(0, 10), (10, 20), (20, 25)]
        return res

    ra, rb = run(True)
    assert rb.admitted_s >= ra.done_s  # held: admitted once A's last launch completed
    ra, rb = run(False)
    assert rb.admitted_s < ra.done_s  # admitted while A's last units were still to run
