"""Serving on the GPU: requests admitted while others are counting share batched launches;
every request's counters equal the same request counted alone (exactly) and, for the small
ones, the oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _trace(k=16, rate=300.0, seed=5):
    from paper_1811_09136_amd.serve import Request
    tr = synth.serving_trace(seed=seed, n_requests=k, rate_per_s=rate, median_edges=2e4, e_hi=2e5)
    reqs = []
    for i, r in enumerate(tr):
        e, n = synth.scaled_chung_lu(r["E"], r["graph_seed"] % (2**31))
        reqs.append(Request(i, r["arrival_s"], e, n, r["m"], r["c"], r["hash_seed"]))
    return reqs


def test_served_equals_alone_and_oracle(cuda):
    import torch
    from paper_1811_09136_amd import rept
    from paper_1811_09136_amd.serve import DeviceExecutor, Server
    reqs = _trace(rate=20000.0)  # arrivals faster than service: requests overlap on the device
    _say(f"serving {len(reqs)} requests")
    ex = DeviceExecutor("cuda:0")
    srv = Server(ex, budget_bytes=8 << 30, max_active=6, chunk_units=150, build_workers=2)
    res = srv.run(reqs)
    assert all(r.status == "ok" for r in res), [r.status for r in res]
    # batches really mixed requests: some launch held several
    assert max(len(ids) for _, ids in srv.trace) > 1
    for r, q in zip(res, reqs):
        g = rept.Graph(rept.to_device_edges(q.edges, cuda), q.n)
        alone = g.count(rept.Params(q.m, q.c, q.seed))
        torch.cuda.synchronize()
        assert np.array_equal(r.glob, alone[0].cpu().numpy())
        assert np.array_equal(r.loc, alone[1].cpu().numpy())
        g.close()
        if len(q.edges) <= 20000:
            og, ol = oracle.rept(q.edges, q.n, q.m, q.c, q.seed)
            assert np.array_equal(r.glob, og) and np.array_equal(r.loc, ol)


def test_oversized_and_invalid_requests_fail_alone(cuda):
    from paper_1811_09136_amd.serve import DeviceExecutor, Request, Server
    reqs = _trace(k=6, rate=1000.0, seed=8)
    bad = reqs[2].edges.copy()
    bad[5] = bad[1][::-1]  # a repeated unordered pair
    reqs[2] = Request(2, reqs[2].arrival_s, bad, reqs[2].n, reqs[2].m, reqs[2].c, reqs[2].seed)
    ex = DeviceExecutor("cuda:0")
    need = [ex.bytes_needed(q) for q in reqs]
    budget = sorted(need)[-2]  # the largest request cannot fit
    big = int(np.argmax(need))
    _say("failure isolation")
    res = Server(ex, budget_bytes=budget, max_active=4, chunk_units=500).run(reqs)
    for i, r in enumerate(res):
        if need[i] > budget:
            assert r.status.startswith("rejected")
        elif i == 2:
            assert r.status.startswith("failed")
        else:
            assert r.status == "ok"
    assert need[big] > budget


@pytest.mark.timeout(600)
def test_served_multi_million_edge_request_against_oracle(cuda):
    """A request of 2.5e6 edges (the served workload's lognormal sizes reach 2e7) counted in many
    unit chunks while smaller requests arrive and join its launches: every result, the large one
    included, equals the oracle's replay."""
    import os
    from paper_1811_09136_amd.serve import DeviceExecutor, Request, Server
    e_big, n_big = synth.scaled_chung_lu(2_500_000, 77)
    reqs = [Request(0, 0.0, e_big, n_big, 50, 200, 901)]
    tr = synth.serving_trace(seed=9, n_requests=10, rate_per_s=2000.0, median_edges=5e4, e_hi=2e5)
    for i, r in enumerate(tr, start=1):
        e, n = synth.scaled_chung_lu(r["E"], r["graph_seed"] % (2**31))
        reqs.append(Request(i, 0.002 + r["arrival_s"], e, n, r["m"], r["c"], r["hash_seed"]))
    _say(f"serving a {len(e_big)}-edge request with {len(reqs) - 1} smaller ones")
    ex = DeviceExecutor("cuda:0", arena_bytes=4 << 30)  # buffers from an arena (with fallback)
    srv = Server(ex, budget_bytes=32 << 30, max_active=16, chunk_units=2048, build_workers=2)
    res = srv.run(reqs)
    assert all(r.status == "ok" for r in res), [r.status for r in res]
    assert res[0].chunks > 1 and max(len(ids) for _, ids in srv.trace) > 1
    W = max(1, min(16, len(os.sched_getaffinity(0))))
    for r, q in zip(res, reqs):
        _say(f"oracle, request {q.rid} ({len(q.edges)} edges, m={q.m}, c={q.c})")
        og, ol = oracle.rept_threads(q.edges, q.n, q.m, q.c, q.seed, workers=W)
        assert np.array_equal(r.glob, og) and np.array_equal(r.loc, ol), q.rid
