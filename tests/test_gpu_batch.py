"""Batched counting on the GPU: a batch equals its jobs counted one by one, equals the oracle,
survives HIP-graph capture and replay, and every autotuner candidate computes the same integers."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _np(out):
    return out[0].cpu().numpy(), out[1].cpu().numpy()


def _mixed_jobs(cuda):
    from paper_1811_09136_amd import rept
    from paper_1811_09136_amd.batch import Job
    specs = []
    g1 = rept.Graph(rept.to_device_edges(synth.config1_stream(), cuda), 2000)
    e2, n2 = synth.scaled_chung_lu(60_000, 7)
    g2 = rept.Graph(rept.to_device_edges(e2, cuda), n2)
    e3 = synth.er(400, 5000, 5, 6)
    g3 = rept.Graph(rept.to_device_edges(e3, cuda), 400)
    jobs = [
        Job(g1, rept.Params(10, 10, 1)),
        Job(g1, rept.Params(10, 10, 2)),                 # replica: same graph, other seed
        Job(g2, rept.Params(5, 20, 3)),
        Job(g2, rept.Params(3, 7, 4, per_proc=True)),
        Job(g3, rept.Params(4, 4, 5), t0=1000, t1=4000, accumulate=True),
        Job(g3, rept.Params(1, 1, 6)),
    ]
    specs = [(synth.config1_stream(), 2000), (synth.config1_stream(), 2000), (e2, n2), (e2, n2), (e3, 400),
             (e3, 400)]
    for j in jobs:
        if j.accumulate:
            out = j.graph.outputs(j.params)
            out[0].zero_()
            out[1].zero_()
            j.out = out
    return jobs, specs


def test_batch_equals_oracle_per_job(cuda):
    import torch
    from paper_1811_09136_amd.batch import run_batched
    jobs, specs = _mixed_jobs(cuda)
    _say("mixed batch of 6 jobs")
    run_batched(jobs)
    torch.cuda.synchronize()
    for j, (e, n) in zip(jobs, specs):
        kw = {}
        if j.t1 != 2**64 - 1:
            kw = dict(t0=j.t0, t1=j.t1)
        og, ol = oracle.rept(e, n, j.params.m, j.params.c, j.params.seed, per_proc=j.params.per_proc, **kw)
        g, l = _np(j.out)
        assert np.array_equal(g, og) and np.array_equal(l, ol)


def test_unit_chunks_sum_to_whole(cuda):
    import torch
    from paper_1811_09136_amd import rept
    from paper_1811_09136_amd.batch import Job, run_batched
    e, n = synth.scaled_chung_lu(200_000, 9)
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    P = rept.Params(10, 20, 11)
    full = g.count(P)
    U = g.info.num_apex
    cuts = [0, 1, 37, U // 3, U // 2, U - 5, U]
    out = g.outputs(P)
    out[0].zero_()
    out[1].zero_()
    _say(f"unit chunks over {U} apexes")
    jobs = [Job(g, P, out=out, unit0=a, unit1=b, accumulate=True) for a, b in zip(cuts[:-1], cuts[1:])]
    run_batched(jobs)  # several chunks of one job in one batch, accumulating into one output
    torch.cuda.synchronize()
    assert torch.equal(out[0], full[0]) and torch.equal(out[1], full[1])


def test_graph_capture_replays(cuda):
    import torch
    from paper_1811_09136_amd.batch import Batch
    jobs, _ = _mixed_jobs(cuda)
    jobs = [j for j in jobs if not j.accumulate]
    b = Batch(jobs)
    b.launch()
    torch.cuda.synchronize()
    ref = [(j.out[0].clone(), j.out[1].clone()) for j in jobs]
    _say("capture + 3 replays")
    b.capture()
    # an eager batch of the same graphs with other outputs, launched between the replays (it
    # forks onto the library's second stream as the captured launch does)
    import dataclasses
    other = Batch([dataclasses.replace(j, out=None, workspace=None, table_ready=False) for j in jobs])
    for r in range(3):
        for j in jobs:  # eager work in between: scribble over the outputs
            j.out[0].fill_(-7)
            j.out[1].fill_(-7)
        other.launch()
        torch.cuda.synchronize()
        for o, (rg, rl) in zip(other.jobs, ref):
            assert torch.equal(o.out[0], rg) and torch.equal(o.out[1], rl), f"eager batch {r}"
        b.replay()
        torch.cuda.synchronize()
        for j, (rg, rl) in zip(jobs, ref):
            assert torch.equal(j.out[0], rg) and torch.equal(j.out[1], rl), f"replay {r}"


def test_autotuner_candidates_agree(cuda, tmp_path):
    import torch
    from paper_1811_09136_amd.batch import Autotuner, Batch, DEFAULT_CANDIDATES
    from paper_1811_09136_amd import rept
    jobs, _ = _mixed_jobs(cuda)
    jobs = [j for j in jobs if not j.accumulate]
    results = []
    for cand in DEFAULT_CANDIDATES:
        _say(f"candidate {cand}")
        b = Batch(jobs, rept.tuning(**cand))
        b.launch()
        torch.cuda.synchronize()
        results.append([(j.out[0].clone(), j.out[1].clone()) for j in jobs])
    for r in results[1:]:
        for (g0, l0), (g1, l1) in zip(results[0], r):
            assert torch.equal(g0, g1) and torch.equal(l0, l1)
    tuner = Autotuner(cache_path=str(tmp_path / "tune.json"))
    best = tuner.best(jobs)
    assert best in DEFAULT_CANDIDATES
    assert Autotuner(cache_path=str(tmp_path / "tune.json")).best(jobs) == best  # cached


def test_reduced_batched_workload_and_replica_statistics(cuda):
    """The batched workload's shape at reduced size: independent power-law streams plus
    hash-seed replicas of one stream (m = c = 20).  Every job matches the oracle; over the
    replicas the estimate is unbiased with Theorem 3's variance tau (m - 1) (c = m)."""
    import torch
    from paper_1811_09136_amd import rept
    from paper_1811_09136_amd.batch import Job, run_batched
    streams, (rep, rep_n), rep_seeds = synth.batch_jobs(seed=4, n_streams=12, n_replicas=96, e_min=1e4, e_max=6e4,
                                                        replica_edges=60_000, replica_nodes=3000)
    P = lambda s: rept.Params(20, 20, int(s))
    graphs = [rept.Graph(rept.to_device_edges(e, cuda), n) for e, n in streams]
    rg = rept.Graph(rept.to_device_edges(rep, cuda), rep_n)
    jobs = [Job(g, P(i + 1)) for i, g in enumerate(graphs)] + [Job(rg, P(s)) for s in rep_seeds]
    _say(f"reduced batched workload: {len(jobs)} jobs")
    run_batched(jobs)
    torch.cuda.synchronize()
    for i, (e, n) in enumerate(streams):
        og, ol = oracle.rept(e, n, 20, 20, i + 1)
        g, l = _np(jobs[i].out)
        assert np.array_equal(g, og) and np.array_equal(l, ol)
    for s, j in list(zip(rep_seeds, jobs[len(streams):]))[:4]:
        og, ol = oracle.rept(rep, rep_n, 20, 20, int(s))
        g, l = _np(j.out)
        assert np.array_equal(g, og) and np.array_equal(l, ol)
    # exact triangle count of the replica stream (m = 1 counts every triangle once)
    tau = int(rg.count(rept.Params(1, 1, 0))[0].item())
    ests = np.array([rept.rept_estimate(rep_n, j.params, _np(j.out)[0], None)[0] for j in jobs[len(streams):]])
    R, m = len(ests), 20
    var = tau * (m - 1)
    assert abs(ests.mean() - tau) < 4 * math.sqrt(var / R)
    assert 0.6 < ests.var(ddof=1) / var < 1.6
