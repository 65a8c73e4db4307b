"""Full-size parity, in the launch configuration bench.py times:
* the 1M/20M power-law workload and the R-MAT scale-24 workload against the oracle's stored
  digests (every counter), plus sampled windows the oracle evaluates edge by edge and
  invariants that hold at any size;
* the 512-job batched workload in one graph-captured launch against the oracle's replay."""
import hashlib
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print("[case]", *a, flush=True)


def _golden_kv(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        out[k.strip()] = v.strip()
    return out


def _digest(glob, loc):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(glob, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(loc, dtype="<i8").tobytes())
    return h.hexdigest()


@pytest.mark.timeout(300)
def test_config2_full_against_oracle_digest(cuda):
    import torch
    from paper_1811_09136_amd import rept
    ref = _golden_kv("config2_oracle.txt")
    e = synth.config2_stream()
    _say("config2 Chung-Lu n=1e6 E=2e7 m=10 c=40 full count")
    g = rept.Graph(rept.to_device_edges(e, cuda), 1_000_000)
    glob, loc = g.count(rept.Params(10, 40, 20181122))
    torch.cuda.synchronize()
    glob, loc = glob.cpu().numpy(), loc.cpu().numpy()
    assert " ".join(str(int(x)) for x in glob) == ref["global"]
    assert " ".join(str(int(x)) for x in loc.sum(axis=1)) == ref["local_row_sums"]
    assert _digest(glob, loc) == ref["sha256"]
    for k in range(4):  # each semi-triangle adds one to each of its three nodes
        assert loc[k].sum() == 3 * glob[10 * k:10 * k + 10].sum()
    g.close()


@pytest.mark.timeout(600)
def test_config3_full_against_oracle_digest_and_windows(cuda):
    """R-MAT scale 24 (2.6e8 stream edges, m = c = 100): the whole count against the oracle's
    stored digest (every global and local counter), then window additivity and sampled windows
    the oracle evaluates edge by edge."""
    import torch
    from paper_1811_09136_amd import rept
    ref = _golden_kv("config3_oracle.txt")
    e = synth.config3_stream()
    E, n = len(e), 1 << 24
    P = rept.Params(100, 100, 20181122)
    _say(f"config3 R-MAT scale 24 E={E} m=100 c=100 build")
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    full = g.count(P)
    torch.cuda.synchronize()
    fg, fl = full[0].cpu().numpy(), full[1].cpu().numpy()
    assert " ".join(str(int(x)) for x in fg) == ref["global"]
    assert " ".join(str(int(x)) for x in fl.sum(axis=1)) == ref["local_row_sums"]
    assert _digest(fg, fl) == ref["sha256"]
    assert int(fl.sum()) == 3 * int(fg.sum())
    del fl
    # additivity: two halves of the stream sum to the whole
    half = g.outputs(P)
    half[0].zero_()
    half[1].zero_()
    g.count_range(P, 0, E // 2, half)
    g.count_range(P, E // 2, E, half)
    torch.cuda.synchronize()
    assert torch.equal(half[0], full[0]) and torch.equal(half[1], full[1])
    del half, full
    # sampled windows, late in the stream (most triangles close there) and mid-stream,
    # accumulated into one output; the oracle evaluates the same edges one by one
    windows = [(E - 1500, E), (E // 2, E // 2 + 1500)]
    out = g.outputs(P)
    out[0].zero_()
    out[1].zero_()
    for t0, t1 in windows:
        _say(f"config3 window [{t0}, {t1})")
        g.count_range(P, t0, t1, out)
    torch.cuda.synchronize()
    ts = np.concatenate([np.arange(t0, t1) for t0, t1 in windows])
    og, ol = oracle.edge_updates(e, n, 100, 100, 20181122, ts)
    assert og.sum() > 0
    assert np.array_equal(out[0].cpu().numpy(), og)
    assert np.array_equal(out[1].cpu().numpy(), ol)
    g.close()


def _host_threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.mark.timeout(900)
def test_config4_full_batch_against_oracle(cuda):
    """The batched workload at full size (256 Chung-Lu streams of 1e4-2e6 edges plus 256 hash-seed
    replicas of one 5e6-edge stream, m = c = 20) in one autotuned, graph-captured launch: every
    job, stream or replica, against the oracle's full replay."""
    import torch
    from paper_1811_09136_amd import rept
    from paper_1811_09136_amd.batch import Autotuner, Batch, Job
    streams, (rep, rep_n), rep_seeds = synth.batch_jobs(seed=4)
    _say(f"config4: {len(streams)} streams + {len(rep_seeds)} replicas, builds")
    graphs = [rept.Graph(rept.to_device_edges(e, cuda), n) for e, n in streams]
    rg = rept.Graph(rept.to_device_edges(rep, cuda), rep_n)
    P = lambda s: rept.Params(20, 20, int(s))
    jobs = [Job(g, P(i + 1)) for i, g in enumerate(graphs)] + [Job(rg, P(s)) for s in rep_seeds]
    shape = Autotuner(reps=1).best(jobs)
    _say(f"config4: batched launch, shape {shape}")
    b = Batch(jobs, rept.tuning(**shape) if shape else None)
    b.capture()
    for j in jobs:
        j.out[0].fill_(-1)
        j.out[1].fill_(-1)
    b.replay()
    torch.cuda.synchronize()
    W = _host_threads()
    for i, ((e, n), j) in enumerate(zip(streams, jobs)):
        if i % 32 == 0:
            _say(f"config4: oracle, stream job {i} ({len(e)} edges)")
        og, ol = oracle.rept_threads(e, n, 20, 20, i + 1, workers=W)
        assert np.array_equal(j.out[0].cpu().numpy(), og), f"stream job {i}"
        assert np.array_equal(j.out[1].cpu().numpy(), ol), f"stream job {i}"
    for r, j in enumerate(jobs[len(streams):]):
        g_, l_ = j.out[0].cpu().numpy(), j.out[1].cpu().numpy()
        assert g_.min() >= 0 and int(l_.sum()) == 3 * int(g_.sum()), f"replica {r}"
        if r % 32 == 0:
            _say(f"config4: oracle, replica {r}")
        og, ol = oracle.rept_threads(rep, rep_n, 20, 20, int(rep_seeds[r]), workers=W)
        assert np.array_equal(g_, og) and np.array_equal(l_, ol), f"replica {r}"
    for g in graphs:
        g.close()
    rg.close()
