"""Algorithm 2 (Section III-B, c > m with c mod m != 0) on the device against the CPU oracle:
the triangle-pair counters (both readings of the counter's value on insert) bit for bit, the
semi-triangle counters of the same launch bit for bit, and the combined estimators at 0 ulp.

Inputs are seeded synthetic streams (module ``synth``).  Each case prints its name and shape
before touching the GPU so that a failing run names its case.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _run(cuda, edges, n, m, c, seed, per_proc=False, tune=None, with_nodes=True):
    import torch
    from paper_1811_09136_amd import rept
    p = rept.Params(m, c, seed, per_proc)
    g = rept.Graph(rept.to_device_edges(edges, cuda), n)
    glob, loc, eta, eta_v = g.count_eta(p, tuning=tune, with_nodes=with_nodes)
    torch.cuda.synchronize()
    res = (glob.cpu().numpy(), loc.cpu().numpy(), eta.cpu().numpy(),
           None if eta_v is None else eta_v.cpu().numpy(), g.info)
    g.close()
    return res


def _check(edges, n, m, c, seed, got, per_proc=False):
    glob, loc, eta, eta_v, _ = got
    og, ol = oracle.rept(edges, n, m, c, seed, per_proc=per_proc)
    assert np.array_equal(glob, og), (glob, og)
    assert np.array_equal(loc, ol)
    ed, el, vd, vl = oracle.rept2_eta(edges, n, m, c, seed)
    assert np.array_equal(eta[0], ed), (eta[0], ed)
    assert np.array_equal(eta[1], el), (eta[1], el)
    if eta_v is not None:
        assert np.array_equal(eta_v[0], vd)
        assert np.array_equal(eta_v[1], vl)
    return og, ol, ed, vd


@pytest.mark.parametrize("m,c,per_proc", [(3, 7, False), (2, 5, True), (10, 15, False), (5, 3, False),
                                          (4, 8, False), (1, 1, False), (2, 3, False), (3, 22, False)])
def test_pair_counters_random_graphs(cuda, m, c, per_proc):
    e = synth.er(300, 3000, 21 + m, 22 + c)
    _say(f"alg2 ER n=300 E=3000 m={m} c={c} per_proc={per_proc}")
    got = _run(cuda, e, 300, m, c, 99 + m * c, per_proc=per_proc)
    _, _, ed, vd = _check(e, 300, m, c, 99 + m * c, got, per_proc=per_proc)
    assert ed.sum() > 0
    # each pair's share is added at both endpoints of its shared edge
    assert vd.sum() == 2 * ed.sum()


def test_pair_counters_hand_streams(cuda):
    """Two triangles sharing {0, 1} (one processor): shared edge first (a pair under both
    readings), shared edge closing the first triangle (a pair only under the printed counter)."""
    for rows, want in [([[0, 1], [0, 2], [1, 2], [0, 3], [1, 3]], ([1], [1])),
                       ([[0, 2], [1, 2], [0, 1], [0, 3], [1, 3]], ([0], [1]))]:
        e = np.array(rows, np.uint32)
        _say(f"alg2 hand stream {rows}")
        got = _run(cuda, e, 4, 1, 1, 0)
        _check(e, 4, 1, 1, 0, got)
        assert got[2][0].tolist() == want[0] and got[2][1].tolist() == want[1]


def test_pair_counters_degenerate(cuda):
    cases = [(np.zeros((0, 2), np.uint32), 5), (np.array([[0, 1]], np.uint32), 2)]
    tri = [(0, 1), (1, 2), (0, 2)]
    for perm in itertools.permutations(range(3)):
        cases.append((np.array([tri[i] for i in perm], np.uint32), 3))
    cases.append((synth.shuffled(synth.complete(12), 5, 6), 12))
    for e, n in cases:
        for m, c in [(1, 1), (2, 3), (1, 3)]:
            _say(f"alg2 degenerate E={len(e)} n={n} m={m} c={c}")
            got = _run(cuda, e, n, m, c, 4)
            _check(e, n, m, c, 4, got)


@pytest.mark.parametrize("tune", [None,
                                  dict(wave_cap=16, block_cap=64, b_chunk=16, threads=256),
                                  dict(wave_cap=32, block_cap=128, b_chunk=64, threads=1024, light_tile=1),
                                  dict(wave_cap=8, block_cap=64, b_chunk=1024, threads=64, blocks=3)])
def test_pair_counters_launch_shapes(cuda, tune):
    """Hub lists split over several hashed chunks and several staged list chunks, per
    workgroup and per wavefront: each pair lands on the right adjacency position."""
    from paper_1811_09136_amd import rept
    e, n = synth.scaled_chung_lu(120_000, 31)
    for m, c in [(3, 5), (2, 3)]:
        _say(f"alg2 Chung-Lu n={n} E={len(e)} m={m} c={c} tune={tune}")
        got = _run(cuda, e, n, m, c, 17, tune=None if tune is None else rept.tuning(**tune))
        assert got[4].max_out_degree > 64
        _check(e, n, m, c, 17, got)


def test_pair_counters_million_edges(cuda):
    """A 1M-edge power-law stream in two hash groups (m = 10, c = 15): every counter exact."""
    e, n = synth.scaled_chung_lu(1_000_000, 41)
    _say(f"alg2 Chung-Lu n={n} E={len(e)} m=10 c=15")
    got = _run(cuda, e, n, 10, 15, 17)
    _check(e, n, 10, 15, 17, got)
    got = _run(cuda, e, n, 10, 15, 17, with_nodes=False)
    assert got[3] is None
    ed, el, _, _ = oracle.rept2_eta(e, n, 10, 15, 17)
    assert np.array_equal(got[2][0], ed) and np.array_equal(got[2][1], el)


@pytest.mark.parametrize("m,c,per_proc", [(10, 15, False), (3, 7, True), (2, 5, False)])
def test_count_then_combined_estimate(cuda, m, c, per_proc):
    """Counts and pair counters from the device, combined estimators from the library on the
    host: equal to the oracle's estimators on the oracle's counts, 0 ulp."""
    from paper_1811_09136_amd import rept
    e = synth.config1_stream() if m == 10 else synth.er(400, 5000, 3 + m, 4 + c)
    n = 2000 if m == 10 else 400
    _say(f"alg2 estimate n={n} E={len(e)} m={m} c={c} per_proc={per_proc}")
    got = _run(cuda, e, n, m, c, 7, per_proc=per_proc)
    og, ol, ed, vd = _check(e, n, m, c, 7, got, per_proc=per_proc)
    p = rept.Params(m, c, 7, per_proc)
    th, tv = rept.rept_estimate_combined(n, p, got[0], got[1], int(got[2][0].sum()), got[3][0])
    oth, otv = oracle.estimate2(n, m, c, og, ol, int(ed.sum()), vd, per_proc=per_proc)
    assert th == oth and np.array_equal(tv.view(np.uint64), otv.view(np.uint64))


def test_pair_counter_errors(cuda):
    import torch
    from paper_1811_09136_amd import rept
    e = synth.er(50, 200, 1, 2)
    g = rept.Graph(rept.to_device_edges(e, cuda), 50)
    p = rept.Params(2, 3, 1)
    need = rept.rept_count_eta_workspace_size(g.handle, p)
    assert need >= rept.rept_count_workspace_size(g.handle, p) + 8 * 2 * len(e)
    glob, loc = g.outputs(p)
    eta = torch.empty((2, 3), dtype=torch.int64, device=cuda)
    ws = torch.empty(need, dtype=torch.uint8, device=cuda)
    sp = torch.cuda.current_stream().cuda_stream
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_count_eta(g.handle, p, glob.data_ptr(), loc.data_ptr(), eta.data_ptr(), None, ws.data_ptr(),
                            need - 256, None, sp)
    assert ei.value.code == rept.REPT_ENOMEM
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_count_eta(g.handle, p, glob.data_ptr(), loc.data_ptr(), eta.data_ptr() + 4, None, ws.data_ptr(),
                            need, None, sp)
    assert ei.value.code == rept.REPT_EINVAL
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_count_eta(g.handle, rept.Params(2, 3, 1, mascot=True), glob.data_ptr(), loc.data_ptr(),
                            eta.data_ptr(), None, ws.data_ptr(), need, None, sp)
    assert ei.value.code == rept.REPT_ENOTSUP
    torch.cuda.synchronize()
    g.close()


@pytest.mark.parametrize("m,c,per_proc", [(2, 19, False), (3, 28, True), (2, 35, False)])
def test_pair_counters_more_than_eight_groups(cuda, m, c, per_proc):
    """Algorithm 2 with more than 8 hash groups (launches of 8 groups, each adding its pair
    counts): every counter equals the oracle's, and the combined estimators agree to 0 ulp."""
    from paper_1811_09136_amd import rept
    e = synth.er(300, 3000, 61 + m, 62 + c)
    _say(f"alg2 ER n=300 E=3000 m={m} c={c} per_proc={per_proc} groups={-(-c // m)}")
    got = _run(cuda, e, 300, m, c, 5 + c, per_proc=per_proc)
    og, ol, ed, vd = _check(e, 300, m, c, 5 + c, got, per_proc=per_proc)
    assert ed.sum() > 0
    p = rept.Params(m, c, 5 + c, per_proc)
    th, tv = rept.rept_estimate_combined(300, p, got[0], got[1], int(got[2][0].sum()), got[3][0])
    oth, otv = oracle.estimate2(300, m, c, og, ol, int(ed.sum()), vd, per_proc=per_proc)
    assert th == oth and np.array_equal(tv.view(np.uint64), otv.view(np.uint64))
