"""Device path vs the CPU oracle, bit-exact on every integer counter.

Inputs are seeded synthetic streams (module ``synth``).  Each case prints its name and shape
before touching the GPU so that a failing run names its case.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _run(cuda, edges, n, m, c, seed, per_proc=False, tune=None, window=None):
    import torch
    from paper_1811_09136_amd import rept
    p = rept.Params(m, c, seed, per_proc)
    g = rept.Graph(rept.to_device_edges(edges, cuda), n)
    if tune is None and window is None:
        glob, loc = g.count(p)
    else:
        out = g.outputs(p)
        out[0].zero_()
        out[1].zero_()
        t0, t1 = (0, len(edges)) if window is None else window
        if tune is None:
            glob, loc = g.count_range(p, t0, t1, out)
        else:
            job = rept.make_job(g, p, out, g.new_workspace(p), t0=t0, t1=t1, accumulate=True)
            ws = torch.empty(rept.rept_batch_workspace_size(1), dtype=torch.uint8, device=cuda)
            rept.rept_batch_count([job], tune, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
            glob, loc = out
    torch.cuda.synchronize()
    res = glob.cpu().numpy(), loc.cpu().numpy(), g.info
    g.close()
    return res


def _check(edges, n, m, c, seed, got, per_proc=False, window=None):
    kw = {}
    if window is not None:
        kw = dict(t0=window[0], t1=window[1])
    og, ol = oracle.rept(edges, n, m, c, seed, per_proc=per_proc, **kw)
    assert np.array_equal(got[0], og), (got[0], og)
    assert np.array_equal(got[1], ol)
    return og, ol


def test_config1_parity(cuda):
    e = synth.config1_stream()
    _say("config1 ER n=2000 E=20000 m=10 c=10")
    got = _run(cuda, e, 2000, 10, 10, 20181122)
    og, ol = _check(e, 2000, 10, 10, 20181122, got)
    assert og.sum() > 0
    # invariant: each semi-triangle adds one to each of its three nodes
    assert ol.sum() == 3 * og.sum()


@pytest.mark.parametrize("m,c,per_proc", [(1, 1, False), (2, 2, False), (3, 7, False), (10, 40, False),
                                          (4, 4, True), (5, 12, True), (2, 16, False), (20, 150, False),
                                          (300, 1500, False), (17, 34, True), (257, 300, False)])
def test_random_graphs(cuda, m, c, per_proc):
    e = synth.er(300, 3000, 11 + m, 12 + c)
    _say(f"ER n=300 E=3000 m={m} c={c} per_proc={per_proc}")
    got = _run(cuda, e, 300, m, c, 1234 + m * c, per_proc=per_proc)
    _check(e, 300, m, c, 1234 + m * c, got, per_proc=per_proc)


@pytest.mark.parametrize("shape", ["complete", "wheel", "friendship", "bipartite", "cycle"])
def test_closed_form_shapes(cuda, shape):
    # m = 1: every triangle is counted once (its first two edges share the only slot)
    mk = {"complete": lambda: (synth.complete(24), 24), "wheel": lambda: (synth.wheel(50), 51),
          "friendship": lambda: (synth.friendship(30), 61), "bipartite": lambda: (synth.complete_bipartite(9, 13), 22),
          "cycle": lambda: (synth.cycle(40), 40)}
    e0, n = mk[shape]()
    e = synth.shuffled(e0, 77, 78)
    _say(f"shape={shape} n={n} E={len(e)} m=1 c=1")
    got = _run(cuda, e, n, 1, 1, 5)
    _check(e, n, 1, 1, 5, got)


def test_windows_additive(cuda):
    e = synth.er(500, 6000, 21, 22)
    cuts = [0, 1, 1000, 2500, 2501, 6000]
    _say("windows ER n=500 E=6000 m=3 c=6")
    full = _run(cuda, e, 500, 3, 6, 9)
    acc_g = np.zeros_like(full[0])
    acc_l = np.zeros_like(full[1])
    for t0, t1 in zip(cuts[:-1], cuts[1:]):
        got = _run(cuda, e, 500, 3, 6, 9, window=(t0, t1))
        _check(e, 500, 3, 6, 9, got, window=(t0, t1))
        acc_g += got[0]
        acc_l += got[1]
    assert np.array_equal(acc_g, full[0]) and np.array_equal(acc_l, full[1])


@pytest.mark.parametrize("tune", [dict(wave_cap=16, block_cap=64, b_chunk=16, threads=256),
                                  dict(wave_cap=32, block_cap=128, b_chunk=64, threads=1024, light_tile=1),
                                  dict(wave_cap=8, block_cap=64, b_chunk=1024, threads=64, blocks=3),
                                  dict(wave_cap=256, block_cap=2048, b_chunk=256, threads=512, blocks=1,
                                       light_tile=64)])
def test_launch_shapes(cuda, tune):
    from paper_1811_09136_amd import rept
    e, n = synth.scaled_chung_lu(120_000, 31)
    _say(f"Chung-Lu n={n} E={len(e)} m=3 c=5 tune={tune}")
    got = _run(cuda, e, n, 3, 5, 17, tune=rept.tuning(**tune))
    assert got[2].max_out_degree > 64  # the chunked workgroup path is exercised
    _check(e, n, 3, 5, 17, got)


def test_hash_slots(cuda):
    import torch
    from paper_1811_09136_amd import rept
    e = synth.config1_stream()
    for m, c in [(10, 40), (7, 7), (1, 3), (255, 1000)]:
        _say(f"hash slots m={m} c={c}")
        p = rept.Params(m, c, 99 + m)
        s = rept.hash_slots(p, rept.to_device_edges(e, cuda))
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy().view(np.uint32), oracle.slots(e, m, p.groups, p.seed))


@pytest.mark.parametrize("case", ["selfloop", "dup_same", "dup_flipped", "range"])
def test_invalid_streams(cuda, case):
    from paper_1811_09136_amd import rept
    e = synth.er(50, 200, 3, 4).copy()
    if case == "selfloop":
        e[100] = (7, 7)
        code = rept.REPT_ESELFLOOP
    elif case == "dup_same":
        e[150] = e[20]
        code = rept.REPT_EDUP
    elif case == "dup_flipped":
        e[150] = e[20][::-1]
        code = rept.REPT_EDUP
    else:
        e[10] = (3, 50)
        code = rept.REPT_ERANGE
    assert oracle.validate(50, e) == code
    _say(f"invalid stream {case}")
    with pytest.raises(rept.ReptError) as ei:
        rept.Graph(rept.to_device_edges(e, cuda), 50)
    assert ei.value.code == code


@pytest.mark.parametrize("K", [40, 100, 300])
@pytest.mark.parametrize("flipped", [False, True])
def test_duplicate_in_each_sort_class(cuda, K, flipped):
    """A duplicate edge inside one adjacency segment of K entries (segments of at most 64
    entries are sorted by one wavefront, longer ones up to 4096 by a workgroup in LDS, with
    networks of 128 and 512 entries here): a K-clique in which every node but 0 and 1 has one
    pendant edge, so node 0 ranks lowest in the clique and its out-list holds the K - 1 other
    clique nodes plus the second copy of {0, 1}."""
    from paper_1811_09136_amd import rept
    clique = [(u, v) for u in range(K) for v in range(u + 1, K)]
    pend = [(i, K + i) for i in range(2, K)]
    dup = (1, 0) if flipped else (0, 1)
    e = np.array(clique + pend + [dup], np.uint32)
    n = 2 * K
    assert oracle.validate(n, e) == rept.REPT_EDUP
    _say(f"duplicate in a segment of {K} entries flipped={flipped}")
    with pytest.raises(rept.ReptError) as ei:
        rept.Graph(rept.to_device_edges(e, cuda), n)
    assert ei.value.code == rept.REPT_EDUP
    # without the duplicate the same stream builds and counts like the oracle
    e = e[:-1]
    got = _run(cuda, e, n, 2, 3, 5)
    _check(e, n, 2, 3, 5, got)
    assert got[2].max_out_degree == K - 1


def test_degenerate_streams(cuda):
    # empty stream, one edge, a path (no triangles), a single triangle in all 6 orders
    cases = [(np.zeros((0, 2), np.uint32), 5), (np.array([[0, 1]], np.uint32), 2),
             (np.array([[0, 1], [1, 2], [2, 3]], np.uint32), 4)]
    import itertools
    tri = [(0, 1), (1, 2), (0, 2)]
    for perm in itertools.permutations(range(3)):
        cases.append((np.array([tri[i] for i in perm], np.uint32), 3))
    for e, n in cases:
        for m, c in [(1, 1), (2, 2), (2, 4)]:
            _say(f"degenerate E={len(e)} n={n} m={m} c={c}")
            got = _run(cuda, e, n, m, c, 3)
            _check(e, n, m, c, 3, got)


def test_lds_budget_rejected(cuda):
    # a staging chunk whose LDS footprint exceeds the 160 KB of a CU is refused, not launched
    import torch
    from paper_1811_09136_amd import rept
    e = synth.er(100, 500, 1, 2)
    g = rept.Graph(rept.to_device_edges(e, cuda), 100)
    p = rept.Params(3, 6, 1)
    out = g.outputs(p)
    job = rept.make_job(g, p, out, g.new_workspace(p))
    ws = torch.empty(rept.rept_batch_workspace_size(1), dtype=torch.uint8, device=cuda)
    _say("LDS budget rejection")
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_batch_count([job], rept.tuning(block_cap=4096, b_chunk=1024, threads=1024), ws.data_ptr(),
                              ws.numel(), None)
    assert ei.value.code == rept.REPT_EINVAL
    # a light tile is loaded one unit per lane: more than 64 units is refused
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_batch_count([job], rept.tuning(light_tile=65), ws.data_ptr(), ws.numel(), None)
    assert ei.value.code == rept.REPT_EINVAL
    g.close()


def test_count_workspace_contract(cuda):
    """The count workspace holds the slot table: too small -> ENOMEM, missing or misaligned ->
    EINVAL; a batch job flagged TABLE_READY reuses the table an earlier launch wrote and gives
    the same integers; a table written for other params is rewritten by a job without the flag."""
    import torch
    from paper_1811_09136_amd import rept
    e = synth.er(400, 5000, 41, 42)
    g = rept.Graph(rept.to_device_edges(e, cuda), 400)
    p = rept.Params(3, 9, 77)
    need = g.workspace_bytes(p)
    assert need >= 2 * 4 * len(e) and need % 256 == 0  # 3 groups -> 4 slots of 16 bits per edge
    out = g.outputs(p)
    small = torch.empty(need - 256, dtype=torch.uint8, device=cuda)
    _say("workspace errors")
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_count(g.handle, p, out[0].data_ptr(), out[1].data_ptr(), small.data_ptr(), small.numel(), None)
    assert ei.value.code == rept.REPT_ENOMEM
    big = torch.empty(need + 512, dtype=torch.uint8, device=cuda)
    for ptr in (0, big.data_ptr() + 8):
        with pytest.raises(rept.ReptError) as ei:
            rept.rept_count(g.handle, p, out[0].data_ptr(), out[1].data_ptr(), ptr, need, None)
        assert ei.value.code == rept.REPT_EINVAL
    og, ol = oracle.rept(e, 400, 3, 9, 77)
    ws = g.new_workspace(p)
    bw = torch.empty(rept.rept_batch_workspace_size(1), dtype=torch.uint8, device=cuda)
    sp = torch.cuda.current_stream().cuda_stream
    _say("table ready reuse")
    for ready in (False, True, True):
        job = rept.make_job(g, p, out, ws, table_ready=ready)
        rept.rept_batch_count([job], None, bw.data_ptr(), bw.numel(), sp)
        torch.cuda.synchronize()
        assert np.array_equal(out[0].cpu().numpy(), og) and np.array_equal(out[1].cpu().numpy(), ol)
    # the same buffer used for other params (a new seed) is rewritten when the flag is absent
    p2 = rept.Params(3, 9, 78)
    og2, ol2 = oracle.rept(e, 400, 3, 9, 78)
    out2 = g.outputs(p2)
    job = rept.make_job(g, p2, out2, ws)
    rept.rept_batch_count([job], None, bw.data_ptr(), bw.numel(), sp)
    torch.cuda.synchronize()
    assert np.array_equal(out2[0].cpu().numpy(), og2) and np.array_equal(out2[1].cpu().numpy(), ol2)
    g.close()


def _orientation_stats(e, n):
    """Statistics of the degree orientation from their definitions: rank = (degree, id); an
    edge points from its lower- to its higher-ranked endpoint."""
    e = e.astype(np.int64)
    deg = np.bincount(e.ravel(), minlength=n)
    key = deg * n + np.arange(n)
    lo = np.where(key[e[:, 0]] < key[e[:, 1]], e[:, 0], e[:, 1])
    hi = np.where(key[e[:, 0]] < key[e[:, 1]], e[:, 1], e[:, 0])
    dout = np.bincount(lo, minlength=n)
    return dict(work=int(np.minimum(dout[lo], dout[hi]).sum()), reverse=int((dout[lo] < dout[hi]).sum()),
                sum_out_sq=int((dout * dout).sum()), max_out=int(dout.max()), units=int((dout >= 2).sum()))


@pytest.mark.parametrize("kind", ["er", "chung_lu"])
def test_build_statistics_match_definitions(cuda, kind):
    from paper_1811_09136_amd import rept
    if kind == "er":
        e, n = synth.er(3000, 30000, 61, 62), 3000
    else:
        e, n = synth.scaled_chung_lu(80_000, 63)
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    ref = _orientation_stats(e, n)
    _say(f"build statistics {kind}")
    i = g.info
    assert (i.oriented_work, i.num_reverse, i.sum_out_sq, i.max_out_degree, i.num_apex) == \
        (ref["work"], ref["reverse"], ref["sum_out_sq"], ref["max_out"], ref["units"])
    g.close()


def test_reduce_local_exact(cuda):
    """The device reduction of the local rows (exact int64), into its own buffer and in place
    over the first row; bad pointers are EINVAL before any launch."""
    import torch
    from paper_1811_09136_amd import rept
    rng = np.random.default_rng(5)
    for rows, n in [(1, 1), (4, 1000), (3, 70001), (40, 5003)]:
        _say(f"reduce_local rows={rows} n={n}")
        loc = rng.integers(0, 2**45, size=(rows, n))
        d = torch.from_numpy(loc).to(cuda)
        out = torch.full((n,), -1, dtype=torch.int64, device=cuda)
        rept.rept_reduce_local(d.data_ptr(), rows, n, out.data_ptr(), None)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), loc.sum(axis=0))
        rept.rept_reduce_local(d.data_ptr(), rows, n, d.data_ptr(), None)
        torch.cuda.synchronize()
        assert np.array_equal(d[0].cpu().numpy(), loc.sum(axis=0))
        assert np.array_equal(d[1:].cpu().numpy(), loc[1:])
    d = torch.zeros(8, dtype=torch.int64, device=cuda)
    for args in [(0, 1, 1, d.data_ptr()), (d.data_ptr(), 0, 1, d.data_ptr()), (d.data_ptr(), 1, 0, d.data_ptr()),
                 (d.data_ptr() + 4, 1, 1, d.data_ptr())]:
        with pytest.raises(rept.ReptError) as ei:
            rept.rept_reduce_local(*args, None)
        assert ei.value.code == rept.REPT_EINVAL


@pytest.mark.parametrize("m,c,per_proc", [(10, 40, False), (3, 7, True)])
def test_count_reduce_estimate_path(cuda, m, c, per_proc):
    """Count, reduce the local rows on the device, estimate from the sums: the estimators equal
    the oracle's on the oracle's rows (0 ulp)."""
    import torch
    from paper_1811_09136_amd import rept
    n = 3000
    e = synth.chung_lu(n, 30000, 2.1, 300.0, seed=31, order_seed=32)
    _say(f"count_reduce_estimate chung_lu n={n} E={len(e)} m={m} c={c} per_proc={per_proc}")
    p = rept.Params(m, c, 77, per_proc)
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    glob, loc = g.count(p)
    sums = torch.empty(n, dtype=torch.int64, device=cuda)
    rept.rept_reduce_local(loc.data_ptr(), p.rows, n, sums.data_ptr(), None)
    torch.cuda.synchronize()
    og, ol = oracle.rept(e, n, m, c, 77, per_proc=per_proc)
    assert np.array_equal(sums.cpu().numpy(), ol.sum(axis=0))
    g.close()
    if c > m and c % m:
        return
    th, tv = rept.rept_estimate_sums(n, p, glob.cpu().numpy(), sums.cpu().numpy())
    oth, otv = oracle.estimate(n, m, c, og, ol)
    assert th == oth and np.array_equal(tv.view(np.uint64), otv.view(np.uint64))


def test_default_shape_shrinks_to_fit(cuda):
    """A graph whose longest out-list exceeds 1024 entries with 8 hash groups: the default
    launch shape (2048-entry chunks) does not fit LDS as chosen and is shrunk, not refused.
    The counts are shape-independent, so they equal those of an explicit smaller shape, and
    each semi-triangle adds one to each of its three nodes."""
    import torch
    from paper_1811_09136_amd import rept
    n = 1100
    iu, ju = np.triu_indices(n, 1)
    e = np.stack([iu, ju], 1).astype(np.uint32)
    rng = np.random.default_rng(99)
    e = e[rng.permutation(len(e))]
    flip = rng.random(len(e)) < 0.5
    e[flip] = e[flip][:, ::-1]
    _say(f"complete graph n={n} E={len(e)} m=2 c=16 (8 groups), default vs explicit shape")
    p = rept.Params(2, 16, 5)
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    assert g.info.max_out_degree > 1024
    outs = []
    for tune in (None, rept.tuning(block_cap=512, b_chunk=64)):
        out = g.outputs(p)
        out[0].zero_()
        out[1].zero_()
        job = rept.make_job(g, p, out, g.new_workspace(p), accumulate=True)
        ws = torch.empty(rept.rept_batch_workspace_size(1), dtype=torch.uint8, device=cuda)
        rept.rept_batch_count([job], tune, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        outs.append((out[0].cpu().numpy(), out[1].cpu().numpy()))
    g.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][0].sum() > 0 and outs[0][1].sum() == 3 * outs[0][0].sum()



@pytest.mark.parametrize("kind", ["two_groups", "alg2", "mascot"])
def test_wide_default_shape_equals_small_shape(cuda, kind):
    """Lists of more than 1024 entries take the wide default shape (1024-thread workgroups, one
    2048-entry table chunk, 1024-list B chunks, the light launch sized to fit its LDS). With two
    hash groups, with Algorithm 2's pair counters and with MASCOT's keep masks, its counts equal
    those of an explicit small shape (which the other tests check against the oracle)."""
    import torch
    from paper_1811_09136_amd import rept
    n = 1100
    e = synth.shuffled(synth.complete(n), 77, flip_seed=78)
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    assert g.info.max_out_degree > 1024
    small = rept.tuning(wave_cap=32, block_cap=256, b_chunk=64, threads=256)
    outs = []
    for tune in (None, small):
        _say(f"K_{n} E={len(e)} {kind} shape={'default' if tune is None else 'small'}")
        if kind == "alg2":
            glob, loc, eta, eta_v = g.count_eta(rept.Params(2, 3, 13), tuning=tune)
            torch.cuda.synchronize()
            outs.append([x.cpu().numpy() for x in (glob, loc, eta, eta_v)])
            continue
        p = rept.Params(2, 8, 13, mascot=True) if kind == "mascot" else rept.Params(10, 20, 13)
        out = g.outputs(p)
        out[0].zero_()
        out[1].zero_()
        job = rept.make_job(g, p, out, g.new_workspace(p), accumulate=True)
        ws = torch.empty(rept.rept_batch_workspace_size(1), dtype=torch.uint8, device=cuda)
        rept.rept_batch_count([job], tune, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        outs.append([out[0].cpu().numpy(), out[1].cpu().numpy()])
    g.close()
    assert all(np.array_equal(a, b) for a, b in zip(outs[0], outs[1]))
    assert outs[0][0].sum() > 0

def test_build_from_host_stream(cuda):
    """A host-resident stream built with rept_build_host: the same graph statistics as the
    device-input build and the oracle's counts; an invalid stream is reported as from the
    device path; buffers too small are refused before any copy."""
    import torch
    from paper_1811_09136_amd import rept
    e = synth.er(500, 6000, 21, 22)
    n, p = 500, rept.Params(5, 15, 3)
    _say(f"host-input build ER n={n} E={len(e)} m=5 c=15")
    pb, sb = rept.rept_query_sizes(n, len(e))
    P = torch.empty(pb, dtype=torch.uint8, device=cuda)
    S = torch.empty(sb, dtype=torch.uint8, device=cuda)
    sp = torch.cuda.current_stream().cuda_stream
    h = rept.rept_build_host(n, e, P.data_ptr(), pb, S.data_ptr(), sb, sp)
    info_h = rept.rept_graph_get_info(h)
    glob = torch.empty(p.c, dtype=torch.int64, device=cuda)
    loc = torch.empty((p.rows, n), dtype=torch.int64, device=cuda)
    wsb = rept.rept_count_workspace_size(h, p)
    ws = torch.empty(wsb, dtype=torch.uint8, device=cuda)
    rept.rept_count(h, p, glob.data_ptr(), loc.data_ptr(), ws.data_ptr(), wsb, sp)
    torch.cuda.synchronize()
    got = glob.cpu().numpy(), loc.cpu().numpy()
    rept.rept_destroy(h)
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    info_d = g.info
    g.close()
    for f in ("num_apex", "max_out_degree", "oriented_work", "num_reverse"):
        assert getattr(info_h, f) == getattr(info_d, f), f
    og, ol = oracle.rept(e, n, 5, 15, 3)
    assert np.array_equal(got[0], og) and np.array_equal(got[1], ol)
    bad = e.copy()
    bad[17] = [9, 9]
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_build_host(n, bad, P.data_ptr(), pb, S.data_ptr(), sb, sp)
    assert ei.value.code == rept.REPT_ESELFLOOP
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_build_host(n, e, P.data_ptr(), pb - 256, S.data_ptr(), sb, sp)
    assert ei.value.code == rept.REPT_ENOMEM


@pytest.mark.parametrize("m,c,per_proc", [(2, 40, False), (3, 29, False), (2, 33, True), (10, 320, False)])
def test_more_than_eight_groups(cuda, m, c, per_proc):
    """Counts with more than 8 hash groups run as successive launches of 8 groups (the last
    group may be partial): every counter equals the oracle's, also over a stream window."""
    import torch
    from paper_1811_09136_amd import rept
    e = synth.er(300, 3000, 51 + m, 52 + c)
    _say(f"ER n=300 E=3000 m={m} c={c} per_proc={per_proc} groups={-(-c // m)}")
    got = _run(cuda, e, 300, m, c, 7 + c, per_proc=per_proc)
    og, ol = _check(e, 300, m, c, 7 + c, got, per_proc=per_proc)
    assert og.sum() > 0
    p = rept.Params(m, c, 7 + c, per_proc)
    g = rept.Graph(rept.to_device_edges(e, cuda), 300)
    out = g.outputs(p)
    out[0].zero_()
    out[1].zero_()
    g.count_range(p, 1000, 2500, out)
    torch.cuda.synchronize()
    wg, wl = oracle.rept(e, 300, m, c, 7 + c, per_proc=per_proc, t0=1000, t1=2500)
    assert np.array_equal(out[0].cpu().numpy(), wg) and np.array_equal(out[1].cpu().numpy(), wl)
    if c % m == 0:  # (c mod m != 0 takes Algorithm 2's estimator, at most 8 groups)
        th, tv = rept.rept_estimate(300, p, out[0].cpu().numpy(), out[1].cpu().numpy())
        oth, otv = oracle.estimate(300, m, c, wg, wl)
        assert th == oth and np.array_equal(tv.view(np.uint64), otv.view(np.uint64))
    g.close()
