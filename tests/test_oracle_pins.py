"""Pins of the CPU oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: closed-form counts, a
definition-level brute force, invariants of Algorithm 1's updates, the sampling probabilities
of Theorem 1, the unbiasedness and variance of Theorem 3, published generator outputs, and a
hand-built stream.  A plausible slip in the oracle (a dropped counter update, counting after
insertion instead of before, a wrong processor index, a transposed edge, a wrong estimator
scale) fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    expects, rows = {}, []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line.startswith("# expect"):
            k, *vals = line[len("# expect"):].split()
            expects[k] = [int(v) for v in vals]
        elif line and not line.startswith("#"):
            rows.append([int(x) for x in line.split()])
    return expects, rows


# ---------------------------------------------------------------------------- P5 hand-built

def test_k4_hand_built_stream():
    exp, rows = _golden("k4_stream.txt")
    e = np.array(rows, dtype=np.uint32)
    g, l = oracle.rept(e, 4, 1, 1, 0)
    assert g.tolist() == exp["global"]
    assert l[0].tolist() == exp["local"]
    # per-edge updates 0,0,1,0,1,2 (counted before insertion)
    per_edge = [int(oracle.edge_updates(e, 4, 1, 1, 0, [t])[0][0]) for t in range(6)]
    assert per_edge == [0, 0, 1, 0, 1, 2]


# ---------------------------------------------------------------------------- hash pins

def test_splitmix64_reference_outputs():
    _, rows = _golden("splitmix64_seed1234567.txt")
    for idx, val in rows:
        assert oracle.splitmix64(1234567, idx) == val


def test_hash_params_are_consecutive_splitmix_draws():
    hp = oracle.hash_params(42, 3)
    p = 2**61 - 1
    assert [int(x) for x in hp.ravel()] == [(oracle.splitmix64(42, i) >> 3) % p for i in range(12)]


def test_hash_basic_properties():
    e = synth.config1_stream()
    s = oracle.slots(e, 10, 4, 7)
    assert s.shape == (4, len(e)) and s.max() < 10
    flipped = np.ascontiguousarray(e[:, ::-1])
    assert np.array_equal(oracle.slots(flipped, 10, 4, 7), s)  # undirected: h(u,v) = h(v,u)
    assert (oracle.slots(e, 1, 2, 7) == 0).all()  # m = 1: one slot
    # groups use independent parameters: their slot sequences differ
    assert (s[0] != s[1]).mean() > 0.8


def test_hash_uniform_and_collision_rates():
    """Theorem 1: r given edges land in one given processor with probability 1/m^r, so two
    distinct edges share a slot with probability 1/m and three with probability 1/m^2."""
    m = 10
    e = synth.er(5000, 200000, 3, 4)
    s = oracle.slots(e, m, 1, 2024)[0].astype(np.int64)
    counts = np.bincount(s, minlength=m)
    expected = len(s) / m
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 40.0  # chi^2 with 9 dof: 40 is far beyond the 0.9999 quantile (~33.7)
    rng = np.random.default_rng(5)
    i = rng.integers(0, len(s), size=(400000, 3))
    i = i[(i[:, 0] != i[:, 1]) & (i[:, 1] != i[:, 2]) & (i[:, 0] != i[:, 2])]
    pair = (s[i[:, 0]] == s[i[:, 1]]).mean()
    triple = ((s[i[:, 0]] == s[i[:, 1]]) & (s[i[:, 1]] == s[i[:, 2]])).mean()
    assert abs(pair - 1 / m) < 0.004
    assert abs(triple - 1 / m**2) < 0.0012


# ---------------------------------------------------------------------------- P1/P4 closed forms

@pytest.mark.parametrize("n", [3, 4, 7, 12])
def test_complete_graph(n):
    e = synth.shuffled(synth.complete(n), 10 + n, 20 + n)
    g, l = oracle.rept(e, n, 1, 1, 0)
    assert g[0] == math.comb(n, 3)
    assert (l[0] == math.comb(n - 1, 2)).all()


@pytest.mark.parametrize("n", [4, 5, 9])
def test_cycle_and_bipartite_have_none(n):
    e = synth.shuffled(synth.cycle(n), 1, 2)
    g, l = oracle.rept(e, n, 1, 1, 0)
    assert g[0] == 0 and l.sum() == 0
    e = synth.shuffled(synth.complete_bipartite(n, n + 1), 3, 4)
    g, l = oracle.rept(e, 2 * n + 1, 1, 1, 0)
    assert g[0] == 0 and l.sum() == 0


@pytest.mark.parametrize("n", [4, 6, 11])
def test_wheel(n):
    e = synth.shuffled(synth.wheel(n), 5, 6)
    g, l = oracle.rept(e, n + 1, 1, 1, 0)
    assert g[0] == n
    assert l[0, 0] == n and (l[0, 1:] == 2).all()


@pytest.mark.parametrize("k", [1, 3, 8])
def test_friendship(k):
    e = synth.shuffled(synth.friendship(k), 7, 8)
    g, l = oracle.rept(e, 2 * k + 1, 1, 1, 0)
    assert g[0] == k
    assert l[0, 0] == k and (l[0, 1:] == 1).all()


@pytest.mark.parametrize("seed", range(4))
def test_m1_equals_exact_triangle_counts(seed):
    """m = 1: every edge is stored, each triangle is counted once (at its last edge), so
    tau^(0) = tau and tau_v^(0) = tau_v; checked against trace(A^3)/6 and diag(A^3)/2."""
    n = 40 + 7 * seed
    e = synth.er(n, 4 * n, 100 + seed, 200 + seed)
    tau, tau_v = brute.exact_counts(e, n)
    g, l = oracle.rept(e, n, 1, 1, seed)
    assert g[0] == tau and np.array_equal(l[0], tau_v)
    # c > m = 1: every group is a full copy
    g, l = oracle.rept(e, n, 1, 3, seed)
    assert (g == tau).all() and all(np.array_equal(l[k], tau_v) for k in range(3))


def test_m1_config1_exact():
    e = synth.config1_stream()
    tau, tau_v = brute.exact_counts(e, 2000)
    g, l = oracle.rept(e, 2000, 1, 1, 0)
    assert g[0] == tau and np.array_equal(l[0], tau_v)


# ---------------------------------------------------------------------------- P3 definition

@pytest.mark.parametrize("seed", range(3))
def test_algorithm1_matches_semi_triangle_definition(seed):
    """Algorithm 1's counters equal the semi-triangle counts of Section III: a triangle counts
    on processor i iff its first two edges are stored by i (any last edge)."""
    n = 24
    e = synth.er(n, 110, 300 + seed, 400 + seed)
    for m in range(1, 7):
        for c in range(1, 3 * m + 1):
            hs = 1000 * seed + 10 * m + c
            sl = oracle.slots(e, m, -(-c // m), hs)
            for per_proc in (False, True):
                g, l = oracle.rept(e, n, m, c, hs, per_proc=per_proc)
                bg, bl = brute.semi_triangle_counts(e, n, m, c, lambda k, t: int(sl[k, t]), per_proc)
                assert np.array_equal(g, bg), (m, c)
                assert np.array_equal(l, bl), (m, c)


def test_slot_override_matches_definition():
    """Arbitrary slot assignments (not from the hash): the replay and the definition agree."""
    rng = np.random.default_rng(9)
    n = 20
    e = synth.er(n, 90, 5, 6)
    for m, c in [(2, 2), (3, 5), (4, 9)]:
        G = -(-c // m)
        for _ in range(5):
            ov = rng.integers(0, m, size=(G, len(e))).astype(np.uint16)
            g, l = oracle.rept(e, n, m, c, 0, slot_override=ov)
            bg, bl = brute.semi_triangle_counts(e, n, m, c, lambda k, t: int(ov[k, t]))
            assert np.array_equal(g, bg) and np.array_equal(l, bl)


def test_semi_triangle_order_semantics():
    """Stream (0,1),(1,2),(0,2) with slots (s1, s2, s3): processor j counts the triangle iff
    s1 = s2 = j, whatever s3 is (its last edge need not be stored)."""
    e = np.array([(0, 1), (1, 2), (0, 2)], dtype=np.uint32)
    for s1, s2, s3 in itertools.product(range(2), repeat=3):
        ov = np.array([[s1, s2, s3]], dtype=np.uint16)
        g, l = oracle.rept(e, 3, 2, 2, 0, slot_override=ov, per_proc=True)
        for j in range(2):
            want = int(s1 == s2 == j)
            assert g[j] == want and (l[j] == want).all()
        g1, _ = oracle.rept(e, 3, 2, 1, 0, slot_override=ov)  # c = 1 < m: only slot 0 exists
        assert g1[0] == int(s1 == s2 == 0)


# ---------------------------------------------------------------------------- P2/P9 invariants

def test_local_sum_is_three_times_global():
    e = synth.config1_stream()
    for m, c, pp in [(10, 10, False), (10, 40, False), (4, 3, True), (3, 11, True)]:
        g, l = oracle.rept(e, 2000, m, c, 77, per_proc=pp)
        if pp:
            assert np.array_equal(l.sum(axis=1), 3 * g)
        else:
            G = -(-c // m)
            for k in range(G):
                assert l[k].sum() == 3 * g[k * m:(k + 1) * m].sum()


def test_windows_are_additive_and_match_per_edge_form():
    e = synth.er(400, 5000, 13, 14)
    n, m, c, s = 400, 3, 7, 5
    full = oracle.rept(e, n, m, c, s)
    cuts = [0, 700, 701, 3000, 5000]
    acc = [np.zeros_like(full[0]), np.zeros_like(full[1])]
    for t0, t1 in zip(cuts[:-1], cuts[1:]):
        w = oracle.rept(e, n, m, c, s, t0=t0, t1=t1)
        pe = oracle.edge_updates(e, n, m, c, s, np.arange(t0, t1))
        assert np.array_equal(w[0], pe[0]) and np.array_equal(w[1], pe[1])
        acc[0] += w[0]
        acc[1] += w[1]
    assert np.array_equal(acc[0], full[0]) and np.array_equal(acc[1], full[1])
    rng = np.random.default_rng(3)
    ts = rng.choice(len(e), 300, replace=False)
    pe = oracle.edge_updates(e, n, m, c, s, ts, per_proc=True)
    tot = [np.zeros(c, np.int64), np.zeros((c, n), np.int64)]
    for t in ts:
        w = oracle.rept(e, n, m, c, s, per_proc=True, t0=int(t), t1=int(t) + 1)
        tot[0] += w[0]
        tot[1] += w[1]
    assert np.array_equal(pe[0], tot[0]) and np.array_equal(pe[1], tot[1])


def test_orientation_and_order_independence_of_inputs():
    """Edges are undirected: flipping every pair changes nothing; reordering the stream
    changes the counts only through which edge is last (m = 1 totals are order-free)."""
    e = synth.er(300, 2500, 1, 2)
    a = oracle.rept(e, 300, 4, 8, 3)
    b = oracle.rept(np.ascontiguousarray(e[:, ::-1]), 300, 4, 8, 3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    r = synth.shuffled(e, 9)
    assert oracle.rept(r, 300, 1, 1, 0)[0][0] == oracle.rept(e, 300, 1, 1, 0)[0][0]


def test_validation_codes():
    e = synth.er(30, 60, 1, 2)
    assert oracle.validate(30, e) == oracle.OK
    bad = e.copy(); bad[5] = (4, 4)
    assert oracle.validate(30, bad) == oracle.ESELFLOOP
    bad = e.copy(); bad[9] = e[3][::-1]
    assert oracle.validate(30, bad) == oracle.EDUP
    bad = e.copy(); bad[0] = (0, 30)
    assert oracle.validate(30, bad) == oracle.ERANGE
    with pytest.raises(oracle.OracleError):
        oracle.rept(bad, 30, 2, 2, 0)


# ---------------------------------------------------------------------------- P10 estimator

def test_estimator_special_cases():
    # m = 1, c = 1: the count itself
    assert oracle.estimate(3, 1, 1, [1349])[0] == 1349.0
    # c = m: m^2/c = m exactly
    th, tv = oracle.estimate(3, 10, 10, [13] * 10, np.array([[1, 2, 3]]))
    assert th == 1300.0 and tv.tolist() == [10.0, 20.0, 30.0]
    # c = 4m (c2 = 0): m / c1 = m^2 / c
    th, _ = oracle.estimate(3, 10, 40, [1] * 40)
    assert th == 100.0
    # c < m: m^2 / c
    th, _ = oracle.estimate(3, 8, 3, [1, 1, 1])
    assert th == 64.0
    with pytest.raises(oracle.OracleError) as ei:
        oracle.estimate(3, 10, 15, [0] * 15)  # c > m, c % m != 0: Algorithm 2's estimator
    assert ei.value.code == oracle.ENOTSUP
    with pytest.raises(oracle.OracleError) as ei:
        oracle.estimate(3, 2, 2, [2**52, 2**52])  # sum reaches 2^53
    assert ei.value.code == oracle.ERANGE
    with pytest.raises(oracle.OracleError):
        oracle.estimate(3, 2, 2, [-1, 0])


@pytest.mark.parametrize("m,c", [(4, 4), (4, 2), (3, 6)])
def test_estimator_unbiased_with_theorem3_variance(m, c):
    """Theorem 3 (and Section III-B for m | c): E[tau_hat] = tau and
    Var[tau_hat] = (tau (m^2 - c) + 2 eta (m - c)) / c for c <= m, tau (m - 1) / c1 for c = c1 m.
    Checked over R independent hash seeds on a graph with many edge-sharing triangles."""
    n = 30
    e = synth.shuffled(synth.er(n, 160, 41, 42), 43)
    tau, tau_v = brute.exact_counts(e, n)
    eta = brute.eta(e, n)
    if c <= m:
        var = (tau * (m * m - c) + 2 * eta * (m - c)) / c
    else:
        var = tau * (m - 1) / (c // m)
    R = 1500
    seeds = synth.u64(7, m * 100 + c, R)
    est = np.empty(R)
    for r in range(R):
        g, _ = oracle.rept(e, n, m, c, int(seeds[r]))
        est[r] = oracle.estimate(n, m, c, g)[0]
    assert abs(est.mean() - tau) < 4.0 * math.sqrt(var / R)
    ratio = est.var(ddof=1) / var
    assert 0.8 < ratio < 1.25, (ratio, tau, eta)


def test_local_estimator_unbiased():
    n = 30
    e = synth.shuffled(synth.er(n, 160, 41, 42), 43)
    tau, tau_v = brute.exact_counts(e, n)
    m, c, R = 3, 3, 1200
    acc = np.zeros(n)
    for r in range(R):
        g, l = oracle.rept(e, n, m, c, 5000 + r)
        acc += oracle.estimate(n, m, c, g, l)[1]
    v = int(np.argmax(tau_v))
    sd = math.sqrt(tau_v[v] * (m - 1) / R)  # Var(tau_v_hat) = tau_v (m - 1) when c = m
    assert abs(acc[v] / R - tau_v[v]) < 4 * sd


def test_threaded_processor_ranges_partition_the_replay():
    """Replaying disjoint processor ranges and summing gives the full replay (processors are
    independent trials, Section III-A); a range leaves the other processors' counters at 0."""
    e = synth.er(60, 400, 71, 72)
    g, l = oracle.rept(e, 60, 3, 7, 99, per_proc=True)
    parts = [oracle.rept_threads(e, 60, 3, 7, 99, per_proc=True, workers=2, procs=r) for r in [(0, 2), (2, 5), (5, 7)]]
    assert np.array_equal(sum(p[0] for p in parts), g) and np.array_equal(sum(p[1] for p in parts), l)
    g02, l02 = parts[0]
    assert not g02[2:].any() and not l02[2:].any()


@pytest.mark.parametrize("m,c,per_proc,window", [(10, 10, False, None), (3, 7, True, None), (4, 13, False, (300, 1700)),
                                                 (1, 1, False, None), (5, 3, True, (0, 900)), (2, 9, False, None)])
def test_threaded_replay_equals_serial(m, c, per_proc, window):
    """The threaded replay (stream validated and hashed once, processors spread over threads,
    private group rows added at the end) equals the single-threaded replay at every thread
    count, for group sums, processor rows and windows."""
    e = synth.er(300, 2500, 81, 82)
    kw = {} if window is None else dict(t0=window[0], t1=window[1])
    g, l = oracle.rept(e, 300, m, c, 123, per_proc=per_proc, **kw)
    for workers in (1, 2, 3, 8, 64):
        gt, lt = oracle.rept_threads(e, 300, m, c, 123, per_proc=per_proc, workers=workers, **kw)
        assert np.array_equal(gt, g) and np.array_equal(lt, l), workers


def test_hash_four_wise_collision_rate_over_seeds():
    """Theorem 3's variance needs the slots of any four distinct edges to be independent
    (zero covariance between semi-triangles on disjoint edge pairs).  For FIXED quadruples of
    structured edges -- consecutive keys and a shared endpoint, where weak families fail --
    over many independent hash functions (one per group): three edges share a slot with
    probability 1/m^2, and given that, the fourth joins them with probability 1/m.  A
    polynomial of degree < 3 fixes the fourth value of consecutive keys by the first three,
    which roughly triples that conditional rate at m = 16."""
    m, G = 16, 200_000
    quads = [np.array([[0, 1], [0, 2], [0, 3], [0, 4]], dtype=np.uint32),        # shared endpoint
             np.array([[5, 9], [5, 10], [5, 11], [5, 12]], dtype=np.uint32),     # consecutive keys
             np.array([[1, 2], [3, 4], [5, 6], [7, 8]], dtype=np.uint32)]        # disjoint edges
    for q in quads:
        s = oracle.slots(q, m, G, 4242).astype(np.int64)  # [G][4]: one hash function per row
        three = (s[:, 1] == s[:, 0]) & (s[:, 2] == s[:, 0])
        r3 = three.mean()
        assert abs(r3 - 1 / m**2) < 4.5 * math.sqrt((1 / m**2) * (1 - 1 / m**2) / G), (q, r3)
        cond = (s[three, 3] == s[three, 0]).mean()
        k = int(three.sum())
        assert abs(cond - 1 / m) < 4.5 * math.sqrt((1 / m) * (1 - 1 / m) / k), (q, cond, k)


# ---------------------------------------------------------------- Algorithm 2 (c2 != 0) ----

def _semi_sets(edges, n, m, c, seed):
    """Per processor i: its semi-triangles as ((a, b, w), (t_ab, t_aw, t_bw)), by definition
    (the first two edges by time hash to i), enumerated from the graph's triangles."""
    G = -(-c // m)
    sl = oracle.slots(edges, m, G, seed)
    out = [[] for _ in range(c)]
    for tri, ts in brute.triangles(edges, n):
        first = sorted(ts)[:2]
        for k in range(G):
            ck = m if k + 1 < G else c - (G - 1) * m
            if sl[k, first[0]] == sl[k, first[1]] and sl[k, first[0]] < ck:
                out[k * m + int(sl[k, first[0]])].append((tri, ts))
    return out


def _eta_by_enumeration(edges, n, m, c, seed):
    """(eta_def[c], eta_lit[c], eta_v_def[n], eta_v_lit[n]) from the semi-triangle sets.
    Definition: unordered pairs of distinct semi-triangles of one processor sharing an edge that
    is the last edge of neither.  Literal (counter set to |N| on insert): each edge g adds
    s_g L_g + C(s_g, 2), with s_g the processor's semi-triangles having g as a non-last edge and
    L_g those having g as the last edge; eta_v adds the same over the edges g containing v."""
    sets = _semi_sets(edges, n, m, c, seed)
    ed, el = np.zeros(c, np.int64), np.zeros(c, np.int64)
    vd, vl = np.zeros(n, np.int64), np.zeros(n, np.int64)
    for i, S in enumerate(sets):
        s, L = {}, {}
        for (a, b, w), (tab, taw, tbw) in S:
            last = max(tab, taw, tbw)
            for (x, y), t in (((a, b), tab), ((a, w), taw), ((b, w), tbw)):
                d = L if t == last else s
                d[(x, y)] = d.get((x, y), 0) + 1
        # the definition, pair by pair
        for p, q in itertools.combinations(range(len(S)), 2):
            (A, ta), (B, tb) = S[p], S[q]
            ea = {frozenset(e): t for e, t in zip(((A[0], A[1]), (A[0], A[2]), (A[1], A[2])), ta)}
            eb = {frozenset(e): t for e, t in zip(((B[0], B[1]), (B[0], B[2]), (B[1], B[2])), tb)}
            for g in set(ea) & set(eb):
                if ea[g] != max(ta) and eb[g] != max(tb):
                    ed[i] += 1
                    for v in set(A) & set(B):
                        vd[v] += 1
        for g, sg in s.items():
            f = sg * L.get(g, 0) + sg * (sg - 1) // 2
            el[i] += f
            vl[g[0]] += f
            vl[g[1]] += f
    return ed, el, vd, vl


def test_alg2_counters_hand_streams():
    """Two triangles {0,1,2}, {0,1,3} sharing {0,1}, one processor (m = c = 1).  When {0,1}
    arrives first it is a non-last edge of both: eta = 1 under both readings.  When it closes
    the first triangle, the definition excludes the pair (eta = 0) but a counter set to |N| = 1
    on insert counts it (literal eta = 1, added at nodes 0 and 1)."""
    e = np.array([[0, 1], [0, 2], [1, 2], [0, 3], [1, 3]], np.uint32)
    ed, el, vd, vl = oracle.rept2_eta(e, 4, 1, 1, 0)
    assert ed.tolist() == [1] and el.tolist() == [1] and vd.tolist() == [1, 1, 0, 0] == vl.tolist()
    e = np.array([[0, 2], [1, 2], [0, 1], [0, 3], [1, 3]], np.uint32)
    ed, el, vd, vl = oracle.rept2_eta(e, 4, 1, 1, 0)
    assert ed.tolist() == [0] and el.tolist() == [1] and vd.tolist() == [0, 0, 0, 0] and vl.tolist() == [1, 1, 0, 0]


@pytest.mark.parametrize("m,c,seed", [(2, 3, 1), (3, 7, 2), (2, 5, 3), (4, 6, 4)])
def test_alg2_counters_match_enumeration(m, c, seed):
    e = synth.er(40, 260, 30 + seed, 40 + seed)
    got = oracle.rept2_eta(e, 40, m, c, seed)
    want = _eta_by_enumeration(e, 40, m, c, seed)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    assert want[0].sum() > 0 and (want[1] >= want[0]).all()


def test_alg2_counters_one_processor_equal_graph_eta():
    """m = c = 1: every triangle is on the one processor, so its definition counter is the
    graph's eta (and eta_v), enumerated independently."""
    e = synth.er(30, 150, 7, 8)
    ed, _, vd, _ = oracle.rept2_eta(e, 30, 1, 1, 0)
    assert ed[0] == brute.eta(e, 30) > 0
    assert all(vd[v] == brute.eta(e, 30, node=v) for v in range(30))


def test_alg2_eta_estimate_unbiased_over_seeds():
    """E(eta^(i)) = eta / m^3 for the definition counter (Section III-B), so the mean over hash
    seeds of m^3 sum_i eta^(i) / c approaches eta; checked at 5 standard errors."""
    e = synth.er(45, 420, 11, 12)
    truth = brute.eta(e, 45)
    m, c = 2, 5
    est = [2 ** 3 * oracle.rept2_eta(e, 45, m, c, s)[0].sum() / c for s in range(400)]
    se = np.std(est) / np.sqrt(len(est))
    assert truth > 0 and abs(np.mean(est) - truth) < 5 * se


def test_alg2_estimator_hand_value_and_limits():
    """m = 2, c = 3 (c1 = c2 = 1), S1 = 8, S2 = 7, eta = 4: t1 = 16, t2 = 28, eh = 32/3,
    v1 = 16, v2 = 48 + 64/3 = 208/3, tau_hat = (208/3 * 16 + 16 * 28) / (16 + 208/3) = 18.25
    exactly in rationals.  Both variances zero: t1 (Q12).  The result is a weighted mean."""
    th, tv = oracle.estimate2(2, 2, 3, [3, 5, 7], [[1, 2], [3, 4]], 4, [1, 1])
    # local v = 1: S1_v = 2, S2_v = 4, eta_v = 1 -> 6.25 in rationals; eta_v m^3 / c = 8/3 is
    # rounded once, so the binary64 result is within a few ulps of it (bound 4 ulps)
    assert th == 18.25 and tv[0] == 3.5 and abs(tv[1] - 6.25) <= 4 * np.spacing(6.25)
    th, _ = oracle.estimate2(1, 2, 3, [0, 0, 9], None, 0, None)
    assert th == 0.0
    rng = np.random.default_rng(3)
    for _ in range(200):
        m = int(rng.integers(2, 9)); c = m * int(rng.integers(1, 4)) + int(rng.integers(1, m))
        g = rng.integers(0, 10**6, size=c)
        th, _ = oracle.estimate2(1, m, c, g, None, int(rng.integers(0, 10**7)), None)
        c1 = c // m
        t1 = g[: c1 * m].sum() * m / c1
        t2 = g[c1 * m:].sum() * m * m / (c % m)
        assert min(t1, t2) * (1 - 1e-12) <= th <= max(t1, t2) * (1 + 1e-12)
    with pytest.raises(oracle.OracleError):
        oracle.estimate2(1, 2, 4, [1, 1, 1, 1], None, 0, None)


def test_alg2_estimator_unbiased_over_seeds():
    """Both parts are unbiased (Section III-B), so the combined global estimate averaged over
    hash seeds approaches the exact triangle count."""
    e = synth.er(60, 700, 21, 22)
    tau, _ = brute.exact_counts(e, 60)
    m, c = 3, 7
    est = []
    for s in range(300):
        g, loc = oracle.rept(e, 60, m, c, s)
        eta = int(oracle.rept2_eta(e, 60, m, c, s)[0].sum())
        est.append(oracle.estimate2(60, m, c, g, None, eta, None)[0])
    se = np.std(est) / np.sqrt(len(est))
    assert tau > 0 and abs(np.mean(est) - tau) < 5 * se


# ------------------------------------------------------------------ parallel MASCOT -------

def test_mascot_one_is_exact():
    """m = 1 (p = 1): every processor keeps every edge, so each processor's counters are the
    exact triangle counts (the adjacency-matrix identity, not an enumeration)."""
    e = synth.er(40, 300, 51, 52)
    tau, tau_v = brute.exact_counts(e, 40)
    g, l = oracle.mascot(e, 40, 1, 3, 9)
    assert tau > 0 and g.tolist() == [tau] * 3
    for i in range(3):
        assert np.array_equal(l[i], tau_v)


@pytest.mark.parametrize("m,c,seed", [(2, 3, 1), (3, 5, 2), (4, 2, 3)])
def test_mascot_counts_semi_triangles_of_independent_samples(m, c, seed):
    """Processor i counts exactly the triangles whose first two edges it sampled (h_i = 0),
    found by enumerating the graph's triangles and testing the hash (a different route from
    the stream replay); its locals add the triangle to its three nodes."""
    e = synth.er(40, 260, 60 + seed, 61 + seed)
    g, l = oracle.mascot(e, 40, m, c, seed)
    sl = oracle.slots(e, m, c, seed)  # group i's hash = processor i's coin
    want_g = np.zeros(c, np.int64)
    want_l = np.zeros((c, 40), np.int64)
    for tri, ts in brute.triangles(e, 40):
        t1, t2 = sorted(ts)[:2]
        for i in range(c):
            if sl[i, t1] == 0 and sl[i, t2] == 0:
                want_g[i] += 1
                for x in tri:
                    want_l[i, x] += 1
    assert np.array_equal(g, want_g) and np.array_equal(l, want_l) and want_g.sum() > 0
    # processors are independent samplers: processor 0 equals REPT with one processor
    g1, l1 = oracle.rept(e, 40, m, 1, seed)
    assert g[0] == g1[0] and np.array_equal(l[0], l1[0])


def test_mascot_estimator_unbiased_with_paper_variance():
    """Section III-C: the mean of c independent MASCOT estimates is unbiased with variance
    (tau (m^2 - 1) + 2 eta (m - 1)) / c, checked over hash seeds; on this graph it is several
    times REPT's tau (m - 1) / c1 at c = m (the comparison the paper draws)."""
    n = 30
    e = synth.shuffled(synth.er(n, 160, 41, 42), 43)
    tau, _ = brute.exact_counts(e, n)
    eta = brute.eta(e, n)
    m, c, R = 3, 3, 1500
    var = (tau * (m * m - 1) + 2 * eta * (m - 1)) / c
    seeds = synth.u64(8, 31, R)
    est = np.empty(R)
    for r in range(R):
        g, _ = oracle.mascot(e, n, m, c, int(seeds[r]))
        est[r] = oracle.estimate_mascot(n, m, c, g)[0]
    assert abs(est.mean() - tau) < 4.0 * math.sqrt(var / R)
    ratio = est.var(ddof=1) / var
    assert 0.8 < ratio < 1.25, (ratio, tau, eta)
    assert var > 2 * tau * (m - 1)


def test_mascot_estimator_values():
    """(S m^2) / c with one rounding each: hand values, exact cases, and ERANGE."""
    th, tv = oracle.estimate_mascot(2, 3, 4, [1, 2, 3, 4], [[1, 0], [0, 0], [2, 0], [0, 1]])
    assert th == 22.5 and tv.tolist() == [6.75, 2.25]
    th, _ = oracle.estimate_mascot(1, 10, 7, [3] * 7)
    assert th == (21.0 * 100.0) / 7.0
    with pytest.raises(oracle.OracleError):
        oracle.estimate_mascot(1, 2, 2, [2**52, 2**52])
    with pytest.raises(oracle.OracleError):
        oracle.estimate_mascot(1, 2, 1, [1], [[-1]])
