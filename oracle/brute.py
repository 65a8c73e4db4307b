"""Definition-level enumerators (test infrastructure only; small inputs).

These restate what REPT counts without replaying the stream:

* ``triangles`` lists every triangle of the stream graph G (Section II) by brute force over
  vertex triples, with the arrival times of its three edges.
* ``semi_triangle_counts`` attributes each triangle to processors by the paper's definition of
  a semi-triangle (Section III, and Theorem 2): a triangle counts on processor i exactly when
  its first two edges on the stream are both stored by processor i, whatever happens to its
  last edge.  Each counted triangle adds one to tau^(i) and one to tau_x^(i) of each of its
  three vertices.
* ``eta`` counts the pairs of distinct triangles that share an edge which is the last edge of
  neither (Table I, Theorem 3), used by the variance pins.

Pure Python / numpy, written for inputs of a few hundred edges at most.
"""
from __future__ import annotations

import numpy as np


def edge_times(edges) -> dict:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return {frozenset((int(u), int(v))): t for t, (u, v) in enumerate(e)}


def triangles(edges, n: int):
    """[(a, b, w), (t_ab, t_aw, t_bw)] for every triangle a < b < w of the graph."""
    times = edge_times(edges)
    adj = [set() for _ in range(n)]
    for key in times:
        u, v = tuple(key)
        adj[u].add(v)
        adj[v].add(u)
    out = []
    for a in range(n):
        for b in sorted(x for x in adj[a] if x > a):
            for w in sorted(x for x in adj[a] & adj[b] if x > b):
                out.append(((a, b, w), (times[frozenset((a, b))], times[frozenset((a, w))],
                                        times[frozenset((b, w))])))
    return out


def semi_triangle_counts(edges, n: int, m: int, c: int, slot_of, per_proc: bool = False):
    """tau^(i) and local counts by the semi-triangle definition.

    slot_of(k, t) -> slot of stream edge t under group k's hash.
    """
    G = -(-c // m)
    glob = np.zeros(c, dtype=np.int64)
    loc = np.zeros((c if per_proc else G, n), dtype=np.int64)
    for (a, b, w), (tab, taw, tbw) in triangles(edges, n):
        first_two = sorted([tab, taw, tbw])[:2]
        for k in range(G):
            ck = m if k + 1 < G else c - (G - 1) * m
            s1, s2 = slot_of(k, first_two[0]), slot_of(k, first_two[1])
            if s1 == s2 and s1 < ck:
                i = k * m + s1
                glob[i] += 1
                row = i if per_proc else k
                for x in (a, b, w):
                    loc[row, x] += 1
    return glob, loc


def exact_counts(edges, n: int):
    """Exact triangle count and per-node counts by the adjacency matrix: tau = trace(A^3)/6 and
    tau_v = (A^3)_vv / 2 (a textbook identity, independent of any enumeration above)."""
    A = np.zeros((n, n), dtype=np.float64)
    for u, v in np.asarray(edges, dtype=np.int64).reshape(-1, 2):
        A[u, v] = A[v, u] = 1.0
    # (A^3)_vv = 2 tau_v; every entry is an integer below n^2, exact in binary64
    d = np.rint(np.einsum("ij,ji->i", A @ A, A)).astype(np.int64)
    return int(d.sum() // 6), d // 2


def eta(edges, n: int, node: int | None = None) -> int:
    """Pairs of distinct triangles sharing an edge g that is the last edge of neither.

    With node given: only pairs of triangles that both contain that node (eta_v)."""
    tris = triangles(edges, n)
    times = edge_times(edges)
    by_edge = {}
    for (a, b, w), ts in tris:
        last = max(ts)
        for x, y in ((a, b), (a, w), (b, w)):
            g = frozenset((x, y))
            if times[g] != last:  # g is not the last edge of this triangle
                by_edge.setdefault(g, []).append((a, b, w))
    total = 0
    for g, lst in by_edge.items():
        if node is not None:
            lst = [t for t in lst if node in t]
        total += len(lst) * (len(lst) - 1) // 2
    return total


def wedge_count(edges, n: int) -> int:
    d = np.bincount(np.asarray(edges, dtype=np.int64).ravel(), minlength=n)
    return int((d * (d - 1) // 2).sum())

