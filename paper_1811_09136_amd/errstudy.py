"""Error studies on the device: NRMSE of REPT and parallel MASCOT over hash-seed replicas of
one stream, against the variances the paper derives (the analogue of its accuracy figures,
Section IV, on synthetic graphs).

- Exact statistics of a graph come from one counting pass with p = 1 (m = c = 1): the one
  processor stores every edge, so its counters are the exact triangle counts tau, tau_v, and
  its Algorithm 2 pair counter (definition reading) is the exact eta, eta_v (the Section I
  figure comparing eta with tau).
- Replicas differ only in the hash seed.  REPT replicas with c <= m or m | c run as one batched
  launch; c mod m != 0 runs rept_count_eta per replica for the combined estimator; parallel
  MASCOT runs in passes of at most 8 processors per launch, each pass with its own seed.
- NRMSE = sqrt(mean((est - truth)^2)) / truth (Section IV-B).  For local counts the paper does
  not state how nodes are combined; here it is the mean over nodes with tau_v > 0 of each
  node's NRMSE.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import rept


# ------------------------------------------------------------------ variances (the paper's) --

def variance_rept(tau: float, eta: float, m: int, c: int) -> float:
    """Var of REPT's estimate: Theorem 3 for c <= m, tau (m - 1) / c1 for c = c1 m
    (Section III-B), and for c2 = c mod m != 0 the variance of the inverse-variance combination
    of the two parts, V1 V2 / (V1 + V2) (Section III-B), with V1 = tau (m - 1) / c1 and V2
    Theorem 3's form on the c2 processors of the last group."""
    if c <= m:
        return (tau * (m * m - c) + 2.0 * eta * (m - c)) / c
    c1, c2 = divmod(c, m)
    v1 = tau * (m - 1) / c1
    if c2 == 0:
        return v1
    v2 = (tau * (m * m - c2) + 2.0 * eta * (m - c2)) / c2
    return 0.0 if v1 + v2 == 0 else v1 * v2 / (v1 + v2)


def variance_mascot(tau: float, eta: float, m: int, c: int) -> float:
    """Var of the mean of c independent MASCOT estimates with p = 1/m (Section III-C)."""
    return (tau * (m * m - 1) + 2.0 * eta * (m - 1)) / c


# ------------------------------------------------------------------ exact statistics --------

@dataclass
class Exact:
    tau: int
    eta: int
    tau_v: np.ndarray  # int64[n]
    eta_v: np.ndarray  # int64[n]


def exact_stats(graph: "rept.Graph", stream=None) -> Exact:
    """tau, eta and their per-node forms from one pass with every edge stored (m = c = 1)."""
    import torch
    g, loc, eta, eta_v = graph.count_eta(rept.Params(1, 1, 0), stream=stream)
    torch.cuda.synchronize()
    return Exact(int(g[0].item()), int(eta[0, 0].item()), loc[0].cpu().numpy(), eta_v[0].cpu().numpy())


# ------------------------------------------------------------------ replicas ----------------

def replica_seeds(seed: int, R: int) -> list[int]:
    return [int(x) for x in np.random.SeedSequence(seed).generate_state(R, np.uint64)]


def _batched_counts(graph, params_list, stream=None):
    """Counts of one graph under several parameter sets in one persistent launch."""
    import torch
    from .batch import Batch, Job
    jobs = [Job(graph, p) for p in params_list]
    Batch(jobs, stream=stream).launch(stream)
    torch.cuda.synchronize()
    return [(j.out[0].cpu().numpy(), j.out[1].cpu().numpy()) for j in jobs]


def replicate_rept(graph, m: int, c: int, seeds: list[int], with_local: bool = True, chunk: int = 64):
    """REPT estimates over the seeds: (tau_hat[R], tau_v_hat[R, n] or None)."""
    n = graph.n
    R = len(seeds)
    est = np.empty(R)
    loc_est = np.empty((R, n)) if with_local else None
    c1, c2 = divmod(c, m)
    if c > m and c2 != 0:
        for r, s in enumerate(seeds):
            p = rept.Params(m, c, s)
            g, l, eta, eta_v = graph.count_eta(p, with_nodes=with_local)
            import torch
            torch.cuda.synchronize()
            gh, lh = g.cpu().numpy(), l.cpu().numpy()
            ev = eta_v[0].cpu().numpy() if with_local else None
            th, tv = rept.rept_estimate_combined(n, p, gh, lh if with_local else None, int(eta[0].sum().item()), ev)
            est[r] = th
            if with_local:
                loc_est[r] = tv
        return est, loc_est
    for r0 in range(0, R, chunk):
        ps = [rept.Params(m, c, s) for s in seeds[r0:r0 + chunk]]
        for k, (gh, lh) in enumerate(_batched_counts(graph, ps)):
            th, tv = rept.rept_estimate(n, ps[k], gh, lh if with_local else None)
            est[r0 + k] = th
            if with_local:
                loc_est[r0 + k] = tv
    return est, loc_est


def replicate_mascot(graph, m: int, c: int, seeds: list[int], with_local: bool = True, chunk: int = 64):
    """Parallel MASCOT estimates over the seeds: c processors in passes of at most 8 (pass q of
    replica r hashes with its own seed), pooled as (m^2 / c) sum_i tau^(i)."""
    n = graph.n
    R = len(seeds)
    passes = [min(8, c - q) for q in range(0, c, 8)]
    S = np.zeros(R, dtype=np.int64)
    Sv = np.zeros((R, n), dtype=np.int64) if with_local else None
    work = [(r, q, cq) for r in range(R) for q, cq in enumerate(passes)]
    for w0 in range(0, len(work), chunk):
        part = work[w0:w0 + chunk]
        ps = [rept.Params(m, cq, replica_seeds(seeds[r], q + 1)[q], mascot=True) for r, q, cq in part]
        for (r, _, _), (gh, lh) in zip(part, _batched_counts(graph, ps)):
            S[r] += int(gh.sum())
            if with_local:
                Sv[r] += lh.sum(axis=0)
    num, den = float(m * m), float(c)
    est = (S.astype(np.float64) * num) / den
    loc_est = (Sv.astype(np.float64) * num) / den if with_local else None
    return est, loc_est


# ------------------------------------------------------------------ the study ---------------

def nrmse(est: np.ndarray, truth: float) -> float:
    return float(np.sqrt(np.mean((np.asarray(est) - truth) ** 2)) / truth)


def study(graph, m: int, cs, R: int, seed: int = 1, methods=("rept", "mascot"), with_local: bool = True,
          exact: Exact | None = None) -> list[dict]:
    """One row per (method, c): empirical NRMSE of the global and local estimates over R
    replicas next to the NRMSE the paper's variance gives."""
    ex = exact or exact_stats(graph)
    if ex.tau == 0:
        raise ValueError("the graph has no triangles")
    seeds = replica_seeds(seed, R)
    tv = ex.tau_v
    nodes = np.nonzero(tv > 0)[0]
    rows = []
    for method in methods:
        for c in cs:
            if method == "rept":
                est, lest = replicate_rept(graph, m, c, seeds, with_local)
                var = variance_rept(ex.tau, ex.eta, m, c)
                var_v = np.array([variance_rept(tv[v], ex.eta_v[v], m, c) for v in nodes])
            else:
                est, lest = replicate_mascot(graph, m, c, seeds, with_local)
                var = variance_mascot(ex.tau, ex.eta, m, c)
                var_v = variance_mascot(tv[nodes].astype(float), ex.eta_v[nodes].astype(float), m, c)
            row = {"method": method, "m": m, "c": c, "R": R, "tau": ex.tau, "eta": ex.eta,
                   "mean_tau_hat": float(est.mean()), "nrmse_global": nrmse(est, ex.tau),
                   "nrmse_global_theory": math.sqrt(var) / ex.tau,
                   "var_ratio": float(np.mean((est - ex.tau) ** 2) / var) if var > 0 else None}
            if with_local and len(nodes):
                per = np.sqrt(np.mean((lest[:, nodes] - tv[nodes]) ** 2, axis=0)) / tv[nodes]
                row["nrmse_local_mean"] = float(per.mean())
                row["nrmse_local_theory_mean"] = float((np.sqrt(var_v) / tv[nodes]).mean())
            rows.append(row)
    return rows


def main(argv=None):
    """python -m paper_1811_09136_amd.errstudy: REPT vs parallel MASCOT on a seeded Chung-Lu
    stream, one JSON row per (method, c)."""
    import argparse
    import json
    import os
    import sys
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--edges", type=int, default=200_000)
    ap.add_argument("--m", type=int, default=10)
    ap.add_argument("--cs", default="5,10,15,20,40")
    ap.add_argument("--replicas", type=int, default=200)
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth  # seeded input generator
    e, n = synth.scaled_chung_lu(args.edges, args.seed)
    g = rept.Graph(rept.to_device_edges(e, torch.device("cuda:0")), n)
    ex = exact_stats(g)
    print(json.dumps({"graph": f"Chung-Lu gamma 2.1, {len(e)} edges, {n} nodes", "tau": ex.tau, "eta": ex.eta,
                      "eta_over_tau": ex.eta / max(ex.tau, 1)}), flush=True)
    for row in study(g, args.m, [int(x) for x in args.cs.split(",")], args.replicas, args.seed, exact=ex):
        print(json.dumps(row), flush=True)
    g.close()


if __name__ == "__main__":
    main()
