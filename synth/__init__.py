"""Seeded synthetic edge streams shared by the oracle tests, the device tests and the bench.

This module generates inputs only; it contains no part of the counting method.  Streams are
``numpy.uint32`` arrays of shape ``[E, 2]`` holding undirected simple edges (no self-loops, no
repeated unordered pair); the stream position ``t`` of an edge is its row index, matching the
problem statement of the paper (Section II: the t-th edge of the stream).

The heavy generators live in ``csrc/synth.c`` (counter-based randomness, OpenMP), compiled to
``libsynth.so`` beside it by :func:`build`.
"""
from __future__ import annotations

import ctypes
import functools
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.synth_er.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u32p]
        lib.synth_er.restype = ctypes.c_int
        lib.synth_chung_lu.argtypes = [ctypes.c_uint32, ctypes.c_uint64, f64p, ctypes.c_uint64,
                                       ctypes.c_uint64, u32p]
        lib.synth_chung_lu.restype = ctypes.c_int
        lib.synth_rmat.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_uint64, u32p]
        lib.synth_rmat.restype = ctypes.c_int64
        lib.synth_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, f64p]
        lib.synth_uniform.restype = None
        lib.synth_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.POINTER(ctypes.c_uint64)]
        lib.synth_u64.restype = None
        _lib = lib
    return _lib


def _u32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


# ----------------------------------------------------------------------------- basic streams

def er(n: int, m_edges: int, seed: int, order_seed: int) -> np.ndarray:
    """Erdos-Renyi G(n, M): M distinct uniform pairs, stream order shuffled by ``order_seed``."""
    out = np.empty((m_edges, 2), dtype=np.uint32)
    rc = _load().synth_er(n, m_edges, seed & (2**64 - 1), order_seed & (2**64 - 1), _u32p(out))
    if rc != 0:
        raise ValueError(f"synth_er failed ({rc})")
    return out


def chung_lu_weights(n: int, num_edges: int, gamma: float, w_max: float) -> np.ndarray:
    """Power-law expected degrees ``w_i = beta * (i + i0) ** (-1/(gamma-1))``.

    ``i0`` is solved by bisection so that the largest weight is ``w_max`` when the weights sum
    to ``2 * num_edges``; ``beta`` then fixes the sum.
    """
    alpha = 1.0 / (gamma - 1.0)
    idx = np.arange(n, dtype=np.float64)
    target = w_max / (2.0 * num_edges)

    def share(i0):
        w = (idx + i0) ** (-alpha)
        return w[0] / w.sum()

    lo, hi = 1e-9, float(n)
    if share(lo) < target:  # even the steepest profile cannot reach w_max: use it as is
        i0 = lo
    else:
        for _ in range(200):
            mid = math.sqrt(lo * hi) if lo > 0 else hi / 2
            if share(mid) > target:
                lo = mid
            else:
                hi = mid
        i0 = math.sqrt(lo * hi)
    w = (idx + i0) ** (-alpha)
    return w * (2.0 * num_edges / w.sum())


def chung_lu(n: int, num_edges: int, gamma: float, w_max: float, seed: int, order_seed: int) -> np.ndarray:
    """Chung-Lu power-law stream: endpoints proportional to the weights, simple, shuffled."""
    w = chung_lu_weights(n, num_edges, gamma, w_max)
    cum = np.zeros(n + 1, dtype=np.float64)
    np.cumsum(w, out=cum[1:])
    out = np.empty((num_edges, 2), dtype=np.uint32)
    rc = _load().synth_chung_lu(n, num_edges, cum.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                seed & (2**64 - 1), order_seed & (2**64 - 1), _u32p(out))
    if rc != 0:
        raise ValueError(f"synth_chung_lu failed ({rc})")
    return out


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int) -> np.ndarray:
    """R-MAT draws, self-loops dropped, first occurrence of each pair kept, generation order."""
    draws = (1 << scale) * edge_factor
    buf = np.empty((draws, 2), dtype=np.uint32)
    kept = _load().synth_rmat(scale, edge_factor, a, b, c, seed & (2**64 - 1), _u32p(buf))
    if kept < 0:
        raise ValueError(f"synth_rmat failed ({kept})")
    return np.ascontiguousarray(buf[:kept])


def uniform(seed: int, stream: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().synth_uniform(seed & (2**64 - 1), stream, count,
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def u64(seed: int, stream: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().synth_u64(seed & (2**64 - 1), stream, count,
                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def shuffled(edges: np.ndarray, order_seed: int, flip_seed: int | None = None) -> np.ndarray:
    """Return ``edges`` in a seeded random stream order (optionally with random orientation)."""
    e = np.asarray(edges, dtype=np.uint32).reshape(-1, 2)
    r = uniform(order_seed, 11, len(e))
    out = np.ascontiguousarray(e[np.argsort(r, kind="stable")])
    if flip_seed is not None:
        f = uniform(flip_seed, 12, len(out)) < 0.5
        out[f] = out[f][:, ::-1]
    return out


# ----------------------------------------------------------------------------- small shapes

def complete(n: int) -> np.ndarray:
    iu = np.triu_indices(n, 1)
    return np.stack(iu, axis=1).astype(np.uint32)


def cycle(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.uint32)
    return np.stack([i, (i + 1) % n], axis=1).astype(np.uint32)


def wheel(n_rim: int) -> np.ndarray:
    """Hub 0 joined to every vertex of the cycle 1..n_rim."""
    rim = cycle(n_rim) + 1
    spokes = np.stack([np.zeros(n_rim, np.uint32), np.arange(1, n_rim + 1, dtype=np.uint32)], axis=1)
    return np.concatenate([rim, spokes]).astype(np.uint32)


def friendship(k: int) -> np.ndarray:
    """k triangles sharing the centre 0: (0, 2i+1), (0, 2i+2), (2i+1, 2i+2)."""
    rows = []
    for i in range(k):
        a, b = 2 * i + 1, 2 * i + 2
        rows += [(0, a), (0, b), (a, b)]
    return np.array(rows, dtype=np.uint32).reshape(-1, 2)


def complete_bipartite(a: int, b: int) -> np.ndarray:
    left = np.repeat(np.arange(a, dtype=np.uint32), b)
    right = np.tile(np.arange(a, a + b, dtype=np.uint32), a)
    return np.stack([left, right], axis=1)


# ----------------------------------------------------------------------------- workloads

CONFIG1 = dict(kind="er", n=2000, E=20000, m=10, c=10)
CONFIG2 = dict(kind="chung_lu", n=1_000_000, E=20_000_000, gamma=2.1, w_max=5.0e4, m=10, c=40)
CONFIG3 = dict(kind="rmat", scale=24, edge_factor=16, a=0.57, b=0.19, c_=0.19, m=100, c=100)


@functools.lru_cache(maxsize=4)
def config1_stream(seed: int = 1) -> np.ndarray:
    """Erdos-Renyi, 2,000 nodes, 20,000 edges, uniformly shuffled stream order."""
    return er(2000, 20000, seed, seed + 1000)


@functools.lru_cache(maxsize=2)
def config2_stream(seed: int = 2) -> np.ndarray:
    """Chung-Lu power law, 1M nodes, 20M edges, exponent 2.1, max expected degree 5e4, shuffled."""
    return chung_lu(1_000_000, 20_000_000, 2.1, 5.0e4, seed, seed + 1000)


@functools.lru_cache(maxsize=1)
def config3_stream(seed: int = 3) -> np.ndarray:
    """R-MAT scale 24, edge factor 16, (0.57, 0.19, 0.19), deduplicated, generation order."""
    return rmat(24, 16, 0.57, 0.19, 0.19, seed)


def scaled_chung_lu(num_edges: int, seed: int, avg_degree: int = 40, gamma: float = 2.1) -> np.ndarray:
    """A smaller stream with the shape of the 1M/20M power-law workload (n = E / 20)."""
    n = max(8, -(-2 * num_edges // avg_degree))
    w_max = min(5.0e4, n / 2)
    return chung_lu(n, num_edges, gamma, w_max, seed, seed + 1000), n


def batch_jobs(seed: int = 4, n_streams: int = 256, n_replicas: int = 256,
               e_min: float = 1e4, e_max: float = 2e6, replica_edges: int = 5_000_000,
               replica_nodes: int = 250_000):
    """The batched workload: independent Chung-Lu streams with log-uniform sizes plus hash-seed
    replicas of one fixed power-law stream.  Returns (streams, replica_stream, replica_seeds)
    where ``streams`` is a list of (edges, n) and ``replica_seeds`` are per-replica hash seeds."""
    u = uniform(seed, 21, n_streams)
    sizes = np.exp(np.log(e_min) + u * (np.log(e_max) - np.log(e_min))).astype(np.int64)
    job_seeds = u64(seed, 22, n_streams)
    streams = []
    for j in range(n_streams):
        e = int(sizes[j])
        n = -(-e // 20)
        w_max = min(5.0e4, n / 2)
        streams.append((chung_lu(n, e, 2.1, w_max, int(job_seeds[j]), int(job_seeds[j]) + 1), n))
    rep = chung_lu(replica_nodes, replica_edges, 2.1, min(5.0e4, replica_nodes / 2), seed + 7, seed + 8) \
        if n_replicas else None
    rep_seeds = u64(seed, 23, n_replicas)
    return streams, (rep, replica_nodes), rep_seeds


def serving_trace(seed: int = 5, n_requests: int = 64, rate_per_s: float = 10.0,
                  median_edges: float = 2e5, sigma: float = 1.0, e_lo: float = 1e3, e_hi: float = 2e7):
    """Poisson arrivals with lognormal stream sizes, m in {10, 50, 100}, c in {m, 4m}.

    Returns a list of dicts {arrival_s, E, n, m, c, graph_seed, hash_seed}.
    """
    u_gap = uniform(seed, 31, n_requests)
    u1 = uniform(seed, 32, n_requests)
    u2 = uniform(seed, 33, n_requests)
    u_m = uniform(seed, 34, n_requests)
    u_c = uniform(seed, 35, n_requests)
    seeds = u64(seed, 36, 2 * n_requests)
    gaps = -np.log1p(-u_gap) / rate_per_s
    arrivals = np.cumsum(gaps)
    # Box-Muller normal from two uniforms
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    sizes = np.clip(np.exp(np.log(median_edges) + sigma * z), e_lo, e_hi).astype(np.int64)
    out = []
    for i in range(n_requests):
        m = (10, 50, 100)[min(2, int(u_m[i] * 3))]
        c = m if u_c[i] < 0.5 else 4 * m
        e = int(sizes[i])
        out.append(dict(arrival_s=float(arrivals[i]), E=e, n=-(-e // 20), m=m, c=c,
                        graph_seed=int(seeds[2 * i]), hash_seed=int(seeds[2 * i + 1])))
    return out
