"""CPU oracle for REPT (arXiv:1811.09136) -- TEST INFRASTRUCTURE ONLY.

The oracle is the plain, slow statement of what the device path computes; only ``tests/``,
``__graft_entry__.smoke()`` and the bench's CPU-baseline leg may call it.  It shares no code
with the device library (``paper_1811_09136_amd``) and never imports it.

* ``rept``          -- Algorithm 1 replayed literally per processor (Section III-A), with the
                       c > m grouping of Section III-B; optional window [t0, t1) of updates.
* ``edge_updates``  -- the per-edge update of Algorithm 1 evaluated from its definition for a
                       list of stream positions (for sampled checks on large streams).
* ``estimate``      -- the estimators of Section III-A / III-B (c <= m, or m divides c).
* ``hash_params`` / ``slots`` -- the edge-to-processor hash (SplitMix64-seeded, 4-independent
                       polynomial over GF(2^61 - 1)).
* ``brute``         -- a definition-level enumerator (module ``oracle.brute``).

Parity pins for every function are in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rept_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ERANGE, ESELFLOOP, EDUP, ENOMEM, ENOTSUP = 0, -1, -2, -3, -4, -5, -7


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc; floating point contraction is off so that the estimator's
    two roundings (product, then quotient) are exactly the ones written."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        vp = ctypes.c_void_p
        L.oracle_splitmix64.argtypes = [u64, u64]
        L.oracle_splitmix64.restype = u64
        L.oracle_hash_params.argtypes = [u64, u32, vp]
        L.oracle_hash_params.restype = None
        L.oracle_slot.argtypes = [vp, u32, u32, u32]
        L.oracle_slot.restype = u32
        L.oracle_slots.argtypes = [u64, u32, u32, vp, u64, vp]
        L.oracle_slots.restype = None
        L.oracle_validate.argtypes = [u32, vp, u64]
        L.oracle_validate.restype = i32
        L.oracle_rept.argtypes = [u32, u32, u32, u64, i32, vp, u64, u64, u64, vp, vp, vp]
        L.oracle_rept.restype = i32
        L.oracle_rept_procs.argtypes = [u32, u32, u32, u64, i32, vp, u64, u64, u64, vp, u32, u32, vp, vp]
        L.oracle_rept_procs.restype = i32
        L.oracle_rept_parallel.argtypes = [u32, u32, u32, u64, i32, vp, u64, u64, u64, u32, u32, u32, vp, vp]
        L.oracle_rept_parallel.restype = i32
        L.oracle_edge_updates.argtypes = [u32, u32, u32, u64, i32, vp, u64, vp, u64, vp, vp]
        L.oracle_edge_updates.restype = i32
        L.oracle_estimate.argtypes = [u32, u32, u32, u32, vp, vp, vp, vp]
        L.oracle_estimate.restype = i32
        L.oracle_rept2_eta.argtypes = [u32, u32, u32, u64, vp, u64, vp, vp, vp, vp]
        L.oracle_rept2_eta.restype = i32
        L.oracle_estimate2.argtypes = [u32, u32, u32, u32, i32, vp, vp, ctypes.c_int64, vp, vp, vp]
        L.oracle_estimate2.restype = i32
        L.oracle_mascot.argtypes = [u32, u32, u32, u64, vp, u64, vp, vp]
        L.oracle_mascot.restype = i32
        L.oracle_estimate_mascot.argtypes = [u32, u32, u32, vp, vp, vp, vp]
        L.oracle_estimate_mascot.restype = i32
        _lib = L
    return _lib


def _edges(edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.uint32).reshape(-1, 2))
    return e


def groups(m: int, c: int) -> int:
    return -(-c // m)


def splitmix64(seed: int, index: int) -> int:
    return int(_load().oracle_splitmix64(seed & (2**64 - 1), index))


def hash_params(seed: int, G: int) -> np.ndarray:
    """Per group (a_0, a_1, a_2, a_3): the 4-independent polynomial hash's coefficients."""
    out = np.zeros((G, 4), dtype=np.uint64)
    _load().oracle_hash_params(seed & (2**64 - 1), G, out.ctypes.data)
    return out


def slots(edges, m: int, G: int, seed: int) -> np.ndarray:
    """h_k(edge t) for every group k < G: array [G, E] of uint32."""
    e = _edges(edges)
    out = np.zeros((G, len(e)), dtype=np.uint32)
    _load().oracle_slots(seed & (2**64 - 1), m, G, e.ctypes.data, len(e), out.ctypes.data)
    return out


def validate(n: int, edges) -> int:
    e = _edges(edges)
    return int(_load().oracle_validate(n, e.ctypes.data, len(e)))


def rept(edges, n: int, m: int, c: int, seed: int, per_proc: bool = False, t0: int = 0,
         t1: int | None = None, slot_override=None):
    """Algorithm 1 per processor.  Returns (global[c], local[rows, n]) as int64, where rows is
    the number of groups (group sums) or c (per_proc)."""
    e = _edges(edges)
    E = len(e)
    t1 = E if t1 is None else t1
    G = groups(m, c)
    rows = c if per_proc else G
    glob = np.zeros(c, dtype=np.int64)
    loc = np.zeros((rows, n), dtype=np.int64)
    ov = None
    if slot_override is not None:
        ov = np.ascontiguousarray(np.asarray(slot_override, dtype=np.uint16).reshape(G, E))
    rc = _load().oracle_rept(n, m, c, seed & (2**64 - 1), int(per_proc), e.ctypes.data, E, t0, t1,
                             None if ov is None else ov.ctypes.data, glob.ctypes.data, loc.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_rept")
    return glob, loc


def rept_threads(edges, n: int, m: int, c: int, seed: int, per_proc: bool = False, t0: int = 0,
                 t1: int | None = None, workers: int = 8, procs: tuple | None = None):
    """Algorithm 1 with the c processors spread over host threads (C threads: the stream is
    validated and hashed once, then each thread replays whole processors).  Processors are
    independent, so the result equals ``rept``.  ``procs = (lo, hi)`` replays only processors
    lo..hi-1 (the others' counters stay 0)."""
    e = _edges(edges)
    E = len(e)
    t1 = E if t1 is None else t1
    G = groups(m, c)
    rows = c if per_proc else G
    p_lo, p_hi = (0, c) if procs is None else procs
    if not 0 <= p_lo <= p_hi <= c:
        raise OracleError(EINVAL, "rept_threads: processor range")
    glob = np.zeros(c, dtype=np.int64)
    loc = np.zeros((rows, n), dtype=np.int64)
    if p_lo == p_hi:
        return glob, loc
    rc = _load().oracle_rept_parallel(n, m, c, seed & (2**64 - 1), int(per_proc), e.ctypes.data, E, t0, t1,
                                      p_lo, p_hi, max(1, int(workers)), glob.ctypes.data, loc.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_rept_parallel")
    return glob, loc


def edge_updates(edges, n: int, m: int, c: int, seed: int, ts, per_proc: bool = False):
    """Per-edge updates of Algorithm 1 from their definition, summed over stream positions ts."""
    e = _edges(edges)
    G = groups(m, c)
    rows = c if per_proc else G
    t = np.ascontiguousarray(np.asarray(ts, dtype=np.uint64).ravel())
    glob = np.zeros(c, dtype=np.int64)
    loc = np.zeros((rows, n), dtype=np.int64)
    rc = _load().oracle_edge_updates(n, m, c, seed & (2**64 - 1), int(per_proc), e.ctypes.data, len(e),
                                     t.ctypes.data, len(t), glob.ctypes.data, loc.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_edge_updates")
    return glob, loc


def estimate(n: int, m: int, c: int, glob, loc=None):
    """(tau_hat, tau_v_hat[n] or None) per Sections III-A/III-B (c <= m or m | c)."""
    g = np.ascontiguousarray(np.asarray(glob, dtype=np.int64))
    th = ctypes.c_double(0.0)
    tv = None
    lp = None
    rows = 0
    if loc is not None:
        lo = np.ascontiguousarray(np.asarray(loc, dtype=np.int64))
        rows = lo.shape[0]
        tv = np.zeros(n, dtype=np.float64)
        lp = lo.ctypes.data
    rc = _load().oracle_estimate(n, m, c, rows, g.ctypes.data, lp, ctypes.addressof(th),
                                 None if tv is None else tv.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_estimate")
    return th.value, tv


def rept2_eta(edges, n: int, m: int, c: int, seed: int):
    """Algorithm 2's triangle-pair counters (Section III-B), both readings of the counter's
    initial value on insert: returns (eta_def[c], eta_lit[c], eta_v_def[n], eta_v_lit[n]),
    eta_v summed over all processors."""
    e = _edges(edges)
    ed = np.zeros(c, dtype=np.int64)
    el = np.zeros(c, dtype=np.int64)
    vd = np.zeros(n, dtype=np.int64)
    vl = np.zeros(n, dtype=np.int64)
    rc = _load().oracle_rept2_eta(n, m, c, seed & (2**64 - 1), e.ctypes.data, len(e), ed.ctypes.data,
                                  el.ctypes.data, vd.ctypes.data, vl.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_rept2_eta")
    return ed, el, vd, vl


def estimate2(n: int, m: int, c: int, glob, loc=None, eta: int = 0, eta_v=None, per_proc: bool = False):
    """Algorithm 2's combined estimators (c > m, m not dividing c): (tau_hat, tau_v_hat[n] or
    None), from the counters, eta (sum of eta^(i)) and eta_v (sums over processors)."""
    g = np.ascontiguousarray(np.asarray(glob, dtype=np.int64))
    th = ctypes.c_double(0.0)
    tv = lp = ep = None
    rows = 0
    if loc is not None and eta_v is not None:
        lo = np.ascontiguousarray(np.asarray(loc, dtype=np.int64))
        ev = np.ascontiguousarray(np.asarray(eta_v, dtype=np.int64))
        rows = lo.shape[0]
        tv = np.zeros(n, dtype=np.float64)
        lp, ep = lo.ctypes.data, ev.ctypes.data
    rc = _load().oracle_estimate2(n, m, c, rows, int(per_proc), g.ctypes.data, lp, int(eta), ep,
                                  ctypes.addressof(th), None if tv is None else tv.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_estimate2")
    return th.value, tv


def mascot(edges, n: int, m: int, c: int, seed: int):
    """Parallel MASCOT (Section III-C): c processors, each keeping every edge independently with
    probability 1/m (processor i keeps e iff h_i(e) = 0, h_i the hash of group i); returns
    (global[c], local[c][n]) of the per-processor counters of Algorithm 1's counting step."""
    e = _edges(edges)
    glob = np.zeros(c, dtype=np.int64)
    loc = np.zeros((c, n), dtype=np.int64)
    rc = _load().oracle_mascot(n, m, c, seed & (2**64 - 1), e.ctypes.data, len(e), glob.ctypes.data,
                               loc.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_mascot")
    return glob, loc


def estimate_mascot(n: int, m: int, c: int, glob, loc=None):
    """Parallel MASCOT's estimators (the mean of the processors' m^2 tau^(i)): (tau_hat,
    tau_v_hat[n] or None)."""
    g = np.ascontiguousarray(np.asarray(glob, dtype=np.int64))
    th = ctypes.c_double(0.0)
    tv = lp = None
    if loc is not None:
        lo = np.ascontiguousarray(np.asarray(loc, dtype=np.int64))
        tv = np.zeros(n, dtype=np.float64)
        lp = lo.ctypes.data
    rc = _load().oracle_estimate_mascot(n, m, c, g.ctypes.data, lp, ctypes.addressof(th),
                                        None if tv is None else tv.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_estimate_mascot")
    return th.value, tv
