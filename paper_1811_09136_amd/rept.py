"""ctypes binding of ``librept.so`` (declared in ``include/rept.h``).

Argument marshalling only: every step of the counting path runs in the HIP library.  PyTorch
provides device memory (``torch.empty(..., device="cuda")``) and streams; nothing here
computes counts.  If the library is missing, :func:`lib` raises -- there is no fallback.

The functions named ``rept_*`` mirror the C calls one to one; :class:`Graph` and the helpers
below them are conveniences built only from those calls.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librept.so")

REPT_OK, REPT_EINVAL, REPT_ERANGE, REPT_ESELFLOOP, REPT_EDUP, REPT_ENOMEM, REPT_EDEVICE, REPT_ENOTSUP = \
    0, -1, -2, -3, -4, -5, -6, -7
REPT_LOCAL_PER_PROC = 1
REPT_MASCOT = 2
REPT_JOB_ACCUMULATE = 1
REPT_JOB_TABLE_READY = 2
UINT64_MAX = 2**64 - 1
UINT32_MAX = 2**32 - 1


class ReptError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {code} ({rept_status_str(code)})")


class rept_params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_uint32), ("c", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class rept_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("num_edges", ctypes.c_uint64), ("num_apex", ctypes.c_uint32),
                ("max_out_degree", ctypes.c_uint32), ("oriented_work", ctypes.c_uint64),
                ("sum_out_sq", ctypes.c_uint64), ("num_reverse", ctypes.c_uint64)]


class rept_job(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("params", rept_params), ("global_", ctypes.c_void_p),
                ("local", ctypes.c_void_p), ("t0", ctypes.c_uint64), ("t1", ctypes.c_uint64),
                ("unit0", ctypes.c_uint32), ("unit1", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64)]


class rept_tuning(ctypes.Structure):
    _fields_ = [("wave_cap", ctypes.c_uint32), ("block_cap", ctypes.c_uint32), ("b_chunk", ctypes.c_uint32),
                ("blocks", ctypes.c_uint32), ("threads", ctypes.c_uint32), ("light_tile", ctypes.c_uint32),
                ("phase_launches", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``librept.so``; raise if it has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1811_09136_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        sz = ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "rept_local_rows": ([P(rept_params)], u32),
            "rept_query_sizes": ([u32, u64, P(sz), P(sz)], i32),
            "rept_build": ([u32, vp, u64, vp, sz, vp, sz, vp, P(vp)], i32),
            "rept_build_host": ([u32, vp, u64, vp, sz, vp, sz, vp, P(vp)], i32),
            "rept_graph_get_info": ([vp, P(rept_graph_info)], i32),
            "rept_count_workspace_size": ([vp, P(rept_params), P(sz)], i32),
            "rept_count": ([vp, P(rept_params), vp, vp, vp, sz, vp], i32),
            "rept_count_range": ([vp, P(rept_params), u64, u64, vp, vp, vp, sz, vp], i32),
            "rept_count_noalloc": ([vp, P(rept_params), vp, vp, vp], i32),
            "rept_estimate": ([u32, P(rept_params), vp, vp, vp, vp], i32),
            "rept_estimate_sums": ([u32, P(rept_params), vp, vp, vp, vp], i32),
            "rept_count_eta_workspace_size": ([vp, P(rept_params), P(sz)], i32),
            "rept_count_eta": ([vp, P(rept_params), vp, vp, vp, vp, vp, sz, P(rept_tuning), vp], i32),
            "rept_estimate_combined": ([u32, P(rept_params), vp, vp, ctypes.c_int64, vp, vp, vp], i32),
            "rept_stream_query_sizes": ([u32, u64, u64, P(sz)], i32),
            "rept_stream_create": ([u32, u64, u64, P(rept_params), vp, sz, vp, vp, vp, P(vp)], i32),
            "rept_stream_append": ([vp, vp, u64, vp], i32),
            "rept_stream_num_edges": ([vp, P(u64)], i32),
            "rept_stream_set_policy": ([vp, u32], i32),
            "rept_stream_paths": ([vp, P(u64), P(u64)], i32),
            "rept_stream_destroy": ([vp], None),
            "rept_reduce_local": ([vp, u32, u32, vp, vp], i32),
            "rept_hash_slots": ([P(rept_params), vp, u64, vp, vp], i32),
            "rept_batch_workspace_size": ([u32, P(sz)], i32),
            "rept_batch_prepare": ([P(rept_job), u32, P(rept_tuning), vp, sz, vp], i32),
            "rept_batch_launch": ([vp, vp], i32),
            "rept_batch_count": ([P(rept_job), u32, P(rept_tuning), vp, sz, vp], i32),
            "rept_destroy": ([vp], None),
            "rept_status_str": ([i32], ctypes.c_char_p),
            "rept_device_cus": ([], u32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


EXPORTED = ["rept_local_rows", "rept_query_sizes", "rept_build", "rept_build_host", "rept_graph_get_info",
            "rept_count_workspace_size", "rept_count", "rept_count_noalloc",
            "rept_count_range", "rept_estimate", "rept_estimate_sums", "rept_count_eta_workspace_size",
            "rept_count_eta", "rept_estimate_combined", "rept_stream_query_sizes", "rept_stream_create",
            "rept_stream_append", "rept_stream_num_edges", "rept_stream_set_policy", "rept_stream_paths",
            "rept_stream_destroy", "rept_reduce_local", "rept_hash_slots", "rept_batch_workspace_size",
            "rept_batch_prepare", "rept_batch_launch", "rept_batch_count", "rept_destroy", "rept_status_str",
            "rept_device_cus"]


def _check(code: int, where: str):
    if code != REPT_OK:
        raise ReptError(code, where)


def _stream_ptr(stream) -> int | None:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


@dataclass(frozen=True)
class Params:
    """REPT sampling parameters: p = 1/m, c processors, hash seed (Table I)."""
    m: int
    c: int
    seed: int
    per_proc: bool = False
    mascot: bool = False  # parallel MASCOT: independent Bernoulli(1/m) samples (Section III-C)

    def c_struct(self) -> rept_params:
        flags = (REPT_LOCAL_PER_PROC if self.per_proc else 0) | (REPT_MASCOT if self.mascot else 0)
        return rept_params(self.m, self.c, self.seed & UINT64_MAX, flags, 0)

    @property
    def groups(self) -> int:
        return self.c if self.mascot else -(-self.c // self.m)

    @property
    def rows(self) -> int:
        return self.c if (self.per_proc or self.mascot) else self.groups


# ------------------------------------------------------------------ same-name wrappers -----

def rept_status_str(code: int) -> str:
    return lib().rept_status_str(int(code)).decode()


def rept_local_rows(params: Params) -> int:
    p = params.c_struct()
    return int(lib().rept_local_rows(ctypes.byref(p)))


def rept_query_sizes(n: int, num_edges: int) -> tuple[int, int]:
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _check(lib().rept_query_sizes(n, num_edges, ctypes.byref(a), ctypes.byref(b)), "rept_query_sizes")
    return a.value, b.value


def rept_build(n: int, edges_ptr: int, num_edges: int, persistent_ptr: int, persistent_bytes: int,
               scratch_ptr: int, scratch_bytes: int, stream_ptr: int | None) -> int:
    h = ctypes.c_void_p(0)
    _check(lib().rept_build(n, edges_ptr, num_edges, persistent_ptr, persistent_bytes, scratch_ptr, scratch_bytes,
                            stream_ptr, ctypes.byref(h)), "rept_build")
    return h.value


def rept_build_host(n: int, host_edges: np.ndarray, persistent_ptr: int, persistent_bytes: int,
                    scratch_ptr: int, scratch_bytes: int, stream_ptr: int | None) -> int:
    """rept_build for a host-resident stream (uint32 [E, 2]); the library copies it over PCIe."""
    e = np.ascontiguousarray(host_edges, dtype=np.uint32)
    if e.ndim != 2 or e.shape[1] != 2:
        raise ValueError("host_edges must be an [E, 2] array")
    h = ctypes.c_void_p(0)
    _check(lib().rept_build_host(n, e.ctypes.data if len(e) else None, len(e), persistent_ptr, persistent_bytes,
                                 scratch_ptr, scratch_bytes, stream_ptr, ctypes.byref(h)), "rept_build_host")
    return h.value


def rept_graph_get_info(handle: int) -> rept_graph_info:
    info = rept_graph_info()
    _check(lib().rept_graph_get_info(handle, ctypes.byref(info)), "rept_graph_get_info")
    return info


def rept_count_workspace_size(handle: int, params: Params) -> int:
    p = params.c_struct()
    b = ctypes.c_size_t(0)
    _check(lib().rept_count_workspace_size(handle, ctypes.byref(p), ctypes.byref(b)), "rept_count_workspace_size")
    return b.value


def rept_count(handle: int, params: Params, global_ptr: int, local_ptr: int, ws_ptr: int, ws_bytes: int,
               stream_ptr: int | None):
    p = params.c_struct()
    _check(lib().rept_count(handle, ctypes.byref(p), global_ptr, local_ptr, ws_ptr, ws_bytes, stream_ptr),
           "rept_count")


def rept_count_noalloc(handle: int, params: Params, global_ptr: int, local_ptr: int, stream_ptr: int | None):
    """rept_count with the slot table in the library's static device array (no workspace)."""
    p = params.c_struct()
    _check(lib().rept_count_noalloc(handle, ctypes.byref(p), global_ptr, local_ptr, stream_ptr), "rept_count_noalloc")


def rept_count_range(handle: int, params: Params, t0: int, t1: int, global_ptr: int, local_ptr: int, ws_ptr: int,
                     ws_bytes: int, stream_ptr: int | None):
    p = params.c_struct()
    _check(lib().rept_count_range(handle, ctypes.byref(p), t0, t1, global_ptr, local_ptr, ws_ptr, ws_bytes,
                                  stream_ptr), "rept_count_range")


def rept_estimate(n: int, params: Params, glob: np.ndarray, loc: np.ndarray | None, tau_v_out=None):
    """Host FP64 estimators; returns (tau_hat, tau_v_hat or None).  `tau_v_out` (float64[n])
    receives the local estimators when given (no allocation per call)."""
    p = params.c_struct()
    g = np.ascontiguousarray(glob, dtype=np.int64)
    th = ctypes.c_double(0.0)
    tv = None
    lp = None
    if loc is not None:
        lo = np.ascontiguousarray(loc, dtype=np.int64)
        if tau_v_out is None:
            tv = np.empty(n, dtype=np.float64)
        else:
            tv = tau_v_out
            if tv.dtype != np.float64 or tv.shape != (n,) or not tv.flags.c_contiguous:
                raise ValueError("tau_v_out must be a contiguous float64 array of n values")
        lp = lo.ctypes.data
    _check(lib().rept_estimate(n, ctypes.byref(p), g.ctypes.data, lp, ctypes.addressof(th),
                               None if tv is None else tv.ctypes.data), "rept_estimate")
    return th.value, tv


def rept_estimate_sums(n: int, params: Params, glob: np.ndarray, sums: np.ndarray | None, tau_v_out=None):
    """Host FP64 estimators from node sums S_v (rept_reduce_local's output); returns
    (tau_hat, tau_v_hat or None), identical to rept_estimate on the rows."""
    p = params.c_struct()
    g = np.ascontiguousarray(glob, dtype=np.int64)
    th = ctypes.c_double(0.0)
    tv = None
    sp = None
    if sums is not None:
        sv = np.ascontiguousarray(sums, dtype=np.int64)
        if sv.shape != (n,):
            raise ValueError("sums must hold n values")
        if tau_v_out is None:
            tv = np.empty(n, dtype=np.float64)
        else:
            tv = tau_v_out
            if tv.dtype != np.float64 or tv.shape != (n,) or not tv.flags.c_contiguous:
                raise ValueError("tau_v_out must be a contiguous float64 array of n values")
        sp = sv.ctypes.data
    _check(lib().rept_estimate_sums(n, ctypes.byref(p), g.ctypes.data, sp, ctypes.addressof(th),
                                    None if tv is None else tv.ctypes.data), "rept_estimate_sums")
    return th.value, tv


def rept_count_eta_workspace_size(handle: int, params: Params) -> int:
    p = params.c_struct()
    b = ctypes.c_size_t(0)
    _check(lib().rept_count_eta_workspace_size(handle, ctypes.byref(p), ctypes.byref(b)),
           "rept_count_eta_workspace_size")
    return b.value


def rept_count_eta(handle: int, params: Params, global_ptr: int, local_ptr: int, eta_ptr: int, eta_v_ptr: int | None,
                   ws_ptr: int, ws_bytes: int, tuning: rept_tuning | None, stream_ptr: int | None):
    p = params.c_struct()
    _check(lib().rept_count_eta(handle, ctypes.byref(p), global_ptr, local_ptr, eta_ptr, eta_v_ptr, ws_ptr, ws_bytes,
                                None if tuning is None else ctypes.byref(tuning), stream_ptr), "rept_count_eta")


def rept_estimate_combined(n: int, params: Params, glob: np.ndarray, loc: np.ndarray | None, eta: int,
                           eta_v: np.ndarray | None, tau_v_out=None):
    """Algorithm 2's combined FP64 estimators (c > m, m not dividing c); returns
    (tau_hat, tau_v_hat or None).  eta: sum of the definition counters; eta_v: int64[n];
    `tau_v_out` (float64[n]) receives the local estimators when given."""
    p = params.c_struct()
    g = np.ascontiguousarray(glob, dtype=np.int64)
    th = ctypes.c_double(0.0)
    tv = lp = ep = None
    if loc is not None and eta_v is not None:
        lo = np.ascontiguousarray(loc, dtype=np.int64)
        ev = np.ascontiguousarray(eta_v, dtype=np.int64)
        if ev.shape != (n,):
            raise ValueError("eta_v must hold n values")
        if tau_v_out is None:
            tv = np.empty(n, dtype=np.float64)
        else:
            tv = tau_v_out
            if tv.dtype != np.float64 or tv.shape != (n,) or not tv.flags.c_contiguous:
                raise ValueError("tau_v_out must be a contiguous float64 array of n values")
        lp, ep = lo.ctypes.data, ev.ctypes.data
    _check(lib().rept_estimate_combined(n, ctypes.byref(p), g.ctypes.data, lp, int(eta), ep, ctypes.addressof(th),
                                        None if tv is None else tv.ctypes.data), "rept_estimate_combined")
    return th.value, tv


def rept_stream_query_sizes(n: int, capacity: int, max_chunk: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().rept_stream_query_sizes(n, capacity, max_chunk, ctypes.byref(b)), "rept_stream_query_sizes")
    return b.value


def rept_stream_create(n: int, capacity: int, max_chunk: int, params: Params, buf_ptr: int, buf_bytes: int,
                       global_ptr: int, local_ptr: int, stream_ptr: int | None) -> int:
    p = params.c_struct()
    h = ctypes.c_void_p(0)
    _check(lib().rept_stream_create(n, capacity, max_chunk, ctypes.byref(p), buf_ptr, buf_bytes, global_ptr,
                                    local_ptr, stream_ptr, ctypes.byref(h)), "rept_stream_create")
    return h.value


def rept_stream_append(handle: int, edges_ptr: int, num_edges: int, stream_ptr: int | None):
    _check(lib().rept_stream_append(handle, edges_ptr, num_edges, stream_ptr), "rept_stream_append")


def rept_stream_num_edges(handle: int) -> int:
    v = ctypes.c_uint64(0)
    _check(lib().rept_stream_num_edges(handle, ctypes.byref(v)), "rept_stream_num_edges")
    return v.value


REPT_STREAM_AUTO, REPT_STREAM_PER_EDGE, REPT_STREAM_RECOUNT = 0, 1, 2
STREAM_POLICIES = {"auto": REPT_STREAM_AUTO, "per_edge": REPT_STREAM_PER_EDGE, "recount": REPT_STREAM_RECOUNT}


def rept_stream_set_policy(handle: int, policy: int):
    _check(lib().rept_stream_set_policy(handle, policy), "rept_stream_set_policy")


def rept_stream_paths(handle: int) -> tuple[int, int]:
    a, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().rept_stream_paths(handle, ctypes.byref(a), ctypes.byref(b)), "rept_stream_paths")
    return a.value, b.value


def rept_stream_destroy(handle: int):
    lib().rept_stream_destroy(handle)


def rept_reduce_local(local_ptr: int, rows: int, n: int, sums_ptr: int, stream_ptr: int | None):
    """sums[v] = sum of the rows of local at v, on the device (exact int64)."""
    _check(lib().rept_reduce_local(local_ptr, rows, n, sums_ptr, stream_ptr), "rept_reduce_local")


def rept_hash_slots(params: Params, edges_ptr: int, num_edges: int, slots_ptr: int, stream_ptr: int | None):
    p = params.c_struct()
    _check(lib().rept_hash_slots(ctypes.byref(p), edges_ptr, num_edges, slots_ptr, stream_ptr), "rept_hash_slots")


def rept_batch_workspace_size(njobs: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().rept_batch_workspace_size(njobs, ctypes.byref(b)), "rept_batch_workspace_size")
    return b.value


def rept_batch_prepare(jobs, tuning: rept_tuning | None, ws_ptr: int, ws_bytes: int, stream_ptr: int | None):
    arr = (rept_job * len(jobs))(*jobs)
    _check(lib().rept_batch_prepare(arr, len(jobs), None if tuning is None else ctypes.byref(tuning), ws_ptr,
                                    ws_bytes, stream_ptr), "rept_batch_prepare")


def rept_batch_launch(ws_ptr: int, stream_ptr: int | None):
    _check(lib().rept_batch_launch(ws_ptr, stream_ptr), "rept_batch_launch")


def rept_batch_count(jobs, tuning: rept_tuning | None, ws_ptr: int, ws_bytes: int, stream_ptr: int | None):
    arr = (rept_job * len(jobs))(*jobs)
    _check(lib().rept_batch_count(arr, len(jobs), None if tuning is None else ctypes.byref(tuning), ws_ptr,
                                  ws_bytes, stream_ptr), "rept_batch_count")


def rept_destroy(handle: int):
    lib().rept_destroy(handle)


def rept_device_cus() -> int:
    return int(lib().rept_device_cus())


# ------------------------------------------------------------------ conveniences ----------

def _alloc(nbytes: int, device):
    import torch
    # 256-byte alignment: the caching allocator returns 512-byte aligned blocks
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def to_device_edges(edges: np.ndarray, device="cuda"):
    """Upload a host [E, 2] uint32 stream (stored as int32 bits; the library reads uint32)."""
    import torch
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.uint32).reshape(-1, 2))
    return torch.from_numpy(e.view(np.int32)).to(device)


class Graph:
    """A built graph on the device (owns its persistent buffer)."""

    def __init__(self, edges_dev, n: int, stream=None):
        import torch
        self.device = edges_dev.device
        self.n = int(n)
        self.num_edges = int(edges_dev.shape[0])
        pbytes, sbytes = rept_query_sizes(self.n, self.num_edges)
        self.persistent_bytes = pbytes
        self.scratch_bytes = sbytes
        self.persistent = _alloc(pbytes, self.device)
        scratch = _alloc(sbytes, self.device)
        sp = _stream_ptr(stream)
        self.handle = rept_build(self.n, edges_dev.data_ptr(), self.num_edges, self.persistent.data_ptr(), pbytes,
                                 scratch.data_ptr(), sbytes, sp)
        # scratch may be reused once rept_build returned (it synchronised its stream)
        del scratch
        self.info = rept_graph_get_info(self.handle)
        self._torch = torch
        self._ws = None  # workspace shared by this graph's count / count_range calls

    def outputs(self, params: Params):
        torch = self._torch
        g = torch.empty(params.c, dtype=torch.int64, device=self.device)
        l = torch.empty((params.rows, self.n), dtype=torch.int64, device=self.device)
        return g, l

    def workspace_bytes(self, params: Params) -> int:
        return rept_count_workspace_size(self.handle, params)

    def new_workspace(self, params: Params):
        """A device workspace (slot table) for one count of this graph under `params`."""
        return _alloc(self.workspace_bytes(params), self.device)

    def _shared_workspace(self, params: Params):
        # one buffer for the calls below, grown on demand; calls on one graph from different
        # streams at the same time must pass their own workspaces
        need = self.workspace_bytes(params)
        if self._ws is None or self._ws.numel() < need:
            self._ws = _alloc(need, self.device)
        return self._ws

    def count(self, params: Params, out=None, stream=None, workspace=None):
        g, l = self.outputs(params) if out is None else out
        ws = self._shared_workspace(params) if workspace is None else workspace
        rept_count(self.handle, params, g.data_ptr(), l.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream))
        return g, l

    def count_range(self, params: Params, t0: int, t1: int, out, stream=None, workspace=None):
        g, l = out
        ws = self._shared_workspace(params) if workspace is None else workspace
        rept_count_range(self.handle, params, t0, t1, g.data_ptr(), l.data_ptr(), ws.data_ptr(), ws.numel(),
                         _stream_ptr(stream))
        return g, l

    def count_eta(self, params: Params, stream=None, with_nodes: bool = True, tuning: rept_tuning | None = None):
        """Counts with Algorithm 2's pair counters: (global[c], local[rows][n], eta[2][c],
        eta_v[2][n] or None); row 0 of eta / eta_v is the definition counter, row 1 the
        counter as printed in Algorithm 2."""
        torch = self._torch
        g, l = self.outputs(params)
        eta = torch.empty((2, params.c), dtype=torch.int64, device=self.device)
        eta_v = torch.empty((2, self.n), dtype=torch.int64, device=self.device) if with_nodes else None
        ws = _alloc(rept_count_eta_workspace_size(self.handle, params), self.device)
        rept_count_eta(self.handle, params, g.data_ptr(), l.data_ptr(), eta.data_ptr(),
                       None if eta_v is None else eta_v.data_ptr(), ws.data_ptr(), ws.numel(), tuning,
                       _stream_ptr(stream))
        self._eta_ws = ws  # kept until the next call: the work on `stream` may still read it
        return g, l, eta, eta_v

    def close(self):
        if getattr(self, "handle", None):
            rept_destroy(self.handle)
            self.handle = None
            self.persistent = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IncrementalStream:
    """A stream appended chunk by chunk on the device; `counts` (global int64[c], local
    int64[rows][n]) always hold Algorithm 1's updates of every edge appended so far."""

    def __init__(self, n: int, capacity: int, max_chunk: int, params: Params, device="cuda", stream=None,
                 policy: str = "auto"):
        """policy: how appends count their edges ("auto", "per_edge" or "recount"; equal results)."""
        import torch
        self.n, self.params, self.device = int(n), params, torch.device(device)
        nbytes = rept_stream_query_sizes(self.n, capacity, max_chunk)
        self.buffer = _alloc(nbytes, self.device)
        self.counts = (torch.empty(params.c, dtype=torch.int64, device=self.device),
                       torch.empty((params.rows, self.n), dtype=torch.int64, device=self.device))
        self.handle = rept_stream_create(self.n, capacity, max_chunk, params, self.buffer.data_ptr(), nbytes,
                                         self.counts[0].data_ptr(), self.counts[1].data_ptr(), _stream_ptr(stream))
        rept_stream_set_policy(self.handle, STREAM_POLICIES[policy])

    def append(self, edges_dev, stream=None):
        """Append a device [W, 2] chunk (int32 bits of uint32 ids).  Raises ReptError (state
        unchanged) if the chunk is invalid."""
        W = int(edges_dev.shape[0])
        if W:
            if not edges_dev.is_contiguous():
                raise ValueError("edges must be contiguous")
            rept_stream_append(self.handle, edges_dev.data_ptr(), W, _stream_ptr(stream))
        self._last = edges_dev  # the chunk stays referenced until the next append

    @property
    def num_edges(self) -> int:
        return rept_stream_num_edges(self.handle)

    def paths(self) -> tuple[int, int]:
        """(appends counted edge by edge, appends counted by a windowed recount)."""
        return rept_stream_paths(self.handle)

    def estimate(self):
        """(tau_hat, tau_v_hat) of the stream so far (synchronises)."""
        import torch
        torch.cuda.synchronize(self.device)
        g, l = self.counts[0].cpu().numpy(), self.counts[1].cpu().numpy()
        return rept_estimate(self.n, self.params, g, l)

    def close(self):
        if getattr(self, "handle", None):
            rept_stream_destroy(self.handle)
            self.handle = None
            self.buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hash_slots(params: Params, edges_dev, stream=None):
    import torch
    E = int(edges_dev.shape[0])
    out = torch.empty((params.groups, E), dtype=torch.int32, device=edges_dev.device)
    rept_hash_slots(params, edges_dev.data_ptr(), E, out.data_ptr(), _stream_ptr(stream))
    return out


def make_job(graph: Graph, params: Params, out, workspace, t0: int = 0, t1: int = UINT64_MAX, unit0: int = 0,
             unit1: int = UINT32_MAX, accumulate: bool = False, table_ready: bool = False) -> rept_job:
    """One batch job.  `workspace` (a device tensor of at least graph.workspace_bytes(params)
    bytes, e.g. graph.new_workspace(params)) must stay alive until the launch completed; with
    `table_ready` it already holds this (graph, params)'s slot table from an earlier launch."""
    g, l = out
    flags = (REPT_JOB_ACCUMULATE if accumulate else 0) | (REPT_JOB_TABLE_READY if table_ready else 0)
    job = rept_job(graph.handle, params.c_struct(), g.data_ptr(), l.data_ptr(), t0, t1, unit0, unit1, flags, 0,
                   workspace.data_ptr(), workspace.numel())
    job._keep = (workspace, g, l)  # the struct holds raw pointers: keep the tensors alive with it
    return job


def tuning(wave_cap=0, block_cap=0, b_chunk=0, blocks=0, threads=0, light_tile=0, phase_launches=0) -> rept_tuning:
    """Launch shape of the counting kernel (zero = library default); see ``rept_tuning`` in rept.h."""
    return rept_tuning(wave_cap, block_cap, b_chunk, blocks, threads, light_tile, phase_launches, 0)
