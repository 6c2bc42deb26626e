"""Thin Python binding of libdfpr.so (``include/dfpr.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Host arrays are numpy arrays; device arrays are torch tensors
on the current HIP device, whose pointers and stream are handed over as
plain integers.  If the library is missing this module raises; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfpr.so")

DFPR_OK = 0
DFPR_E_ARG = -1
DFPR_E_RANGE = -2
DFPR_E_NOMEM = -3
DFPR_E_DEVICE = -4
DFPR_E_BUSY = -5
DFPR_E_LIMIT = -6
FP64 = 0
FP32_KAHAN = 1
SYNC = 0
ASYNC = 1
LOOP_LAUNCHES = 0
LOOP_DEVICE = 1
FTOL_ADAPTIVE = -1.0

EXPORTED = [
    "dfpr_params_default", "dfpr_load_graph", "dfpr_free_graph", "dfpr_set_stream",
    "dfpr_graph_info", "dfpr_apply_batch", "dfpr_apply_batch_device",
    "dfpr_pagerank_static", "dfpr_pagerank_naive_dynamic",
    "dfpr_pagerank_dynamic_frontier", "dfpr_pagerank_dynamic_frontier_device",
    "dfpr_pagerank_dynamic_frontier_device_noalloc",
    "dfpr_mark_affected", "dfpr_get_affected", "dfpr_get_ranks", "dfpr_set_ranks",
    "dfpr_export_csr", "dfpr_last_error", "dfpr_profile_reset", "dfpr_profile_read",
    "dfpr_pagerank_dynamic_traversal", "dfpr_mark_reachable",
    "dfpr_server_create", "dfpr_server_free", "dfpr_server_add_graph", "dfpr_server_submit",
    "dfpr_server_run", "dfpr_server_result", "dfpr_server_set_large_edges",
]


class DfprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dfpr error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("tol", ctypes.c_double),
                ("frontier_tol", ctypes.c_double), ("max_iters", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("loop", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("refine_sweeps", ctypes.c_int32), ("loop_iterations", ctypes.c_int32),
                ("final_linf", ctypes.c_double), ("ms_device", ctypes.c_double),
                ("affected_initial", ctypes.c_int64), ("affected_final", ctypes.c_int64),
                ("vertices_processed", ctypes.c_int64), ("edges_processed", ctypes.c_int64),
                ("ms_mark", ctypes.c_double), ("ms_iter", ctypes.c_double),
                ("ms_apply", ctypes.c_double), ("frontier_tol_used", ctypes.c_double)]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("rows", ctypes.c_int64), ("edges", ctypes.c_int64),
                ("expanded_rows", ctypes.c_int64), ("expanded_edges", ctypes.c_int64),
                ("marked", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("wall_ms", ctypes.c_double),
                ("updates_per_s", ctypes.c_double), ("latency_p50_ms", ctypes.c_double),
                ("latency_p99_ms", ctypes.c_double), ("latency_mean_ms", ctypes.c_double),
                ("queue_p50_ms", ctypes.c_double), ("queue_p99_ms", ctypes.c_double),
                ("max_active", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("peak_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RequestResult(ctypes.Structure):
    _fields_ = [("graph_id", ctypes.c_int32), ("status", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("refine_sweeps", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("arrival_ms", ctypes.c_double), ("admit_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double), ("applied", ctypes.c_int64 * 2),
                ("edges_processed", ctypes.c_int64), ("affected", ctypes.c_int64),
                ("final_linf", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "applied"}
        d["applied"] = (int(self.applied[0]), int(self.applied[1]))
        return d


@dataclass
class Stats:
    iterations: int
    converged: bool
    refine_sweeps: int
    final_linf: float
    ms_device: float
    affected_initial: int
    affected_final: int
    vertices_processed: int
    edges_processed: int
    ms_mark: float
    ms_iter: float
    ms_apply: float
    loop_iterations: int = 0
    frontier_tol_used: float = 0.0


def _stats(s):
    return Stats(s.iterations, bool(s.converged), s.refine_sweeps, s.final_linf, s.ms_device,
                 s.affected_initial, s.affected_final, s.vertices_processed, s.edges_processed,
                 s.ms_mark, s.ms_iter, s.ms_apply, s.loop_iterations, s.frontier_tol_used)


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64


def lib():
    """Open libdfpr.so.  torch is imported first so that the process holds a
    single HIP runtime, shared by torch tensors and the library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python paper_2401_03256_amd/build.py")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    L.dfpr_params_default.argtypes = [_P]
    L.dfpr_params_default.restype = None
    L.dfpr_load_graph.argtypes = [_I32, _I64, _P, _P, ctypes.POINTER(_P)]
    L.dfpr_free_graph.argtypes = [_P]
    L.dfpr_free_graph.restype = None
    L.dfpr_set_stream.argtypes = [_P, _P]
    L.dfpr_graph_info.argtypes = [_P, _P, _P]
    batch = [_I64, _P, _P, _I64, _P, _P]
    L.dfpr_apply_batch.argtypes = [_P, *batch, _P]
    L.dfpr_apply_batch_device.argtypes = [_P, *batch, _P]
    L.dfpr_pagerank_static.argtypes = [_P, _P, _P, _P]
    L.dfpr_pagerank_naive_dynamic.argtypes = [_P, _P, _P, _P, _P]
    L.dfpr_pagerank_dynamic_frontier.argtypes = [_P, _P, *batch, _P, _P, _P]
    L.dfpr_pagerank_dynamic_frontier_device.argtypes = [_P, _P, *batch, _P, _P, _P]
    L.dfpr_pagerank_dynamic_frontier_device_noalloc.argtypes = [_P, _P, *batch, _P, _P, _P]
    L.dfpr_mark_affected.argtypes = [_P, *batch, _P]
    L.dfpr_pagerank_dynamic_traversal.argtypes = [_P, _P, *batch, _P, _P, _P]
    L.dfpr_mark_reachable.argtypes = [_P, *batch, _P]
    L.dfpr_get_affected.argtypes = [_P, _P]
    L.dfpr_get_ranks.argtypes = [_P, _P, ctypes.c_int]
    L.dfpr_set_ranks.argtypes = [_P, _P, ctypes.c_int]
    L.dfpr_export_csr.argtypes = [_P, ctypes.c_int, _P, _P]
    L.dfpr_profile_reset.argtypes = [_P, ctypes.c_int]
    L.dfpr_profile_read.argtypes = [_P, _P]
    L.dfpr_server_create.argtypes = [_I32, _I64, ctypes.POINTER(_P)]
    L.dfpr_server_free.argtypes = [_P]
    L.dfpr_server_free.restype = None
    L.dfpr_server_set_large_edges.argtypes = [_P, _I64]
    L.dfpr_server_add_graph.argtypes = [_P, _P, _P, _P]
    L.dfpr_server_submit.argtypes = [_P, _I32, ctypes.c_double, *batch, _P]
    L.dfpr_server_run.argtypes = [_P, _P]
    L.dfpr_server_result.argtypes = [_P, _I64, _P]
    L.dfpr_last_error.argtypes = []
    L.dfpr_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != DFPR_OK:
        raise DfprError(rc, lib().dfpr_last_error().decode())


def _hp(a):
    return None if a is None else a.ctypes.data_as(_P)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def params(alpha=None, tol=None, frontier_tol=None, max_iters=None, precision=None,
           mode=None, loop=None) -> Params:
    p = Params()
    lib().dfpr_params_default(ctypes.byref(p))
    if alpha is not None:
        p.alpha = alpha
    if tol is not None:
        p.tol = tol
        if frontier_tol is None:
            p.frontier_tol = tol / 1e5
    if frontier_tol is not None:
        p.frontier_tol = frontier_tol
    if max_iters is not None:
        p.max_iters = max_iters
    if precision is not None:
        p.precision = precision
    if mode is not None:
        p.mode = mode
    if loop is not None:
        p.loop = loop
    return p


def _batch_arrays(batch):
    """Deletion and insertion pairs as int32 arrays; each side's two arrays
    must have the same length (the library reads that many of each)."""
    ds, dd, is_, id_ = (_i32(batch.del_src), _i32(batch.del_dst), _i32(batch.ins_src),
                        _i32(batch.ins_dst))
    if ds.ndim != 1 or ds.shape != dd.shape or is_.ndim != 1 or is_.shape != id_.shape:
        raise ValueError("a batch needs 1-D source and target arrays of equal length")
    return ds, dd, is_, id_


def _dev_ptr(t, dtype=None, numel=None):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device arguments must be contiguous tensors on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"device argument of dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"device argument of {t.numel()} elements, expected {numel}")
    return _P(t.data_ptr())


class Graph:
    """A graph resident on the GPU (both CSRs, ranks, work lists)."""

    def __init__(self, n, src, dst):
        src, dst = _i32(src), _i32(dst)
        if src.shape != dst.shape:
            raise ValueError("src/dst length mismatch")
        h = _P()
        _check(lib().dfpr_load_graph(int(n), int(src.size), _hp(src), _hp(dst), ctypes.byref(h)))
        self._h = h
        self.n = int(n)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dfpr_free_graph(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def m(self) -> int:
        m = _I64()
        _check(lib().dfpr_graph_info(self._h, None, ctypes.byref(m)))
        return int(m.value)

    def set_stream(self, stream_ptr):
        _check(lib().dfpr_set_stream(self._h, _P(stream_ptr) if stream_ptr else None))

    def use_torch_stream(self):
        import torch
        self.set_stream(torch.cuda.current_stream().cuda_stream)

    # -- graph updates ----------------------------------------------------
    def apply_batch(self, batch):
        ds, dd, is_, id_ = _batch_arrays(batch)
        applied = np.zeros(2, np.int64)
        _check(lib().dfpr_apply_batch(self._h, ds.size, _hp(ds), _hp(dd), is_.size, _hp(is_),
                                      _hp(id_), _hp(applied)))
        return int(applied[0]), int(applied[1])

    def apply_batch_device(self, ds, dd, is_, id_):
        """Torch int32 tensors on the GPU."""
        import torch
        nd, ni = ds.numel(), is_.numel()
        applied = np.zeros(2, np.int64)
        _check(lib().dfpr_apply_batch_device(
            self._h, nd, _dev_ptr(ds, torch.int32), _dev_ptr(dd, torch.int32, nd), ni,
            _dev_ptr(is_, torch.int32), _dev_ptr(id_, torch.int32, ni), _hp(applied)))
        return int(applied[0]), int(applied[1])

    # -- rank engines -----------------------------------------------------
    def static(self, p: Params | None = None, out=True):
        st = _Stats()
        R = np.empty(self.n, np.float64) if out else None
        _check(lib().dfpr_pagerank_static(self._h, ctypes.byref(p) if p else None, _hp(R),
                                          ctypes.byref(st)))
        return R, _stats(st)

    def naive_dynamic(self, prev=None, p: Params | None = None, out=True):
        st = _Stats()
        prev = self._ranks_arg(prev)
        R = np.empty(self.n, np.float64) if out else None
        _check(lib().dfpr_pagerank_naive_dynamic(self._h, ctypes.byref(p) if p else None,
                                                 _hp(prev), _hp(R), ctypes.byref(st)))
        return R, _stats(st)

    def dynamic_frontier(self, batch, prev=None, p: Params | None = None, out=True):
        ds, dd, is_, id_ = _batch_arrays(batch)
        prev = self._ranks_arg(prev)
        R = np.empty(self.n, np.float64) if out else None
        st = _Stats()
        _check(lib().dfpr_pagerank_dynamic_frontier(
            self._h, ctypes.byref(p) if p else None, ds.size, _hp(ds), _hp(dd), is_.size,
            _hp(is_), _hp(id_), _hp(prev), _hp(R), ctypes.byref(st)))
        return R, _stats(st)

    def dynamic_frontier_device(self, ds, dd, is_, id_, prev=None, out=None,
                                p: Params | None = None, noalloc=False):
        """Batch as torch int32 GPU tensors; prev/out optional float64 GPU
        tensors.  noalloc: the entry point that makes no allocation."""
        import torch
        nd, ni = ds.numel(), is_.numel()
        st = _Stats()
        fn = (lib().dfpr_pagerank_dynamic_frontier_device_noalloc if noalloc
              else lib().dfpr_pagerank_dynamic_frontier_device)
        _check(fn(self._h, ctypes.byref(p) if p else None, nd, _dev_ptr(ds, torch.int32),
                  _dev_ptr(dd, torch.int32, nd), ni, _dev_ptr(is_, torch.int32),
                  _dev_ptr(id_, torch.int32, ni), _dev_ptr(prev, torch.float64, self.n),
                  _dev_ptr(out, torch.float64, self.n), ctypes.byref(st)))
        return _stats(st)

    # -- inspection ---------------------------------------------------------
    def dynamic_traversal(self, batch, prev=None, p: Params | None = None, out=True):
        """Dynamic Traversal PageRank (comparator) after apply_batch(batch)."""
        ds, dd, is_, id_ = _batch_arrays(batch)
        prev = self._ranks_arg(prev)
        R = np.empty(self.n, np.float64) if out else None
        st = _Stats()
        _check(lib().dfpr_pagerank_dynamic_traversal(
            self._h, ctypes.byref(p) if p else None, ds.size, _hp(ds), _hp(dd), is_.size,
            _hp(is_), _hp(id_), _hp(prev), _hp(R), ctypes.byref(st)))
        return R, _stats(st)

    def mark_reachable(self, batch):
        ds, dd, is_, id_ = _batch_arrays(batch)
        flags = np.zeros(self.n, np.uint8)
        _check(lib().dfpr_mark_reachable(self._h, ds.size, _hp(ds), _hp(dd), is_.size, _hp(is_),
                                         _hp(id_), _hp(flags)))
        return flags

    def mark_affected(self, batch):
        ds, dd, is_, id_ = _batch_arrays(batch)
        flags = np.zeros(self.n, np.uint8)
        _check(lib().dfpr_mark_affected(self._h, ds.size, _hp(ds), _hp(dd), is_.size, _hp(is_),
                                        _hp(id_), _hp(flags)))
        return flags

    def affected(self):
        flags = np.zeros(self.n, np.uint8)
        _check(lib().dfpr_get_affected(self._h, _hp(flags)))
        return flags

    def ranks(self):
        R = np.empty(self.n, np.float64)
        _check(lib().dfpr_get_ranks(self._h, _hp(R), 0))
        return R

    def ranks_device(self, out):
        import torch
        _check(lib().dfpr_get_ranks(self._h, _dev_ptr(out, torch.float64, self.n), 1))
        return out

    def _ranks_arg(self, R):
        """A host rank vector as n contiguous doubles (the library reads n)."""
        if R is None:
            return None
        R = np.ascontiguousarray(R, np.float64)
        if R.shape != (self.n,):
            raise ValueError(f"rank vector of shape {R.shape}, expected ({self.n},)")
        return R

    def set_ranks(self, R=None):
        R = self._ranks_arg(R)
        _check(lib().dfpr_set_ranks(self._h, _hp(R), 0))

    def profile_reset(self, enable=True):
        _check(lib().dfpr_profile_reset(self._h, 1 if enable else 0))

    def profile(self) -> Profile:
        pr = Profile()
        _check(lib().dfpr_profile_read(self._h, ctypes.byref(pr)))
        return pr

    def csr(self, out: bool):
        off = np.zeros(self.n + 1, np.int64)
        idx = np.zeros(max(self.m, 1), np.int32)
        _check(lib().dfpr_export_csr(self._h, 1 if out else 0, _hp(off), _hp(idx)))
        return off, idx[: self.m]

    # -- checkpoint ---------------------------------------------------------
    def save(self, path):
        """Checkpoint: the current graph (out-CSR, self-loops included) and
        the resident ranks, the only state carried from one snapshot to the
        next (Algorithm 1 takes R^{t-1}), in one .npz file."""
        off, idx = self.csr(out=True)
        np.savez(path, n=np.int64(self.n), out_offsets=off, out_idx=idx, ranks=self.ranks())

    @classmethod
    def load(cls, path):
        """A graph and its ranks from save(); the file holds plain arrays
        and is read without unpickling."""
        with np.load(path, allow_pickle=False) as z:
            n = int(z["n"])
            off = z["out_offsets"]
            src = np.repeat(np.arange(n, dtype=np.int32), np.diff(off))
            g = cls(n, src, z["out_idx"])
            g.set_ranks(z["ranks"])
        return g


class Server:
    """Serving form: resident graphs, update requests served by continuous
    batching (``dfpr_server_*`` in include/dfpr.h)."""

    def __init__(self, max_slots=8, hbm_budget_bytes=64 << 30):
        h = _P()
        _check(lib().dfpr_server_create(int(max_slots), int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self._graphs = []

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dfpr_server_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_large_edges(self, edges: int) -> None:
        """Graphs of at least `edges` edges run in the large lane."""
        _check(lib().dfpr_server_set_large_edges(self._h, int(edges)))

    def add_graph(self, graph: Graph, p: Params | None = None) -> int:
        gid = _I32()
        _check(lib().dfpr_server_add_graph(self._h, graph.handle, ctypes.byref(p) if p else None,
                                           ctypes.byref(gid)))
        self._graphs.append(graph)
        return int(gid.value)

    def submit(self, gid, arrival_ms, batch) -> int:
        ds, dd, is_, id_ = _batch_arrays(batch)
        rid = _I64()
        _check(lib().dfpr_server_submit(self._h, int(gid), float(arrival_ms), ds.size, _hp(ds),
                                        _hp(dd), is_.size, _hp(is_), _hp(id_), ctypes.byref(rid)))
        return int(rid.value)

    def run(self) -> dict:
        st = ServerStats()
        _check(lib().dfpr_server_run(self._h, ctypes.byref(st)))
        return st.as_dict()

    def result(self, rid) -> dict:
        r = RequestResult()
        _check(lib().dfpr_server_result(self._h, int(rid), ctypes.byref(r)))
        return r.as_dict()
