"""ctypes binding of libtl (include/tl.h): argument marshalling only.

Device buffers are torch tensors on the current HIP device; their raw
pointers and the current stream are handed to the C-ABI.  Every step of the
listing path runs in the library's HIP kernels.  If libtl.so is missing the
import fails: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtl.so")

TL_OK, TL_EINVAL, TL_ENOMEM, TL_ECAPACITY, TL_EHIP, TL_EABORT = range(6)
ALGOS = {"A++": 0, "A+-": 1, "A--": 2}


class TLError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_lib.tl_strerror(code).decode()} ({_lib.tl_last_error().decode()})")
        self.code = code


class Summary(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("hash", ctypes.c_uint64),
                ("work", ctypes.c_uint64), ("scanned", ctypes.c_uint64)]

    def __repr__(self):
        return (f"Summary(count={self.count}, hash=0x{self.hash:016x}, work={self.work}, "
                f"scanned={self.scanned})")


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_batch_jobs", ctypes.c_uint32),
                ("max_batch_edges", ctypes.c_uint64), ("solo_edges", ctypes.c_uint64),
                ("pipeline", ctypes.c_uint32), ("list_threads", ctypes.c_uint32)]


class Job(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint64), ("src", ctypes.c_void_p),
                ("dst", ctypes.c_void_p), ("rank", ctypes.c_void_p), ("algo", ctypes.c_int),
                ("key", ctypes.c_uint64)]


JOB_PENDING = -1


class JobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("count", ctypes.c_uint64), ("hash", ctypes.c_uint64),
                ("work", ctypes.c_uint64), ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64), ("batch_id", ctypes.c_uint64),
                ("batch_jobs", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "submitted", "jobs_done", "batches", "rejected", "cancelled", "split_batches", "reserved",
        "peak_reserved", "pending", "max_batch_jobs_seen", "upload_ns", "orient_ns", "list_ns",
        "resident_hits", "resident_graphs", "resident_bytes", "resident_dropped")]


class ListStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "light_items", "heavy_items", "light_seeds", "heavy_seeds", "heavy_work", "heavy_pivots",
        "heavy_staged", "heavy_triangles", "tasks", "items_bitmap", "items_array", "items_global",
        "items_reverse", "items_hash", "items_bucket", "items_split", "slices", "slices_redone",
        "items_long", "items_short", "items_single", "split_below", "split_below_global", "heavy_task_staged", "split_groups",
        "split_below_groups")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


CHUNK_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p)


class NeighResult(ctypes.Structure):
    _fields_ = [("cpm_start", ctypes.c_uint64), ("cpm", ctypes.c_uint64), ("passes", ctypes.c_uint32),
                ("visits", ctypes.c_uint32), ("moves", ctypes.c_uint64), ("seconds", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(or python -m paper_2203_04774_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.tl_orient.argtypes = [u32, vp, vp, u64, vp, vp, ctypes.POINTER(vp)]
    lib.tl_cost.argtypes = [vp, i32, vp, ctypes.POINTER(u64)]
    lib.tl_list.argtypes = [vp, i32, vp, u64, CHUNK_FN, vp, vp, ctypes.POINTER(Summary)]
    lib.tl_list_range.argtypes = [vp, i32, u32, u32, vp, u64, CHUNK_FN, vp, vp, ctypes.POINTER(Summary)]
    lib.tl_list_count_noalloc.argtypes = [vp, i32, vp, ctypes.POINTER(Summary)]
    lib.tl_csr_size.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u64)]
    lib.tl_csr_copy_to_host.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.tl_csr_free.argtypes = [vp]
    lib.tl_csr_free.restype = None
    lib.tl_set_chunk_triangles.argtypes = [u64]
    lib.tl_set_tuning.argtypes = [ctypes.c_char_p, u64]
    lib.tl_get_tuning.argtypes = [ctypes.c_char_p, ctypes.POINTER(u64)]
    lib.tl_order.argtypes = [vp, i32, vp, vp]
    lib.tl_order.restype = i32
    lib.tl_order_neigh.argtypes = [vp, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32, vp,
                                   ctypes.POINTER(NeighResult), vp]
    lib.tl_order_neigh.restype = i32
    lib.tl_batch_orient.argtypes = [u32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.tl_batch_from_graphs.argtypes = [u32, vp, vp, ctypes.POINTER(vp)]
    lib.tl_batch_list.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.tl_batch_size.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u64)]
    lib.tl_batch_free.argtypes = [vp]
    lib.tl_batch_free.restype = None
    lib.tl_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.tl_server_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(u64)]
    lib.tl_server_poll.argtypes = [vp, u64, ctypes.c_int64, ctypes.POINTER(JobResult)]
    lib.tl_server_cancel.argtypes = [vp, u64]
    lib.tl_server_pause.argtypes = [vp, i32]
    lib.tl_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.tl_server_job_bytes.argtypes = [u32, u64]
    lib.tl_server_job_bytes.restype = u64
    lib.tl_server_destroy.argtypes = [vp]
    lib.tl_server_destroy.restype = None
    for f in ("tl_server_create", "tl_server_submit", "tl_server_poll", "tl_server_cancel", "tl_server_pause",
              "tl_server_get_stats"):
        getattr(lib, f).restype = i32
    lib.tl_last_list_stats.argtypes = [ctypes.POINTER(ListStats)]
    lib.tl_last_list_stats.restype = i32
    lib.tl_release_cached_memory.argtypes = []
    lib.tl_release_cached_memory.restype = i32
    lib.tl_strerror.argtypes = [i32]
    lib.tl_strerror.restype = ctypes.c_char_p
    lib.tl_last_error.restype = ctypes.c_char_p
    for f in ("tl_orient", "tl_cost", "tl_list", "tl_list_range", "tl_csr_size",
              "tl_csr_copy_to_host", "tl_set_chunk_triangles", "tl_set_tuning", "tl_get_tuning",
              "tl_batch_orient", "tl_batch_list", "tl_batch_size"):
        getattr(lib, f).restype = i32
    return lib


_lib = _load()
_NULL_CB = CHUNK_FN()


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t: torch.Tensor | None, what: str):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype not in (torch.int32, torch.uint32):
        raise ValueError(f"{what} must be int32/uint32")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(rc, what):
    if rc != TL_OK:
        raise TLError(rc, what)


class Csr:
    """Oriented graph handle returned by :func:`orient` (owns device memory)."""

    def __init__(self, handle):
        self._h = handle
        n, m = ctypes.c_uint32(), ctypes.c_uint64()
        _check(_lib.tl_csr_size(handle, ctypes.byref(n), ctypes.byref(m)), "tl_csr_size")
        self.n, self.m = int(n.value), int(m.value)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("handle already freed")
        return self._h

    def free(self):
        if self._h is not None:
            _lib.tl_csr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def to_host(self):
        """(off_fwd, adj_fwd, off_bwd, adj_bwd, inv) as numpy arrays."""
        import numpy as np
        fo = np.zeros(self.n + 1, np.uint64)
        bo = np.zeros(self.n + 1, np.uint64)
        fa = np.zeros(max(self.m, 1), np.uint32)
        ba = np.zeros(max(self.m, 1), np.uint32)
        inv = np.zeros(max(self.n, 1), np.uint32)
        _check(_lib.tl_csr_copy_to_host(self.handle, fo.ctypes.data, fa.ctypes.data, bo.ctypes.data,
                                        ba.ctypes.data, inv.ctypes.data), "tl_csr_copy_to_host")
        return fo, fa[:self.m], bo, ba[:self.m], inv[:self.n]


def orient(n: int, src: torch.Tensor, dst: torch.Tensor, rank: torch.Tensor, stream=None) -> Csr:
    """tl_orient: edges (src[i], dst[i]) and rank (device int32 tensors)."""
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in length")
    h = ctypes.c_void_p()
    _check(_lib.tl_orient(n, _dptr(src, "src"), _dptr(dst, "dst"), src.numel(), _dptr(rank, "rank"),
                          _stream_ptr(stream), ctypes.byref(h)), "tl_orient")
    return Csr(h)


ORDERS = {"degree": 0, "split": 1, "core": 2, "check": 3}


def order(g: Csr, kind: str = "degree", out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """tl_order: a new ordering (device int32 rank tensor of g.n entries)
    computed on the device from the oriented graph g."""
    if out is None:
        out = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")[: g.n]
    elif out.numel() != g.n:
        raise ValueError("out must have g.n entries")
    ptr = _dptr(out, "out") if g.n else None
    _check(_lib.tl_order(g.handle, ORDERS[kind], ptr, _stream_ptr(stream)), "tl_order")
    return out


def order_neigh(g: Csr, eps: float = 0.01, max_passes: int = 100, max_visits: int = 0,
                out: torch.Tensor | None = None, stream=None):
    """tl_order_neigh: Neigh (Algorithm 3) from the ordering g is oriented
    by; returns (device int32 rank tensor, NeighResult)."""
    if out is None:
        out = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")[: g.n]
    elif out.numel() != g.n:
        raise ValueError("out must have g.n entries")
    ptr = _dptr(out, "out") if g.n else None
    res = NeighResult()
    _check(_lib.tl_order_neigh(g.handle, float(eps), int(max_passes), int(max_visits), ptr, ctypes.byref(res),
                               _stream_ptr(stream)), "tl_order_neigh")
    return out, res


def cost(g: Csr, algo: str = "A++", stream=None) -> int:
    out = ctypes.c_uint64()
    _check(_lib.tl_cost(g.handle, ALGOS[algo], _stream_ptr(stream), ctypes.byref(out)), "tl_cost")
    return int(out.value)


def list_triangles(g: Csr, algo: str = "A++", out: torch.Tensor | None = None, on_chunk=None,
                   pivot_range=None, stream=None, allow_capacity_error=False) -> Summary:
    """tl_list / tl_list_range.

    out       optional device int32 tensor of shape (cap, 3): receives the
              triangles (original ids, a < b < c)
    on_chunk  optional callable(ptr: int, k: int) -> bool|None; return True
              to stop; receives library-owned device chunks
    """
    s = Summary()
    cap = 0
    if out is not None:
        if out.dim() != 2 or out.shape[1] != 3:
            raise ValueError("out must have shape (cap, 3)")
        cap = out.shape[0]
    cb = _NULL_CB
    if on_chunk is not None:
        def _tramp(ptr, k, user):
            try:
                return 1 if on_chunk(int(ptr), int(k)) else 0
            except Exception:
                return 1
        cb = CHUNK_FN(_tramp)
    optr = _dptr(out, "out") if out is not None else None
    if pivot_range is None:
        rc = _lib.tl_list(g.handle, ALGOS[algo], optr, cap, cb, None, _stream_ptr(stream), ctypes.byref(s))
    else:
        lo, hi = pivot_range
        rc = _lib.tl_list_range(g.handle, ALGOS[algo], lo, hi, optr, cap, cb, None, _stream_ptr(stream),
                                ctypes.byref(s))
    if rc == TL_ECAPACITY and allow_capacity_error:
        return s
    _check(rc, "tl_list")
    return s


def list_count_noalloc(g: Csr, algo: str = "A++", stream=None) -> Summary:
    """tl_list_count_noalloc: count, digest and work with no device
    allocation (scratch from the library's fixed device array)."""
    s = Summary()
    _check(_lib.tl_list_count_noalloc(g.handle, ALGOS[algo], _stream_ptr(stream), ctypes.byref(s)),
           "tl_list_count_noalloc")
    return s


class Batch:
    """Handle of a batch of graphs returned by :func:`batch_orient`."""

    def __init__(self, handle):
        self._h = handle
        k, n, m = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        _check(_lib.tl_batch_size(handle, ctypes.byref(k), ctypes.byref(n), ctypes.byref(m)), "tl_batch_size")
        self.k, self.n, self.m = int(k.value), int(n.value), int(m.value)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("handle already freed")
        return self._h

    def list(self, algo: str = "A++", use_graph: bool = True, out_dev: torch.Tensor | None = None,
             stream=None):
        """tl_batch_list: returns a (k, 3) uint64 numpy array of per-graph
        (count, digest, work); out_dev (device int64 tensor of 3k entries)
        also receives the table on the stream when given."""
        import numpy as np
        table = np.zeros(3 * self.k, np.uint64)
        dptr = None
        if out_dev is not None:
            if not out_dev.is_cuda or out_dev.dtype not in (torch.int64, torch.uint64) \
                    or out_dev.numel() != 3 * self.k or not out_dev.is_contiguous():
                raise ValueError("out_dev must be a contiguous device int64 tensor of 3k entries")
            dptr = ctypes.c_void_p(out_dev.data_ptr())
        _check(_lib.tl_batch_list(self.handle, ALGOS[algo], 1 if use_graph else 0, table.ctypes.data, dptr,
                                  _stream_ptr(stream)), "tl_batch_list")
        return table.reshape(self.k, 3)

    def free(self):
        if self._h is not None:
            _lib.tl_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def batch_orient(n, m, src: torch.Tensor, dst: torch.Tensor, rank: torch.Tensor, stream=None) -> Batch:
    """tl_batch_orient: n, m per-graph sizes (host sequences); src/dst the
    graphs' edges back to back (local ids), rank their orderings back to
    back (device int32 tensors)."""
    import numpy as np
    n_h = np.ascontiguousarray(n, np.uint32)
    m_h = np.ascontiguousarray(m, np.uint64)
    if n_h.shape != m_h.shape or n_h.ndim != 1 or len(n_h) == 0:
        raise ValueError("n and m must be 1-d of the same non-zero length")
    if src.numel() != int(m_h.sum()) or dst.numel() != src.numel():
        raise ValueError("src/dst length differs from sum(m)")
    if rank.numel() != int(n_h.sum()):
        raise ValueError("rank length differs from sum(n)")
    h = ctypes.c_void_p()
    _check(_lib.tl_batch_orient(len(n_h), n_h.ctypes.data, m_h.ctypes.data, _dptr(src, "src"), _dptr(dst, "dst"),
                                _dptr(rank, "rank"), _stream_ptr(stream), ctypes.byref(h)), "tl_batch_orient")
    return Batch(h)


def batch_from_graphs(graphs, stream=None) -> Batch:
    """tl_batch_from_graphs: a batch of oriented graph handles (Csr), whose
    union is built by copying their arrays; the handles stay the caller's."""
    if len(graphs) == 0:
        raise ValueError("no graphs")
    arr = (ctypes.c_void_p * len(graphs))(*[g.handle for g in graphs])
    h = ctypes.c_void_p()
    _check(_lib.tl_batch_from_graphs(len(graphs), ctypes.cast(arr, ctypes.c_void_p), _stream_ptr(stream),
                                     ctypes.byref(h)), "tl_batch_from_graphs")
    return Batch(h)


class Server:
    """tl_server_*: a listing server on the current device.  Job arrays are
    host numpy uint32 arrays; they are kept referenced here until the job's
    final result has been polled."""

    def __init__(self, hbm_budget: int, max_batch_jobs: int = 0, max_batch_edges: int = 0,
                 solo_edges: int = 0, pipeline: bool = True, list_threads: int = 0):
        cfg = ServerConfig(int(hbm_budget), int(max_batch_jobs), int(max_batch_edges), int(solo_edges),
                           1 if pipeline else 0, int(list_threads))
        h = ctypes.c_void_p()
        _check(_lib.tl_server_create(ctypes.byref(cfg), ctypes.byref(h)), "tl_server_create")
        self._h = h
        self._keep = {}

    def submit(self, n, src, dst, rank, algo: str = "A++", key: int = 0) -> int:
        """key != 0 names the graph and ordering: it is kept resident on the
        device and later jobs with the same key are listed from it."""
        import numpy as np
        s = np.ascontiguousarray(src, np.uint32)
        d = np.ascontiguousarray(dst, np.uint32)
        r = np.ascontiguousarray(rank, np.uint32)
        if s.shape != d.shape or len(r) != n:
            raise ValueError("src/dst lengths differ or rank length != n")
        job = Job(int(n), len(s), s.ctypes.data if len(s) else None, d.ctypes.data if len(d) else None,
                  r.ctypes.data if len(r) else None, ALGOS[algo], int(key))
        jid = ctypes.c_uint64()
        _check(_lib.tl_server_submit(self._h, ctypes.byref(job), ctypes.byref(jid)), "tl_server_submit")
        self._keep[int(jid.value)] = (s, d, r)
        return int(jid.value)

    def poll(self, jid: int, wait_us: int = -1) -> JobResult:
        out = JobResult()
        _check(_lib.tl_server_poll(self._h, jid, wait_us, ctypes.byref(out)), "tl_server_poll")
        if out.status != JOB_PENDING:
            self._keep.pop(jid, None)
        return out

    def cancel(self, jid: int) -> int:
        """TL_OK if the job was cancelled, TL_EINVAL if it was admitted already."""
        return int(_lib.tl_server_cancel(self._h, jid))

    def pause(self, paused: bool = True):
        _check(_lib.tl_server_pause(self._h, 1 if paused else 0), "tl_server_pause")

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.tl_server_get_stats(self._h, ctypes.byref(st)), "tl_server_get_stats")
        return {k: int(getattr(st, k)) for k, _ in ServerStats._fields_}

    @staticmethod
    def job_bytes(n: int, m: int) -> int:
        """The device footprint admission charges for a job (tl_server_job_bytes)."""
        return int(_lib.tl_server_job_bytes(int(n), int(m)))

    def close(self):
        if self._h is not None:
            _lib.tl_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release_cached_memory():
    """tl_release_cached_memory: hand cached device blocks back to the driver."""
    _check(_lib.tl_release_cached_memory(), "tl_release_cached_memory")


def set_chunk_triangles(k: int):
    _check(_lib.tl_set_chunk_triangles(k), "tl_set_chunk_triangles")


def last_list_stats() -> dict:
    """Work split and slice counts of this thread's most recent listing
    (tl_last_list_stats)."""
    st = ListStats()
    _check(_lib.tl_last_list_stats(ctypes.byref(st)), "tl_last_list_stats")
    return st.as_dict()


def set_tuning(key: str, value: int):
    """tl_set_tuning: launch parameters (results never depend on them)."""
    _check(_lib.tl_set_tuning(key.encode(), int(value)), f"tl_set_tuning({key})")


def get_tuning(key: str) -> int:
    v = ctypes.c_uint64()
    _check(_lib.tl_get_tuning(key.encode(), ctypes.byref(v)), f"tl_get_tuning({key})")
    return int(v.value)


def raw_lib():
    """The loaded ctypes library (for callers that marshal pointers themselves)."""
    return _lib
