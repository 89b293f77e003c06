"""CPU oracle for triangle listing under a vertex ordering -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never does.  The C source, ``oracle.c``, is a plain single-threaded
statement of what Lecuyer et al., "Tailored vertex ordering for faster
triangle listing in large graphs", list and count: every triangle once,
found from the definition (an edge plus a vertex adjacent to both ends,
under the orientation by the ordering), grouped by the pivot role that
Algorithm 1 (A++), Algorithm 2 (A+-) or the A-- variant gives one of its
vertices; the work of Property 1 and Definition 1's costs; and the paper's
orderings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

APP, APM, AMM = 0, 1, 2
ALGOS = {"A++": APP, "A+-": APM, "A--": AMM}

u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile oracle.c (plain -O2, no vectorisation flags, single thread)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp,
                           os.path.join(_HERE, "oracle.c")])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    lib.orc_list.restype = ctypes.c_int
    lib.orc_list.argtypes = [u32, u64, u32p, u32p, u32p, ctypes.c_int, u32, u32, vp, u64, u64p]
    lib.orc_cost.restype = ctypes.c_int
    lib.orc_cost.argtypes = [u32, u64, u32p, u32p, u32p, u64p]
    lib.orc_oriented_csr.restype = ctypes.c_int
    lib.orc_oriented_csr.argtypes = [u32, u64, u32p, u32p, u32p, u64p, u32p, u64p, u32p, u32p]
    lib.orc_list_ranges.restype = ctypes.c_int
    lib.orc_list_ranges.argtypes = [u32, u64, u32p, u32p, u32p, ctypes.c_int, u32, u32p, u32p, vp, vp, u64p]
    lib.orc_graph_new.restype = vp
    lib.orc_graph_new.argtypes = [u32, u64, u32p, u32p, u32p, ctypes.POINTER(ctypes.c_int)]
    lib.orc_graph_list.restype = ctypes.c_int
    lib.orc_graph_list.argtypes = [vp, ctypes.c_int, u32, u32, vp, u64, u64p]
    lib.orc_graph_bin.restype = ctypes.c_int
    lib.orc_graph_bin.argtypes = [vp, ctypes.c_int, u32, u32, u32, u32p, u64p]
    lib.orc_graph_work.restype = u64
    lib.orc_graph_work.argtypes = [vp, ctypes.c_int, u32, u32]
    lib.orc_graph_m.restype = u64
    lib.orc_graph_m.argtypes = [vp]
    lib.orc_graph_free.restype = None
    lib.orc_graph_free.argtypes = [vp]
    lib.orc_triangle_hash.restype = u64
    lib.orc_triangle_hash.argtypes = [u32, u32, u32]
    lib.orc_mix64.restype = u64
    lib.orc_mix64.argtypes = [u64]
    for f in ("orc_degree_order", "orc_split_order", "orc_coreness", "orc_core_order"):
        getattr(lib, f).restype = ctypes.c_int
        getattr(lib, f).argtypes = [u32, u64, u32p, u32p, u32p]
    lib.orc_neigh_order.restype = ctypes.c_int
    lib.orc_neigh_order.argtypes = [u32, u64, u32p, u32p, u32p, ctypes.c_double, u32, u32, u32p,
                                    ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32)]
    lib.orc_check_order.restype = ctypes.c_int
    lib.orc_check_order.argtypes = [u32, u64, u32p, u32p, u32p, ctypes.POINTER(ctypes.c_uint8)]
    _lib = lib
    return lib


class OracleError(ValueError):
    pass


def _check(rc):
    if rc == -1:
        raise OracleError("invalid input (vertex id >= n or rank not a permutation)")
    if rc == -2:
        raise MemoryError("oracle: out of host memory")


@dataclass
class Listing:
    count: int
    hash: int
    work: int
    m: int
    triangles: np.ndarray | None  # (count, 3) uint32, canonical, discovery order

    def sorted_triangles(self) -> np.ndarray:
        t = self.triangles
        if t is None or len(t) == 0:
            return np.zeros((0, 3), np.uint32)
        order = np.lexsort((t[:, 2], t[:, 1], t[:, 0]))
        return t[order]


def _arrs(src, dst, rank):
    return (np.ascontiguousarray(src, np.uint32), np.ascontiguousarray(dst, np.uint32),
            np.ascontiguousarray(rank, np.uint32))


def list_triangles(n, src, dst, rank, algo="A++", pivot_lo=0, pivot_hi=None,
                   want_triangles=True, cap=None) -> Listing:
    """The triangles whose pivot for the form -- A++ (Algorithm 1): the
    vertex of largest rank; A+- (Algorithm 2): smallest; A--: middle -- has
    rank in [pivot_lo, pivot_hi), with the paper's work over those pivots."""
    lib = _load()
    s, d, r = _arrs(src, dst, rank)
    if pivot_hi is None:
        pivot_hi = n
    out = np.zeros(4, np.uint64)
    tri = None
    if want_triangles:
        if cap is None:
            # first pass for the size, then list
            _check(lib.orc_list(n, len(s), s, d, r, ALGOS[algo], pivot_lo, pivot_hi, None, 0, out))
            cap = int(out[0])
        tri = np.zeros((max(cap, 1), 3), np.uint32)
        _check(lib.orc_list(n, len(s), s, d, r, ALGOS[algo], pivot_lo, pivot_hi,
                            tri.ctypes.data, cap, out))
        tri = tri[:min(cap, int(out[0]))]
    else:
        _check(lib.orc_list(n, len(s), s, d, r, ALGOS[algo], pivot_lo, pivot_hi, None, 0, out))
    return Listing(int(out[0]), int(out[1]), int(out[2]), int(out[3]), tri)


def list_ranges(n, src, dst, rank, algo, ranges, caps=None):
    """list_triangles over several pivot ranges with one graph build.

    ranges: list of (lo, hi); caps: None (counts only) or a list of
    capacities, in which case each range's triangles are returned too.
    Returns a list of Listing."""
    lib = _load()
    s, d, r = _arrs(src, dst, rank)
    nr = len(ranges)
    lo = np.ascontiguousarray([a for a, _ in ranges], np.uint32)
    hi = np.ascontiguousarray([b for _, b in ranges], np.uint32)
    out = np.zeros(4 * nr, np.uint64)
    bufs, ptrs, capa = None, None, None
    if caps is not None:
        bufs = [np.zeros((max(int(c), 1), 3), np.uint32) for c in caps]
        ptrs = (ctypes.c_void_p * nr)(*[b.ctypes.data for b in bufs])
        capa = np.ascontiguousarray(caps, np.uint64)
    _check(lib.orc_list_ranges(n, len(s), s, d, r, ALGOS[algo], nr, lo, hi,
                               ctypes.cast(ptrs, ctypes.c_void_p) if ptrs is not None else None,
                               capa.ctypes.data if capa is not None else None, out))
    res = []
    for i in range(nr):
        c = int(out[4 * i])
        tri = bufs[i][:min(c, int(caps[i]))] if bufs is not None else None
        res.append(Listing(c, int(out[4 * i + 1]), int(out[4 * i + 2]), int(out[4 * i + 3]), tri))
    return res


class BuiltGraph:
    """A graph built once by the oracle, listed over many pivot ranges."""

    def __init__(self, n, src, dst, rank):
        lib = _load()
        s, d, r = _arrs(src, dst, rank)
        rc = ctypes.c_int(0)
        self.n = n
        self._h = lib.orc_graph_new(n, len(s), s, d, r, ctypes.byref(rc))
        _check(rc.value)

    def list(self, algo="A++", lo=0, hi=None, cap=0) -> Listing:
        lib = _load()
        hi = self.n if hi is None else hi
        out = np.zeros(4, np.uint64)
        tri = np.zeros((max(cap, 1), 3), np.uint32) if cap else None
        _check(lib.orc_graph_list(self._h, ALGOS[algo], lo, hi, tri.ctypes.data if cap else None, cap, out))
        c = int(out[0])
        return Listing(c, int(out[1]), int(out[2]), int(out[3]), tri[:min(c, cap)] if cap else None)

    def work(self, algo="A++", lo=0, hi=None) -> int:
        """The paper's work (Property 1) over pivots of rank in [lo, hi)."""
        hi = self.n if hi is None else hi
        return int(_load().orc_graph_work(self._h, ALGOS[algo], lo, hi))

    @property
    def m(self) -> int:
        return int(_load().orc_graph_m(self._h))

    def bin(self, algo, cuts, src_lo=0, src_hi=None) -> np.ndarray:
        """(count, hash) per bin [cuts[i], cuts[i+1]) of pivot ranks for the
        form, over the triangles whose smallest rank lies in [src_lo,
        src_hi); summing over a partition of the source ranks gives every
        bin for the whole graph.  Returns a (len(cuts)-1, 2) uint64 array."""
        lib = _load()
        hi = self.n if src_hi is None else src_hi
        c = np.ascontiguousarray(cuts, np.uint32)
        out = np.zeros(2 * (len(c) - 1), np.uint64)
        _check(lib.orc_graph_bin(self._h, ALGOS[algo], src_lo, hi, len(c) - 1, c, out))
        return out.reshape(-1, 2)

    def close(self):
        if self._h:
            _load().orc_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Cost:
    cpp: int   # C++ = sum d+ d+
    cpm: int   # C+- = sum d+ d-
    cmm: int   # sum d- d-
    m: int
    sum_dplus: int
    sum_dminus: int

    def for_algo(self, algo: str) -> int:
        return {"A++": self.cpp, "A+-": self.cpm, "A--": self.cmm}[algo]


def cost(n, src, dst, rank) -> Cost:
    lib = _load()
    s, d, r = _arrs(src, dst, rank)
    out = np.zeros(6, np.uint64)
    _check(lib.orc_cost(n, len(s), s, d, r, out))
    return Cost(*[int(x) for x in out])


def oriented_csr(n, src, dst, rank):
    """(fwd_off, fwd_adj, bwd_off, bwd_adj, inv) in rank space."""
    lib = _load()
    s, d, r = _arrs(src, dst, rank)
    c = cost(n, s, d, r)
    fo = np.zeros(n + 1, np.uint64)
    bo = np.zeros(n + 1, np.uint64)
    fa = np.zeros(max(c.m, 1), np.uint32)
    ba = np.zeros(max(c.m, 1), np.uint32)
    inv = np.zeros(max(n, 1), np.uint32)
    _check(lib.orc_oriented_csr(n, len(s), s, d, r, fo, fa, bo, ba, inv))
    return fo, fa[:c.m], bo, ba[:c.m], inv[:n]


def degree_order(n, src, dst) -> np.ndarray:
    """Degree ordering of the simple graph (Section 2.2): non-decreasing
    degree, ties by id; returns rank (rank[u] = position of u)."""
    lib = _load()
    s = np.ascontiguousarray(src, np.uint32)
    d = np.ascontiguousarray(dst, np.uint32)
    rank = np.zeros(max(n, 1), np.uint32)
    _check(lib.orc_degree_order(n, len(s), s, d, rank))
    return rank[:n]


def split_order(n, src, dst) -> np.ndarray:
    """Split ordering (Section 3.3.3) built from the non-increasing degree
    ordering (the degree ordering read backwards); returns rank."""
    lib = _load()
    s = np.ascontiguousarray(src, np.uint32)
    d = np.ascontiguousarray(dst, np.uint32)
    rank = np.zeros(max(n, 1), np.uint32)
    _check(lib.orc_split_order(n, len(s), s, d, rank))
    return rank[:n]


def coreness(n, src, dst) -> np.ndarray:
    """Coreness of every vertex of the simple graph (Section 1.3)."""
    lib = _load()
    s = np.ascontiguousarray(src, np.uint32)
    d = np.ascontiguousarray(dst, np.uint32)
    core = np.zeros(max(n, 1), np.uint32)
    _check(lib.orc_coreness(n, len(s), s, d, core))
    return core[:n]


def core_order(n, src, dst) -> np.ndarray:
    """Core ordering: non-decreasing coreness, ties by id; returns rank."""
    lib = _load()
    s = np.ascontiguousarray(src, np.uint32)
    d = np.ascontiguousarray(dst, np.uint32)
    rank = np.zeros(max(n, 1), np.uint32)
    _check(lib.orc_core_order(n, len(s), s, d, rank))
    return rank[:n]


def check_order(n, src, dst, with_side=False):
    """Check ordering (Section 3.3.2): vertices by non-increasing degree
    (the degree ordering read backwards), each put right after the
    beginning block or right before the end block, whichever gives it the
    smaller C+- share (ties: beginning).  Returns rank, or (rank, side)
    with side[u] = 0 for beginning, 1 for end."""
    lib = _load()
    s = np.ascontiguousarray(src, np.uint32)
    d = np.ascontiguousarray(dst, np.uint32)
    rank = np.zeros(max(n, 1), np.uint32)
    side = np.zeros(max(n, 1), np.uint8)
    _check(lib.orc_check_order(n, len(s), s, d, rank, side.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return (rank[:n], side[:n]) if with_side else rank[:n]


def neigh_order(n, src, dst, rank_in, eps=0.01, max_passes=100, max_visits=0):
    """Neigh (Algorithm 3) from the ordering rank_in; returns (rank, C+-,
    passes).  Every candidate place is priced from scratch: small graphs
    only.  max_visits > 0 stops after that many vertex visits."""
    lib = _load()
    s = np.ascontiguousarray(src, np.uint32)
    d = np.ascontiguousarray(dst, np.uint32)
    r0 = np.ascontiguousarray(rank_in, np.uint32)
    rank = np.zeros(max(n, 1), np.uint32)
    c = ctypes.c_uint64(0)
    p = ctypes.c_uint32(0)
    _check(lib.orc_neigh_order(n, len(s), s, d, r0, float(eps), max_passes, max_visits, rank, ctypes.byref(c),
                               ctypes.byref(p)))
    return rank[:n], int(c.value), int(p.value)


def triangle_hash(a: int, b: int, c: int) -> int:
    return int(_load().orc_triangle_hash(a, b, c))


def mix64(z: int) -> int:
    return int(_load().orc_mix64(z))


def hash_of(triangles) -> int:
    """Wrapping 64-bit sum of the per-triangle digest (canonical input)."""
    h = 0
    for a, b, c in np.asarray(triangles).reshape(-1, 3):
        h = (h + triangle_hash(int(a), int(b), int(c))) & 0xFFFFFFFFFFFFFFFF
    return h
