"""Seeded synthetic inputs: undirected graphs and vertex orderings.

This module is shared by the oracle-side tests and the GPU path, and holds
none of the listing method's arithmetic: it only produces edge lists and
rank arrays.  Large generators run in C (``gen.c``, built with gcc/OpenMP);
the closed-form fixture graphs are plain numpy.

Conventions
-----------
* A graph is ``(n, src, dst)``: ``src``/``dst`` are ``uint32`` numpy arrays
  with ``src[i] < dst[i]`` (each undirected edge once, no loops, sorted).
* An ordering is ``rank``: a ``uint32`` permutation of ``[0, n)``; vertex ``u``
  gets index ``rank[u]`` (the paper's pi_u, 0-based; Section 1.3).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_lib = None

u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile gen.c into libgraphgen.so (always recompiles)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    u64, u32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
    lib.gg_rmat.restype = u64
    lib.gg_rmat.argtypes = [ctypes.c_int, u64, dbl, dbl, dbl, u64, u32p, u32p]
    lib.gg_chung_lu.restype = u64
    lib.gg_chung_lu.argtypes = [u32, dbl, dbl, u64, u64, u32p, u32p]
    lib.gg_simplify.restype = u64
    lib.gg_simplify.argtypes = [u32, u64, u32p, u32p, u32p, u32p]
    lib.gg_degrees.restype = None
    lib.gg_degrees.argtypes = [u32, u64, u32p, u32p, u32p]
    lib.gg_degree_order.restype = None
    lib.gg_degree_order.argtypes = [u32, u32p, u32p]
    lib.gg_random_order.restype = None
    lib.gg_random_order.argtypes = [u32, u64, u32p]
    lib.gg_core_order.restype = None
    lib.gg_core_order.argtypes = [u32, u64, u32p, u32p, u32p, ctypes.c_void_p]
    lib.gg_num_threads.restype = ctypes.c_int
    f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
    u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
    lib.gg_chung_lu_batch.restype = None
    lib.gg_chung_lu_batch.argtypes = [u32, u32p, f64p, u64p, u64p, dbl, u64p, u32p, u32p, u32p]
    _lib = lib
    return lib


class Graph:
    """A simple undirected graph: n vertices, edges (src[i], dst[i]), src < dst."""

    __slots__ = ("n", "src", "dst", "name")

    def __init__(self, n, src, dst, name=""):
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.uint32)
        self.dst = np.ascontiguousarray(dst, dtype=np.uint32)
        self.name = name

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def __repr__(self):
        return f"Graph({self.name!r}, n={self.n}, m={self.m})"


# ------------------------------------------------------------------ graphs

def rmat(scale: int, edge_factor: int = 8, a=0.57, b=0.19, c=0.19, seed: int = 1) -> Graph:
    """RMAT over 2^scale vertices, edge_factor * 2^scale samples, symmetrised,
    loops and duplicates dropped (no label scrambling)."""
    lib = _load()
    samples = edge_factor << scale
    src = np.empty(samples, np.uint32)
    dst = np.empty(samples, np.uint32)
    m = lib.gg_rmat(scale, samples, a, b, c, seed, src, dst)
    # prefix views, not copies: at scale 26 a copy would cost another 8 GB
    return Graph(1 << scale, src[:m], dst[:m], f"rmat{scale}-ef{edge_factor}-s{seed}")


def chung_lu(n: int, gamma: float = 2.1, mean_degree: float = 20.0, seed: int = 1,
             i0: float = 10.0) -> Graph:
    """Chung-Lu power-law graph: round(n * mean_degree / 2) endpoint pairs,
    each endpoint drawn with probability ~ (i + i0)^(-1/(gamma-1)); loops and
    duplicates dropped."""
    lib = _load()
    samples = int(round(n * mean_degree / 2.0))
    src = np.empty(max(samples, 1), np.uint32)
    dst = np.empty(max(samples, 1), np.uint32)
    m = lib.gg_chung_lu(n, gamma, i0, samples, seed, src, dst) if samples else 0
    return Graph(n, src[:m], dst[:m], f"chunglu-n{n}-g{gamma}-k{mean_degree}-s{seed}")


def simplify(n: int, src, dst, name="") -> Graph:
    """Drop loops and duplicate undirected pairs from an arbitrary edge list."""
    lib = _load()
    s = np.ascontiguousarray(src, np.uint32)
    d = np.ascontiguousarray(dst, np.uint32)
    os_ = np.empty(max(len(s), 1), np.uint32)
    od = np.empty(max(len(s), 1), np.uint32)
    m = lib.gg_simplify(n, len(s), s, d, os_, od) if len(s) else 0
    return Graph(n, os_[:m].copy(), od[:m].copy(), name)


# --------------------------------------------------------------- orderings

def degrees(g: Graph) -> np.ndarray:
    lib = _load()
    deg = np.empty(max(g.n, 1), np.uint32)
    if g.n:
        lib.gg_degrees(g.n, g.m, g.src, g.dst, deg)
    return deg[:g.n]


def degree_order(g: Graph) -> np.ndarray:
    """Non-decreasing degree, ties by vertex id (rank = sorted position)."""
    lib = _load()
    deg = degrees(g)
    rank = np.empty(max(g.n, 1), np.uint32)
    if g.n:
        lib.gg_degree_order(g.n, np.ascontiguousarray(deg), rank)
    return rank[:g.n]


def random_order(n: int, seed: int = 1) -> np.ndarray:
    """Uniform random permutation from the counter-based stream."""
    lib = _load()
    rank = np.empty(max(n, 1), np.uint32)
    if n:
        lib.gg_random_order(n, seed, rank)
    return rank[:n]


def core_order(g: Graph, return_core: bool = False):
    """Degeneracy order: min-current-degree peeling, smallest id first."""
    lib = _load()
    rank = np.empty(max(g.n, 1), np.uint32)
    core = np.empty(max(g.n, 1), np.uint32)
    if g.n:
        lib.gg_core_order(g.n, g.m, g.src, g.dst, rank, core.ctypes.data)
    if return_core:
        return rank[:g.n], core[:g.n]
    return rank[:g.n]


def ordering(g: Graph, kind: str, seed: int = 1) -> np.ndarray:
    if kind == "degree":
        return degree_order(g)
    if kind == "core":
        return core_order(g)
    if kind == "random":
        return random_order(g.n, seed)
    if kind == "identity":
        return np.arange(g.n, dtype=np.uint32)
    raise ValueError(f"unknown ordering {kind!r}")


# ------------------------------------------------- workload recipes

def config_rmat12(seed: int = 1) -> Graph:
    """RMAT scale 12, edge factor 8, a/b/c/d = .57/.19/.19/.05."""
    return rmat(12, 8, seed=seed)


def config_chunglu20(seed: int = 1) -> Graph:
    """Chung-Lu n = 2^20, gamma 2.1, mean degree 20."""
    return chung_lu(1 << 20, 2.1, 20.0, seed=seed)


def config_rmat26(seed: int = 1) -> Graph:
    """RMAT scale 26, edge factor 16, a/b/c/d = .57/.19/.19/.05."""
    return rmat(26, 16, seed=seed)


def batch_graph_params(i: int, base_seed: int = 1000):
    """Parameters of graph i of the batched workload: n log-uniform in
    [100, 50000], gamma uniform in [2.0, 2.8], mean degree uniform in [8, 40]."""
    rs = np.random.Generator(np.random.PCG64(base_seed + i))
    n = int(math.floor(math.exp(rs.uniform(math.log(100), math.log(50000)))))
    gamma = float(rs.uniform(2.0, 2.8))
    k = float(rs.uniform(8.0, 40.0))
    return n, gamma, k, base_seed + i


def batch_graph(i: int, base_seed: int = 1000) -> Graph:
    n, gamma, k, seed = batch_graph_params(i, base_seed)
    return chung_lu(n, gamma, k, seed=seed)


def serve_job_params(j: int, base_seed: int = 5000) -> dict:
    """Job j of the serving workload: RMAT or Chung-Lu (equally likely), a
    target edge count log-uniform in [10^3, 10^7], degree or core order
    (equally likely); Chung-Lu exponent uniform in [2.0, 2.8]."""
    rs = np.random.Generator(np.random.PCG64(base_seed + j))
    kind = "rmat" if rs.random() < 0.5 else "chunglu"
    m = int(math.floor(math.exp(rs.uniform(math.log(1e3), math.log(1e7)))))
    order = "degree" if rs.random() < 0.5 else "core"
    gamma = float(rs.uniform(2.0, 2.8))
    return dict(j=j, kind=kind, m_target=m, order=order, gamma=gamma, seed=base_seed + j)


def serve_job(j: int, base_seed: int = 5000):
    """(graph, rank, params) of serving job j: RMAT with scale
    ceil(log2(m/8)) and edge factor 8, or Chung-Lu with n = m/10 and mean
    degree 20."""
    p = serve_job_params(j, base_seed)
    if p["kind"] == "rmat":
        scale = max(1, math.ceil(math.log2(p["m_target"] / 8)))
        g = rmat(scale, 8, seed=p["seed"])
    else:
        g = chung_lu(max(p["m_target"] // 10, 2), p["gamma"], 20.0, seed=p["seed"])
    return g, ordering(g, p["order"]), p


class GraphBatch:
    """k graphs stored back to back: graph i has n[i] vertices, its edges
    (local ids) at [ebase[i], ebase[i+1]) of src/dst and its ordering at
    [vbase[i], vbase[i+1]) of rank."""

    def __init__(self, n, ebase, src, dst, rank, first=0, base_seed=1000):
        self.n = np.ascontiguousarray(n, np.uint32)
        self.ebase = np.ascontiguousarray(ebase, np.uint64)
        self.vbase = np.zeros(len(self.n) + 1, np.uint64)
        np.cumsum(self.n, out=self.vbase[1:])
        self.src, self.dst, self.rank = src, dst, rank
        self.first, self.base_seed = first, base_seed

    @property
    def k(self) -> int:
        return len(self.n)

    @property
    def m(self) -> np.ndarray:
        return np.diff(self.ebase)

    def graph(self, i) -> Graph:
        a, b = int(self.ebase[i]), int(self.ebase[i + 1])
        return Graph(int(self.n[i]), self.src[a:b], self.dst[a:b], f"batch{self.first + i}")

    def ranks(self, i) -> np.ndarray:
        return self.rank[int(self.vbase[i]):int(self.vbase[i + 1])]


def batch(k: int, first: int = 0, base_seed: int = 1000) -> GraphBatch:
    """Graphs first .. first+k-1 of the batched workload (each equal to
    batch_graph(i)) with their degree orders, generated in parallel."""
    lib = _load()
    params = [batch_graph_params(first + i, base_seed) for i in range(k)]
    n = np.array([p[0] for p in params], np.uint32)
    gamma = np.array([p[1] for p in params], np.float64)
    samples = np.array([int(round(p[0] * p[2] / 2.0)) for p in params], np.uint64)
    seeds = np.array([p[3] for p in params], np.uint64)
    total = int(samples.sum())
    src = np.empty(max(total, 1), np.uint32)
    dst = np.empty(max(total, 1), np.uint32)
    rank = np.empty(max(int(n.sum()), 1), np.uint32)
    ebase = np.empty(k + 1, np.uint64)
    lib.gg_chung_lu_batch(k, n, gamma, samples, seeds, 10.0, ebase, src, dst, rank)
    m = int(ebase[-1])
    return GraphBatch(n, ebase, src[:m], dst[:m], rank[:int(n.sum())], first, base_seed)


def num_threads() -> int:
    return int(_load().gg_num_threads())
