"""GPU orderings (tl_order) against the oracle's: the degree ordering,
Split (Section 3.3.3), the core ordering (Section 1.3) and Check (Section
3.3.2), and the full listing with the ordering computed on the device; the
library's Neigh (Algorithm 3, run on the host) against the oracle's."""
import numpy as np
import pytest

import graphgen
import graphs as G
import oracle
from gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_04774_amd as tl
    return tl


def gpu_order(tl, n, s, d, kind, start_rank=None):
    r0 = np.arange(n, dtype=np.uint32) if start_rank is None else start_rank
    g = tl.orient(n, dev(s), dev(d), dev(r0))
    try:
        return tl.order(g, kind).cpu().numpy().view(np.uint32)
    finally:
        g.free()


def test_split_worked_example(tl):
    n, s, d, orders, names = G.fig2()
    deg = gpu_order(tl, n, s, d, "degree")
    assert [int(u) for u in np.argsort(deg)][::-1] == orders[3][0]  # (e,b,g,a,f,d,c)
    split = gpu_order(tl, n, s, d, "split")
    assert [int(u) for u in np.argsort(split)] == orders[4][0]      # (e,g,f,c,d,a,b)


@pytest.mark.parametrize("seed", range(6))
def test_orders_match_oracle_with_noisy_input(tl, seed):
    rs = np.random.default_rng(seed)
    n = int(rs.integers(50, 3000))
    s = rs.integers(0, n, 6 * n).astype(np.uint32)
    d = rs.integers(0, n, 6 * n).astype(np.uint32)  # loops and repeats included
    start = rs.permutation(n).astype(np.uint32)      # any orientation gives the same degrees
    assert np.array_equal(gpu_order(tl, n, s, d, "degree", start), oracle.degree_order(n, s, d))
    assert np.array_equal(gpu_order(tl, n, s, d, "split", start), oracle.split_order(n, s, d))
    assert np.array_equal(gpu_order(tl, n, s, d, "core", start), oracle.core_order(n, s, d))
    assert np.array_equal(gpu_order(tl, n, s, d, "check", start), oracle.check_order(n, s, d))


@pytest.mark.parametrize("which", ["rmat12", "chunglu20"])
def test_orders_match_oracle_on_workloads(tl, which):
    g = graphgen.config_rmat12() if which == "rmat12" else graphgen.config_chunglu20()
    assert np.array_equal(gpu_order(tl, g.n, g.src, g.dst, "degree"), oracle.degree_order(g.n, g.src, g.dst))
    assert np.array_equal(gpu_order(tl, g.n, g.src, g.dst, "split"), oracle.split_order(g.n, g.src, g.dst))
    assert np.array_equal(gpu_order(tl, g.n, g.src, g.dst, "core"), oracle.core_order(g.n, g.src, g.dst))
    assert np.array_equal(gpu_order(tl, g.n, g.src, g.dst, "check"), oracle.check_order(g.n, g.src, g.dst))


def test_check_worked_example(tl):
    """Check on the Figure 2 graph: (e,g,a,f,d,c,b), worked by hand."""
    n, s, d, orders, names = G.fig2()
    r = gpu_order(tl, n, s, d, "check")
    assert [names[int(u)] for u in np.argsort(r)] == list("egafdcb")


def test_check_shapes(tl):
    for (n, s, d) in [G.complete(9), G.wheel(12), G.grid(5, 7), G.star(10), G.cycle(13),
                      G.complete_bipartite(5, 8), (6, np.arange(5, dtype=np.uint32), np.arange(1, 6, dtype=np.uint32))]:
        assert np.array_equal(gpu_order(tl, n, s, d, "check"), oracle.check_order(n, s, d))


def test_core_closed_forms(tl):
    for (n, s, d) in [G.complete(9), G.wheel(12), G.grid(5, 7), G.star(10), G.cycle(13)]:
        assert np.array_equal(gpu_order(tl, n, s, d, "core"), oracle.core_order(n, s, d))


def test_small_and_empty(tl):
    for n in (1, 2):
        s = np.zeros(0, np.uint32)
        assert np.array_equal(gpu_order(tl, n, s, s, "degree"), np.arange(n, dtype=np.uint32))
        assert np.array_equal(gpu_order(tl, n, s, s, "split"), oracle.split_order(n, s, s))
        assert np.array_equal(gpu_order(tl, n, s, s, "core"), np.arange(n, dtype=np.uint32))
        assert np.array_equal(gpu_order(tl, n, s, s, "check"), oracle.check_order(n, s, s))


@pytest.mark.parametrize("kind,algo", [("split", "A+-"), ("degree", "A++"), ("core", "A+-"), ("check", "A+-")])
def test_full_listing_on_device(tl, kind, algo):
    """Edges -> orientation by id -> ordering on the device -> orientation
    by that ordering -> listing; equal to the oracle under the oracle's
    ordering."""
    g = graphgen.config_rmat12(seed=2)
    g0 = tl.orient(g.n, dev(g.src), dev(g.dst), dev(np.arange(g.n, dtype=np.uint32)))
    rank = tl.order(g0, kind)
    g0.free()
    g1 = tl.orient(g.n, dev(g.src), dev(g.dst), rank)
    try:
        got = tl.list_triangles(g1, algo)
        c = tl.cost(g1, algo)
    finally:
        g1.free()
    r = {"split": oracle.split_order, "degree": oracle.degree_order, "core": oracle.core_order,
         "check": oracle.check_order}[kind](
        g.n, g.src, g.dst)
    L = oracle.list_triangles(g.n, g.src, g.dst, r, algo, want_triangles=False)
    assert (got.count, got.hash, got.work) == (L.count, L.hash, L.work)
    assert c == oracle.cost(g.n, g.src, g.dst, r).for_algo(algo)


def test_bad_kind(tl):
    import ctypes
    n, s, d = G.complete(4)
    g = tl.orient(n, dev(s), dev(d), dev(np.arange(n, dtype=np.uint32)))
    try:
        out = dev(np.zeros(n, np.uint32))
        rc = tl.raw_lib().tl_order(g.handle, 9, ctypes.c_void_p(out.data_ptr()), None)
        assert rc == tl.tl.TL_EINVAL
    finally:
        g.free()


def neigh(tl, n, s, d, start_rank, **kw):
    g = tl.orient(n, dev(s), dev(d), dev(start_rank))
    try:
        r, res = tl.order_neigh(g, **kw)
        return r.cpu().numpy().view(np.uint32), res
    finally:
        g.free()


def test_neigh_figure2_first_move(tl):
    """Figure 2: from (a,...,g), C+- = 9, a moves right after e, C+- = 6."""
    n, s, d, orders, names = G.fig2()
    r, res = neigh(tl, n, s, d, G.order_to_rank(orders[0][0]), max_visits=1)
    assert [int(u) for u in np.argsort(r)] == orders[1][0]
    assert (res.cpm_start, res.cpm, res.visits, res.moves) == (9, 6, 1, 1)


@pytest.mark.parametrize("seed", range(8))
def test_neigh_matches_oracle(tl, seed):
    """The library's Neigh (linked list with labels, costs from degrees)
    against the oracle's (every candidate priced from scratch), from random
    starting orders, on graphs given with loops and repeated edges."""
    rs = np.random.default_rng(1600 + seed)
    n = int(rs.integers(30, 400))
    k = int(rs.integers(2, 8)) * n
    s = rs.integers(0, n, k).astype(np.uint32)
    d = (s + rs.integers(0, max(n // 8, 2), k)).astype(np.uint32) % n  # some locality, loops included
    r0 = rs.permutation(n).astype(np.uint32)
    eps, passes = [(0.0, 1000), (0.01, 1000), (0.3, 1000), (0.0, 1)][seed % 4]
    got, res = neigh(tl, n, s, d, r0, eps=eps, max_passes=passes)
    want, cpm, npass = oracle.neigh_order(n, s, d, r0, eps=eps, max_passes=passes)
    assert np.array_equal(got, want)
    assert (res.cpm, res.passes) == (cpm, npass)
    assert res.cpm_start == oracle.cost(n, s, d, r0).cpm


def test_neigh_matches_oracle_on_a_heavy_tailed_graph(tl):
    g = graphgen.chung_lu(600, 2.1, 10.0, seed=9)
    r0 = oracle.degree_order(g.n, g.src, g.dst)
    got, res = neigh(tl, g.n, g.src, g.dst, r0, eps=0.01)
    want, cpm, npass = oracle.neigh_order(g.n, g.src, g.dst, r0, eps=0.01)
    assert np.array_equal(got, want) and (res.cpm, res.passes) == (cpm, npass)
    assert cpm < oracle.cost(g.n, g.src, g.dst, r0).cpm


def test_neigh_full_listing_and_errors(tl):
    import ctypes
    g = graphgen.chung_lu(500, 2.3, 12.0, seed=4)
    r0 = np.arange(g.n, dtype=np.uint32)
    g0 = tl.orient(g.n, dev(g.src), dev(g.dst), dev(r0))
    try:
        rank, res = tl.order_neigh(g0, eps=0.01)
        rc = tl.raw_lib().tl_order_neigh(g0.handle, ctypes.c_double(1.5), 10, 0, ctypes.c_void_p(rank.data_ptr()),
                                         None, None)
        assert rc != 0  # eps outside [0, 1)
    finally:
        g0.free()
    g1 = tl.orient(g.n, dev(g.src), dev(g.dst), rank)
    try:
        got = tl.list_triangles(g1, "A+-")
    finally:
        g1.free()
    want_rank, cpm, _ = oracle.neigh_order(g.n, g.src, g.dst, r0, eps=0.01)
    L = oracle.list_triangles(g.n, g.src, g.dst, want_rank, "A+-", want_triangles=False)
    assert (got.count, got.hash, got.work) == (L.count, L.hash, L.work) and L.work == cpm == res.cpm
