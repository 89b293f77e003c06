"""GPU orderings (tl_order) against the oracle's: the degree ordering,
Split (Section 3.3.3), the core ordering (Section 1.3) and Check (Section
3.3.2), and the full listing with the ordering computed on the device."""
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
