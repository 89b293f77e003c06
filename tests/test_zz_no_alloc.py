"""GPU test of tl_list_count_noalloc (the count-only listing that allocates
nothing): through the C-ABI, its summary equals tl_list's count-only
summary of the same handle, on two calls in a row where the second graph is
smaller than the first (the shared scratch keeps the first call's
contents), for every form; a graph whose plan exceeds the fixed scratch is
refused with TL_ECAPACITY and nothing launched."""
import numpy as np
import pytest

import graphgen
import graphs as G
from gpu_util import dev

pytestmark = pytest.mark.gpu

ALGOS = ["A++", "A+-", "A--"]


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_04774_amd as tl
    return tl


def summary(s):
    return (int(s.count), int(s.hash), int(s.work), int(s.scanned))


def oriented(tl, n, src, dst, rank):
    return tl.orient(n, dev(src), dev(dst), dev(rank))


@pytest.mark.parametrize("algo", ALGOS)
def test_noalloc_equals_tl_list_two_calls(tl, algo):
    g1 = graphgen.config_rmat12(seed=2)
    r1 = graphgen.degree_order(g1)
    n2, s2, d2 = G.erdos_renyi(300, 0.05, 11)
    r2 = np.random.default_rng(11).permutation(n2).astype(np.uint32)
    big = oriented(tl, g1.n, g1.src, g1.dst, r1)
    small = oriented(tl, n2, s2, d2, r2)
    try:
        want_big = summary(tl.list_triangles(big, algo))
        want_small = summary(tl.list_triangles(small, algo))
        assert want_big[0] > 0 and want_small[0] > 0
        got_big = summary(tl.list_count_noalloc(big, algo))
        got_small = summary(tl.list_count_noalloc(small, algo))  # second call, smaller input
        assert got_big == want_big
        assert got_small == want_small
        # and again in the other order, with heavy pivots forced (tasks in the scratch)
        saved = tl.get_tuning("heavy_min")
        tl.set_tuning("heavy_min", 1)
        try:
            want_big_h = summary(tl.list_triangles(big, algo))
            assert summary(tl.list_count_noalloc(big, algo)) == want_big_h == want_big
            assert summary(tl.list_count_noalloc(small, algo)) == want_small
        finally:
            tl.set_tuning("heavy_min", saved)
    finally:
        big.free()
        small.free()


def test_noalloc_empty_and_edgeless(tl):
    g = oriented(tl, 4, np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.arange(4, dtype=np.uint32))
    try:
        assert summary(tl.list_count_noalloc(g, "A++")) == (0, 0, 0, 0)
    finally:
        g.free()


def test_noalloc_refuses_graph_beyond_scratch(tl):
    gr = graphgen.config_chunglu20(seed=1)  # ~9.6 M edges: far beyond the fixed scratch
    r = graphgen.degree_order(gr)
    g = oriented(tl, gr.n, gr.src, gr.dst, r)
    try:
        with pytest.raises(tl.TLError) as e:
            tl.list_count_noalloc(g, "A++")
        assert e.value.code == tl.tl.TL_ECAPACITY
        # the regular entry point still lists it
        assert tl.list_triangles(g, "A++").count == 105669988
    finally:
        g.free()
