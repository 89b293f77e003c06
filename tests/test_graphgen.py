"""Checks of the seeded input generators (graphs and orderings)."""
import numpy as np
import pytest

import graphgen
import graphs as G


def is_simple_sorted(g):
    s, d = g.src.astype(np.int64), g.dst.astype(np.int64)
    if g.m == 0:
        return True
    keys = (s << 32) | d
    return bool(np.all(s < d) and np.all(d < g.n) and np.all(np.diff(keys) > 0))


def test_rmat_simple_and_deterministic():
    a = graphgen.rmat(10, 8, seed=3)
    b = graphgen.rmat(10, 8, seed=3)
    c = graphgen.rmat(10, 8, seed=4)
    assert a.n == 1024 and is_simple_sorted(a)
    assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
    assert not (a.m == c.m and np.array_equal(a.src, c.src))
    # a/b/c/d = .57/.19/.19/.05 makes low ids heavy
    deg = graphgen.degrees(a)
    assert deg[:64].mean() > 4 * deg[-512:].mean()


def test_chung_lu_simple_and_heavy_tailed():
    g = graphgen.chung_lu(20000, 2.1, 20.0, seed=2)
    assert is_simple_sorted(g)
    deg = graphgen.degrees(g)
    assert 0.8 * 20 < deg.mean() < 1.05 * 20
    assert deg.max() > 30 * deg.mean()


def test_simplify():
    g = graphgen.simplify(5, [0, 1, 2, 2, 3, 4], [1, 0, 2, 3, 2, 0])
    assert g.src.tolist() == [0, 0, 2] and g.dst.tolist() == [1, 4, 3]


@pytest.mark.parametrize("seed", range(4))
def test_degree_order(seed):
    g = graphgen.chung_lu(3000, 2.3, 10.0, seed=seed)
    r = graphgen.degree_order(g)
    assert np.array_equal(np.sort(r), np.arange(g.n))
    deg = graphgen.degrees(g)
    by_rank = np.argsort(r)
    key = deg[by_rank].astype(np.int64) * g.n + by_rank
    assert np.all(np.diff(key) > 0)   # degree ascending, ties by id


def brute_coreness(n, src, dst):
    adj = [set() for _ in range(n)]
    for a, b in zip(src.tolist(), dst.tolist()):
        adj[a].add(b)
        adj[b].add(a)
    core = [0] * n
    k = 0
    alive = set(range(n))
    while alive:
        k += 1
        changed = True
        while changed:
            changed = False
            for v in list(alive):
                if len(adj[v] & alive) < k:
                    alive.remove(v)
                    core[v] = k - 1
                    changed = True
    return core


@pytest.mark.parametrize("seed", range(4))
def test_core_order(seed):
    n, s, d = G.erdos_renyi(60, 0.15, seed)
    g = graphgen.Graph(n, s, d)
    r, core = graphgen.core_order(g, return_core=True)
    assert np.array_equal(np.sort(r), np.arange(n))
    assert core.tolist() == brute_coreness(n, s, d)
    by_rank = np.argsort(r)
    assert np.all(np.diff(core[by_rank].astype(np.int64)) >= 0)


def test_random_order_permutation():
    r = graphgen.random_order(1000, seed=5)
    assert np.array_equal(np.sort(r), np.arange(1000))
    assert not np.array_equal(r, graphgen.random_order(1000, seed=6))


def test_batch_params_ranges():
    for i in range(50):
        n, gamma, k, seed = graphgen.batch_graph_params(i)
        assert 100 <= n <= 50000 and 2.0 <= gamma <= 2.8 and 8 <= k <= 40
