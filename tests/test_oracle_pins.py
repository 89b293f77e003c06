"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each check is independent of the oracle's own code: brute-force enumeration,
trace(A^3)/6, closed forms, the printed values of the Figure 2 example and
the Split example (Section 3.3.3), the Check result worked by hand on the
Figure 2 graph together with the optimum its caption states (re-found by
trying every ordering), Neigh's first move in the Figure 2 caption and the
local optimality of its result, the costs stated for the gadget graphs of
Appendices A and B, the linear-cost property of Appendix B, and splitmix64's
published output sequence for the digest's mixing function.
"""
import itertools
import math

import numpy as np
import pytest

import graphs as G
import oracle

ALGOS = ["A++", "A+-", "A--"]
MASK = (1 << 64) - 1


def rand_graph(seed, n=None, p=None):
    rs = np.random.default_rng(seed)
    n = n if n is not None else int(rs.integers(3, 45))
    p = p if p is not None else float(rs.uniform(0.05, 0.6))
    return G.erdos_renyi(n, p, seed)


def rand_rank(n, seed):
    rs = np.random.default_rng(seed + 99991)
    return rs.permutation(n).astype(np.uint32)


# ---------------------------------------------------------------- digest

def test_mix64_matches_published_splitmix64_sequence():
    # splitmix64 from state 0 outputs f(k * 0x9e3779b97f4a7c15), k = 1, 2, 3;
    # these three values are the generator's published first outputs.
    golden = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    for k, want in enumerate(golden, start=1):
        assert oracle.mix64((k * 0x9E3779B97F4A7C15) & MASK) == want


def test_digest_is_sum_over_bruteforce_set():
    n, s, d = rand_graph(7, n=30, p=0.4)
    bf = G.brute_force_triangles(n, s, d)
    res = oracle.list_triangles(n, s, d, rand_rank(n, 7), "A+-")
    assert res.hash == oracle.hash_of(bf)
    # a duplicated triangle changes the digest (add, not xor, combination)
    dup = np.vstack([bf, bf[:1]])
    assert oracle.hash_of(dup) != res.hash


# ------------------------------------------------------ triangle set pins

@pytest.mark.parametrize("seed", range(25))
@pytest.mark.parametrize("algo", ALGOS)
def test_matches_brute_force(seed, algo):
    n, s, d = rand_graph(seed)
    bf = G.brute_force_triangles(n, s, d)
    res = oracle.list_triangles(n, s, d, rand_rank(n, seed), algo)
    assert res.count == len(bf)
    assert np.array_equal(res.sorted_triangles(), bf)
    # every listed triple is canonical and unique
    t = res.triangles
    assert np.all(t[:, 0] < t[:, 1]) and np.all(t[:, 1] < t[:, 2])


@pytest.mark.parametrize("seed", range(10))
def test_count_matches_trace_a3(seed):
    n, s, d = rand_graph(100 + seed, n=60)
    assert oracle.list_triangles(n, s, d, rand_rank(n, seed), "A++",
                                 want_triangles=False).count == G.trace_count(n, s, d)


@pytest.mark.parametrize("nv", range(3, 10))
def test_complete_graph_closed_forms(nv):
    n, s, d = G.complete(nv)
    for seed in range(3):
        r = rand_rank(n, seed)
        for algo in ALGOS:
            assert oracle.list_triangles(n, s, d, r, algo).count == math.comb(nv, 3)
        c = oracle.cost(n, s, d, r)
        # every order gives out-degrees 0..n-1 once each
        assert c.cpp == (nv - 1) * nv * (2 * nv - 1) // 6
        assert c.cpm == math.comb(nv, 3)


@pytest.mark.parametrize("nv", range(4, 14))
def test_wheel(nv):
    n, s, d = G.wheel(nv)
    want = 4 if nv == 4 else nv - 1   # W_4 is K_4
    for algo in ALGOS:
        assert oracle.list_triangles(n, s, d, rand_rank(n, nv), algo).count == want


@pytest.mark.parametrize("builder", [lambda: G.grid(7, 9), lambda: G.complete_bipartite(6, 8),
                                     lambda: G.random_bipartite(15, 20, 0.4, 3),
                                     lambda: G.cycle(10), lambda: G.star(12)])
def test_triangle_free(builder):
    n, s, d = builder()
    for algo in ALGOS:
        res = oracle.list_triangles(n, s, d, rand_rank(n, 1), algo)
        assert res.count == 0 and res.hash == 0


def test_fig2_triangles_and_printed_costs():
    n, s, d, orders, names = G.fig2()
    bf = G.brute_force_triangles(n, s, d)
    as_names = sorted("".join(names[i] for i in t) for t in bf.tolist())
    assert as_names == ["abe", "ade", "bcg"]
    for order, cpm in orders:
        r = G.order_to_rank(order)
        assert oracle.cost(n, s, d, r).cpm == cpm
        for algo in ALGOS:
            assert np.array_equal(oracle.list_triangles(n, s, d, r, algo).sorted_triangles(), bf)


@pytest.mark.parametrize("dd,want", G.ld_golden())
def test_ld_gadget_cost(dd, want):
    n, s, d, order = G.ld_gadget(dd)
    r = G.order_to_rank(order)
    c = oracle.cost(n, s, d, r)
    assert c.cpp == want
    # triangles of L_d: inside the clique K (d+1 vertices) and each v_i with
    # any two clique vertices
    res = oracle.list_triangles(n, s, d, r, "A++")
    assert res.count == math.comb(dd + 1, 3) + dd * math.comb(dd + 1, 2)
    assert res.count == len(G.brute_force_triangles(n, s, d))


@pytest.mark.parametrize("seed", range(6))
def test_gphi_gadget(seed):
    n, s, d, order = G.gphi_gadget(n_vars=6 + seed, n_clauses=4 + 2 * seed, seed=seed)
    m_clauses = 4 + 2 * seed
    r = G.order_to_rank(order)
    assert oracle.cost(n, s, d, r).cpm == 2 * m_clauses
    for k in range(20):
        assert oracle.cost(n, s, d, rand_rank(n, 1000 * seed + k)).cpm >= 2 * m_clauses
    assert oracle.list_triangles(n, s, d, r, "A+-").count == m_clauses


# ------------------------------------------------------- cost and work

@pytest.mark.parametrize("seed", range(15))
def test_work_equals_cost(seed):
    n, s, d = rand_graph(200 + seed)
    r = rand_rank(n, seed)
    c = oracle.cost(n, s, d, r)
    for algo in ALGOS:
        assert oracle.list_triangles(n, s, d, r, algo, want_triangles=False).work == c.for_algo(algo)


@pytest.mark.parametrize("seed", range(10))
def test_linear_cost_invariant(seed):
    # Appendix B property: the successor counts sum to |E| for every order
    n, s, d = rand_graph(300 + seed)
    m = len({(min(a, b), max(a, b)) for a, b in zip(s.tolist(), d.tolist()) if a != b})
    for k in range(5):
        c = oracle.cost(n, s, d, rand_rank(n, k))
        assert c.sum_dplus == m and c.sum_dminus == m and c.m == m


@pytest.mark.parametrize("seed", range(10))
def test_reversal_identities(seed):
    n, s, d = rand_graph(400 + seed)
    r = rand_rank(n, seed)
    rev = (n - 1 - r.astype(np.int64)).astype(np.uint32)
    c, cr = oracle.cost(n, s, d, r), oracle.cost(n, s, d, rev)
    assert cr.cpm == c.cpm
    assert cr.cpp == c.cmm and cr.cmm == c.cpp


# ---------------------------------------------------------- invariance

@pytest.mark.parametrize("seed", range(5))
def test_invariance_over_orders_and_algorithms(seed):
    n, s, d = rand_graph(500 + seed, n=40, p=0.3)
    ref = oracle.list_triangles(n, s, d, np.arange(n, dtype=np.uint32), "A++")
    for k in range(20):
        r = rand_rank(n, 37 * seed + k)
        for algo in ALGOS:
            res = oracle.list_triangles(n, s, d, r, algo)
            assert (res.count, res.hash) == (ref.count, ref.hash)
            assert np.array_equal(res.sorted_triangles(), ref.sorted_triangles())


@pytest.mark.parametrize("algo", ALGOS)
def test_pivot_ranges_partition(algo):
    n, s, d = rand_graph(77, n=40, p=0.35)
    r = rand_rank(n, 5)
    full = oracle.list_triangles(n, s, d, r, algo)
    cuts = [0, 3, 11, 12, 25, n]
    cnt = hsh = wrk = 0
    parts = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        p = oracle.list_triangles(n, s, d, r, algo, lo, hi)
        cnt += p.count
        hsh = (hsh + p.hash) & MASK
        wrk += p.work
        parts.append(p.triangles)
    assert (cnt, hsh, wrk) == (full.count, full.hash, full.work)
    allp = np.vstack(parts)
    assert np.array_equal(allp[np.lexsort((allp[:, 2], allp[:, 1], allp[:, 0]))],
                          full.sorted_triangles())


# ------------------------------------------------------------- inputs

def test_loops_and_duplicates_dropped():
    n, s, d = G.complete(6)
    s2 = np.concatenate([s, d, np.arange(6, dtype=np.uint32), s[:4]])
    d2 = np.concatenate([d, s, np.arange(6, dtype=np.uint32), d[:4]])
    r = rand_rank(n, 3)
    a = oracle.list_triangles(n, s, d, r, "A+-")
    b = oracle.list_triangles(n, s2, d2, r, "A+-")
    assert (a.count, a.hash, a.m) == (b.count, b.hash, b.m) == (20, a.hash, 15)


def test_invalid_inputs_rejected():
    n, s, d = G.complete(5)
    with pytest.raises(oracle.OracleError):
        oracle.list_triangles(n, s, d, np.array([0, 1, 1, 2, 3], np.uint32))
    with pytest.raises(oracle.OracleError):
        oracle.list_triangles(n, s, d, np.array([0, 1, 2, 3, 5], np.uint32))
    bad = s.copy()
    bad[0] = 9
    with pytest.raises(oracle.OracleError):
        oracle.list_triangles(n, bad, d, np.arange(5, dtype=np.uint32))


def test_empty_and_tiny_graphs():
    for nv in range(0, 4):
        n, s, d = G.complete(nv)
        r = np.arange(nv, dtype=np.uint32)
        res = oracle.list_triangles(n, s, d, r, "A++")
        assert res.count == (1 if nv == 3 else 0)


@pytest.mark.parametrize("seed", range(5))
def test_oriented_csr_rows(seed):
    n, s, d = rand_graph(600 + seed)
    r = rand_rank(n, seed)
    fo, fa, bo, ba, inv = oracle.oriented_csr(n, s, d, r)
    _, pairs = G.simple_degrees(n, s, d)
    want_f = [[] for _ in range(n)]
    want_b = [[] for _ in range(n)]
    for a, b in pairs:
        lo, hi = sorted((int(r[a]), int(r[b])))
        want_f[lo].append(hi)
        want_b[hi].append(lo)
    for x in range(n):
        assert fa[fo[x]:fo[x + 1]].tolist() == sorted(want_f[x])
        assert ba[bo[x]:bo[x + 1]].tolist() == sorted(want_b[x])
        assert r[inv[x]] == x


# ------------------------------------------------------------ orderings


def test_split_worked_example():
    """Section 3.3.3: the non-increasing degree ordering (e,b,g,a,f,d,c) of
    the Figure 2 graph has C+- = 7; Split turns it into (e,g,f,c,d,a,b)
    with C+- = 4 (both printed in the paper, fixture lines 4 and 5)."""
    n, s, d, orders, names = G.fig2()
    start, start_cpm = orders[3]
    split_order, split_cpm = orders[4]
    deg_rank = oracle.degree_order(n, s, d)
    assert [int(u) for u in np.argsort(deg_rank)][::-1] == start
    assert oracle.cost(n, s, d, G.order_to_rank(start)).cpm == start_cpm == 7
    split = oracle.split_order(n, s, d)
    assert [int(u) for u in np.argsort(split)] == split_order
    assert oracle.cost(n, s, d, split).cpm == split_cpm == 4


def _with_noise(n, s, d, seed):
    """The same graph given with loops and repeated (also reversed) edges."""
    rs = np.random.default_rng(seed)
    k = len(s) // 3
    idx = rs.integers(0, max(len(s), 1), k)
    loops = rs.integers(0, n, 5).astype(np.uint32)
    return (np.concatenate([s, d[idx], loops]).astype(np.uint32),
            np.concatenate([d, s[idx], loops]).astype(np.uint32))


@pytest.mark.parametrize("seed", range(8))
def test_degree_order_definition(seed):
    n, s, d = rand_graph(900 + seed)
    s2, d2 = _with_noise(n, s, d, seed)
    r = oracle.degree_order(n, s2, d2)
    assert sorted(r.tolist()) == list(range(n))
    nbr = [set() for _ in range(n)]
    for a, b in zip(s.tolist(), d.tolist()):
        if a != b:
            nbr[a].add(b)
            nbr[b].add(a)
    deg = [len(x) for x in nbr]
    order = np.argsort(r)
    keys = [(deg[u], int(u)) for u in order]
    assert all(keys[i] < keys[i + 1] for i in range(n - 1))


@pytest.mark.parametrize("seed", range(8))
def test_split_reads_degree_order_from_both_ends(seed):
    """Split's order read from both ends inward, alternately (first, last,
    second, second to last, ...), is the non-increasing degree ordering."""
    n, s, d = rand_graph(950 + seed)
    s2, d2 = _with_noise(n, s, d, seed)
    split = np.argsort(oracle.split_order(n, s2, d2))
    delta = np.argsort(oracle.degree_order(n, s2, d2))[::-1]
    zig = []
    lo, hi = 0, n - 1
    while lo <= hi:
        zig.append(int(split[lo]))
        if lo != hi:
            zig.append(int(split[hi]))
        lo += 1
        hi -= 1
    assert zig == [int(u) for u in delta]


def _coreness_by_definition(n, s, d):
    """c_u = the largest k such that u lies in the k-core, each k-core found
    by deleting vertices of degree < k until none is left (Section 1.3)."""
    nbr = [set() for _ in range(n)]
    for a, b in zip(s.tolist(), d.tolist()):
        if a != b:
            nbr[a].add(b)
            nbr[b].add(a)
    core = [0] * n
    k = 1
    while True:
        alive = set(range(n))
        changed = True
        while changed:
            changed = False
            for u in list(alive):
                if len(nbr[u] & alive) < k:
                    alive.discard(u)
                    changed = True
        if not alive:
            return core
        for u in alive:
            core[u] = k
        k += 1


def test_coreness_closed_forms():
    assert oracle.coreness(*G.complete(7)).tolist() == [6] * 7
    assert oracle.coreness(*G.wheel(10)).tolist() == [3] * 10
    assert oracle.coreness(*G.grid(4, 6)).tolist() == [2] * 24
    assert oracle.coreness(*G.star(9)).tolist() == [1] * 9
    assert oracle.coreness(*G.cycle(11)).tolist() == [2] * 11
    path = (6, np.arange(5, dtype=np.uint32), np.arange(1, 6, dtype=np.uint32))
    assert oracle.coreness(*path).tolist() == [1] * 6
    one = (3, np.array([0], np.uint32), np.array([1], np.uint32))  # vertex 2 isolated
    assert oracle.coreness(*one).tolist() == [1, 1, 0]


@pytest.mark.parametrize("seed", range(10))
def test_coreness_matches_definition(seed):
    n, s, d = rand_graph(1100 + seed)
    s2, d2 = _with_noise(n, s, d, seed)
    assert oracle.coreness(n, s2, d2).tolist() == _coreness_by_definition(n, s, d)


@pytest.mark.parametrize("seed", range(4))
def test_core_order_sorts_by_coreness_then_id(seed):
    n, s, d = rand_graph(1200 + seed)
    core = oracle.coreness(n, s, d)
    order = np.argsort(oracle.core_order(n, s, d))
    keys = [(int(core[u]), int(u)) for u in order]
    assert all(keys[i] < keys[i + 1] for i in range(n - 1))


def test_coreness_agrees_with_the_generators_peeling():
    """Two independent peelings (the oracle's buckets, the input generators'
    heap) give the same coreness on a 20,000-vertex heavy-tailed graph."""
    import graphgen
    g = graphgen.chung_lu(20000, 2.1, 12.0, seed=5)
    _, core = graphgen.core_order(g, return_core=True)
    assert np.array_equal(oracle.coreness(g.n, g.src, g.dst), core)


# ------------------------------------------------------------ Check


def _cpm_python(n, s, d, rank):
    """C+- of an ordering by direct counting (Definition 1)."""
    nbr = [set() for _ in range(n)]
    for a, b in zip(s.tolist(), d.tolist()):
        if a != b:
            nbr[a].add(b)
            nbr[b].add(a)
    tot = 0
    for u in range(n):
        plus = sum(1 for v in nbr[u] if rank[v] > rank[u])
        tot += plus * (len(nbr[u]) - plus)
    return tot


def test_check_worked_example():
    """Check (Section 3.3.2) on the Figure 2 graph, worked by hand.  The
    vertices come by non-increasing degree, (e,b,g,a,f,d,c) (the order
    printed with C+- = 7).  e: nothing placed, C_b = C_e = 0, beginning.
    b: N_b = {e}, N_? = {a,c,g}: C_b = 3 > C_e = 0, end.  g: N_e = {b},
    N_? = {c,f}: C_b = 0 < C_e = 2, beginning.  a: N_b = {e}, N_e = {b},
    N_? = {d}: C_b = C_e = 2, beginning.  f and d: every neighbour at the
    beginning, C_b = C_e = 0, beginning.  c: N_b = {g}, N_e = {b}: C_b =
    C_e = 1, beginning.  Result (e,g,a,f,d,c,b); its C+- = 3 is the optimum
    the Figure 2 caption states, found again here by trying all 5,040
    orderings."""
    n, s, d, orders, names = G.fig2()
    rank, side = oracle.check_order(n, s, d, with_side=True)
    assert [names[int(u)] for u in np.argsort(rank)] == list("egafdcb")
    assert [int(x) for x in side] == [0, 1, 0, 0, 0, 0, 0]  # a..g: only b at the end
    opt_order, opt_cpm = orders[2]
    assert oracle.cost(n, s, d, rank).cpm == opt_cpm == 3
    best = min(_cpm_python(n, s, d, np.array(p)) for p in itertools.permutations(range(n)))
    assert best == 3


def test_check_small_closed_forms():
    # path 0-1-2-3: by non-increasing degree 2, 1, 3, 0; 1 finds 2 at the
    # beginning and one unplaced neighbour (C_b = 1 > C_e = 0): end
    path = (4, np.array([0, 1, 2], np.uint32), np.array([1, 2, 3], np.uint32))
    rank = oracle.check_order(*path)
    assert rank.tolist() == [2, 3, 0, 1]
    assert oracle.cost(*path, rank).cpm == 0
    # star: the centre first, then every leaf (one neighbour, at the
    # beginning: C_b = C_e = 0) after it, by decreasing id
    n, s, d = G.star(9)
    order = np.argsort(oracle.check_order(n, s, d))
    centre = int(np.bincount(np.concatenate([s, d])).argmax())
    assert order[0] == centre
    assert order[1:].tolist() == sorted([u for u in range(n) if u != centre], reverse=True)
    # edgeless: every vertex at the beginning, in the order taken
    rank = oracle.check_order(5, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert rank.tolist() == [4, 3, 2, 1, 0]


@pytest.mark.parametrize("seed", range(8))
def test_check_structure_and_greedy_choice(seed):
    """On random graphs (given with loops and repeated edges): the result is
    a permutation; the beginning block holds its vertices in the order they
    were taken and the end block in reverse; and every vertex's own C+-
    share in the final ordering is the smaller of its two options, with the
    options recounted from the final sides and the order of placement."""
    n, s, d = rand_graph(1300 + seed)
    s2, d2 = _with_noise(n, s, d, seed)
    rank, side = oracle.check_order(n, s2, d2, with_side=True)
    assert sorted(rank.tolist()) == list(range(n))
    taken = np.argsort(oracle.degree_order(n, s, d))[::-1]  # non-increasing degree
    when = np.empty(n, np.int64)
    when[taken] = np.arange(n)
    begin = [int(u) for u in taken if side[u] == 0]
    end = [int(u) for u in taken if side[u] == 1]
    assert [int(u) for u in np.argsort(rank)] == begin + end[::-1]
    nbr = [set() for _ in range(n)]
    for a, b in zip(s.tolist(), d.tolist()):
        if a != b:
            nbr[a].add(b)
            nbr[b].add(a)
    total = 0
    for u in range(n):
        nb = sum(1 for v in nbr[u] if when[v] < when[u] and side[v] == 0)
        ne = sum(1 for v in nbr[u] if when[v] < when[u] and side[v] == 1)
        nq = len(nbr[u]) - nb - ne
        cb, ce = nb * (ne + nq), (nb + nq) * ne
        plus = sum(1 for v in nbr[u] if rank[v] > rank[u])
        share = plus * (len(nbr[u]) - plus)
        assert share == min(cb, ce)
        assert side[u] == (0 if cb <= ce else 1)
        total += share
    assert oracle.cost(n, s, d, rank).cpm == total == _cpm_python(n, s, d, rank)


# ------------------------------------------------------------ Neigh


def _candidates(order, u, nbrs):
    """Neigh's candidate orders for u (Algorithm 3): u right before its first
    neighbour, or right after its p-th, neighbours taken in the order."""
    rest = [x for x in order if x != u]
    ns = sorted(nbrs, key=rest.index)
    out = [rest[:rest.index(ns[0])] + [u] + rest[rest.index(ns[0]):]]
    for v in ns:
        i = rest.index(v) + 1
        out.append(rest[:i] + [u] + rest[i:])
    return out


def test_neigh_first_move_is_figure2s():
    """Figure 2: from (a,b,...,g), C+- = 9, vertex a moves right after e,
    giving (b,c,d,e,a,f,g) with C+- = 6 (both orders and costs printed in
    the caption).  The four places among a's neighbours are priced here
    independently; after e is the only cheapest."""
    n, s, d, orders, names = G.fig2()
    start, start_cpm = orders[0]
    moved, moved_cpm = orders[1]
    a = names.index("a")
    nbrs = {int(y) for x, y in zip(s, d) if x == a} | {int(x) for x, y in zip(s, d) if y == a}
    costs = [oracle.cost(n, s, d, G.order_to_rank(c)).cpm for c in _candidates(start, a, nbrs)]
    assert costs[0] == start_cpm == 9 and costs[-1] == moved_cpm == 6
    assert costs.index(min(costs)) == len(costs) - 1 and costs.count(6) == 1
    rank, cpm, _ = oracle.neigh_order(n, s, d, G.order_to_rank(start), max_visits=1)
    assert [int(u) for u in np.argsort(rank)] == moved and cpm == 6


@pytest.mark.parametrize("seed", range(6))
def test_neigh_ends_in_a_local_optimum(seed):
    """Run to a standstill (eps = 0), no vertex has a cheaper place among its
    neighbours (every candidate priced by Definition 1 via the pinned
    cost), and C+- never rose from the start."""
    rs = np.random.default_rng(1400 + seed)
    n = int(rs.integers(20, 60))
    s, d = G.erdos_renyi(n, float(rs.uniform(0.05, 0.2)), 1400 + seed)[1:]
    r0 = rs.permutation(n).astype(np.uint32)
    rank, cpm, passes = oracle.neigh_order(n, s, d, r0, eps=0.0, max_passes=1000)
    assert passes < 1000
    assert sorted(rank.tolist()) == list(range(n))
    assert cpm == oracle.cost(n, s, d, rank).cpm <= oracle.cost(n, s, d, r0).cpm
    order = [int(u) for u in np.argsort(rank)]
    nbr = [set() for _ in range(n)]
    for a, b in zip(s.tolist(), d.tolist()):
        if a != b:
            nbr[a].add(b)
            nbr[b].add(a)
    for u in range(n):
        if nbr[u]:
            for c in _candidates(order, u, nbr[u]):
                assert oracle.cost(n, s, d, G.order_to_rank(c)).cpm >= cpm


def test_neigh_keeps_an_optimal_order():
    """From an order of minimum C+- (found by trying all orders of a 7-vertex
    graph), every vertex is already at a cheapest place: nothing moves."""
    rs = np.random.default_rng(1500)
    n = 7
    s, d = G.erdos_renyi(n, 0.5, 1500)[1:]
    best = min(itertools.permutations(range(n)), key=lambda p: _cpm_python(n, s, d, np.array(p)))
    r0 = np.array(best, np.uint32)
    rank, cpm, passes = oracle.neigh_order(n, s, d, r0, eps=0.0)
    assert np.array_equal(rank, r0) and passes == 1
    assert cpm == _cpm_python(n, s, d, r0)


# ------------------------------------------- pivot ranges and their helpers
#
# A form lists, for pivots of rank in [lo, hi), the triangles whose vertex in
# the form's pivot role has such a rank: the largest rank for A++
# (Algorithm 1's outer vertex w), the smallest for A+- (Algorithm 2's u), the
# middle one for A-- (v).  These tests compute that set by brute force and
# the paper's work by its per-seed-edge count (Property 1) straight from the
# edge set, and hold every range entry point of the oracle to them.

def _py_f(z):
    # splitmix64's output function, from its published definition
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def _py_digest(a, b, c):
    # the digest convention the library header states:
    # h(a,b,c) = f(f((a << 32) | b) + c) with 64-bit wrap-around
    return _py_f((_py_f((a << 32) | b) + c) & MASK)


def _py_digest_sum(tri):
    h = 0
    for a, b, c in np.asarray(tri).reshape(-1, 3).tolist():
        h = (h + _py_digest(a, b, c)) & MASK
    return h


def _pivot_rank(tri, rank, algo):
    rk = np.sort(rank[np.asarray(tri, np.int64).reshape(-1, 3)].astype(np.int64), axis=1)
    return rk[:, {"A++": 2, "A+-": 0, "A--": 1}[algo]]


def _bf_range(n, s, d, rank, algo, lo, hi):
    bf = G.brute_force_triangles(n, s, d)
    if len(bf) == 0:
        return bf
    pr = _pivot_rank(bf, rank, algo)
    return bf[(pr >= lo) & (pr < hi)]


def _py_work(n, s, d, rank, algo, lo, hi):
    dp, dm = G.oriented_degrees(n, s, d, rank)
    _, pairs = G.simple_degrees(n, s, d)
    w = 0
    for a, b in pairs:
        x, y = (a, b) if rank[a] < rank[b] else (b, a)  # oriented x -> y
        if algo == "A++":    # pivot y, seed x scans N+(x)
            piv, cost = rank[y], dp[x]
        elif algo == "A+-":  # pivot x, seed y scans N+(y)
            piv, cost = rank[x], dp[y]
        else:                # pivot x (middle), seed y scans N-(y)
            piv, cost = rank[x], dm[y]
        if lo <= piv < hi:
            w += int(cost)
    return w


def test_digest_convention_pin():
    # convention pin: the oracle's per-triangle digest is exactly the stated
    # composition, including the carry of the inner sum and extreme ids
    for a, b, c in [(0, 1, 2), (1, 2, 3), (7, 1000, 65536), (12345, 67890, 4000000000),
                    (0xFFFFFFFD, 0xFFFFFFFE, 0xFFFFFFFF), (0, 0x80000000, 0xFFFFFFFF)]:
        assert oracle.triangle_hash(a, b, c) == _py_digest(a, b, c), (a, b, c)
    # the composition is not symmetric in its arguments: a swapped inner pair,
    # or an xor in place of the sum, gives another value
    assert _py_digest(1, 2, 3) != _py_digest(2, 1, 3)
    assert _py_digest(1, 2, 3) != _py_f(_py_f((1 << 32) | 2) ^ 3)


CUT_SETS = [[0, 5, 6, 17, 30, 45], [0, 1, 2, 3, 45], [0, 22, 45], [10, 12, 40]]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("algo", ALGOS)
def test_pivot_range_is_the_roles_set(seed, algo):
    n, s, d = rand_graph(900 + seed, n=45, p=0.3)
    r = rand_rank(n, 900 + seed)
    for cuts in CUT_SETS:
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            want = _bf_range(n, s, d, r, algo, lo, hi)
            got = oracle.list_triangles(n, s, d, r, algo, lo, hi)
            assert got.count == len(want), (lo, hi)
            assert np.array_equal(got.sorted_triangles(), want), (lo, hi)
            assert got.hash == _py_digest_sum(want)
            assert got.work == _py_work(n, s, d, r, algo, lo, hi)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("algo", ALGOS)
def test_built_graph_and_list_ranges_match_brute_force(seed, algo):
    n, s, d = rand_graph(950 + seed, n=45, p=0.35)
    r = rand_rank(n, 950 + seed)
    g = oracle.BuiltGraph(n, s, d, r)
    try:
        assert g.m == len(G.simple_degrees(n, s, d)[1])
        for cuts in CUT_SETS:
            ranges = list(zip(cuts[:-1], cuts[1:]))
            want = [_bf_range(n, s, d, r, algo, lo, hi) for lo, hi in ranges]
            caps = [len(w) + 3 for w in want]
            many = oracle.list_ranges(n, s, d, r, algo, ranges, caps)
            for (lo, hi), w, cap, lr in zip(ranges, want, caps, many):
                one = g.list(algo, lo, hi, cap=cap)
                work = _py_work(n, s, d, r, algo, lo, hi)
                for res in (one, lr):
                    assert (res.count, res.hash, res.work) == (len(w), _py_digest_sum(w), work), (lo, hi)
                    assert np.array_equal(res.sorted_triangles(), w), (lo, hi)
                assert g.work(algo, lo, hi) == work
            # a buffer shorter than the range keeps the first triangles only
            lo, hi = ranges[0]
            if len(want[0]) > 1:
                short = g.list(algo, lo, hi, cap=1)
                assert short.count == len(want[0]) and len(short.triangles) == 1
    finally:
        g.close()


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("algo", ALGOS)
def test_bins_over_source_ranges_match_brute_force(seed, algo):
    n, s, d = rand_graph(980 + seed, n=45, p=0.35)
    r = rand_rank(n, 980 + seed)
    bf = G.brute_force_triangles(n, s, d)
    g = oracle.BuiltGraph(n, s, d, r)
    try:
        for cuts in CUT_SETS:
            tot = np.zeros((len(cuts) - 1, 2), np.uint64)
            for a, b in [(0, 9), (9, 10), (10, 31), (31, n)]:  # a partition of the source ranks
                tot += g.bin(algo, cuts, a, b)
            pr = _pivot_rank(bf, r, algo) if len(bf) else np.zeros(0, np.int64)
            for i, (lo, hi) in enumerate(zip(cuts[:-1], cuts[1:])):
                sel = bf[(pr >= lo) & (pr < hi)] if len(bf) else bf
                assert int(tot[i, 0]) == len(sel), (cuts, i)
                assert int(tot[i, 1]) == _py_digest_sum(sel), (cuts, i)
            # source ranges alone: the triangles whose smallest rank lies there
            part = g.bin("A+-", [0, n], 10, 31)
            sel = bf[(_pivot_rank(bf, r, "A+-") >= 10) & (_pivot_rank(bf, r, "A+-") < 31)] if len(bf) else bf
            assert int(part[0, 0]) == len(sel)
    finally:
        g.close()
