"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

Integer results are compared bit for bit: sorted triangle lists where they
are materialised, and (count, digest, work) always; CSR arrays element by
element; costs exactly.
"""
import math

import numpy as np
import pytest

import graphgen
import graphs as G
import oracle
from gpu_util import dev, edge_fingerprint, load_expected, packed_sorted, sort_rows, sorted_sha256_device

pytestmark = pytest.mark.gpu

ALGOS = ["A++", "A+-", "A--"]


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_04774_amd as tl
    return tl


def gpu_run(tl, n, src, dst, rank, algo, want_list=True, cap=None):
    import torch
    g = tl.orient(n, dev(src), dev(dst), dev(rank))
    try:
        if not want_list:
            return tl.list_triangles(g, algo), None, g.m
        if cap is None:
            s0 = tl.list_triangles(g, algo)
            cap = max(int(s0.count), 1)
        out = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
        s = tl.list_triangles(g, algo, out=out)
        tri = out[: s.count].cpu().numpy().view(np.uint32)
        return s, tri, g.m
    finally:
        g.free()


def assert_same(tl, n, src, dst, rank, algo):
    s, tri, m = gpu_run(tl, n, src, dst, rank, algo)
    ref = oracle.list_triangles(n, src, dst, rank, algo)
    assert m == ref.m
    assert (s.count, s.hash, s.work) == (ref.count, ref.hash, ref.work)
    assert s.scanned <= s.work
    got = sort_rows(tri)
    assert np.array_equal(got, ref.sorted_triangles())
    return s


def rand_case(seed):
    rs = np.random.default_rng(seed)
    n = int(rs.integers(3, 300))
    p = float(rs.uniform(0.02, 0.5)) if n < 80 else float(rs.uniform(0.01, 0.1))
    n, s, d = G.erdos_renyi(n, p, seed)
    rank = rs.permutation(n).astype(np.uint32)
    return n, s, d, rank


# ---------------------------------------------------------------- small

@pytest.mark.parametrize("seed", range(20))
@pytest.mark.parametrize("algo", ALGOS)
def test_random_graphs(tl, seed, algo):
    n, s, d, r = rand_case(seed)
    assert_same(tl, n, s, d, r, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_closed_forms(tl, algo):
    for nv in [3, 4, 5, 17, 64, 65, 130]:
        n, s, d = G.complete(nv)
        r = np.random.default_rng(nv).permutation(n).astype(np.uint32)
        st = assert_same(tl, n, s, d, r, algo)
        assert st.count == math.comb(nv, 3)
    for nv in [4, 5, 9, 100]:
        n, s, d = G.wheel(nv)
        st = assert_same(tl, n, s, d, np.arange(n, dtype=np.uint32), algo)
        assert st.count == (4 if nv == 4 else nv - 1)
    for builder in [lambda: G.grid(30, 40), lambda: G.complete_bipartite(20, 70), lambda: G.star(5000)]:
        n, s, d = builder()
        r = np.random.default_rng(1).permutation(n).astype(np.uint32)
        st = assert_same(tl, n, s, d, r, algo)
        assert st.count == 0 and st.hash == 0


@pytest.mark.parametrize("algo", ALGOS)
def test_paper_examples(tl, algo):
    n, s, d, orders, _ = G.fig2()
    for order, _cpm in orders:
        assert_same(tl, n, s, d, G.order_to_rank(order), algo)
    for dd in range(1, 7):
        n, s, d, order = G.ld_gadget(dd)
        assert_same(tl, n, s, d, G.order_to_rank(order), algo)
    n, s, d, order = G.gphi_gadget(8, 12, 3)
    assert_same(tl, n, s, d, G.order_to_rank(order), algo)


def test_costs_match_oracle_and_paper(tl):
    n, s, d, orders, _ = G.fig2()
    for order, cpm in orders:
        r = G.order_to_rank(order)
        g = tl.orient(n, dev(s), dev(d), dev(r))
        assert tl.cost(g, "A+-") == cpm
        c = oracle.cost(n, s, d, r)
        assert (tl.cost(g, "A++"), tl.cost(g, "A--")) == (c.cpp, c.cmm)
        g.free()
    for seed in range(10):
        n, s, d, r = rand_case(100 + seed)
        g = tl.orient(n, dev(s), dev(d), dev(r))
        c = oracle.cost(n, s, d, r)
        assert [tl.cost(g, a) for a in ALGOS] == [c.cpp, c.cpm, c.cmm]
        g.free()


def test_loops_duplicates_and_both_directions(tl):
    rs = np.random.default_rng(5)
    n, s, d = G.erdos_renyi(120, 0.1, 5)
    # both directions, self-loops, and repeats of a hub's edges
    s2 = np.concatenate([s, d, np.arange(0, n, 3, dtype=np.uint32), s[:50], s[:50]])
    d2 = np.concatenate([d, s, np.arange(0, n, 3, dtype=np.uint32), d[:50], d[:50]])
    perm = rs.permutation(len(s2))
    s2, d2 = s2[perm].copy(), d2[perm].copy()
    r = rs.permutation(n).astype(np.uint32)
    for algo in ALGOS:
        assert_same(tl, n, s2, d2, r, algo)
    # a long row (> 64 entries) full of repeats
    hub = np.zeros(3000, np.uint32)
    leaves = (np.arange(3000) % 700 + 1).astype(np.uint32)
    nn = 701
    r = np.arange(nn, dtype=np.uint32)
    s3 = np.concatenate([hub, s % nn])
    d3 = np.concatenate([leaves, d % nn])
    for algo in ALGOS:
        assert_same(tl, nn, s3, d3, r, algo)


@pytest.mark.parametrize("seed", range(6))
def test_csr_parity(tl, seed):
    n, s, d, r = rand_case(200 + seed)
    if seed == 5:
        n, s, d = G.star(70000)        # one row of 69999 entries
        r = np.arange(n, dtype=np.uint32)
    g = tl.orient(n, dev(s), dev(d), dev(r))
    fo, fa, bo, ba, inv = g.to_host()
    rfo, rfa, rbo, rba, rinv = oracle.oriented_csr(n, s, d, r)
    assert np.array_equal(fo, rfo) and np.array_equal(fa, rfa)
    assert np.array_equal(bo, rbo) and np.array_equal(ba, rba)
    assert np.array_equal(inv, rinv)
    g.free()


def test_empty_and_tiny(tl):
    for nv in range(0, 4):
        n, s, d = G.complete(nv)
        r = np.arange(nv, dtype=np.uint32)
        for algo in ALGOS:
            st, tri, m = gpu_run(tl, n, s, d, r, algo, want_list=False)
            assert st.count == (1 if nv == 3 else 0)
    # isolated vertices only
    st, _, m = gpu_run(tl, 10, np.zeros(0, np.uint32), np.zeros(0, np.uint32),
                       np.arange(10, dtype=np.uint32), "A++", want_list=False)
    assert m == 0 and st.count == 0


def test_invalid_inputs(tl):
    n, s, d = G.complete(6)
    with pytest.raises(tl.TLError) as e:
        tl.orient(n, dev(s), dev(d), dev(np.array([0, 1, 2, 3, 4, 4], np.uint32)))
    assert e.value.code == 1
    with pytest.raises(tl.TLError) as e:
        tl.orient(n, dev(s), dev(d), dev(np.array([0, 1, 2, 3, 4, 6], np.uint32)))
    assert e.value.code == 1
    bad = s.copy()
    bad[3] = 6
    with pytest.raises(tl.TLError) as e:
        tl.orient(n, dev(bad), dev(d), dev(np.arange(6, dtype=np.uint32)))
    assert e.value.code == 1


def test_capacity_error_reports_size(tl):
    import torch
    n, s, d = G.complete(30)
    r = np.arange(n, dtype=np.uint32)
    g = tl.orient(n, dev(s), dev(d), dev(r))
    out = torch.empty((100, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(tl.TLError) as e:
        tl.list_triangles(g, "A++", out=out)
    assert e.value.code == 3
    st = tl.list_triangles(g, "A++", out=out, allow_capacity_error=True)
    assert st.count == math.comb(30, 3)
    g.free()


def test_chunked_output_and_abort(tl):
    import torch
    n, s, d = G.erdos_renyi(200, 0.2, 9)
    r = np.random.default_rng(9).permutation(n).astype(np.uint32)
    ref = oracle.list_triangles(n, s, d, r, "A+-")
    g = tl.orient(n, dev(s), dev(d), dev(r))
    tl.set_chunk_triangles(997)
    try:
        parts = []

        def sink(ptr, k):
            # copy the library-owned chunk out before returning
            buf = torch.empty((k, 3), dtype=torch.int32, device="cuda")
            import ctypes
            hip = ctypes.CDLL("libamdhip64.so")
            hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
            assert hip.hipMemcpy(buf.data_ptr(), ptr, k * 12, 3) == 0   # device to device
            parts.append(buf.cpu().numpy().view(np.uint32))
            return False

        st = tl.list_triangles(g, "A+-", on_chunk=sink)
        assert len(parts) > 1
        assert (st.count, st.hash) == (ref.count, ref.hash)
        assert np.array_equal(sort_rows(np.vstack(parts)), ref.sorted_triangles())
        calls = []
        with pytest.raises(tl.TLError) as e:
            tl.list_triangles(g, "A+-", on_chunk=lambda p, k: calls.append(k) or True)
        assert e.value.code == 5 and len(calls) == 1
    finally:
        tl.set_chunk_triangles(1 << 24)
        g.free()


@pytest.mark.parametrize("algo", ALGOS)
def test_chunked_slices_redone_after_overflow(tl, algo):
    """With chunk_growth above 1, callback slices grow while triangles are
    rare.  A sparse part listed first and a clique listed last (highest
    ranks) make a grown slice find more triangles than the device chunk
    holds; it is probed again shorter, and the callbacks, at most K
    triangles each, still hold exactly the oracle's list."""
    import ctypes
    import itertools

    import torch
    rs = np.random.default_rng(21)
    ns, nk, K = 3000, 48, 500
    u, v = rs.integers(0, ns, 9000), rs.integers(0, ns, 9000)
    keep = u != v
    sparse = np.stack([np.minimum(u, v)[keep], np.maximum(u, v)[keep]], 1)
    clique = np.array(list(itertools.combinations(range(ns, ns + nk), 2)))
    pairs = np.unique(np.vstack([sparse, clique]), axis=0).astype(np.uint32)
    n, s, d = ns + nk, pairs[:, 0].copy(), pairs[:, 1].copy()
    r = np.concatenate([rs.permutation(ns), ns + np.arange(nk)]).astype(np.uint32)
    ref = oracle.list_triangles(n, s, d, r, algo)
    g = tl.orient(n, dev(s), dev(d), dev(r))
    tl.set_chunk_triangles(K)
    saved = {k: tl.get_tuning(k) for k in ("chunk_growth", "chunk_margin")}
    tl.set_tuning("chunk_growth", 4)
    tl.set_tuning("chunk_margin", 125)
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        parts = []

        def sink(ptr, k):
            assert 0 < k <= K
            buf = torch.empty((k, 3), dtype=torch.int32, device="cuda")
            assert hip.hipMemcpy(buf.data_ptr(), ptr, k * 12, 3) == 0
            parts.append(buf.cpu().numpy().view(np.uint32))
            return False

        st = tl.list_triangles(g, algo, on_chunk=sink)
        stats = tl.last_list_stats()
        assert (st.count, st.hash, st.work) == (ref.count, ref.hash, ref.work)
        assert np.array_equal(sort_rows(np.vstack(parts)), ref.sorted_triangles())
        assert stats["slices_redone"] >= 1
        # a slice is handed out K triangles at a time
        assert len(parts) >= -(-st.count // K)
        # fewer slices than the one-item-one-triangle bound would need
        assert stats["slices"] < -(-st.scanned // K)
    finally:
        for k, v in saved.items():
            tl.set_tuning(k, v)
        tl.set_chunk_triangles(1 << 24)
        g.free()


@pytest.mark.parametrize("algo", ALGOS)
def test_pivot_ranges_partition(tl, algo):
    n, s, d = G.erdos_renyi(150, 0.15, 4)
    r = np.random.default_rng(4).permutation(n).astype(np.uint32)
    g = tl.orient(n, dev(s), dev(d), dev(r))
    full = tl.list_triangles(g, algo)
    cuts = [0, 1, 40, 41, 99, 150]
    tot_c = tot_h = tot_w = 0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        p = tl.list_triangles(g, algo, pivot_range=(lo, hi))
        ref = oracle.list_triangles(n, s, d, r, algo, lo, hi, want_triangles=False)
        assert (p.count, p.hash, p.work) == (ref.count, ref.hash, ref.work)
        tot_c += p.count
        tot_h = (tot_h + p.hash) % (1 << 64)
        tot_w += p.work
    assert (tot_c, tot_h, tot_w) == (full.count, full.hash, full.work)
    g.free()


def test_deterministic_repeats(tl):
    gr = graphgen.config_rmat12(seed=2)
    r = graphgen.degree_order(gr)
    g = tl.orient(gr.n, dev(gr.src), dev(gr.dst), dev(r))
    res = {(s.count, s.hash, s.work) for s in (tl.list_triangles(g, "A++") for _ in range(5))}
    assert len(res) == 1
    g.free()


# ------------------------------------------------------- workload sizes

@pytest.mark.parametrize("seed", range(1, 6))
def test_rmat12_all_orders_and_algorithms(tl, seed):
    """RMAT scale 12 (edge factor 8): full sorted lists against the oracle."""
    gr = graphgen.config_rmat12(seed=seed)
    exp = load_expected()[f"rmat12_s{seed}"]
    assert (gr.m, edge_fingerprint(gr.src, gr.dst)) == (exp["m"], exp["edges"])
    for kind in ["degree", "core", "random"]:
        r = graphgen.ordering(gr, kind, seed=1)
        for algo in ALGOS:
            st = assert_same(tl, gr.n, gr.src, gr.dst, r, algo)
            e = exp["orders"][kind]["list"][algo]
            assert (st.count, st.hash, st.work) == (e["count"], e["hash"], e["work"])


@pytest.fixture(scope="module")
def chunglu20():
    gr = graphgen.config_chunglu20(seed=1)
    exp = load_expected()["chunglu20_s1"]
    assert (gr.m, edge_fingerprint(gr.src, gr.dst)) == (exp["m"], exp["edges"])
    return gr, exp


@pytest.mark.parametrize("kind", ["degree", "core", "random"])
def test_chunglu20_summaries_and_cost(tl, chunglu20, kind):
    """Chung-Lu n=2^20: count, digest, work and cost of every algorithm."""
    gr, exp = chunglu20
    r = graphgen.ordering(gr, kind, seed=1)
    g = tl.orient(gr.n, dev(gr.src), dev(gr.dst), dev(r))
    try:
        for algo in ALGOS:
            assert tl.cost(g, algo) == exp["orders"][kind]["cost"][algo]
            st = tl.list_triangles(g, algo)
            e = exp["orders"][kind]["list"][algo]
            assert (st.count, st.hash, st.work) == (e["count"], e["hash"], e["work"])
    finally:
        g.free()


def test_chunglu20_csr_parity(tl, chunglu20):
    gr, _ = chunglu20
    r = graphgen.random_order(gr.n, seed=1)
    g = tl.orient(gr.n, dev(gr.src), dev(gr.dst), dev(r))
    fo, fa, bo, ba, inv = g.to_host()
    g.free()
    rfo, rfa, rbo, rba, rinv = oracle.oriented_csr(gr.n, gr.src, gr.dst, r)
    assert np.array_equal(fo, rfo) and np.array_equal(fa, rfa)
    assert np.array_equal(bo, rbo) and np.array_equal(ba, rba)
    assert np.array_equal(inv, rinv)


@pytest.mark.parametrize("algo", ["A++", "A+-"])
def test_chunglu20_full_sorted_list(tl, chunglu20, algo):
    """Chung-Lu n=2^20, degree order: the whole triangle list, sorted."""
    gr, _ = chunglu20
    r = graphgen.degree_order(gr)
    st, tri, _ = gpu_run(tl, gr.n, gr.src, gr.dst, r, algo)
    ref = oracle.list_triangles(gr.n, gr.src, gr.dst, r, algo)
    assert (st.count, st.hash, st.work) == (ref.count, ref.hash, ref.work)
    assert np.array_equal(packed_sorted(tri), packed_sorted(ref.triangles))


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["random", "degree", "core"])
def test_chunglu20_sorted_lists_every_order(tl, chunglu20, kind):
    """Chung-Lu n=2^20 under the random, degree and core orders, every form:
    the whole list written to one device buffer, sorted on the device, equal
    to the oracle's sorted list (its SHA-256, stored; the triangle set is the
    same for every ordering and form)."""
    import torch
    gr, exp = chunglu20
    r = graphgen.ordering(gr, kind, seed=1)
    g = tl.orient(gr.n, dev(gr.src), dev(gr.dst), dev(r))
    try:
        T = exp["orders"][kind]["list"]["A++"]["count"]
        out = torch.empty((T, 3), dtype=torch.int32, device="cuda")
        for algo in ALGOS:
            out.fill_(-1)
            st = tl.list_triangles(g, algo, out=out)
            e = exp["orders"][kind]["list"][algo]
            assert (st.count, st.hash, st.work) == (e["count"], e["hash"], e["work"]), algo
            assert sorted_sha256_device(out, 21) == exp["sorted_sha256"], algo
    finally:
        g.free()


# ---------------------------------------------------- every probe path

TUNINGS = {
    "all-light": {"heavy_min": 1 << 40},
    "bitmap": {"heavy_min": 1, "force_mode": 0},
    "array": {"heavy_min": 1, "force_mode": 1},
    "global": {"heavy_min": 1, "force_mode": 2},
    "reverse": {"heavy_min": 1, "force_mode": 3},
    "hash": {"heavy_min": 1, "force_mode": 4},
    "bucket": {"heavy_min": 1, "force_mode": 5},
    "split": {"heavy_min": 1, "force_mode": 6},
    "split-auto": {"heavy_min": 1, "split": 2},
    "tiny-tasks-static": {"heavy_min": 1, "slice_min": 64, "slice_mult": 1, "queue": 0, "splits": 0},
    "tiny-tasks-queue": {"heavy_min": 1, "slice_min": 64, "slice_mult": 1, "queue": 1, "splits": 1},
}
# every scanned list of up to 255 entries (the largest setting) taken whole
# by the plan: elements outside the window must fail each membership test
# like any non-member
for _name in ["all-light", "bitmap", "array", "global", "reverse", "hash", "bucket", "split", "split-auto"]:
    TUNINGS[_name + "+whole-lists"] = {**TUNINGS[_name], "plan_full": 255}
TUNINGS["no-whole-lists"] = {"plan_full": 0}
# one light wavefront per 64 items (the smallest share): many light
# wavefronts, hence many emission blocks and holes, even on small graphs
TUNINGS["all-light-many-waves"] = {"heavy_min": 1 << 40, "light_wave_items": 64}
TUNINGS["many-light-waves"] = {"light_wave_items": 64}


def wide_hub_case(seed):
    """1.5M vertices; a hub adjacent to 20,000 of them spread over the whole
    rank range, random edges among those; the hub ranked last."""
    rs = np.random.default_rng(seed)
    n = 1_500_000
    nodes = rs.choice(n, 20_000, replace=False).astype(np.uint32)
    hub = nodes[0]
    a = rs.choice(nodes[1:], 80_000)
    b = rs.choice(nodes[1:], 80_000)
    src = np.concatenate([np.full(len(nodes) - 1, hub, np.uint32), a]).astype(np.uint32)
    dst = np.concatenate([nodes[1:], b]).astype(np.uint32)
    g = graphgen.simplify(n, src, dst)
    rank = rs.permutation(n).astype(np.uint32)
    top = int(np.where(rank == n - 1)[0][0])
    rank[top], rank[hub] = rank[hub], n - 1
    return n, g.src, g.dst, rank


@pytest.fixture
def tuned(tl, request):
    cfg = TUNINGS[request.param]
    saved = {k: tl.get_tuning(k) for k in cfg}
    for k, v in cfg.items():
        tl.set_tuning(k, v)
    yield request.param
    for k, v in saved.items():
        tl.set_tuning(k, v)


@pytest.mark.parametrize("tuned", list(TUNINGS), indirect=True)
@pytest.mark.parametrize("algo", ALGOS)
def test_probe_paths(tl, tuned, algo):
    """Each membership mode and task schedule, forced, against the oracle:
    random graphs (short and long windows), closed forms, RMAT-12 under the
    three orderings, and a chunked listing whose slices clip tasks."""
    for seed in range(6):
        n, s, d, r = rand_case(700 + seed)
        assert_same(tl, n, s, d, r, algo)
    n, s, d = G.complete(150)
    assert_same(tl, n, s, d, np.random.default_rng(3).permutation(n).astype(np.uint32), algo)
    n, s, d = G.wheel(3000)
    assert_same(tl, n, s, d, np.arange(n, dtype=np.uint32)[::-1].copy(), algo)
    gr = graphgen.config_rmat12(seed=3)
    for kind in ["degree", "random"]:
        assert_same(tl, gr.n, gr.src, gr.dst, graphgen.ordering(gr, kind, seed=2), algo)
    # pivot lists spread over rank windows far wider than 8192 slices
    gc = graphgen.chung_lu(60000, 2.1, 10.0, seed=9)
    assert_same(tl, gc.n, gc.src, gc.dst, graphgen.random_order(gc.n, seed=4), algo)
    # a hub whose neighbours span 1.5M ranks: its list's window is wider than an LDS bitmap
    n, s, d, r = wide_hub_case(11)
    assert_same(tl, n, s, d, r, algo)
    # chunked: slices of 5000 items cut through heavy tasks
    import torch
    r = graphgen.degree_order(gr)
    ref = oracle.list_triangles(gr.n, gr.src, gr.dst, r, algo)
    g = tl.orient(gr.n, dev(gr.src), dev(gr.dst), dev(r))
    tl.set_chunk_triangles(5000)
    try:
        parts = []
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]

        def sink(ptr, k):
            buf = torch.empty((k, 3), dtype=torch.int32, device="cuda")
            assert hip.hipMemcpy(buf.data_ptr(), ptr, k * 12, 3) == 0
            parts.append(buf.cpu().numpy().view(np.uint32))
            return False

        st = tl.list_triangles(g, algo, on_chunk=sink)
        assert (st.count, st.hash, st.work) == (ref.count, ref.hash, ref.work)
        assert np.array_equal(sort_rows(np.vstack(parts)), ref.sorted_triangles())
    finally:
        tl.set_chunk_triangles(1 << 24)
        g.free()


@pytest.mark.parametrize("case", ["rmat12", "pow2-dups", "tiny", "empty-edges", "chunglu-random"])
def test_orient_sort_and_scatter_agree(tl, case):
    """The two ways of building the CSRs (radix sort of packed keys, or
    per-vertex counters and scatter) give identical arrays, and both equal
    the oracle's oriented graph."""
    rs = np.random.default_rng(17)
    if case == "rmat12":
        g = graphgen.config_rmat12(seed=4)
        n, s, d = g.n, g.src, g.dst
        r = graphgen.degree_order(g)
    elif case == "pow2-dups":  # n a power of two; loops and repeated pairs in the input
        n = 1024
        s = rs.integers(0, n, 9000).astype(np.uint32)
        d = rs.integers(0, n, 9000).astype(np.uint32)
        r = rs.permutation(n).astype(np.uint32)
    elif case == "tiny":
        n, s, d = 1, np.zeros(1, np.uint32), np.zeros(1, np.uint32)
        r = np.zeros(1, np.uint32)
    elif case == "empty-edges":
        n, s, d = 5, np.zeros(0, np.uint32), np.zeros(0, np.uint32)
        r = rs.permutation(n).astype(np.uint32)
    else:
        g = graphgen.chung_lu(200000, 2.1, 10.0, seed=3)
        n, s, d = g.n, g.src, g.dst
        r = graphgen.random_order(n, seed=5)
    saved = tl.get_tuning("orient_sort")
    arrays, listed = [], []
    try:
        for way in (1, 0):
            tl.set_tuning("orient_sort", way)
            c = tl.orient(n, dev(s), dev(d), dev(r))
            arrays.append(c.to_host())
            # the A++ plan ends each window at the pivot's own place in the
            # scanned list, which each way records while orienting
            sm = tl.list_triangles(c, "A++")
            listed.append((sm.count, sm.hash, sm.work))
            c.free()
    finally:
        tl.set_tuning("orient_sort", saved)
    for a, b in zip(arrays[0], arrays[1]):
        assert np.array_equal(a, b)
    ref = oracle.list_triangles(n, s, d, r, "A++", want_triangles=False)
    assert listed[0] == listed[1] == (ref.count, ref.hash, ref.work)
    fo, fa, bo, ba, inv = oracle.oriented_csr(n, s, d, r)
    got = arrays[0]
    assert np.array_equal(got[0], fo) and np.array_equal(got[1], fa)
    assert np.array_equal(got[2], bo) and np.array_equal(got[3], ba)
    assert np.array_equal(got[4], inv)
