"""GPU parity of the batched form: many graphs oriented and listed as one.

Every graph's (count, digest, work) from one batched pass must equal the
oracle's for that graph alone (Algorithms 1 and 2 and the A-- variant,
digests over the graph's own ids), for direct launches and for replays of
the captured HIP graph, and equal what the plain per-graph calls return.
"""
import numpy as np
import pytest

import graphgen
import graphs as G
import oracle
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


def pack(graphs):
    """[(n, src, dst, rank)] -> per-graph sizes and back-to-back arrays."""
    n = np.array([g[0] for g in graphs], np.uint32)
    m = np.array([len(g[1]) for g in graphs], np.uint64)
    cat = lambda i: (np.concatenate([np.asarray(g[i], np.uint32) for g in graphs])
                     if sum(len(g[i]) for g in graphs) else np.zeros(0, np.uint32))
    return n, m, cat(1), cat(2), cat(3)


def oracle_table(graphs, algo):
    rows = []
    for (n, s, d, r) in graphs:
        L = oracle.list_triangles(n, s, d, r, algo, want_triangles=False)
        rows.append((L.count, L.hash, L.work))
    return np.array(rows, np.uint64).reshape(-1, 3)


def orient_batch(tl, graphs):
    n, m, s, d, r = pack(graphs)
    return tl.batch_orient(n, m, dev(s), dev(d), dev(r))


def fixture_graphs():
    rs = np.random.default_rng(7)
    out = []
    for (n, s, d) in [G.complete(6), G.wheel(9), G.grid(4, 5), G.complete_bipartite(3, 4), G.star(7),
                      G.erdos_renyi(60, 0.2, 3), G.cycle(3), G.fig2()[:3], G.ld_gadget(5)[:3]]:
        out.append((n, s, d, rs.permutation(n).astype(np.uint32)))
    out.append((1, np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(1, np.uint32)))
    out.append((5, np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.arange(5, dtype=np.uint32)))
    # loops and repeated edges in the input are dropped per graph
    out.append((4, np.array([0, 1, 2, 1, 0, 3, 3], np.uint32), np.array([1, 2, 0, 0, 0, 0, 1], np.uint32),
                np.array([3, 1, 0, 2], np.uint32)))
    return out


@pytest.mark.parametrize("algo", ALGOS)
def test_fixture_batch_matches_oracle(tl, algo):
    graphs = fixture_graphs()
    b = orient_batch(tl, graphs)
    try:
        want = oracle_table(graphs, algo)
        assert np.array_equal(b.list(algo, use_graph=False), want)
        assert np.array_equal(b.list(algo, use_graph=True), want)
    finally:
        b.free()


def workload_graphs(k, first=0):
    B = graphgen.batch(k, first=first)
    return B, [(B.graph(i).n, B.graph(i).src, B.graph(i).dst, B.ranks(i)) for i in range(k)]


@pytest.mark.parametrize("algo", ALGOS)
def test_workload_batch_matches_oracle(tl, algo):
    # graphs 0..11 of the batched workload (n log-uniform in [100, 50000])
    B, graphs = workload_graphs(12)
    b = tl.batch_orient(B.n, B.m, dev(B.src), dev(B.dst), dev(B.rank))
    try:
        want = oracle_table(graphs, algo)
        got = b.list(algo, use_graph=True)
        assert np.array_equal(got, want)
    finally:
        b.free()


def test_graph_replays_are_stable(tl):
    """The captured pass replayed several times, with eager work between the
    replays, gives the same table every time."""
    import torch
    B, graphs = workload_graphs(6, first=100)
    b = tl.batch_orient(B.n, B.m, dev(B.src), dev(B.dst), dev(B.rank))
    try:
        want = oracle_table(graphs, "A++")
        out = torch.zeros(3 * b.k, dtype=torch.int64, device="cuda")
        for it in range(4):
            got = b.list("A++", use_graph=True, out_dev=out)
            assert np.array_equal(got, want), it
            assert np.array_equal(out.cpu().numpy().view(np.uint64).reshape(-1, 3), want), it
            x = torch.randn(1 << 20, device="cuda")
            torch.cuda.synchronize()
            assert float((x * 0).sum()) == 0.0
            out.zero_()
        # the eager form interleaved with replays of every algorithm
        for algo in ALGOS:
            t1 = b.list(algo, use_graph=True)
            t2 = b.list(algo, use_graph=False)
            assert np.array_equal(t1, t2)
    finally:
        b.free()


def test_batch_equals_plain_calls(tl):
    """Each graph listed alone by tl_orient + tl_list gives its batch row."""
    B, graphs = workload_graphs(10, first=300)
    b = tl.batch_orient(B.n, B.m, dev(B.src), dev(B.dst), dev(B.rank))
    try:
        table = b.list("A++")
    finally:
        b.free()
    for i, (n, s, d, r) in enumerate(graphs):
        g = tl.orient(n, dev(s), dev(d), dev(r))
        try:
            x = tl.list_triangles(g, "A++")
        finally:
            g.free()
        assert (x.count, x.hash, x.work) == tuple(int(v) for v in table[i]), i


def test_single_graph_batch_equals_plain(tl):
    n, s, d = G.erdos_renyi(300, 0.1, 11)
    r = np.random.default_rng(5).permutation(n).astype(np.uint32)
    b = orient_batch(tl, [(n, s, d, r)])
    try:
        for algo in ALGOS:
            row = b.list(algo)[0]
            L = oracle.list_triangles(n, s, d, r, algo, want_triangles=False)
            assert tuple(int(v) for v in row) == (L.count, L.hash, L.work)
    finally:
        b.free()


def test_batch_rejects_bad_input(tl):
    n, m = np.array([3, 3], np.uint32), np.array([1, 1], np.uint64)
    good_r = np.array([0, 1, 2, 2, 1, 0], np.uint32)
    with pytest.raises(tl.TLError) as e:  # endpoint 3 >= n of the first graph
        tl.batch_orient(n, m, dev(np.array([0, 0], np.uint32)), dev(np.array([3, 1], np.uint32)), dev(good_r))
    assert e.value.code == tl.tl.TL_EINVAL
    with pytest.raises(tl.TLError) as e:  # rank 3 outside [0, 3)
        tl.batch_orient(n, m, dev(np.array([0, 0], np.uint32)), dev(np.array([1, 1], np.uint32)),
                        dev(np.array([0, 1, 3, 2, 1, 0], np.uint32)))
    assert e.value.code == tl.tl.TL_EINVAL
    with pytest.raises(tl.TLError) as e:  # not a permutation inside the second graph
        tl.batch_orient(n, m, dev(np.array([0, 0], np.uint32)), dev(np.array([1, 1], np.uint32)),
                        dev(np.array([0, 1, 2, 1, 1, 0], np.uint32)))
    assert e.value.code == tl.tl.TL_EINVAL


BINS = [
    {"batch_heavy_min": 1},                      # every pivot with work in the LDS bin where it fits
    {"batch_heavy_min": 1 << 62},                # no LDS bin
    {"batch_heavy_min": 64, "batch_heavy_block": 256, "batch_heavy_per_cu": 1},
    {"batch_heavy_min": 512, "batch_heavy_block": 1024, "batch_light_per_cu": 1},
]


@pytest.fixture
def restore_tuning(tl):
    keys = ["batch_heavy_min", "batch_heavy_block", "batch_heavy_per_cu", "batch_light_per_cu"]
    saved = {k: tl.get_tuning(k) for k in keys}
    yield
    for k, v in saved.items():
        tl.set_tuning(k, v)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("bins", BINS, ids=["all-lds", "no-lds", "small-lds", "big-lds"])
def test_bins_and_shapes_do_not_change_results(tl, algo, bins, restore_tuning):
    B, graphs = workload_graphs(8, first=40)
    graphs += fixture_graphs()
    n, m, s, d, r = pack(graphs[8:])
    n = np.concatenate([B.n, n])
    m = np.concatenate([B.m, m])
    b = tl.batch_orient(n, m, dev(np.concatenate([B.src, s])), dev(np.concatenate([B.dst, d])),
                        dev(np.concatenate([B.rank, r])))
    try:
        want = oracle_table(graphs, algo)
        for k, v in bins.items():
            tl.set_tuning(k, v)
        assert np.array_equal(b.list(algo, use_graph=False), want)
        assert np.array_equal(b.list(algo, use_graph=True), want)
    finally:
        b.free()


def test_graph_recaptured_after_tuning_change(tl, restore_tuning):
    B, graphs = workload_graphs(5, first=200)
    b = tl.batch_orient(B.n, B.m, dev(B.src), dev(B.dst), dev(B.rank))
    try:
        want = oracle_table(graphs, "A++")
        tl.set_tuning("batch_heavy_min", 1 << 62)
        assert np.array_equal(b.list("A++"), want)
        tl.set_tuning("batch_heavy_min", 1)
        assert np.array_equal(b.list("A++"), want)
        tl.set_tuning("batch_heavy_block", 1024)
        assert np.array_equal(b.list("A++"), want)
    finally:
        b.free()


def test_batch_tuning_keys(tl, restore_tuning):
    with pytest.raises(tl.TLError):
        tl.set_tuning("batch_heavy_block", 300)
    with pytest.raises(tl.TLError):
        tl.set_tuning("batch_light_per_cu", 0)
    tl.set_tuning("batch_heavy_per_cu", 1)
    assert tl.get_tuning("batch_heavy_per_cu") == 1


@pytest.mark.slow
def test_full_workload_table(tl):
    """All 20,000 graphs of the batched workload (157 M vertices, 1.83 G
    edges, union edge indices near 2^31) oriented as one union and listed by
    one captured pass: the whole per-graph table, and its first 2,000 rows,
    equal the oracle's (SHA-256 of the little-endian uint64 rows, stored by
    tests/golden/make_expected_batch.py)."""
    import hashlib
    import json
    import os

    from gpu_util import GOLDEN
    with open(os.path.join(GOLDEN, "oracle_batch.json")) as f:
        gold = json.load(f)["prefixes"]
    K = 20000
    B = graphgen.batch(K)
    assert (int(B.n.sum()), int(B.ebase[-1])) == (gold[str(K)]["vertices"], gold[str(K)]["edges"])
    b = tl.batch_orient(B.n, B.m, dev(B.src), dev(B.dst), dev(B.rank))
    del B
    try:
        table = b.list("A++", use_graph=True)
    finally:
        b.free()
        tl.release_cached_memory()
    sha = lambda t: hashlib.sha256(np.ascontiguousarray(t, "<u8").tobytes()).hexdigest()
    assert sha(table[:2000]) == gold["2000"]["table_sha256"]
    assert sha(table) == gold[str(K)]["table_sha256"]
    assert int(table[:, 0].sum()) == gold[str(K)]["triangles"]
    assert int(table[:, 2].sum()) == gold[str(K)]["work"]


@pytest.mark.parametrize("algo", ALGOS)
def test_batch_from_oriented_graphs_equals_union_orientation(tl, algo):
    """tl_batch_from_graphs (the union copied from graphs oriented one by
    one) lists the same per-graph table as tl_batch_orient and the oracle."""
    B, graphs = workload_graphs(10, first=300)
    graphs = graphs + fixture_graphs()
    handles = [tl.orient(n, dev(s), dev(d), dev(r)) for (n, s, d, r) in graphs]
    try:
        want = oracle_table(graphs, algo)
        b = tl.batch_from_graphs(handles)
        try:
            assert np.array_equal(b.list(algo, use_graph=False), want)
            assert np.array_equal(b.list(algo, use_graph=True), want)
        finally:
            b.free()
        b2 = orient_batch(tl, graphs)
        try:
            assert np.array_equal(b2.list(algo, use_graph=True), want)
        finally:
            b2.free()
    finally:
        for h in handles:
            h.free()


def test_batch_from_graphs_rejects_bad_input(tl):
    """Through the C-ABI: k = 0 and a NULL handle give TL_EINVAL."""
    import ctypes
    lib = tl.raw_lib()
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.tl_batch_from_graphs(0, ctypes.cast(arr, ctypes.c_void_p), None, ctypes.byref(h)) == tl.tl.TL_EINVAL
    assert lib.tl_batch_from_graphs(1, ctypes.cast(arr, ctypes.c_void_p), None, ctypes.byref(h)) == tl.tl.TL_EINVAL
    assert not h.value
    with pytest.raises(ValueError):
        tl.batch_from_graphs([])
