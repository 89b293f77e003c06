"""GPU parity on RMAT scale 26 (edge factor 16, about 1.05 billion simple
edges), degree order, A++: exact count, digest and work of the whole
listing (count only, and with every triangle streamed through 2^30-triangle
device chunks whose count and digest are recomputed on the device from the
emitted triples), the costs of Definition 1, per-range counts and digests
over a partition of the pivot ranks, and the sorted triangle lists of
sampled rank ranges, against the oracle's results stored by
tests/golden/make_expected_rmat26.py.
"""
import ctypes
import json
import os

import pytest

import graphgen
from gpu_util import GOLDEN, MASK64, dev, digest_sum_torch, edge_fingerprint, sorted_sha256_device

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_04774_amd as tl
    with open(os.path.join(GOLDEN, "oracle_rmat26.json")) as f:
        gold = json.load(f)
    g = graphgen.config_rmat26(seed=1)
    assert edge_fingerprint(g.src, g.dst) == gold["edges"]
    rank = graphgen.degree_order(g)
    src, dst, r = dev(g.src), dev(g.dst), dev(rank)
    n = g.n
    del g
    csr = tl.orient(n, src, dst, r)
    del src, dst, r
    torch.cuda.synchronize()
    yield tl, csr, gold
    csr.free()
    tl.release_cached_memory()


def test_rmat26_total(setup):
    tl, csr, gold = setup
    assert (csr.n, csr.m) == (gold["n"], gold["m"])
    s = tl.list_triangles(csr, "A++")
    want = gold["list"]["A++"]
    assert (s.count, s.hash, s.work) == (want["count"], want["hash"], want["work"])
    assert tl.cost(csr, "A++") == gold["cost"]["A++"]
    assert tl.cost(csr, "A+-") == gold["cost"]["A+-"]


def test_rmat26_streamed_chunks(setup):
    """The listing the benchmark times: every triangle streamed through
    library-owned chunks of 2^30 triangles.  Each chunk is copied out in the
    callback and checked on the device: canonical rows (a < b < c < n), and
    its count and digest summed from the triples themselves, so that the
    stream (slices, clipped tasks, holes and moves) is checked, not only the
    kernel's own accumulators."""
    import torch
    tl, csr, gold = setup
    K = 1 << 30
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    buf = torch.empty((K, 3), dtype=torch.int32, device="cuda")
    seen = {"chunks": 0, "count": 0, "hash": 0, "bad": 0}

    def sink(ptr, k):
        assert 0 < k <= K
        assert hip.hipMemcpy(buf.data_ptr(), ptr, k * 12, 3) == 0  # device to device
        t = buf[:k].to(torch.int64)
        ok = (t[:, 0] >= 0) & (t[:, 0] < t[:, 1]) & (t[:, 1] < t[:, 2]) & (t[:, 2] < csr.n)
        seen["bad"] += int((~ok).sum().item())
        seen["count"] += k
        seen["hash"] = (seen["hash"] + digest_sum_torch(buf[:k])) & MASK64
        seen["chunks"] += 1
        return False

    tl.set_chunk_triangles(K)
    try:
        s = tl.list_triangles(csr, "A++", on_chunk=sink)
    finally:
        tl.set_chunk_triangles(1 << 24)
    del buf
    want = gold["list"]["A++"]
    assert (s.count, s.hash, s.work) == (want["count"], want["hash"], want["work"])
    assert seen["bad"] == 0
    assert (seen["count"], seen["hash"]) == (want["count"], want["hash"])
    st = tl.last_list_stats()
    # every slice is handed out in one or more calls of at most K triangles
    assert seen["chunks"] >= st["slices"] >= want["count"] // (st_room(tl) * K)


def st_room(tl):
    return tl.get_tuning("chunk_room")


def test_rmat26_partition(setup):
    """Counts, digests and work over consecutive pivot-rank ranges, each the
    union of some of the stored partition's pieces."""
    tl, csr, gold = setup
    parts = gold["partition"]
    # merge the stored pieces into about 24 ranges of similar triangle counts
    total = sum(p[2] for p in parts)
    ranges, cur = [], None
    for lo, hi, count, h, w in parts:
        if cur is None:
            cur = [lo, hi, 0, 0, 0]
        cur[1] = hi
        cur[2] += count
        cur[3] = (cur[3] + h) & MASK64
        cur[4] += w
        if cur[2] >= total // 24:
            ranges.append(cur)
            cur = None
    if cur is not None:
        ranges.append(cur)
    assert ranges[0][0] == 0 and ranges[-1][1] == csr.n
    for lo, hi, count, h, w in ranges:
        s = tl.list_triangles(csr, "A++", pivot_range=(lo, hi))
        assert (s.count, s.hash, s.work) == (count, h, w), (lo, hi)


def test_rmat26_sampled_sorted_lists(setup):
    import torch
    tl, csr, gold = setup
    checked = 0
    for smp in gold["samples"]:
        s0 = tl.list_triangles(csr, "A++", pivot_range=(smp["lo"], smp["hi"]))
        assert (s0.count, s0.hash, s0.work) == (smp["count"], smp["hash"], smp["work"])
        if "sorted_sha256" not in smp:
            continue
        out = torch.empty((max(smp["count"], 1), 3), dtype=torch.int32, device="cuda")
        s = tl.list_triangles(csr, "A++", out=out, pivot_range=(smp["lo"], smp["hi"]))
        assert s.count == smp["count"]
        assert sorted_sha256_device(out[: s.count], 26) == smp["sorted_sha256"], (smp["lo"], smp["hi"])
        checked += smp["count"] > 0
    assert checked >= 4
