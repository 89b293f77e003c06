"""Writes oracle_rmat26.json: the oracle's result on RMAT scale 26.

RMAT scale 26, edge factor 16, a/b/c/d = .57/.19/.19/.05, seed 1, degree
order, A++.  Calls only the oracle and the seeded generators.

The oracle builds the graph once, in this process; worker processes forked
from it share that build and list disjoint pivot-rank ranges with the plain
single-threaded oracle.  The ranges partition the triangles (the outer
iterations of Algorithm 1 are independent), so counts, digests and work add
up exactly -- a property the CPU test-suite checks on small graphs.  Sampled
ranges, chosen to hold triangles from a few hundred to tens of millions, also
get the SHA-256 of their sorted triangle list.

Usage: python tests/golden/make_expected_rmat26.py [workers]
(about 19 GB for the shared build, plus each worker's output buffers)
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import graphgen  # noqa: E402
import oracle  # noqa: E402
from gpu_util import edge_fingerprint  # noqa: E402

MASK = (1 << 64) - 1
G = {}


def sorted_digest(tri: np.ndarray) -> str:
    """SHA-256 of the triangles as little-endian uint32 triples in ascending
    lexicographic order."""
    t = np.asarray(tri, np.uint32).reshape(-1, 3)
    if len(t):
        t = t[np.lexsort((t[:, 2], t[:, 1], t[:, 0]))]
    return hashlib.sha256(np.ascontiguousarray(t).astype("<u4").tobytes()).hexdigest()


def work(job):
    kind, lo, hi, cap = job
    t = time.time()
    L = G["bg"].list("A++", lo, hi, cap=cap)
    out = {"kind": kind, "lo": lo, "hi": hi, "count": L.count, "hash": L.hash, "work": L.work, "m": L.m,
           "secs": round(time.time() - t, 2)}
    if cap and L.count <= cap:
        out["sorted_sha256"] = sorted_digest(L.triangles)
    return out


def partition_cuts(n):
    """Pivot-rank cuts: the bottom half in 8 pieces, then halving widths
    toward the top ranks, where the hubs' work concentrates; the top 8,192
    ranks in pieces of 64 and the top 32 one by one."""
    cuts = [n * i // 16 for i in range(9)]
    top = n // 2
    w = n // 4
    while w >= 8192:
        top += w
        cuts.append(top)
        w //= 2
    cuts += list(range(n - 8192, n - 32, 64)) + [n - k for k in range(0, 33)]
    return sorted(set(c for c in cuts if 0 <= c <= n))


def sample_ranges(n):
    """(lo, hi, cap): rank ranges whose sorted lists are stored by digest."""
    return [(n - 4194304, n - 4194304 + 65536, 1 << 20),   # low-degree pivots (few triangles)
            (n - 1048576, n - 1048576 + 16384, 1 << 22),
            (n - 131072, n - 131072 + 2048, 1 << 22),
            (n - 65536, n - 65536 + 256, 1 << 22),
            (n - 4096, n - 4096 + 16, 1 << 26),
            (n - 32, n - 31, 1 << 26)]                       # one hub pivot (tens of millions)


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    t0 = time.time()
    g = graphgen.config_rmat26(seed=1)
    rank = graphgen.degree_order(g)
    print(f"generated {g} and degree order in {time.time() - t0:.0f}s", flush=True)
    n = g.n
    G["bg"] = oracle.BuiltGraph(n, g.src, g.dst, rank)
    print(f"oracle graph built in {time.time() - t0:.0f}s", flush=True)
    cuts = partition_cuts(n)
    jobs = [("part", a, b, 0) for a, b in zip(cuts[:-1], cuts[1:])]
    jobs += [("sample", a, b, cap) for a, b, cap in sample_ranges(n)]
    jobs.sort(key=lambda j: -(j[1]))  # heavy top ranges first
    res = []
    # fork: the workers share the parent's oracle build (read only)
    with mp.get_context("fork").Pool(workers) as pool:
        for r in pool.imap_unordered(work, jobs):
            res.append(r)
            print(f"[{time.time() - t0:.0f}s] {r['kind']} [{r['lo']},{r['hi']}) count={r['count']} "
                  f"({r['secs']:.0f}s)", flush=True)
    parts = [r for r in res if r["kind"] == "part"]
    total = {"count": sum(r["count"] for r in parts), "hash": sum(r["hash"] for r in parts) & MASK,
             "work": sum(r["work"] for r in parts)}
    c = oracle.cost(n, g.src, g.dst, rank)
    out = {"workload": "RMAT scale 26, edge factor 16, a/b/c/d=.57/.19/.19/.05, seed 1, degree order, A++",
           "n": n, "m": g.m, "edges": edge_fingerprint(g.src, g.dst), "cost": {"A++": c.cpp, "A+-": c.cpm},
           "list": {"A++": total},
           "samples": sorted([r for r in res if r["kind"] == "sample"], key=lambda r: r["lo"]),
           "partition": sorted([[r["lo"], r["hi"], r["count"], r["hash"], r["work"]] for r in parts])}
    with open(os.path.join(HERE, "oracle_rmat26.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"done in {time.time() - t0:.0f}s: {total}", flush=True)


if __name__ == "__main__":
    main()
