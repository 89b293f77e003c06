"""Writes oracle_rmat26.json: the oracle's result on RMAT scale 26.

RMAT scale 26, edge factor 16, a/b/c/d = .57/.19/.19/.05, seed 1, degree
order, A++.  Calls only the oracle and the seeded generators.

The full listing is split into disjoint pivot-rank ranges that worker
processes list with the plain single-threaded oracle (each worker builds the
graph once); the ranges partition the triangles (the outer iterations of
Algorithm 1 are independent), so counts, digests and work add up exactly --
a property the CPU test-suite checks on small graphs.  A few sampled ranges
also get the SHA-256 of their sorted triangle list.

Usage: python tests/golden/make_expected_rmat26.py [workers]   (~27 GB per worker)
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


def init_worker():
    G["bg"] = oracle.BuiltGraph(G["n"], G["src"], G["dst"], G["rank"])


def work(job):
    kind, lo, hi, cap = job
    t = time.time()
    L = G["bg"].list("A++", lo, hi, cap=cap)
    out = {"kind": kind, "lo": lo, "hi": hi, "count": L.count, "hash": L.hash, "work": L.work, "m": L.m,
           "secs": time.time() - t}
    if cap and L.count <= cap:
        out["sorted_sha256"] = sorted_digest(L.triangles)
    return out


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 2
    t0 = time.time()
    g = graphgen.config_rmat26(seed=1)
    rank = graphgen.degree_order(g)
    print(f"generated {g} and degree order in {time.time() - t0:.0f}s", flush=True)
    n = g.n
    G.update(n=n, src=g.src, dst=g.dst, rank=rank)
    # full partition: the bottom half in 8 pieces, then halving widths toward
    # the top ranks, where the hubs' work concentrates
    cuts = [n * i // 16 for i in range(9)]
    top = n // 2
    w = n // 4
    while w >= 1:
        top += w
        cuts.append(top)
        w //= 2
    cuts = sorted(set(cuts + [n - k for k in range(0, 33)]))
    jobs = [("part", a, b, 0) for a, b in zip(cuts[:-1], cuts[1:])]
    samples = [(n // 4, n // 4 + 4096), (n // 2, n // 2 + 4096), (n - 65536, n - 65536 + 256), (n - 16, n - 12)]
    jobs += [("sample", a, b, 40_000_000) for a, b in samples]
    jobs.sort(key=lambda j: -(j[1]))  # heavy top ranges first
    res = []
    with mp.get_context("fork").Pool(workers, initializer=init_worker) as pool:
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
           "partition": sorted([[r["lo"], r["hi"], r["count"]] for r in parts])}
    with open(os.path.join(HERE, "oracle_rmat26.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"done in {time.time() - t0:.0f}s: {total}", flush=True)


if __name__ == "__main__":
    main()
