"""Writes oracle_expected.json: the oracle's results on the synthetic workloads.

Calls only the oracle and the seeded generators.  Usage:
    python tests/golden/make_expected.py
Each entry holds the input's size and fingerprint (so a test detects a
generator change), Definition 1's costs, for every listing algorithm the
oracle's (count, digest, work), and the SHA-256 of the graph's sorted
triangle list (little-endian uint32 triples in ascending lexicographic
order), taken from the oracle's degree-ordered A+- listing: the triangle set
does not depend on the ordering or the form (Section 2.1), which the CPU
tests pin.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402
from gpu_util import edge_fingerprint  # noqa: E402

WORKLOADS = {
    # RMAT scale 12, edge factor 8, a/b/c/d = .57/.19/.19/.05, seeds 1..5
    **{f"rmat12_s{s}": (lambda s=s: graphgen.config_rmat12(seed=s)) for s in range(1, 6)},
    # Chung-Lu n = 2^20, gamma 2.1, mean degree 20, seed 1
    "chunglu20_s1": lambda: graphgen.config_chunglu20(seed=1),
}
ORDERS = ["degree", "core", "random"]
ALGOS = ["A++", "A+-", "A--"]


def main():
    out = {}
    for name, make in WORKLOADS.items():
        g = make()
        entry = {"n": g.n, "m": g.m, "edges": edge_fingerprint(g.src, g.dst), "orders": {}}
        for kind in ORDERS:
            r = graphgen.ordering(g, kind, seed=1)
            c = oracle.cost(g.n, g.src, g.dst, r)
            od = {"cost": {"A++": c.cpp, "A+-": c.cpm, "A--": c.cmm}, "list": {}}
            for algo in ALGOS:
                t = time.time()
                want = kind == "degree" and algo == "A+-"
                L = oracle.list_triangles(g.n, g.src, g.dst, r, algo, want_triangles=want)
                assert L.work == c.for_algo(algo)
                if want:
                    tri = L.sorted_triangles()
                    entry["sorted_sha256"] = hashlib.sha256(
                        np.ascontiguousarray(tri).astype("<u4").tobytes()).hexdigest()
                od["list"][algo] = {"count": L.count, "hash": L.hash, "work": L.work}
                print(f"{name} {kind} {algo}: T={L.count} work={L.work} ({time.time() - t:.1f}s)", flush=True)
            entry["orders"][kind] = od
        out[name] = entry
    with open(os.path.join(HERE, "oracle_expected.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
