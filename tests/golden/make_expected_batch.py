"""Writes oracle_batch.json: the oracle's per-graph results on the batched
workload (graphs i = 0..K-1, each a Chung-Lu graph drawn by
graphgen.batch_graph(i), degree order, A++).  Calls only the oracle and the
seeded generators.

For every graph i the oracle gives (count, digest, work); the table of K
rows is stored as the SHA-256 of its little-endian uint64 bytes (row-major:
count, digest, work) for the prefixes K = 2000 and K = 20000, together with
the totals and the first rows written out.

Usage: python tests/golden/make_expected_batch.py [workers] [K]
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

import graphgen  # noqa: E402
import oracle  # noqa: E402

PREFIXES = (2000, 20000)


def one(i):
    g = graphgen.batch_graph(i)
    r = graphgen.degree_order(g)
    L = oracle.list_triangles(g.n, g.src, g.dst, r, "A++", want_triangles=False)
    return i, g.n, g.m, L.count, L.hash, L.work


def table_sha(rows):
    return hashlib.sha256(np.ascontiguousarray(rows, "<u8").tobytes()).hexdigest()


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    K = int(sys.argv[2]) if len(sys.argv) > 2 else max(PREFIXES)
    os.environ["OMP_NUM_THREADS"] = "1"
    t0 = time.time()
    rows = np.zeros((K, 3), np.uint64)
    sizes = np.zeros((K, 2), np.uint64)
    with mp.Pool(workers) as pool:
        for done, (i, n, m, c, h, w) in enumerate(pool.imap_unordered(one, range(K), chunksize=8)):
            rows[i] = (c, h, w)
            sizes[i] = (n, m)
            if (done + 1) % 1000 == 0:
                print(f"[{time.time() - t0:.0f}s] {done + 1}/{K} graphs", flush=True)
    out = {
        "workload": "Chung-Lu graphs i = 0..K-1 (graphgen.batch_graph(i): n log-uniform in [100, 50000], "
                    "gamma U(2.0, 2.8), mean degree U(8, 40), seed 1000+i), degree order, A++",
        "table_layout": "K rows of little-endian uint64 (count, digest, work); sha256 of the bytes",
        "prefixes": {},
        "first_rows": [[int(v) for v in rows[i]] for i in range(min(K, 16))],
        "oracle_seconds": time.time() - t0,
    }
    for p in PREFIXES:
        if p <= K:
            out["prefixes"][str(p)] = {
                "table_sha256": table_sha(rows[:p]),
                "triangles": int(rows[:p, 0].sum()),
                "work": int(rows[:p, 2].sum()),
                "vertices": int(sizes[:p, 0].sum()),
                "edges": int(sizes[:p, 1].sum()),
            }
    with open(os.path.join(HERE, "oracle_batch.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["prefixes"]), flush=True)


if __name__ == "__main__":
    main()
