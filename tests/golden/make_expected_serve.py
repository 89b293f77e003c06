"""Writes oracle_serve.json: the oracle's result for every job of the
serving workload's job pool (graphgen.serve_job(j), j = 0..P-1: RMAT or
Chung-Lu, 10^3..10^7 target edges, degree or core order, A++).  Calls only
the oracle and the seeded generators.

Usage: python tests/golden/make_expected_serve.py [workers] [P]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402


def one(j):
    g, rank, p = graphgen.serve_job(j)
    t = time.time()
    L = oracle.list_triangles(g.n, g.src, g.dst, rank, "A++", want_triangles=False)
    return dict(p, n=g.n, m=g.m, count=L.count, hash=L.hash, work=L.work, oracle_s=round(time.time() - t, 3))


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    P = int(sys.argv[2]) if len(sys.argv) > 2 else 128
    os.environ["OMP_NUM_THREADS"] = "1"
    t0 = time.time()
    rows = []
    with mp.Pool(workers) as pool:
        for r in pool.imap_unordered(one, range(P)):
            rows.append(r)
            print(f"[{time.time() - t0:.0f}s] job {r['j']} {r['kind']} m={r['m']} {r['order']} "
                  f"count={r['count']}", flush=True)
    rows.sort(key=lambda r: r["j"])
    out = {"workload": "serving job pool: graphgen.serve_job(j), j = 0..P-1, A++", "P": P, "jobs": rows}
    with open(os.path.join(HERE, "oracle_serve.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(f"done in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
