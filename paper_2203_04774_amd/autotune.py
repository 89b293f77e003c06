"""Autotuner of the batched pass: the pivot-bin threshold and the workgroup
shapes of its two probe kernels.

The batched pass (tl_batch_list) sends a pivot to the LDS-bitmap bin when
its pruned items reach ``batch_heavy_min`` (and its list's rank span fits
the bitmap); the rest go to the flattened lane-per-item kernel.  This
module times the pass on a seeded batch for candidate values of

    batch_heavy_min     bin threshold (items per pivot; 2^62 = no LDS bin)
    batch_heavy_block   threads per LDS-bin workgroup (256, 512, 1024)
    batch_heavy_per_cu  LDS-bin workgroups per CU (1, 2)
    batch_light_per_cu  lane-bin workgroups (256 threads) per CU

by coordinate descent (each key swept with the others fixed, twice over),
checks that every candidate gives the same per-graph table (results never
depend on the launch parameters), and writes the fastest setting to
``tuned_batch.json`` beside this file.  ``apply()`` loads that file into the
library (tl_set_tuning).

Usage (on the GPU):  python -m paper_2203_04774_amd.autotune [--graphs K]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "tuned_batch.json")

CANDIDATES = {
    "batch_heavy_min": [256, 1024, 4096, 16384, 65536, 1 << 62],
    "batch_heavy_block": [256, 512, 1024],
    "batch_heavy_per_cu": [1, 2],
    "batch_light_per_cu": [4, 8, 16, 32],
}
TL_PHASE_BATCH = 6


def _pass_ms(tl, b, algo, reps):
    lib = tl.raw_lib()
    lib.tl_timing_read.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    times, table = [], None
    for _ in range(reps):
        lib.tl_timing_reset()
        lib.tl_timing_enable(1)
        t = b.list(algo, use_graph=False)
        lib.tl_timing_enable(0)
        ms = ctypes.c_double()
        lib.tl_timing_read(TL_PHASE_BATCH, ctypes.byref(ms), None)
        times.append(ms.value)
        if table is None:
            table = t
        elif not np.array_equal(t, table):
            raise RuntimeError("per-graph table changed between runs")
    return float(np.median(times)), table


def tune(tl, b, algo="A++", reps=3, rounds=2, log=print) -> dict:
    """Coordinate descent over CANDIDATES on an oriented batch b."""
    best = {k: tl.get_tuning(k) for k in CANDIDATES}
    for k, v in best.items():
        tl.set_tuning(k, v)
    base_ms, ref = _pass_ms(tl, b, algo, reps)
    trials = [{"settings": dict(best), "ms": base_ms}]
    best_ms = base_ms
    for r in range(rounds):
        for key, values in CANDIDATES.items():
            for v in values:
                if v == best[key]:
                    continue
                tl.set_tuning(key, v)
                ms, table = _pass_ms(tl, b, algo, reps)
                if not np.array_equal(table, ref):
                    raise RuntimeError(f"{key}={v} changed the per-graph table")
                trials.append({"settings": dict(best, **{key: v}), "ms": ms})
                log(f"[autotune] round {r} {key}={v}: {ms:.3f} ms (best {best_ms:.3f})")
                if ms < best_ms:
                    best_ms, best[key] = ms, v
                tl.set_tuning(key, best[key])
    return {"settings": best, "ms": best_ms, "default_ms": base_ms, "trials": trials}


def apply(path: str = TUNED) -> dict | None:
    """Loads tuned settings into the library; returns them (None if no file)."""
    if not os.path.exists(path):
        return None
    import paper_2203_04774_amd as tl
    with open(path) as f:
        d = json.load(f)
    for k, v in d["settings"].items():
        tl.set_tuning(k, int(v))
    return d["settings"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", type=int, default=4000, help="graphs of the batched workload to tune on")
    ap.add_argument("--algo", default="A++")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TUNED)
    args = ap.parse_args()
    import torch

    import graphgen
    import paper_2203_04774_amd as tl

    t0 = time.time()
    B = graphgen.batch(args.graphs)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda")
    b = tl.batch_orient(B.n, B.m, dev(B.src), dev(B.dst), dev(B.rank))
    print(f"[autotune] {args.graphs} graphs, {b.m} edges ready in {time.time() - t0:.1f}s", flush=True)
    res = tune(tl, b, args.algo, args.reps)
    b.free()
    res.update(workload=f"batched workload graphs 0..{args.graphs - 1} (graphgen.batch), degree order",
               algo=args.algo, device=torch.cuda.get_device_name(0))
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: res[k] for k in ("settings", "ms", "default_ms")}), flush=True)


if __name__ == "__main__":
    main()
