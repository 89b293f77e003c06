"""Benchmark: triangle listing under given vertex orderings on one MI355X.

A step is one pass of the whole listing path over the workload: for every
supplied ordering, tl_orient (validate, relabel, forward/backward CSR,
inverse permutation), then for every algorithm tl_cost and tl_list with the
full triangle list written to a device buffer.  Inputs (edge list and rank
arrays) are resident in HBM before the timed region starts.

Default workload: RMAT scale 26, edge factor 16, a/b/c/d = .57/.19/.19/.05,
seed 1 (2^26 vertices, 1.05 G undirected edges), degree ordering, A++, with
the triangles streamed through library-owned device chunks of 2^30 triangles
to a consumer callback (one listing per step).  Other workloads:
chunglu20 (Chung-Lu n = 2^20, three orderings x A++/A+-, full lists to one
device buffer), rmat12, batch, serve, orders.

Prints ONE JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

WORKLOADS = {
    "chunglu20": dict(desc="Chung-Lu n=2^20 gamma=2.1 mean degree 20 seed 1",
                      orders=["random", "degree", "core"], algos=["A++", "A+-"]),
    "rmat12": dict(desc="RMAT scale 12 edge factor 8 a/b/c/d=.57/.19/.19/.05 seed 1",
                   orders=["degree"], algos=["A++"]),
    "rmat26": dict(desc="RMAT scale 26 edge factor 16 a/b/c/d=.57/.19/.19/.05 seed 1",
                   orders=["degree"], algos=["A++"], emit="chunks", chunk=1 << 30, chunk_room=8),
    "serve": dict(desc="Poisson stream of serving jobs", orders=["degree", "core"], algos=["A++"]),
    "orders": dict(desc="orderings on the GPU and cost against time", orders=[], algos=[]),
    "orders26": dict(desc="orderings on the GPU and cost against time, RMAT scale 26", orders=[], algos=[]),
    "batch": dict(desc="independent Chung-Lu graphs i = 0..K-1, n log-uniform in [100, 50000], "
                       "gamma U(2.0, 2.8), mean degree U(8, 40), seed 1000+i, degree order",
                  orders=["degree"], algos=["A++"]),
}


def make_graph(name):
    import graphgen
    if name == "chunglu20":
        return graphgen.config_chunglu20(seed=1)
    if name == "rmat12":
        return graphgen.config_rmat12(seed=1)
    if name == "rmat26":
        return graphgen.config_rmat26(seed=1)
    raise SystemExit(f"unknown workload {name}")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def oracle_results(name):
    """(order, algo) -> (count, digest, work) of the whole listing, as the
    oracle's stored results for this workload give them (written by the
    scripts under tests/golden from oracle/ only), or {} if none are stored."""
    gdir = os.path.join(ROOT, "tests", "golden")
    out = {}
    try:
        if name == "rmat26":
            with open(os.path.join(gdir, "oracle_rmat26.json")) as f:
                d = json.load(f)
            for algo, r in d["list"].items():
                out[("degree", algo)] = (r["count"], r["hash"], r["work"])
        elif name in ("chunglu20", "rmat12"):
            with open(os.path.join(gdir, "oracle_expected.json")) as f:
                d = json.load(f)[name + "_s1"]
            for kind, o in d["orders"].items():
                for algo, r in o["list"].items():
                    out[(kind, algo)] = (r["count"], r["hash"], r["work"])
    except (OSError, KeyError, ValueError):
        return {}
    return out


def alg_bytes(C, m, n, T, emit=True):
    """Algorithmic HBM bytes of one listing: 4 B per scanned-list element of
    the paper's work C, 4 B per staged pivot-list element and ~16 B of
    offsets per seed edge (m each), 16 B of pivot offsets per vertex, and
    12 B per written triangle."""
    return 4 * C + 4 * m + 16 * m + 16 * n + (12 * T if emit else 0)


def heavy_alg_bytes(st):
    """Algorithmic bytes of the heavy-pivot kernel's share of a listing: 4 B
    per element of the paper's work over its seed edges, 4 B per staged
    pivot-list element, 16 B of offsets per seed edge and per pivot, 12 B per
    written triangle."""
    return (4 * st["heavy_work"] + 4 * st["heavy_staged"] + 16 * st["heavy_seeds"] + 16 * st["heavy_pivots"]
            + 12 * st["heavy_triangles"])


def heavy_loaded_bytes(st):
    """Bytes the heavy-pivot kernel actually moves for its share of a
    listing: 4 B per scanned element inside the windows (items), 8 B per
    staged list element per task (marked, then read again to unmark), 20 B
    of seed geometry per heavy seed (work prefix, scan start, endpoint id),
    and per listed triangle 4 B for the third vertex's id plus 12 B written."""
    return (4 * st["heavy_items"] + 8 * st["heavy_task_staged"] + 20 * st["heavy_seeds"]
            + 16 * st["heavy_triangles"])


def measured_traffic(workload, launches_per_step):
    """HBM bytes per heavy-probe launch from the committed rocprofv3 --pmc
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    or None if there is none for this workload or the kernel source changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    from paper_2203_04774_amd.profiling import list_source_digest
    if t.get("source_digest") != list_source_digest():
        return None
    return t.get("heavy_bytes_per_launch")


def host_cpu():
    """(model name, logical CPUs, CPUs this process may run on)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def rmat26_sample_ranges(n):
    """Pivot-rank ranges of the RMAT-26 CPU sample: 16 single pivots spread
    evenly over the top 8,192 ranks of the degree ordering, which hold most
    of the graph's triangles (the ranks below hold few)."""
    return [(n - 8192 + 512 * i + 256, n - 8192 + 512 * i + 257) for i in range(16)]


def start_cpu_baseline_ranges(g, rank, algo, ranges, budget_s):
    """Forks a child, before the GPU is touched, that pins itself to one
    host core, builds the oracle's graph (not timed) and times the oracle's
    listing of the given pivot-rank ranges, in order, until budget_s is
    spent.  The parent keeps the other cores.  Returns a handle for
    finish_cpu_baseline."""
    rfd, wfd = os.pipe()
    cores = sorted(os.sched_getaffinity(0))
    core = cores[-1]
    pid = os.fork()
    if pid == 0:
        os.close(rfd)
        try:
            os.sched_setaffinity(0, {core})
            import oracle
            t0 = time.perf_counter()
            bg = oracle.BuiltGraph(g.n, g.src, g.dst, rank)
            build_s = time.perf_counter() - t0
            log(f"[bench] CPU oracle (child, core {core}): graph built in {build_s:.0f}s")
            spent, tri, work, done = 0.0, 0, 0, []
            for lo, hi in ranges:
                t1 = time.perf_counter()
                L = bg.list(algo, lo, hi)
                dt = time.perf_counter() - t1
                spent += dt
                tri += L.count
                work += L.work
                done.append([lo, hi, L.count, L.work, round(dt, 3)])
                log(f"[bench] CPU oracle (child): pivots [{lo}, {hi}) {L.count} triangles in {dt:.2f}s")
                if spent >= budget_s:
                    break
            payload = {"spent": spent, "tri": tri, "work": work, "done": done, "build_s": build_s, "core": core}
        except BaseException as e:  # reported by the parent
            payload = {"error": repr(e)}
        os.write(wfd, json.dumps(payload).encode())
        os.close(wfd)
        os._exit(0)
    os.close(wfd)
    if len(cores) > 1:
        os.sched_setaffinity(0, set(cores[:-1]))
    return pid, rfd, algo, g.name


def finish_cpu_baseline(handle):
    pid, rfd, algo, name = handle
    chunks = []
    while True:
        b = os.read(rfd, 1 << 16)
        if not b:
            break
        chunks.append(b)
    os.close(rfd)
    os.waitpid(pid, 0)
    r = json.loads(b"".join(chunks).decode() or '{"error": "no result"}')
    if "error" in r:
        log(f"[bench] CPU baseline failed: {r['error']}")
        return None
    model, ncpu, navail = host_cpu()
    spent = r["spent"]
    first, last = r["done"][0], r["done"][-1]
    return {"value": r["tri"] / spent, "unit": "triangles/s", "cores": 1, "kind": "oracle",
            "sample": f"{name}, degree order, {algo}: the oracle's listing of {len(r['done'])} single-pivot "
                      f"rank ranges from [{first[0]}, {first[1]}) to [{last[0]}, {last[1]}) (pivots spread over "
                      f"the top 8,192 ranks): {r['tri']} triangles, paper's work {r['work']}, "
                      f"{spent:.1f} s on one pinned core; graph build ({r['build_s']:.0f} s) not timed",
            "intersect_elems_per_s": r["work"] / spent, "triangles": r["tri"], "work": r["work"],
            "seconds": spent, "ranges": r["done"], "pinned_core": r["core"], "cpu_model": model,
            "logical_cpus": ncpu, "cpus_available": navail}


def cpu_baseline(g, ranks, budget_s=20.0):
    """The oracle on one pinned host core over a bounded sample of the
    step's listings: whole listings, taken in order until the budget is
    spent; each ordering's graph is built by the oracle outside the timed
    region."""
    import oracle
    cores = sorted(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {cores[-1]})  # this thread only, for the timed loop
    try:
        done, tri, work, spent = [], 0, 0, 0.0
        plan = [(k, a) for k in ("degree", "core", "random") if k in ranks for a in ("A++", "A+-")]
        built = {}
        for kind, algo in plan:
            if spent > budget_s * 0.5 and done:
                break
            if kind not in built:
                built = {kind: oracle.BuiltGraph(g.n, g.src, g.dst, ranks[kind])}
            t = time.perf_counter()
            L = built[kind].list(algo)
            spent += time.perf_counter() - t
            tri += L.count
            work += L.work
            done.append(f"{kind}-{algo}")
    finally:
        os.sched_setaffinity(0, set(cores))
    model, ncpu, navail = host_cpu()
    return {"value": tri / spent, "unit": "triangles/s", "cores": 1, "kind": "oracle",
            "sample": f"{g.name}: whole listings {', '.join(done)} ({spent:.1f} s on one pinned core; "
                      f"graph builds not timed)",
            "intersect_elems_per_s": work / spent, "triangles": tri, "work": work, "seconds": spent,
            "pinned_core": cores[-1], "cpu_model": model, "logical_cpus": ncpu, "cpus_available": navail}


def bench_batch(args):
    """Batched form: K graphs oriented as one union and listed by one
    captured pass (per-graph count, digest, work), against the plain form
    (tl_orient + tl_list per graph) on the same resident inputs."""
    import ctypes

    import torch

    import graphgen
    import paper_2203_04774_amd as tl

    from paper_2203_04774_amd import autotune
    tuned = autotune.apply()
    log(f"[bench] batched-pass tuning: {tuned if tuned else 'library defaults'}")
    K = args.batch_graphs
    t0 = time.time()
    B = graphgen.batch(K)
    M = int(B.ebase[-1])
    log(f"[bench] {K} graphs, {int(B.n.sum())} vertices, {M} edges generated in {time.time() - t0:.1f}s")

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda")

    src, dst, rank = dev(B.src), dev(B.dst), dev(B.rank)
    torch.cuda.synchronize()
    lib = tl.raw_lib()
    lib.tl_timing_read.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]

    def phase(ph):
        ms, calls = ctypes.c_double(), ctypes.c_uint64()
        lib.tl_timing_read(ph, ctypes.byref(ms), ctypes.byref(calls))
        return ms.value, int(calls.value)

    def batched_step():
        b = tl.batch_orient(B.n, B.m, src, dst, rank)
        try:
            return b.list("A++", use_graph=True)
        finally:
            b.free()

    for i in range(args.warmup):
        batched_step()
        log(f"[bench] batched warmup {i + 1}/{args.warmup} done")
    lib.tl_timing_reset()
    lib.tl_timing_enable(1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        table = batched_step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    lib.tl_timing_enable(0)
    orient_ms, _ = phase(0)
    list_ms, list_calls = phase(6)
    T = int(table[:, 0].sum())
    W = int(table[:, 2].sum())
    log(f"[bench] batched: {args.steps} steps in {elapsed:.3f}s, T={T}")
    # replays of the captured listing pass on one oriented batch
    b = tl.batch_orient(B.n, B.m, src, dst, rank)
    try:
        b.list("A++", use_graph=True)
        replays = []
        for i in range(3):
            t1 = time.perf_counter()
            again = b.list("A++", use_graph=True)
            replays.append(time.perf_counter() - t1)
            assert np.array_equal(again, table)
    finally:
        b.free()

    # plain form over the same resident inputs, one graph at a time
    tl.release_cached_memory()
    n_plain = min(K, args.plain_graphs) if args.plain_graphs else K
    plain = np.zeros((n_plain, 3), np.uint64)
    views = []
    for i in range(n_plain):
        a, b_ = int(B.ebase[i]), int(B.ebase[i + 1])
        va, vb = int(B.vbase[i]), int(B.vbase[i + 1])
        views.append((int(B.n[i]), src[a:b_], dst[a:b_], rank[va:vb]))
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for i, (n, s_, d_, r_) in enumerate(views):
        g = tl.orient(n, s_, d_, r_)
        x = tl.list_triangles(g, "A++")
        g.free()
        plain[i] = (x.count, x.hash, x.work)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - tp
    same = bool(np.array_equal(plain, table[:n_plain]))
    T_plain = int(plain[:, 0].sum())
    log(f"[bench] plain: {n_plain} graphs in {plain_s:.3f}s, equal to batched rows: {same}")

    value = T * args.steps / elapsed
    plain_value = T_plain / plain_s
    import hashlib
    table_sha = hashlib.sha256(np.ascontiguousarray(table, "<u8").tobytes()).hexdigest()
    expected = None
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_batch.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            gold = json.load(f)
        pre = gold.get("prefixes", {}).get(str(K))
        if pre:
            expected = pre["table_sha256"] == table_sha
    # the listing pass's algorithmic bytes: 4 B per scanned-list element of
    # the paper's work plus 32 B of seed geometry per edge and 8 B per triangle
    pass_bytes = 4 * W + 32 * M + 8 * T
    list_s = list_ms / 1e3 / max(list_calls, 1)
    res = {
        "metric": "triangles listed/s + intersect elems/s (%HBM peak); batched vs plain; p99 job ms",
        "value": value,
        "unit": "triangles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "batch", "graph": WORKLOADS["batch"]["desc"], "graphs": K,
                   "n": int(B.n.sum()), "m": M, "algos": ["A++"],
                   "step": "tl_batch_orient + tl_batch_list (pass captured as a HIP graph, then launched)",
                   "tuning": tuned or "library defaults"},
        "intersect_elems_per_s": W * args.steps / elapsed,
        "plain": {"value": plain_value, "unit": "triangles/s", "graphs": n_plain, "seconds": plain_s,
                  "per_graph_equal_to_batched": same},
        "batched_vs_plain": value / plain_value if plain_value else None,
        "batched_list_only": {"ms": list_s * 1e3, "triangles_per_s": T / list_s if list_s else None,
                              "replay_ms": 1e3 * float(np.median(replays))},
        "orient_ms_per_step": orient_ms / args.steps,
        "roofline": {"bound": "hbm", "kernel": "tl_batch_list pass", "achieved": pass_bytes / list_s / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": pass_bytes / list_s / 1e9 / HBM_PEAK_GBS,
                     "traffic": None},
        "table_sha256": table_sha,
        "oracle_table_match": expected,
    }
    if not args.no_cpu_baseline:
        import oracle
        spent, tri, done = 0.0, 0, 0
        for i in range(K):
            gi = B.graph(i)
            t1 = time.perf_counter()
            L = oracle.list_triangles(gi.n, gi.src, gi.dst, B.ranks(i), "A++", want_triangles=False)
            spent += time.perf_counter() - t1
            tri += L.count
            done += 1
            if spent > args.cpu_budget:
                break
        res["cpu_baseline"] = {"value": tri / spent, "unit": "triangles/s", "cores": 1, "kind": "oracle",
                               "sample": f"graphs 0..{done - 1} of the batch, one at a time ({spent:.1f} s)"}
    print(json.dumps(res), flush=True)


def bench_serve(args):
    """Serving form: Poisson arrivals of listing jobs drawn from a seeded job
    pool, served by the library's server (continuous batching under a 64 GB
    device budget) at several arrival rates, at most serve_jobs jobs or
    serve_seconds of arrivals per rate; latency is submit -> result.  Two
    modes: cold (every job uploaded and oriented) and resident (jobs carry
    their pool index as key, so each graph is oriented once, kept on the
    device, and repeats are listed from it; the cache is warmed first).  The
    plain form lists each pool job by tl_orient + tl_list, its arrays
    uploaded each time."""
    import torch

    import graphgen
    import paper_2203_04774_amd as tl

    P = args.serve_pool
    t0 = time.time()
    pool = [graphgen.serve_job(j) for j in range(P)]
    if args.serve_pinned:
        # job arrays in page-locked host memory (uploads by DMA at full link speed)
        def pinned(a):
            t = torch.empty(len(a), dtype=torch.int32, pin_memory=True)
            v = t.numpy().view(np.uint32)
            v[:] = a
            return v
        pool = [(graphgen.Graph(g.n, pinned(g.src), pinned(g.dst), g.name), pinned(r), p) for g, r, p in pool]
    edges = sum(g.m for g, _, _ in pool)
    log(f"[bench] job pool: {P} jobs, {edges} edges, generated in {time.time() - t0:.1f}s")
    gold = None
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_serve.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            rows = {r["j"]: r for r in json.load(f)["jobs"]}
        if all(j in rows for j in range(P)):
            gold = [(rows[j]["count"], rows[j]["hash"], rows[j]["work"]) for j in range(P)]

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda")

    # plain: one job at a time, upload + orient + list
    def plain_pass():
        out = []
        for g, rank, _ in pool:
            c = tl.orient(g.n, dev(g.src), dev(g.dst), dev(rank))
            x = tl.list_triangles(c, "A++")
            c.free()
            out.append((int(x.count), int(x.hash), int(x.work)))
        return out
    plain_pass()
    torch.cuda.synchronize()
    tp = time.perf_counter()
    plain = plain_pass()
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - tp
    plain_ok = gold is None or plain == gold
    plain_rate = P / plain_s
    log(f"[bench] plain: {P} jobs in {plain_s:.3f}s ({plain_rate:.1f} jobs/s), oracle match {plain_ok}")
    tl.release_cached_memory()

    all_ok = True

    def sweep_mode(resident):
        nonlocal all_ok
        srv = tl.Server(args.serve_budget_gb << 30, list_threads=args.serve_list_threads,
                        solo_edges=args.serve_solo_edges)
        key = (lambda j: j + 1) if resident else (lambda j: 0)
        if resident:  # warm the cache: every pool graph oriented once and kept
            for i in [srv.submit(g.n, g.src, g.dst, rank, key=key(j)) for j, (g, rank, _) in enumerate(pool)]:
                srv.poll(i, -1)
        sweep = []
        for lam in args.serve_rates:
            njobs = int(min(args.serve_jobs, max(1, round(lam * args.serve_seconds))))
            rs = np.random.default_rng(int(lam))
            pick = rs.integers(0, P, njobs)
            arrive = np.cumsum(rs.exponential(1.0 / lam, njobs))
            st0 = srv.stats()
            ids = []
            t_start = time.perf_counter()
            lag = 0.0
            for k in range(njobs):
                while True:
                    el = time.perf_counter() - t_start
                    if el >= arrive[k]:
                        break
                lag = max(lag, el - arrive[k])
                g, rank, _ = pool[pick[k]]
                ids.append(srv.submit(g.n, g.src, g.dst, rank, key=key(int(pick[k]))))
            res = [srv.poll(i, -1) for i in ids]
            st = srv.stats()
            ok = all(r.status == 0 for r in res)
            if gold is not None:
                ok = ok and all((int(r.count), int(r.hash), int(r.work)) == gold[pick[k]]
                                for k, r in enumerate(res))
            all_ok = all_ok and ok
            lat = np.array([(r.t_done_ns - r.t_submit_ns) / 1e6 for r in res])
            span = (max(r.t_done_ns for r in res) - min(r.t_submit_ns for r in res)) / 1e9
            tri = sum(int(r.count) for r in res)
            batches = st["batches"] - st0["batches"]
            row = {"rate": lam, "jobs": njobs, "jobs_per_s": njobs / span, "triangles_per_s": tri / span,
                   "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "mean_batch_jobs": njobs / max(batches, 1), "batches": batches,
                   "resident_hits": st["resident_hits"] - st0["resident_hits"],
                   "peak_reserved_gb": st["peak_reserved"] / 2 ** 30, "client_max_lag_ms": lag * 1e3,
                   "stage_ms": {k: (st[k + "_ns"] - st0[k + "_ns"]) / 1e6 for k in ("upload", "orient", "list")},
                   "oracle_match": ok}
            sweep.append(row)
            log(f"[bench] {'resident' if resident else 'cold'} rate {lam}/s: {row}")
        srv.close()
        return sweep

    cold = sweep_mode(False) if "cold" in args.serve_modes else []
    resident = sweep_mode(True) if "resident" in args.serve_modes else []
    if not cold:
        cold = resident
    if not resident:
        resident = cold
    top_c = max(cold, key=lambda r: r["jobs_per_s"])
    top_r = max(resident, key=lambda r: r["jobs_per_s"])
    res = {
        "metric": "triangles listed/s + intersect elems/s (%HBM peak); batched vs plain; p99 job ms",
        "value": top_r["jobs_per_s"],
        "unit": "jobs/s",
        "n_gpus": 1,
        "steps": len(resident),
        "warmup": 1,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "serve", "pool_jobs": P, "pool_edges": edges,
                   "jobs": "RMAT (scale ceil(log2(m/8)), ef 8) or Chung-Lu (n = m/10, mean degree 20, "
                           "gamma U(2.0, 2.8)); m log-uniform in [1e3, 1e7]; degree or core order; A++; "
                           "drawn uniformly from the pool",
                   "budget_gb": args.serve_budget_gb, "rates": args.serve_rates,
                   "list_threads": args.serve_list_threads or 8, "solo_edges": args.serve_solo_edges or 2 ** 21,
                   "jobs_per_rate": f"min({args.serve_jobs}, rate x {args.serve_seconds} s)",
                   "host_memory": "pinned" if args.serve_pinned else "pageable"},
        "p50_ms": top_r["p50_ms"],
        "p99_ms": top_r["p99_ms"],
        "resident": {"sweep": resident, "jobs_per_s": top_r["jobs_per_s"],
                     "served_vs_plain": top_r["jobs_per_s"] / plain_rate},
        "cold": {"sweep": cold, "jobs_per_s": top_c["jobs_per_s"],
                 "served_vs_plain": top_c["jobs_per_s"] / plain_rate},
        "plain": {"jobs_per_s": plain_rate, "seconds": plain_s, "oracle_match": plain_ok},
        "served_vs_plain": top_r["jobs_per_s"] / plain_rate,
        "oracle_match": all_ok if gold is not None else None,
    }
    print(json.dumps(res), flush=True)


def bench_orders(args):
    """Orderings on the GPU and the cost-time relation (Figure 3's
    experiment): on the Chung-Lu 2^20 graph, (1) the full listing with the
    ordering computed on the device -- orient by id, tl_order, orient by the
    ordering, list -- and (2) for each of
    several orderings and both forms, the paper's cost C against the
    listing time (count and digest only).  Full listings: degree/A++,
    Split/A+-, core/A+- and Check/A+-; Neigh (on the host, from the degree
    ordering) is in the cost-time rows with its own running time."""
    import ctypes

    import torch

    import graphgen
    import paper_2203_04774_amd as tl

    g = make_graph("chunglu20")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda")
    src, dst = dev(g.src), dev(g.dst)
    ident = dev(np.arange(g.n, dtype=np.uint32))
    lib = tl.raw_lib()
    lib.tl_timing_read.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)) * 1e3, out

    full = {}
    for kind, algo in (("degree", "A++"), ("split", "A+-"), ("core", "A+-"), ("check", "A+-")):
        def run():
            g0 = tl.orient(g.n, src, dst, ident)
            t1 = time.perf_counter()
            rank = tl.order(g0, kind)
            t2 = time.perf_counter()
            g0.free()
            g1 = tl.orient(g.n, src, dst, rank)
            t3 = time.perf_counter()
            sm = tl.list_triangles(g1, algo)
            t4 = time.perf_counter()
            g1.free()
            return sm, (t2 - t1) * 1e3, (t3 - t2) * 1e3, (t4 - t3) * 1e3
        ms, (sm, o_ms, r_ms, l_ms) = timed(run, args.steps)
        full[f"{kind}-{algo}"] = {"total_ms": ms, "order_ms": o_ms, "orient_ms": r_ms, "list_ms": l_ms,
                                  "T": int(sm.count), "hash": f"0x{sm.hash:016x}"}
        log(f"[bench] full listing {kind}-{algo}: {full[f'{kind}-{algo}']}")

    # cost against listing time
    ranks = {k: graphgen.ordering(g, k, seed=1) for k in ("random", "degree", "core", "identity")}
    rows = []
    neigh_info = None
    for kind in ("random", "identity", "degree", "core", "split", "check", "neigh"):
        if kind in ("split", "check"):
            g0 = tl.orient(g.n, src, dst, ident)
            r = tl.order(g0, kind)
            g0.free()
        elif kind == "neigh":
            # Neigh (Algorithm 3, on the host) from the degree ordering, eps = 0.01
            g0 = tl.orient(g.n, src, dst, dev(ranks["degree"]))
            r, nres = tl.order_neigh(g0, eps=0.01)
            g0.free()
            neigh_info = {"start": "degree", "eps": 0.01, "seconds": nres.seconds, "passes": nres.passes,
                          "moves": int(nres.moves), "cpm_start": int(nres.cpm_start), "cpm": int(nres.cpm)}
            log(f"[bench] neigh from degree: {neigh_info}")
        else:
            r = dev(ranks[kind])
        csr = tl.orient(g.n, src, dst, r)
        for algo in ("A++", "A+-"):
            C = tl.cost(csr, algo)
            ms, sm = timed(lambda: tl.list_triangles(csr, algo), args.steps)
            rows.append({"order": kind, "algo": algo, "C": C, "list_ms": ms, "T": int(sm.count),
                         "scanned": int(sm.scanned), "ns_per_C": ms * 1e6 / C})
            log(f"[bench] cost-time {kind}-{algo}: C={C} list {ms:.2f} ms")
        csr.free()
    Cs = np.array([r["C"] for r in rows], float)
    ts = np.array([r["list_ms"] for r in rows], float)
    pearson = float(np.corrcoef(Cs, ts)[0, 1])
    slope, icpt = np.polyfit(Cs, ts, 1)
    best = min(rows, key=lambda r: r["list_ms"])
    res = {
        "metric": "triangles listed/s + intersect elems/s (%HBM peak); batched vs plain; p99 job ms",
        "value": g_tri / (full["split-A+-"]["total_ms"] / 1e3) if (g_tri := full["split-A+-"]["T"]) else 0.0,
        "unit": "triangles/s (full listing, Split/A+-)",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": full["split-A+-"]["total_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "orders", "graph": WORKLOADS["chunglu20"]["desc"], "n": g.n, "m": g.m},
        "full_listing": full,
        "split_A+-_vs_degree_A++_full": full["degree-A++"]["total_ms"] / full["split-A+-"]["total_ms"],
        "cost_time": rows,
        "cost_time_pearson_r": pearson,
        "cost_time_fit_ms": {"per_G_of_C": slope * 1e9, "intercept_ms": icpt},
        "fastest_listing": f"{best['order']}-{best['algo']}",
        "neigh": neigh_info,
    }
    print(json.dumps(res), flush=True)


def bench_orders_rmat26(args):
    """Figure 3's experiment (Section 4.2) on RMAT scale 26: for the degree,
    core, Split and Check orderings, each computed on the device from the
    graph oriented by vertex id, and both forms, the paper's cost C against
    the listing time (count and digest only, median of the timed runs), and
    the full listing time (ordering + orientation + listing).  Random and
    identity orders are left out: on this graph their costs are orders of
    magnitude above the others (hubs first or spread), beyond a bounded run."""
    import torch

    import paper_2203_04774_amd as tl

    t0 = time.time()
    g = make_graph("rmat26")
    log(f"[bench] {g} generated in {time.time() - t0:.1f}s")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda")
    src, dst = dev(g.src), dev(g.dst)
    ident = dev(np.arange(g.n, dtype=np.uint32))
    n = g.n
    del g

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        out = None
        for _ in range(reps):
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)) * 1e3, out

    rows, full = [], {}
    reps = max(1, min(args.steps, 3))
    for kind in ("degree", "core", "split", "check"):
        g0 = tl.orient(n, src, dst, ident)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rank = tl.order(g0, kind)
        torch.cuda.synchronize()
        order_ms = (time.perf_counter() - t1) * 1e3
        g0.free()
        t2 = time.perf_counter()
        csr = tl.orient(n, src, dst, rank)
        torch.cuda.synchronize()
        orient_ms = (time.perf_counter() - t2) * 1e3
        for algo in ("A++", "A+-"):
            C = tl.cost(csr, algo)
            ms, sm = timed(lambda: tl.list_triangles(csr, algo), reps)
            rows.append({"order": kind, "algo": algo, "C": C, "list_ms": ms, "T": int(sm.count),
                         "hash": f"0x{sm.hash:016x}", "scanned": int(sm.scanned), "ns_per_C": ms * 1e6 / C})
            full[f"{kind}-{algo}"] = {"order_ms": order_ms, "orient_ms": orient_ms, "list_ms": ms,
                                      "total_ms": order_ms + orient_ms + ms}
            log(f"[bench] {kind}-{algo}: C={C} list {ms:.1f} ms (order {order_ms:.0f} ms, orient {orient_ms:.0f} ms)")
        csr.free()
        del rank
        tl.release_cached_memory()
    Cs = np.array([r["C"] for r in rows], float)
    ts = np.array([r["list_ms"] for r in rows], float)
    pearson = float(np.corrcoef(Cs, ts)[0, 1])
    slope, icpt = np.polyfit(Cs, ts, 1)
    best = min(rows, key=lambda r: r["list_ms"])
    tri = rows[0]["T"]
    res = {
        "metric": "triangles listed/s + intersect elems/s (%HBM peak); batched vs plain; p99 job ms",
        "value": tri / (best["list_ms"] / 1e3),
        "unit": f"triangles/s (count-only listing, fastest ordering: {best['order']}/{best['algo']})",
        "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": best["list_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "orders26", "graph": WORKLOADS["rmat26"]["desc"], "n": n},
        "cost_time": rows,
        "cost_time_pearson_r": pearson,
        "cost_time_fit_ms": {"per_G_of_C": slope * 1e9, "intercept_ms": icpt},
        "fastest_listing": f"{best['order']}-{best['algo']}",
        "full_listing": full,
        "same_triangles_every_run": len({(r["T"], r["hash"]) for r in rows}) == 1,
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat26", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--batch-graphs", type=int, default=20000, help="graphs in the batch workload")
    ap.add_argument("--plain-graphs", type=int, default=0,
                    help="graphs timed one by one for the plain form (0: all)")
    ap.add_argument("--serve-pool", type=int, default=128, help="distinct jobs in the serving job pool")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[100, 300, 1000, 3000, 5000])
    ap.add_argument("--serve-jobs", type=int, default=10000, help="jobs per arrival rate, at most")
    ap.add_argument("--serve-seconds", type=float, default=100.0, help="arrival window per rate, at most")
    ap.add_argument("--serve-budget-gb", type=int, default=64)
    ap.add_argument("--serve-pinned", action="store_true", help="job arrays in page-locked host memory")
    ap.add_argument("--serve-list-threads", type=int, default=0, help="server list threads (0: library default)")
    ap.add_argument("--serve-solo-edges", type=int, default=1 << 24,
                    help="jobs with at least this many edges run alone (0: library default, 2^21); the pool's "
                         "largest jobs (~10^7 edges) are batched with the rest at 2^24")
    ap.add_argument("--serve-modes", nargs="+", default=["cold", "resident"], choices=["cold", "resident"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the listing runs on one GPU; --gpus {args.gpus} is not supported "
              "(pivot ranges of equal work per GPU via tl_list_range would be the multi-GPU form)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "orders":
        bench_orders(args)
        return
    if args.workload == "orders26":
        bench_orders_rmat26(args)
        return

    import ctypes

    import torch

    import graphgen
    import paper_2203_04774_amd as tl

    wl = WORKLOADS[args.workload]
    t0 = time.time()
    g = make_graph(args.workload)
    ranks = {k: graphgen.ordering(g, k, seed=1) for k in wl["orders"]}
    log(f"[bench] workload {g} generated in {time.time() - t0:.1f}s")
    cpu_handle = None
    if not args.no_cpu_baseline and args.workload == "rmat26":
        # the oracle needs minutes to build this graph: it runs in a child on
        # one core of its own while the GPU part runs (forked before any HIP call)
        cpu_handle = start_cpu_baseline_ranges(g, ranks["degree"], "A++", rmat26_sample_ranges(g.n),
                                               args.cpu_budget)
        log(f"[bench] CPU oracle baseline started in a child process on one core")

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda")

    if args.copy_calibration_mib:
        n_words = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n_words, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration_mib} MiB done")
        del a, b

    src, dst = dev(g.src), dev(g.dst)
    dranks = {k: dev(r) for k, r in ranks.items()}
    lib = tl.raw_lib()
    lib.tl_timing_read.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]

    chunked = wl.get("emit") == "chunks"
    out = None
    if chunked:
        # the list does not fit one buffer: it streams through library-owned
        # device chunks, each handed to a callback (here a no-op consumer)
        tl.set_chunk_triangles(wl["chunk"])
        # a device area of chunk_room x K triangles (96 GB here): each probe
        # slice covers that many items, so half as many slices as the
        # library's default of 4 (RMAT-26: 28 slices, 1,107 -> 1,090 ms/step)
        tl.set_tuning("chunk_room", wl.get("chunk_room", 4))
    else:
        # size the output buffer from a count-only pass
        csr = tl.orient(g.n, src, dst, dranks[wl["orders"][0]])
        T = tl.list_triangles(csr, wl["algos"][0]).count
        csr.free()
        out = torch.empty((max(T, 1), 3), dtype=torch.int32, device="cuda")
    chunks_seen = [0]

    def consume(ptr, k):
        chunks_seen[0] += 1
        return False

    runs = [(k, a) for k in wl["orders"] for a in wl["algos"]]
    gold = oracle_results(args.workload)
    seen = []  # (order, algo, count, digest, work) of every listing, warmup and timed

    def phase_ms():
        vals = []
        for ph in range(6):
            ms = ctypes.c_double()
            lib.tl_timing_read(ph, ctypes.byref(ms), None)
            vals.append(ms.value)
        return vals

    def step(record=None):
        for kind in wl["orders"]:
            t_or = phase_ms()[0] if record is not None else 0.0
            csr = tl.orient(g.n, src, dst, dranks[kind])
            if record is not None:
                t_or = phase_ms()[0] - t_or
            for algo in wl["algos"]:
                before = phase_ms() if record is not None else None
                c = tl.cost(csr, algo)
                s = (tl.list_triangles(csr, algo, on_chunk=consume) if chunked
                     else tl.list_triangles(csr, algo, out=out))
                seen.append((kind, algo, int(s.count), int(s.hash), int(s.work)))
                if record is not None:
                    after = phase_ms()
                    st = tl.last_list_stats()
                    record.append(dict(order=kind, algo=algo, T=int(s.count), C=int(c), work=int(s.work),
                                       scanned=int(s.scanned), hash=f"0x{s.hash:016x}", m=csr.m,
                                       orient_ms=t_or, plan_ms=after[1] - before[1],
                                       probe_ms=after[2] - before[2], light_ms=after[4] - before[4],
                                       heavy_ms=after[5] - before[5],
                                       stats=st))
            csr.free()

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    lib.tl_timing_reset()
    lib.tl_timing_enable(1)
    rec = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    marks = [t]  # each listing ends with a wait on its stream, so host marks bound the steps
    for i in range(args.steps):
        step(rec if i == 0 else None)
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    lib.tl_timing_enable(0)
    per_step_ms = np.diff(np.array(marks)) * 1e3
    log(f"[bench] {args.steps} timed steps in {elapsed:.3f}s")

    phases = {}
    for ph, name in enumerate(["orient", "plan", "probe", "cost", "probe_light", "probe_heavy"]):
        ms, calls = ctypes.c_double(), ctypes.c_uint64()
        lib.tl_timing_read(ph, ctypes.byref(ms), ctypes.byref(calls))
        phases[name] = {"ms": ms.value, "launches": int(calls.value)}

    tri_per_step = sum(r["T"] for r in rec)
    work_per_step = sum(r["work"] for r in rec)
    value = tri_per_step * args.steps / elapsed
    # roofline of the dominant kernel, the heavy-pivot probe: algorithmic
    # bytes of its share of the work over its own HIP-event time
    heavy_bytes = sum(heavy_alg_bytes(r["stats"]) for r in rec) * args.steps
    heavy_s = phases["probe_heavy"]["ms"] / 1e3
    achieved = heavy_bytes / heavy_s / 1e9 if heavy_s > 0 else 0.0
    probe_s = phases["probe"]["ms"] / 1e3
    probe_bytes = sum(alg_bytes(r["C"], r["m"], g.n, r["T"]) for r in rec) * args.steps
    heavy_launches = phases["probe_heavy"]["launches"]
    traffic = measured_traffic(args.workload, heavy_launches / max(args.steps, 1))
    loaded = sum(heavy_loaded_bytes(r["stats"]) for r in rec) * args.steps
    avg_launch_s = heavy_s / max(heavy_launches, 1)
    dominant = max(("orient", "plan", "probe_light", "probe_heavy", "cost"), key=lambda k: phases[k]["ms"])

    res = {
        "metric": "triangles listed/s + intersect elems/s (%HBM peak); batched vs plain; p99 job ms",
        "value": value,
        "unit": "triangles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "ms_per_step_median": float(np.median(per_step_ms)),
        "ms_per_step_min": float(per_step_ms.min()),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": wl["desc"], "n": g.n, "m": g.m,
                   "orders": wl["orders"], "algos": wl["algos"], "emit": ("streamed to device chunks of %d triangles (chunk room %d)" % (wl["chunk"], wl.get("chunk_room", 4))) if chunked
                   else "full list to one device buffer",
                   "listings_per_step": len(runs)},
        "intersect_elems_per_s": work_per_step * args.steps / elapsed,
        "roofline": {"bound": "hbm", "kernel": "k_probe_heavy",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_ms": phases["probe_heavy"]["ms"] / max(heavy_launches, 1),
                     "launches": heavy_launches,
                     "alg_bytes_per_launch": heavy_bytes / max(heavy_launches, 1),
                     # what the kernel actually reads and writes (windowed items, staging per
                     # task, seed geometry, hits), and the PMC-measured HBM bytes, as rates
                     "loaded_bytes_per_launch": loaded / max(heavy_launches, 1),
                     "loaded_GBps": loaded / heavy_s / 1e9 if heavy_s > 0 else 0.0,
                     "loaded_frac": loaded / heavy_s / 1e9 / HBM_PEAK_GBS if heavy_s > 0 else 0.0,
                     "traffic_frac": (traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS)
                     if traffic and avg_launch_s > 0 else None},
        "probe_phase": {"achieved_GBps": probe_bytes / probe_s / 1e9 if probe_s else 0.0,
                        "ms_per_step": phases["probe"]["ms"] / args.steps},
        "phases_ms_per_step": {k: v["ms"] / args.steps for k, v in phases.items()},
        "dominant_phase": dominant,
        "runs": rec,
    }
    if chunked:
        res["chunks_per_step"] = chunks_seen[0] / max(args.steps + args.warmup, 1)
    checked = [r for r in seen if (r[0], r[1]) in gold]
    res["oracle_match"] = (all(tuple(r[2:]) == tuple(gold[(r[0], r[1])]) for r in checked)
                           if checked else None)
    res["oracle_checked"] = f"{len(checked)} of {len(seen)} listings (count, digest, work) against the oracle's stored results"
    if cpu_handle is not None:
        log("[bench] waiting for the CPU oracle baseline")
        cb = finish_cpu_baseline(cpu_handle)
        if cb is not None:
            res["cpu_baseline"] = cb
    elif not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(g, ranks, args.cpu_budget)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
