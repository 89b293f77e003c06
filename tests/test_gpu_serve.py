"""GPU tests of the listing server (continuous batching under a device
memory budget).

Every served result must equal the oracle's for that job alone, whatever
batch it was listed in (exact: counts, digests and work are integers);
admission, rejection, cancellation and malformed input are forced from the
host.  Expected values come from tests/golden/oracle_serve.json (written by
make_expected_serve.py, which calls only the oracle).
"""
import json
import os

import numpy as np
import pytest

import graphgen
import graphs as G
import oracle
from gpu_util import GOLDEN

pytestmark = pytest.mark.gpu

GB = 1 << 30


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_04774_amd as tl
    return tl


@pytest.fixture(scope="module")
def pool():
    """Small jobs of the serving pool (target m <= 300000) with their
    oracle results."""
    with open(os.path.join(GOLDEN, "oracle_serve.json")) as f:
        gold = {r["j"]: r for r in json.load(f)["jobs"]}
    jobs = []
    for j in sorted(gold):
        if gold[j]["m_target"] > 300_000:
            continue
        g, rank, p = graphgen.serve_job(j)
        assert (g.n, g.m) == (gold[j]["n"], gold[j]["m"])
        jobs.append((j, g, rank, (gold[j]["count"], gold[j]["hash"], gold[j]["work"])))
        if len(jobs) == 40:
            break
    return jobs


def result_tuple(r):
    return (int(r.count), int(r.hash), int(r.work))


def run_burst(tl, srv, jobs):
    """Queue all jobs while admission is paused, then let them in."""
    srv.pause(True)
    ids = [srv.submit(g.n, g.src, g.dst, rank) for (_, g, rank, _) in jobs]
    srv.pause(False)
    return [srv.poll(i, -1) for i in ids]


def test_served_results_match_oracle(tl, pool):
    srv = tl.Server(8 * GB)
    try:
        res = run_burst(tl, srv, pool)
        for (j, _, _, want), r in zip(pool, res):
            assert r.status == 0, j
            assert result_tuple(r) == want, j
            assert r.t_submit_ns <= r.t_admit_ns <= r.t_start_ns <= r.t_done_ns
        st = srv.stats()
        assert st["jobs_done"] == len(pool)
        assert st["batches"] < len(pool)  # jobs were batched together
        assert st["peak_reserved"] <= 8 * GB
    finally:
        srv.close()


def test_same_result_alone_and_in_the_mix(tl, pool):
    j, g, rank, want = pool[3]
    srv = tl.Server(8 * GB)
    try:
        alone = srv.poll(srv.submit(g.n, g.src, g.dst, rank), -1)
        assert alone.status == 0 and alone.batch_jobs == 1
        mix = pool[:20] + [pool[3]] + pool[20:]
        res = run_burst(tl, srv, mix)
        inmix = res[20]
        assert inmix.status == 0 and inmix.batch_jobs > 1
        assert result_tuple(alone) == result_tuple(inmix) == want
        for (jj, _, _, w), r in zip(mix, res):
            assert result_tuple(r) == w, jj
    finally:
        srv.close()


def test_jobs_arriving_while_others_run_are_admitted(tl, pool):
    """Submissions interleaved with completions: later jobs join later
    batches while earlier ones are on the device."""
    srv = tl.Server(8 * GB)
    try:
        ids = []
        for k, (_, g, rank, _) in enumerate(pool):
            ids.append(srv.submit(g.n, g.src, g.dst, rank))
            if k == 10:
                first = srv.poll(ids[0], -1)
                assert first.status == 0
        res = [first] + [srv.poll(i, -1) for i in ids[1:]]
        for (j, _, _, want), r in zip(pool, res):
            assert r.status == 0 and result_tuple(r) == want, j
    finally:
        srv.close()


@pytest.mark.parametrize("pipeline", [False, True])
@pytest.mark.parametrize("solo_edges", [0, 1000])
@pytest.mark.parametrize("list_threads", [1, 4])
def test_batching_modes_agree(tl, pool, pipeline, solo_edges, list_threads):
    """Every batching mode, with one or several batches listed at once,
    gives each job the oracle's result."""
    srv = tl.Server(8 * GB, max_batch_jobs=7, solo_edges=solo_edges, pipeline=pipeline, list_threads=list_threads)
    try:
        res = run_burst(tl, srv, pool[:16])
        for (j, _, _, want), r in zip(pool[:16], res):
            assert r.status == 0 and result_tuple(r) == want, j
        if solo_edges == 1000:
            assert all(r.batch_jobs == 1 for r in res)
    finally:
        srv.close()


def test_tight_budget_queues_and_rejects(tl, pool):
    sizes = [tl.Server.job_bytes(g.n, g.m) for (_, g, _, _) in pool[:12]]
    budget = sorted(sizes)[-2] + 1  # the largest job can never fit; the rest run a few at a time
    big = int(np.argmax(sizes))
    srv = tl.Server(budget)
    try:
        res = run_burst(tl, srv, pool[:12])
        for k, ((j, _, _, want), r) in enumerate(zip(pool[:12], res)):
            if k == big:
                assert r.status == tl.tl.TL_ENOMEM
            else:
                assert r.status == 0 and result_tuple(r) == want, j
        st = srv.stats()
        assert st["rejected"] == 1 and st["peak_reserved"] <= budget
    finally:
        srv.close()


def test_malformed_job_fails_alone(tl, pool):
    bad_rank = np.zeros(pool[4][1].n, np.uint32)  # not a permutation
    srv = tl.Server(8 * GB)
    try:
        srv.pause(True)
        ids = []
        for k, (_, g, rank, _) in enumerate(pool[:10]):
            ids.append(srv.submit(g.n, g.src, g.dst, bad_rank if k == 4 else rank))
        n, s, d = G.complete(5)  # an endpoint out of range
        ids.append(srv.submit(3, s, d, np.arange(3, dtype=np.uint32)))
        srv.pause(False)
        res = [srv.poll(i, -1) for i in ids]
        for k, ((j, _, _, want), r) in enumerate(zip(pool[:10], res)):
            if k == 4:
                assert r.status == tl.tl.TL_EINVAL
            else:
                assert r.status == 0 and result_tuple(r) == want, j
        assert res[-1].status == tl.tl.TL_EINVAL
        assert srv.stats()["split_batches"] >= 1
    finally:
        srv.close()


def test_cancel_waiting_job(tl, pool):
    srv = tl.Server(8 * GB)
    try:
        srv.pause(True)
        ids = [srv.submit(g.n, g.src, g.dst, rank) for (_, g, rank, _) in pool[:3]]
        assert srv.cancel(ids[1]) == tl.tl.TL_OK
        srv.pause(False)
        res = [srv.poll(i, -1) for i in ids]
        assert res[1].status == tl.tl.TL_EABORT
        for k in (0, 2):
            assert res[k].status == 0 and result_tuple(res[k]) == pool[k][3]
        assert srv.cancel(ids[0]) == tl.tl.TL_EINVAL  # final and handed out: unknown now
        assert srv.stats()["cancelled"] == 1
    finally:
        srv.close()


def test_all_algorithms_served(tl, pool):
    srv = tl.Server(8 * GB)
    try:
        jobs = pool[:6]
        srv.pause(True)
        ids = [(a, k, srv.submit(g.n, g.src, g.dst, rank, algo=a))
               for k, (_, g, rank, _) in enumerate(jobs) for a in ("A++", "A+-", "A--")]
        srv.pause(False)
        for a, k, i in ids:
            r = srv.poll(i, -1)
            _, g, rank, _ = jobs[k]
            L = oracle.list_triangles(g.n, g.src, g.dst, rank, a, want_triangles=False)
            assert r.status == 0 and result_tuple(r) == (L.count, L.hash, L.work), (a, k)
    finally:
        srv.close()


def test_destroy_with_waiting_jobs(tl, pool):
    srv = tl.Server(8 * GB)
    srv.pause(True)
    for (_, g, rank, _) in pool[:5]:
        srv.submit(g.n, g.src, g.dst, rank)
    srv.close()  # cancels the waiting jobs and returns


@pytest.mark.slow
def test_large_jobs_under_64gb_budget(tl):
    """The pool's jobs of 2^21 edges and more (listed alone, by the plain
    path with its heavy forms) mixed with small ones, under the workload's
    64 GB device budget: every result equals the oracle's."""
    with open(os.path.join(GOLDEN, "oracle_serve.json")) as f:
        gold = {r["j"]: r for r in json.load(f)["jobs"]}
    big = [j for j in sorted(gold) if gold[j]["m"] >= (1 << 21)]
    small = [j for j in sorted(gold) if gold[j]["m"] < 100_000][:24]
    assert len(big) >= 10
    order = [x for pair in zip(big, small) for x in pair] + small[len(big):]
    jobs = []
    for j in order:
        g, rank, _ = graphgen.serve_job(j)
        assert (g.n, g.m) == (gold[j]["n"], gold[j]["m"])
        jobs.append((j, g, rank, (gold[j]["count"], gold[j]["hash"], gold[j]["work"])))
    srv = tl.Server(64 * GB)
    try:
        res = run_burst(tl, srv, jobs)
        for (j, g, _, want), r in zip(jobs, res):
            assert r.status == 0, j
            assert result_tuple(r) == want, j
            if g.m >= (1 << 21):
                assert r.batch_jobs == 1, j  # the solo path
        st = srv.stats()
        assert st["jobs_done"] == len(jobs)
        assert st["peak_reserved"] <= 64 * GB
    finally:
        srv.close()


def test_keyed_jobs_stay_resident(tl, pool):
    """Jobs with a key: the first of each key is oriented and kept resident,
    the repeats are listed from the resident graph (no upload, no
    orientation); every result equals the oracle's, alone or in the mix."""
    jobs = pool[:24]
    srv = tl.Server(8 * GB)
    try:
        ids = [srv.submit(g.n, g.src, g.dst, rank, key=j + 1) for (j, g, rank, _) in jobs]
        first = [srv.poll(i, -1) for i in ids]
        for (j, _, _, want), r in zip(jobs, first):
            assert r.status == 0 and result_tuple(r) == want, j
        st0 = srv.stats()
        assert st0["resident_graphs"] == len(jobs)
        # repeats, in another order, in bursts: all resident
        order = list(reversed(jobs)) * 3
        res = run_burst_keyed(tl, srv, order)
        for (j, _, _, want), r in zip(order, res):
            assert r.status == 0 and result_tuple(r) == want, j
        st = srv.stats()
        assert st["resident_hits"] - st0["resident_hits"] == len(order)
        assert st["batches"] - st0["batches"] < len(order)  # repeats were batched together
        assert st["peak_reserved"] <= 8 * GB
    finally:
        srv.close()


def run_burst_keyed(tl, srv, jobs):
    srv.pause(True)
    ids = [srv.submit(g.n, g.src, g.dst, rank, key=j + 1) for (j, g, rank, _) in jobs]
    srv.pause(False)
    return [srv.poll(i, -1) for i in ids]


def test_keyed_and_unkeyed_mixed(tl, pool):
    jobs = pool[:16]
    srv = tl.Server(8 * GB)
    try:
        srv.pause(True)
        ids = []
        for k, (j, g, rank, _) in enumerate(jobs * 2):
            ids.append(srv.submit(g.n, g.src, g.dst, rank, key=(j + 1) if k % 3 else 0))
        srv.pause(False)
        for (j, _, _, want), i in zip(jobs * 2, ids):
            r = srv.poll(i, -1)
            assert r.status == 0 and result_tuple(r) == want, j
    finally:
        srv.close()


def test_resident_graphs_dropped_under_a_tight_budget(tl, pool):
    """A budget that holds only a few resident graphs: the least recently
    used are dropped to admit new jobs, and results stay exact."""
    jobs = pool[:12]
    one = max(tl.Server.job_bytes(g.n, g.m) for (_, g, _, _) in jobs)
    budget = int(1.4 * one)  # one job at a time and about one resident graph beside it
    srv = tl.Server(budget)
    try:
        for rep in range(2):
            res = run_burst_keyed(tl, srv, jobs)
            for (j, _, _, want), r in zip(jobs, res):
                assert r.status == 0 and result_tuple(r) == want, (rep, j)
        st = srv.stats()
        assert st["resident_dropped"] >= 1
        assert st["peak_reserved"] <= budget
    finally:
        srv.close()


def test_keyed_malformed_job_fails_alone(tl, pool):
    bad_rank = np.zeros(pool[2][1].n, np.uint32)
    srv = tl.Server(8 * GB)
    try:
        srv.pause(True)
        ids = []
        for k, (j, g, rank, _) in enumerate(pool[:6]):
            ids.append(srv.submit(g.n, g.src, g.dst, bad_rank if k == 2 else rank, key=1000 + k))
        srv.pause(False)
        for k, ((j, _, _, want), i) in enumerate(zip(pool[:6], ids)):
            r = srv.poll(i, -1)
            if k == 2:
                assert r.status == tl.tl.TL_EINVAL
            else:
                assert r.status == 0 and result_tuple(r) == want, j
        assert srv.stats()["resident_graphs"] == 5
    finally:
        srv.close()
