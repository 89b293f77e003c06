"""Consistency of the stored oracle results (CPU only).

The RMAT scale 26 results were written piece by piece by
tests/golden/make_expected_rmat26.py (oracle only); the pieces must tile the
pivot ranks [0, n) and add up to the stored whole listing, since the count,
the wrap-around digest sum and the work are all additive over pivot ranges
(each triangle is listed once, at its pivot; Definition 1 sums over pivots).
bench.py checks its listings against the same stored totals."""
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
MASK64 = (1 << 64) - 1


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_rmat26_pieces_tile_the_ranks_and_sum_to_the_listing():
    g = _load("oracle_rmat26.json")
    parts = g["partition"]
    assert parts[0][0] == 0 and parts[-1][1] == g["n"]
    assert all(parts[i][1] == parts[i + 1][0] for i in range(len(parts) - 1))
    assert all(lo < hi for lo, hi, *_ in parts)
    whole = g["list"]["A++"]
    assert sum(p[2] for p in parts) == whole["count"]
    assert sum(p[3] for p in parts) & MASK64 == whole["hash"]
    assert sum(p[4] for p in parts) == whole["work"]
    # A++'s work is the paper's cost C++ of the same ordering
    assert whole["work"] == g["cost"]["A++"]


def test_rmat26_samples_lie_inside_the_ranks():
    g = _load("oracle_rmat26.json")
    assert len(g["samples"]) >= 4
    for smp in g["samples"]:
        assert 0 <= smp["lo"] < smp["hi"] <= g["n"]
        assert smp["count"] >= 0 and smp["work"] >= 0
        if smp["count"] == 0:
            assert smp["hash"] == 0


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("workload", ["rmat26", "chunglu20", "rmat12"])
def test_bench_reads_the_stored_results(workload):
    res = _bench().oracle_results(workload)
    assert res
    if workload == "rmat26":
        w = _load("oracle_rmat26.json")["list"]["A++"]
        assert res[("degree", "A++")] == (w["count"], w["hash"], w["work"])
    else:
        d = _load("oracle_expected.json")[workload + "_s1"]
        for (kind, algo), v in res.items():
            r = d["orders"][kind]["list"][algo]
            assert v == (r["count"], r["hash"], r["work"])
        # every order lists the same triangles
        assert len({(c, h) for c, h, _ in res.values()}) == 1
