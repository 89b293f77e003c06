"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2203_04774_amd.profiling stats  <kernel_stats.csv> <out.md> <command...>
    python -m paper_2203_04774_amd.profiling traffic <fetch_counter_collection.csv> \
        <write_counter_collection.csv> <calibration MiB> <workload> <out.json> <command...>

`counters` averages the counters of `--pmc` passes per dispatch for the
probe and plan kernels.  `stats` turns a `--kernel-trace --stats` kernel_stats.csv into a short
markdown table.  `traffic` combines two `--pmc FETCH_SIZE` / `--pmc
WRITE_SIZE` runs of `bench.py --steps 1 --warmup 0 --copy-calibration-mib N`:
the plain device copy of N MiB at the start of the run calibrates the
counters (bytes the copy must move / bytes the counter reports), and the
heavy-pivot probe kernel's per-dispatch bytes are scaled by that factor.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0] if not name.startswith("void ") else name[5:].split("(")[0]


def list_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("list.hip", "dev_util.h", "probe_common.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats(csv_path: str, out_md: str, command: str, top: int = 25) -> None:
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
             f"Total kernel time {total / 1e6:.2f} ms over {sum(int(r['Calls']) for r in rows)} dispatches.", "",
             "| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_dispatch(path: str):
    """{dispatch_id: (kernel, value_kib)} summed over counter instances."""
    out = {}
    for r in csv.DictReader(open(path)):
        d = int(r["Dispatch_Id"])
        k, v = out.get(d, (r["Kernel_Name"], 0.0))
        out[d] = (k, v + float(r["Counter_Value"]))
    return out


def traffic(fetch_csv: str, write_csv: str, calib_mib: float, workload: str, out_json: str, command: str) -> dict:
    fetch, write = _per_dispatch(fetch_csv), _per_dispatch(write_csv)
    calib_bytes = calib_mib * (1 << 20)

    def copy_factor(d):
        # the calibration copy is the first rocclr copy kernel of about the calibration size
        for _, (k, v) in sorted(d.items()):
            if "copyBuffer" in k and v * 1024 > 0.25 * calib_bytes:
                return calib_bytes / (v * 1024), v * 1024
        raise SystemExit("no calibration copy found")

    f_fac, f_raw = copy_factor(fetch)
    w_fac, w_raw = copy_factor(write)
    per_kernel = defaultdict(lambda: {"launches": 0, "fetch": 0.0, "write": 0.0})
    for src, key, fac in ((fetch, "fetch", f_fac), (write, "write", w_fac)):
        for _, (k, v) in src.items():
            name = short_name(k)
            per_kernel[name][key] += v * 1024 * fac
            if key == "fetch":
                per_kernel[name]["launches"] += 1
    # the emitting heavy-pivot kernels: k_probe_heavy<form, true, lean>
    heavy = [n for n in per_kernel if n.startswith("k_probe_heavy<") and n.split(",")[1].strip() == "true"]
    hb = sum(per_kernel[n]["fetch"] + per_kernel[n]["write"] for n in heavy)
    hl = sum(per_kernel[n]["launches"] for n in heavy)
    res = {
        "workload": workload,
        "command": command,
        "source_digest": list_source_digest(),
        "calibration": {"copy_bytes": calib_bytes, "fetch_counter_bytes": f_raw, "write_counter_bytes": w_raw,
                        "fetch_factor": f_fac, "write_factor": w_fac},
        "heavy_kernels": heavy,
        "heavy_launches": hl,
        "heavy_bytes_per_launch": hb / hl if hl else None,
        "per_kernel_bytes_per_launch": {n: {"fetch": v["fetch"] / max(v["launches"], 1),
                                            "write": v["write"] / max(v["launches"], 1),
                                            "launches": v["launches"]}
                                        for n, v in sorted(per_kernel.items(), key=lambda kv: -kv[1]["fetch"])[:20]},
    }
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    return res


def traffic_md(json_path: str, out_md: str) -> None:
    """Renders a traffic JSON (from traffic()) as a short markdown table."""
    with open(json_path) as f:
        d = json.load(f)
    c = d["calibration"]
    lines = [f"# HBM traffic per kernel launch, {d['workload']} workload", "",
             "Commands (two separate counter runs):", "", "```"]
    lines += [part.strip() for part in d["command"].split(" ; ")]
    lines += ["```", "",
              f"Calibration: the run starts with a plain {c['copy_bytes'] / 2**30:.0f} GiB device copy; "
              f"FETCH_SIZE reported {c['fetch_counter_bytes']:.0f} bytes for it (factor {c['fetch_factor']:.3f}), "
              f"WRITE_SIZE {c['write_counter_bytes']:.0f} bytes (factor {c['write_factor']:.3f}). Every kernel's "
              "counter value is scaled by these factors.", "",
              f"Kernel source digest (list.hip, dev_util.h, probe_common.h): `{d['source_digest']}`; bench.py "
              "reports these bytes as `roofline.traffic` only while the digest matches the sources.", "",
              f"Emitting heavy-pivot kernel ({', '.join(d['heavy_kernels'])}): "
              f"{d['heavy_bytes_per_launch'] / 1e9:.3f} GB per launch over {d['heavy_launches']} launches.", "",
              "| kernel | launches | fetched GB / launch | written GB / launch |", "|---|---:|---:|---:|"]
    for k, v in d["per_kernel_bytes_per_launch"].items():
        lines.append(f"| `{k}` | {v['launches']} | {v['fetch'] / 1e9:.3f} | {v['write'] / 1e9:.3f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(csv_paths, out_md: str, command: str, kernels=("k_probe_heavy", "k_probe_light", "k_plan")) -> dict:
    """Per-dispatch averages of every counter in one or more `--pmc` runs
    (counter_collection.csv files, one per pass), for the kernels whose
    names start with one of `kernels`; writes a markdown table and returns
    {kernel: {counter: average per dispatch}}."""
    acc = defaultdict(lambda: defaultdict(float))   # (kernel) -> counter -> sum over dispatches
    disp = defaultdict(lambda: defaultdict(set))    # (kernel) -> counter -> dispatch ids
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            if not k.startswith(tuple(kernels)):
                continue
            c = r["Counter_Name"]
            acc[k][c] += float(r["Counter_Value"])
            disp[k][c].add(int(r["Dispatch_Id"]))
    res = {k: {c: acc[k][c] / len(disp[k][c]) for c in acc[k]} for k in acc}
    names = sorted({c for k in res for c in res[k]})
    lines = ["# rocprofv3 counters per dispatch", "", "Commands (one counter pass each):", "", "```"]
    lines += [part.strip() for part in command.split(" ; ")]
    lines += ["```", "", "Average per dispatch of each counter (summed over the counter's hardware instances).", "",
              "| kernel | dispatches | " + " | ".join(names) + " |", "|---|---:|" + "---:|" * len(names)]
    for k in sorted(res):
        n = max(len(v) for v in disp[k].values())
        lines.append(f"| `{k}` | {n} | " + " | ".join(f"{res[k].get(c, float('nan')):.4g}" for c in names) + " |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return res


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6], " ".join(sys.argv[7:]))
    elif sys.argv[1] == "traffic-md":
        traffic_md(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "counters":
        # counters <out.md> <csv> [<csv> ...] -- <command>
        i = sys.argv.index("--")
        counters(sys.argv[3:i], sys.argv[2], " ".join(sys.argv[i + 1:]))
    else:
        raise SystemExit(__doc__)
