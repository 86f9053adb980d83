#!/usr/bin/env python3
"""Summarises rocprofv3 --pmc CSV output (one directory per counter pass)
into per-kernel means, scaled to bytes with a copy-kernel calibration.

Usage: counters_summary.py OUT.json --copy-fetch DIR --copy-write DIR
           --pass NAME=DIR [--pass ...] [--extra FACTS.json] [--note TEXT]
           [--command TEXT ...]

The profiling script settles its population, idles for a second, then makes
the counted sweeps: dispatches before the first gap of at least half a
second between dispatch starts are left out (a pass with no such gap is
taken whole).  FACTS.json (the profiling script's own output) names the sweep kernel
and the attempts of the counted sweeps; that kernel gets the attempts per
dispatch.

FETCH_SIZE and WRITE_SIZE are reported by the profiler in KiB per
dispatch; the calibration passes ran an elementwise int32 copy that reads
and writes exactly 1 GiB, so bytes = counter KiB x 1024 x (2^30 / the copy's
counter value in bytes).  Every other counter is averaged per dispatch as
it is.  Kernel names are shortened to the part before the argument list."""
import argparse
import collections
import csv
import glob
import json
import os
import statistics


def short(name):
    """The kernel's name and template arguments, without namespace, return
    type or argument list."""
    for p in ("void ", "pamc::(anonymous namespace)::"):
        name = name.replace(p, "")
    depth = 0
    for i, ch in enumerate(name):
        depth += (ch == "<") - (ch == ">")
        if ch == "(" and depth == 0:
            return name[:i].strip()
    return name.strip()


GAP_NS = 500_000_000


def load(d):
    files = glob.glob(os.path.join(d, "*_counter_collection.csv"))
    if not files:
        raise SystemExit(f"no counter CSV under {d}")
    rows = sorted(csv.DictReader(open(files[0])), key=lambda r: int(r["Dispatch_Id"]))
    starts = sorted({(int(r["Start_Timestamp"]), r["Dispatch_Id"]) for r in rows})
    first = None  # the first dispatch after the settling gap
    for (t0, _), (t1, i1) in zip(starts, starts[1:]):
        if t1 - t0 >= GAP_NS:
            first = t1
            break
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(dict)
    for row in rows:
        k = short(row["Kernel_Name"])
        if first is not None and int(row["Start_Timestamp"]) < first:
            continue
        per[k][row["Counter_Name"]].append(float(row["Counter_Value"]))
        dur[k][row["Dispatch_Id"]] = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
    return per, dur


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--pass", dest="passes", action="append", default=[])
    ap.add_argument("--note", default="")
    ap.add_argument("--command", action="append", default=[], help="a command that made the passes")
    ap.add_argument("--extra", default=None, help="the profiling script's JSON output (kernel, attempts, ...)")
    a = ap.parse_args()
    cf, _ = load(a.copy_fetch)
    cw, _ = load(a.copy_write)
    (cfk,), (cwk,) = list(cf), list(cw)
    gib = float(1 << 30)
    fetch_scale = gib / (statistics.mean(cf[cfk]["FETCH_SIZE"]) * 1024)
    write_scale = gib / (statistics.mean(cw[cwk]["WRITE_SIZE"]) * 1024)
    kernels = collections.defaultdict(dict)
    for spec in a.passes:
        name, d = spec.split("=", 1)
        per, dur = load(d)
        for k, ctrs in per.items():
            e = kernels[k]
            for c, xs in ctrs.items():
                e[c] = statistics.mean(xs)
                e.setdefault("dispatches", len(xs))
            e.setdefault("mean_dispatch_ns_under_counters", statistics.mean(dur[k].values()))
    for k, e in kernels.items():
        if "FETCH_SIZE" in e:
            e["hbm_fetch_bytes_per_dispatch"] = e["FETCH_SIZE"] * 1024 * fetch_scale
        if "WRITE_SIZE" in e:
            e["hbm_write_bytes_per_dispatch"] = e["WRITE_SIZE"] * 1024 * write_scale
        if "FETCH_SIZE" in e and "WRITE_SIZE" in e:
            e["hbm_bytes_per_dispatch"] = e["hbm_fetch_bytes_per_dispatch"] + e["hbm_write_bytes_per_dispatch"]
    facts = json.load(open(a.extra)) if a.extra else {}
    main_k = facts.get("kernel")
    if main_k in kernels and facts.get("attempts"):
        kernels[main_k]["attempts_per_dispatch"] = facts["attempts"] / kernels[main_k]["dispatches"]
        if "hbm_bytes_per_dispatch" in kernels[main_k]:
            kernels[main_k]["hbm_bytes_per_attempt"] = (kernels[main_k]["hbm_bytes_per_dispatch"] /
                                                        kernels[main_k]["attempts_per_dispatch"])
    out = {"note": a.note, "commands": a.command, "facts": facts,
           "copy_calibration": {"kernel": cfk[:80], "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                                "FETCH_SIZE_KiB": statistics.mean(cf[cfk]["FETCH_SIZE"]),
                                "WRITE_SIZE_KiB": statistics.mean(cw[cwk]["WRITE_SIZE"]),
                                "fetch_scale": fetch_scale, "write_scale": write_scale},
           "kernels": kernels}
    json.dump(out, open(a.out, "w"), indent=1, sort_keys=True)
    for k, e in kernels.items():
        print(k, {x: round(v, 1) for x, v in e.items()})


if __name__ == "__main__":
    main()
