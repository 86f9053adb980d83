#!/usr/bin/env python3
"""Summarises rocprofv3 --pmc CSV output (one directory per counter pass)
into per-kernel means, scaled to bytes with a copy-kernel calibration.

Usage: counters_summary.py OUT.json --copy-fetch DIR --copy-write DIR
           --pass NAME=DIR[:SKIP] [--pass ...] [--note TEXT] [--command TEXT ...]

SKIP drops each kernel's first SKIP dispatches of that pass (the settling
sweeps the profiling driver makes before the counted ones).

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
    name = name.split("(pamc::")[0].split("(int,")[0]
    for p in ("void ", "pamc::(anonymous namespace)::"):
        name = name.replace(p, "")
    return name.strip()


def load(d, skip=0):
    files = glob.glob(os.path.join(d, "*_counter_collection.csv"))
    if not files:
        raise SystemExit(f"no counter CSV under {d}")
    rows = sorted(csv.DictReader(open(files[0])), key=lambda r: int(r["Dispatch_Id"]))
    seen = collections.defaultdict(list)  # kernel -> dispatch ids in order
    for row in rows:
        k = short(row["Kernel_Name"])
        if row["Dispatch_Id"] not in seen[k]:
            seen[k].append(row["Dispatch_Id"])
    keep = {k: set(ids[skip:]) for k, ids in seen.items()}
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(dict)
    for row in rows:
        k = short(row["Kernel_Name"])
        if row["Dispatch_Id"] not in keep[k]:
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
    ap.add_argument("--extra", default=None, help="JSON file of further facts to record (flip rates, ...)")
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
        skip = 0
        if ":" in d:
            d, sk = d.rsplit(":", 1)
            skip = int(sk)
        per, dur = load(d, skip)
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
    out = {"note": a.note, "commands": a.command,
           **({"facts": json.load(open(a.extra))} if a.extra else {}),
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
