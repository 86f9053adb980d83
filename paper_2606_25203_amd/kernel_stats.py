#!/usr/bin/env python3
"""Writes the text summary of a rocprofv3 --kernel-trace --stats run: one
row per kernel (calls, total ms, mean us, share of the kernel time), with
the title, the command that made the run and a note in the header.

Usage: kernel_stats.py OUT.txt STATS_DIR --title TEXT --command TEXT [--note TEXT]
STATS_DIR holds the run's *_kernel_stats.csv."""
import argparse
import csv
import glob
import os

from counters_summary import short


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("stats_dir")
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--note", default="")
    a = ap.parse_args()
    files = glob.glob(os.path.join(a.stats_dir, "*_kernel_stats.csv"))
    if not files:
        raise SystemExit(f"no kernel statistics under {a.stats_dir}")
    rows = list(csv.DictReader(open(files[0])))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics: {a.title}", f"# command: {a.command}"]
    if a.note:
        lines.append(f"# {a.note}")
    lines += ["", f"{'kernel':48s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>9s} {'pct':>6s}"]
    for r in rows:
        t = float(r["TotalDurationNs"])
        lines.append(f"{short(r['Name'])[:48]:48s} {int(r['Calls']):6d} {t / 1e6:10.2f} "
                     f"{float(r['AverageNs']) / 1e3:9.2f} {100 * t / total:6.2f}")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
