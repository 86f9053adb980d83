#!/usr/bin/env python3
"""Time-to-solution protocol of the benchmark section (Eq. 5).

A workload's target cut is fixed once, from the plain path, and recorded:

  python -m paper_2606_25203_amd.tts record --workload c1 [--seeds 32]

runs the workload's schedule (paper_2606_25203_amd.workloads) on one
instance, one run after another from seeds 0 .. S-1, and stores the median
of the runs' final best cuts M* as the target in targets.json beside this
file (with the seeds, the finals and the schedule).

  python -m paper_2606_25203_amd.tts scan --workload c1 [--runs 100] [--sa] [--out FILE]

then makes independent runs (seeds 1000, 1001, ...) that stop once M*
reaches the recorded target.  A run's compute time T_com is the device time
from the start of the run to the end of the beta step whose M* first met the
target (step granularity); a run that never meets it has none.  For every
candidate T (each observed T_com) the success probability P_s(T) is the
fraction of all runs with T_com <= T, Eq. 5 gives
TTS(T) = T ln(1 - 0.99) / ln(1 - P_s(T)), and the smallest TTS over the
candidates is reported.  Eq. 5 has no finite value at P_s = 1; there (and
for any P_s >= 0.99) one run already succeeds with 99 % probability, so
TTS(T) = T.  --sa runs the same schedule without resampling or augmentation
(R independent annealing chains) against the same target.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TARGETS = os.path.join(HERE, "targets.json")
SCAN_SEED0 = 1000


def tts(T: float, ps: float) -> float:
    """Eq. 5 at one candidate (T, P_s); infinite for P_s = 0, T for
    P_s >= 0.99."""
    if ps <= 0.0:
        return math.inf
    if ps >= 0.99:
        return T
    return T * math.log(1.0 - 0.99) / math.log(1.0 - ps)


def scan(times, n_runs: int):
    """The P_s scan: one row (T, P_s(T), TTS(T)) per distinct observed
    T_com, ascending, and the row of smallest TTS (None if no run
    succeeded).  times holds the T_com of the successful runs only."""
    if n_runs <= 0:
        raise ValueError("no runs")
    if len(times) > n_runs:
        raise ValueError("more successes than runs")
    rows = []
    for T in sorted(set(times)):
        ps = sum(1 for t in times if t <= T) / n_runs
        rows.append((T, ps, tts(T, ps)))
    best = min(rows, key=lambda r: r[2]) if rows else None
    return rows, best


def recorded_target(name: str):
    """The recorded target cut of a workload, or None."""
    try:
        with open(TARGETS) as f:
            return int(json.load(f)[name]["target"])
    except (OSError, KeyError, ValueError):
        return None


def _pamc():
    from paper_2606_25203_amd import pamc
    return pamc


def record(name: str, seeds: int):
    from paper_2606_25203_amd.workloads import make_instance, workload
    pamc = _pamc()
    w = workload(name)
    inst = make_instance(pamc, w, 0)
    sched = pamc.schedule(**w["sched"])
    finals = []
    for s in range(seeds):
        inst.reset(s)
        finals.append(int(inst.anneal(sched).best_cut))
        print(f"record {name}: seed {s} final M* {finals[-1]}", file=sys.stderr, flush=True)
    inst.close()
    target = int(statistics.median_low(finals))
    try:
        with open(TARGETS) as f:
            data = json.load(f)
    except OSError:
        data = {}
    data[name] = {"target": target, "rule": "median (lower) of the final M* of the plain path",
                  "seeds": list(range(seeds)), "finals": finals, "schedule": w["sched"], "workload": w["desc"]}
    with open(TARGETS, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    return data[name]


def run_scan(name: str, runs: int, sa: bool):
    from paper_2606_25203_amd.workloads import make_instance, workload
    pamc = _pamc()
    w = workload(name)
    target = recorded_target(name)
    if target is None:
        raise SystemExit(f"no recorded target for {name}: run 'record' first")
    kw = dict(w["sched"])
    if sa:
        kw.update(resample=0, augmented=0)
    kw.update(target=target, stop_at_target=1)
    sched = pamc.schedule(**kw)
    inst = make_instance(pamc, w, 0)
    inst.reset(SCAN_SEED0 + runs)  # one untimed run first (code paths, graph capture)
    inst.anneal(sched)
    per_run = []
    t_all = time.perf_counter()
    for k in range(runs):
        seed = SCAN_SEED0 + k
        t0 = time.perf_counter()
        inst.reset(seed)
        res = inst.anneal(sched)
        wall = time.perf_counter() - t0
        hit = res.seconds_to_target if res.step_reached >= 0 else None
        per_run.append({"seed": seed, "final": int(res.best_cut), "step_reached": int(res.step_reached),
                        "t_com_s": hit, "device_s": res.seconds_total, "host_wall_s": wall})
        print(f"scan {name}{' sa' if sa else ''}: run {k} seed {seed} M* {res.best_cut} "
              f"step {res.step_reached} T_com {hit}", file=sys.stderr, flush=True)
    total = time.perf_counter() - t_all
    inst.close()
    times = [r["t_com_s"] for r in per_run if r["t_com_s"] is not None]
    rows, best = scan(times, runs)
    return {"workload": w["desc"], "mode": "SA (no resampling, no augmentation)" if sa else "PAMC as scheduled",
            "target": target, "runs": runs, "seeds": [SCAN_SEED0, SCAN_SEED0 + runs - 1],
            "successes": len(times), "ps_final": len(times) / runs,
            "tts99_s": None if best is None else best[2],
            "at": None if best is None else {"T_com_s": best[0], "P_s": best[1]},
            "t_com_p50_s": statistics.median(times) if times else None,
            "scan": [{"T_s": T, "P_s": ps, "TTS_s": (None if math.isinf(v) else v)} for T, ps, v in rows],
            "host_wall_all_runs_s": total, "per_run": per_run}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("what", choices=["record", "scan"])
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--seeds", type=int, default=32, help="record: runs whose median is the target")
    ap.add_argument("--runs", type=int, default=100, help="scan: independent runs")
    ap.add_argument("--sa", action="store_true", help="scan: no resampling (independent chains)")
    ap.add_argument("--out", default=None, help="scan: write the result JSON here")
    a = ap.parse_args()
    if a.what == "record":
        r = record(a.workload, a.seeds)
        print(json.dumps({"workload": a.workload, "target": r["target"], "finals": r["finals"]}))
        return
    out = run_scan(a.workload, a.runs, a.sa)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k not in ("scan", "per_run")}))


if __name__ == "__main__":
    main()
