#!/usr/bin/env python3
"""Runs one hot kernel of a workload many times, for hardware-counter passes
(rocprofv3 --pmc) and kernel statistics.

Each workload builds its instance exactly as the benchmark does, then calls
only the primitive that launches the kernel of interest, so a counter pass
sees that kernel (and the small per-call setup kernels) and nothing else:
  c2   pamc_sweep on the 100 x 200 +-1 torus, R = 4096 (k_sweep_pull)
  c4   pamc_sweep on the Max-3-Cut embedding of G(7000, 21000), R = 2048
       (k_sweep_push, incremental fields)
  c3   pamc_sweep on the dense +-1 n = 100,000 instance, R = 256 (k_dense_*)
  c1   pamc_sweep on G(800, 19176), R = 256
Before the counted sweeps the population is brought to the inverse
temperature the workload's runs spend most sweeps near, so flip rates (and
hence bytes) are representative.  Prints one JSON line: sweeps, attempts,
launches per sweep, flips (from the library's counters) and wall time.

Run with PAMC_NO_TORCH=1 to keep torch's HIP runtime out of the process.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--beta", type=float, default=None, help="inverse temperature of the counted sweeps")
    ap.add_argument("--no-events", action="store_true",
                    help="no library timing events or flip counters (for counter passes; the trajectory, "
                         "hence the flips, is the same as with them)")
    args = ap.parse_args()
    import synth
    from paper_2606_25203_amd import pamc

    if args.workload == "c2":
        inst = pamc.Instance.csr(synth.torus(100, 200, seed=1), replicas=4096, seed=0)
        beta = 2.0
    elif args.workload == "c4":
        inst = pamc.Instance.max3cut(synth.random_graph(7000, 21000, seed=1), replicas=2048, seed=0)
        beta = 2.0
    elif args.workload == "c1":
        inst = pamc.Instance.csr(synth.random_graph(800, 19176, seed=1), replicas=256, seed=0)
        beta = 1.5
    else:
        inst = pamc.Instance.dense_random(100_000, 1, replicas=256, seed=0)
        beta = 1.5 / math.sqrt(100_000)
    if args.beta is not None:
        beta = args.beta
    info = inst.info()
    inst.sweep(beta, 5)  # settle at beta (not counted in the summary below)
    inst.synchronize()
    if not args.no_events:
        pamc.pamc_profile_enable(inst.h, True)
    print(f"profile_kernels: {args.workload} n={info.n} R={info.replicas} beta={beta:.4g}, "
          f"{args.sweeps} sweeps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    inst.sweep(beta, args.sweeps)
    inst.synchronize()
    wall = time.perf_counter() - t0
    prof = pamc.pamc_profile_read(inst.h) if not args.no_events else \
        {"attempts": args.sweeps * info.n * info.replicas, "flips": -1, "launches": -1, "ms": -1.0}
    out = {"workload": args.workload, "n": info.n, "replicas": info.replicas, "beta": beta,
           "sweeps": args.sweeps, "attempts": prof["attempts"], "flips": prof["flips"],
           "flip_rate": prof["flips"] / max(prof["attempts"], 1), "launches": prof["launches"],
           "kernel_ms": prof["ms"], "wall_s": wall, "pull": info.pull, "nnz": info.nnz,
           "tiles_per_wave": info.tiles_per_wave, "quads_per_wave": info.quads_per_wave,
           "coupling_mode": info.coupling_mode}
    inst.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
