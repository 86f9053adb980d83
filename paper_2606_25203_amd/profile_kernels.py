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
  c1   pamc_sweep on G(800, 19176), R = 256 (k_sweep_tile: all sweeps of a
       call in one launch)
  c4p  pamc_sweep on G(7000, 21000) with 3-state Potts labels, R = 2048
       (k_sweep_potts<3>)
Before the counted sweeps the population is brought to the inverse
temperature the workload's runs spend most sweeps near, so flip rates (and
hence bytes) are representative; then the script idles for a second, a gap
the counter summary uses to leave the settling dispatches out.  Prints one
JSON line: sweeps, attempts, launches, flips (from the library's counters),
wall time, the name of the sweep kernel and the hash of the kernel sources
(--facts-out also writes it to a file).

Run with PAMC_NO_TORCH=1 to keep torch's HIP runtime out of the process.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_25203_amd", "csrc")
sys.path.insert(0, ROOT)

SETTLE_GAP_S = 1.0


def kernel_source_sha256(src):
    """Hash of one kernel source file and the device headers it includes:
    counters taken on other sources no longer describe the kernels."""
    h = hashlib.sha256()
    for f in (src, "pamc_device.hpp", "instance.hpp"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sweep_kernel(info, potts=False):
    """The name rocprofv3 gives (up to the argument list) to the kernel that
    makes an instance's sweeps, from the instance's chosen shape."""
    if info.dense:
        return "k_dense_step<0>"
    if potts:
        return f"k_sweep_potts<{info.potts_K}>"
    if info.tile_sweeps == 2:  # one instance (at most 128 tiles): a work-group per 16-replica group
        return "k_sweep_tmma_g<8>"
    if info.tile_sweeps:
        return f"k_sweep_tile<{info.coupling_mode}>"
    if info.pull:
        wide = "true" if 2 * info.X + 1 > 2048 else "false"
        return (f"k_sweep_pull<{info.coupling_mode}, {info.tiles_per_wave}, {wide}, "
                f"{'true' if info.hubs else 'false'}>")
    return "k_sweep_push"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c4p"])
    ap.add_argument("--facts-out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--sweeps", type=int, default=20, help="sweeps per call")
    ap.add_argument("--calls", type=int, default=1, help="counted calls of the sweep primitive")
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
    elif args.workload == "c4p":
        inst = pamc.Instance.potts(synth.random_graph(7000, 21000, seed=1), 3, replicas=2048, seed=0,
                                   potts_rule=0, gamma=1.0)
        beta = 2.0
    else:
        inst = pamc.Instance.dense_random(100_000, 1, replicas=256, seed=0)
        beta = 1.5 / math.sqrt(100_000)
    if args.beta is not None:
        beta = args.beta
    info = inst.info()
    inst.sweep(beta, 5)  # settle at beta (not counted in the summary below)
    inst.synchronize()
    time.sleep(SETTLE_GAP_S)
    if not args.no_events:
        pamc.pamc_profile_enable(inst.h, True)
    print(f"profile_kernels: {args.workload} n={info.n} R={info.replicas} beta={beta:.4g}, "
          f"{args.calls} x {args.sweeps} sweeps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.calls):
        inst.sweep(beta, args.sweeps)
    inst.synchronize()
    wall = time.perf_counter() - t0
    total = args.calls * args.sweeps
    prof = pamc.pamc_profile_read(inst.h) if not args.no_events else \
        {"attempts": total * info.n * info.replicas, "flips": -1, "launches": -1, "ms": -1.0}
    out = {"workload": args.workload, "n": info.n, "replicas": info.replicas, "beta": beta,
           "sweeps": total, "sweeps_per_call": args.sweeps, "attempts": prof["attempts"], "flips": prof["flips"],
           "flip_rate": prof["flips"] / max(prof["attempts"], 1), "launches": prof["launches"],
           "kernel_ms": prof["ms"], "wall_s": wall, "pull": info.pull, "nnz": info.nnz,
           "tiles_per_wave": info.tiles_per_wave, "quads_per_wave": info.quads_per_wave,
           "coupling_mode": info.coupling_mode, "tile_sweeps": info.tile_sweeps, "hubs": info.hubs,
           "kernel": sweep_kernel(info, args.workload == "c4p"), "settle_gap_s": SETTLE_GAP_S,
           "source_sha256": kernel_source_sha256("dense.hip" if info.dense else "sparse.hip")}
    inst.close()
    print(json.dumps(out), flush=True)
    if args.facts_out:
        with open(args.facts_out, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
