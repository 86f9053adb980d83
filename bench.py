#!/usr/bin/env python3
"""Throughput of the augmented PAMC hot path on one MI355X.

Default workload (the one the JSON line is quoted on): augmented PAMC
(adaptive reheat + cluster moves) on a 100 x 200 toroidal grid with +-1
weights (n = 20,000, degree 4), R = 4096 replicas, 500 beta steps of 10
sweeps (beta0 = 0.1, dbeta = 0.02, restart every 400 steps, n_top = 128, 4
independent-set trials, cooldown 25).  One bench step is one complete run on
the resident instance: population initialisation from a fresh seed, then the
500 steps (resampling, cluster moves, threshold tables, sweeps, best-cut
reduction, controller), all on the device.

Other workloads (--workload): c1 = plain PAMC on the n = 800 random graph;
c3 = plain PAMC on the dense n = 100,000 +-1 instance; c4 = augmented PAMC on
the Max-3-Cut embedding of a 7,000-vertex graph (the decoded 3-cuts are
reported as final_3cuts); c4p / c4c = the same graph with 3-state Potts
labels (softmax-perturbed argmax / cascaded p-bits).

Printed (one JSON line): flip attempts per second over the timed runs,
time-to-target p50/p99 (target = median final best cut of the timed runs),
the dominant kernel's roofline position measured with HIP events around
every launch of it, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_I8_PEAK_TOPS = 5000.0
CSRC = os.path.join(ROOT, "paper_2606_25203_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def tts99(hit_times, n_runs):
    """Eq. 5: TTS(T) = T ln(1 - 0.99) / ln(1 - P_s(T)) with P_s(T) the
    fraction of runs that reached the target within T (device time from the
    start of the run), minimised over the observed hit times T.  None when no
    run reached the target."""
    best = None
    for T in sorted(hit_times):
        ps = sum(1 for t in hit_times if t <= T) / n_runs
        tts = T if ps >= 0.99 else T * math.log(0.01) / math.log(1.0 - ps)
        best = tts if best is None else min(best, tts)
    return best


def sweep_bytes_per_attempt(p_flip: float, degree: float, pull: bool) -> float:
    """Algorithmic HBM bytes of one (replica, vertex) visit of the sparse sweep.
    Incremental fields (push): read the spin (1 B) and the field (4 B); on a
    flip (probability p) write the spin (1 B) and read-modify-write every
    neighbour field (8 B each).  Gathered fields (pull): read the spin (1 B)
    and, over a sweep, every other spin once more as a neighbour (1 B); write
    the spin on a flip.  The CSR row (column + coupling, 8 B per neighbour)
    is shared by the 64 lanes of a wavefront in both."""
    csr = 8.0 * degree / 64.0
    if pull:
        return 2.0 + p_flip + csr
    return 5.0 + p_flip * (1.0 + 8.0 * degree) + csr


VALU_PEAK_TSLOTS = 256 * 64 * 2.4e9 / 1e12   # 39.3 T int32 lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz


def alu_slots_per_attempt(degree: float, coupling_mode: int) -> float:
    """Vector-ALU issue slots (lane-ops, a 32x32->64 product counting 4 as it
    issues at quarter rate) of one (replica, vertex) visit of the
    gathered-field sweep.  Philox4x32-10: one 4-word block per 4 attempts,
    10 rounds of two 32x32->64 products and two three-input xors, i.e.
    (10 x (2 x 4 + 2)) / 4 = 25 slots.  Field: one int8 dot product per
    neighbour (coupling mode 2), else byte extract + multiply + add.
    Decision: spin extract, s*h, clamp (2), table address, compare, spin
    flip select, energy select + add: 9 slots."""
    per_neighbour = 1.0 if coupling_mode == 2 else 3.0
    return 25.0 + per_neighbour * degree + 9.0


def potts_slots_per_attempt(degree: float, K: int, X: int) -> float:
    """Vector-ALU issue slots (lane-ops, 32x32->64 products counting 4,
    binary64 operations 2) of one Potts label visit of k_sweep_potts<3>, from
    the compiled loop: 506 slots per quad of 4 vertices outside the gather
    loops (Philox4x32-10 blocks shared by the quad, the binary64 weights and
    comparisons, the label updates; both rules' code counted, so an upper
    bound), i.e. 126.5 per visit, plus per gathered-CSR entry (rows padded to
    multiples of 4) 23/4 slots when the K label sums fit 32/K-bit fields of
    one integer (X < 2^(32/K - 1): byte extract, shift, add) and 47/4
    otherwise (K compare-select-adds)."""
    per_entry = 23.0 / 4.0 if X < (1 << (32 // K - 1)) else 47.0 / 4.0
    return 126.5 + per_entry * 4.0 * math.ceil(degree / 4.0)


def counters_traffic(name: str, src: str):
    """HBM bytes per launch from a committed rocprofv3 FETCH/WRITE pass, or
    None if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{name}_counters.json")
    try:
        with open(path) as f:
            c = json.load(f)
        sha = hashlib.sha256(open(os.path.join(CSRC, src), "rb").read()).hexdigest()
        if c.get("source_sha256") != sha:
            return None
        return c["hbm_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


# ----------------------------------------------------------------- workloads
def workload(name):
    import synth
    if name == "c2":
        g = synth.torus(100, 200, seed=1)
        return dict(kind="csr", graph=g, R=4096, steps=500, sweeps=10,
                    sched=dict(beta0=0.1, dbeta=0.02, steps=500, sweeps=10, augmented=1, z_rst=400, n_top=128,
                               mis_trials=4, tau=25),
                    desc="augmented PAMC, 100x200 torus +-1 weights (n=20000, degree 4), R=4096, "
                         "500 beta steps x 10 sweeps",
                    counters="sweep_torus100x200_R4096", cpu=dict(R=64, step_s=1.2))
    if name == "c1":
        g = synth.random_graph(800, 19176, seed=1)
        return dict(kind="csr", graph=g, R=256, steps=50, sweeps=5,
                    sched=dict(beta0=0.1, dbeta=2.9 / 49, steps=50, sweeps=5),
                    desc="plain PAMC, random graph n=800 m=19176 w=+1, R=256, 50 beta steps 0.1->3.0 x 5 sweeps",
                    counters="sweep_gnm800_R256", cpu=dict(R=256, step_s=0.3))
    if name == "c3":
        n = 100_000
        return dict(kind="dense", n=n, R=256, steps=200, sweeps=1,
                    sched=dict(beta0=0.1 / math.sqrt(n), dbeta=2.9 / math.sqrt(n) / 199, steps=200, sweeps=1),
                    desc="plain PAMC, dense +-1 Ising n=100000 (int8 J, 10 GB), R=256, "
                         "200 beta steps 0.1/sqrt(n)->3.0/sqrt(n) x 1 sweep",
                    counters="dense_gemm_n100000_R256", cpu=None)
    if name == "c4":
        g = synth.random_graph(7000, 21000, seed=1)
        return dict(kind="max3cut", graph=g, R=2048, steps=300, sweeps=10,
                    sched=dict(beta0=0.1, dbeta=0.02, steps=300, sweeps=10, augmented=1, z_rst=400, n_top=64,
                               mis_trials=4, tau=25),
                    desc="augmented PAMC, Max-3-Cut one-hot embedding of G(7000, 21000) (n=21001), R=2048, "
                         "300 beta steps x 10 sweeps",
                    counters="sweep_max3cut7000_R2048", cpu=dict(R=64, step_s=1.5))
    if name in ("c4p", "c4c"):
        # the paper's own Max-3-Cut formulation on C4's graph: one 3-state
        # Potts label per vertex (n = 7000 instead of the embedding's 21001)
        g = synth.random_graph(7000, 21000, seed=1)
        cascade = name == "c4c"
        return dict(kind="potts", graph=g, K=3, potts_rule=1 if cascade else 0, gamma=0.0 if cascade else 1.0,
                    R=2048, steps=300, sweeps=10,
                    sched=dict(beta0=0.1, dbeta=0.02, steps=300, sweeps=10, augmented=1, z_rst=400, n_top=64,
                               mis_trials=4, tau=25),
                    desc="augmented PAMC, Max-3-Cut with 3-state Potts labels (" +
                         ("cascaded p-bit sampler" if cascade else "softmax-perturbed argmax, gamma=1") +
                         ") on G(7000, 21000), R=2048, 300 beta steps x 10 sweeps",
                    counters="sweep_potts7000_R2048", cpu=dict(R=64, step_s=0.6))
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, seconds_budget: float):
    import oracle
    if w["cpu"] is None:
        return None
    rr = w["cpu"]["R"]
    g = w["graph"]
    if w["kind"] == "max3cut":
        o = oracle.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, rr, 0)
        n = 3 * g.n + 1
    elif w["kind"] == "potts":
        o = oracle.Oracle.potts(g.n, g.row_ptr, g.col, g.w, w["K"], rr, 0, rule=w["potts_rule"], gamma=w["gamma"])
        n = g.n
    else:
        o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, rr, 0)
        n = g.n
    steps = max(1, min(w["steps"], int(round(seconds_budget / w["cpu"]["step_s"]))))
    kw = dict(w["sched"])
    kw.update(steps=steps, n_top=max(1, min(kw.get("n_top", 1), rr // 32)))
    t0 = time.perf_counter()
    o.anneal(oracle.default_schedule(**kw))
    dt = time.perf_counter() - t0
    att = steps * w["sweeps"] * n * rr
    return {"value": att / dt, "unit": "flip attempts/s", "cores": 1, "kind": "oracle",
            "sample": f"same instance, R={rr} replicas, first {steps} beta steps x {w['sweeps']} sweeps "
                      f"({att:.3g} attempts in {dt:.1f} s, single thread)"}


# ------------------------------------------------------ batched and served
BATCH_SEEDS = {"c1": 256, "c2": 8, "c4": 16}


def make_instance(pamc, w, seed, fields=None):
    if w["kind"] == "csr":
        return pamc.Instance.csr(w["graph"], replicas=w["R"], seed=seed, fields=fields)
    if w["kind"] == "max3cut":
        return pamc.Instance.max3cut(w["graph"], replicas=w["R"], seed=seed, fields=fields)
    raise SystemExit("batched runs take sparse workloads")


def bench_batched(pamc, torch, name, count=None):
    """The same set of runs (one instance, count seeds) made one after the
    other through pamc_anneal and together through pamc_anneal_batch;
    instances are built and initialised before the clock starts in both."""
    w = workload(name)
    count = count or BATCH_SEEDS[name]
    sched = pamc.schedule(**w["sched"])
    seeds = list(range(1000, 1000 + count))
    insts = [make_instance(pamc, w, s) for s in seeds]
    n = insts[0].info().n
    # warm-up of both paths on the first instance
    insts[0].anneal(sched)
    pamc.anneal_batch(insts[:2], [sched] * 2)
    for i, s in zip(insts, seeds):
        i.reset(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [i.anneal(sched) for i in insts]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for i, s in zip(insts, seeds):
        i.reset(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batched = pamc.anneal_batch(insts, [sched] * count)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    for i in insts:
        i.close()
    att = sum(r.steps_run for r in plain) * w["sweeps"] * n * w["R"]
    same = all(a.best_cut == b.best_cut and a.sum_lnq == b.sum_lnq and a.steps_run == b.steps_run
               for a, b in zip(plain, batched))
    return {"workload": w["desc"], "runs": count, "plain_attempts_per_s": att / t_plain,
            "batched_attempts_per_s": att / t_batch, "speedup": t_plain / t_batch,
            "plain_s": t_plain, "batched_s": t_batch, "identical_results": same,
            "cuts": sorted(r.best_cut for r in batched)[count // 2]}


C5_SCHED = dict(beta0=0.1, dbeta=2.9 / 199, steps=200, sweeps=5)


def bench_served(pamc, torch, count, budget_gb=16.0, slots=256, tick_steps=8, seed=5):
    """A prefix of the request stream (n log-uniform in [800, 20000], half
    random graphs of average degree 4-50, half +-1 tori; R = 512, 200 beta
    steps x 5 sweeps each): plain = one request after the other through
    instance creation + pamc_anneal; served = the server, with every
    request arriving at t = 0, then with Poisson arrivals at 0.8 x and
    2.5 x the plain path's measured request rate.  Wall time includes
    building each instance in every mode.  The plain path's latencies under
    the same arrivals follow from its measured per-request times (one
    request at a time, in arrival order)."""
    import synth
    R = 512
    sched = pamc.schedule(**C5_SCHED)
    reqs = synth.request_stream(count, 1.0, seed)
    # warm-up
    wi = pamc.Instance.csr(reqs[0].graph, replicas=R, seed=1)
    wi.anneal(pamc.schedule(**dict(C5_SCHED, steps=3)))
    wi.close()
    torch.cuda.synchronize()
    attempts = sum(q.graph.n for q in reqs) * R * C5_SCHED["steps"] * C5_SCHED["sweeps"]
    t0 = time.perf_counter()
    plain, service = {}, []
    for q in reqs:
        t1 = time.perf_counter()
        inst = pamc.Instance.csr(q.graph, replicas=R, seed=q.seed)
        plain[q.index] = inst.anneal(sched).best_cut
        inst.close()
        service.append(time.perf_counter() - t1)
    t_plain = time.perf_counter() - t0
    log(f"served bench: plain {count} requests in {t_plain:.2f} s")
    out = {"requests": count, "replicas": R, "beta_steps": C5_SCHED["steps"], "sweeps": C5_SCHED["sweeps"],
           "mean_n": sum(q.graph.n for q in reqs) / count, "hbm_budget_gb": budget_gb, "max_slots": slots,
           "plain_attempts_per_s": attempts / t_plain, "plain_requests_per_s": count / t_plain}
    def plain_latencies(arrivals):
        # the plain path is one request at a time in arrival order
        done, lat = 0.0, []
        for a, sv in zip(arrivals, service):
            done = max(done, a) + sv
            lat.append(done - a)
        return lat

    for mode, load in (("burst", None), ("poisson", 0.8), ("poisson_overload", 2.5)):
        rate = load * count / t_plain if load else None
        arrivals = [0.0] * count if load is None else [q.arrival_s / rate for q in reqs]
        srv = pamc.Server(int(budget_gb * (1 << 30)), slots, replicas=R)
        tickets = {}
        t0 = time.perf_counter()
        nxt = 0
        while True:
            now = time.perf_counter() - t0
            while nxt < count and arrivals[nxt] <= now:
                q = reqs[nxt]
                tickets[srv.submit(q.graph, q.seed, sched)] = q.index
                nxt += 1
            active, queued = srv.tick(tick_steps)
            if nxt >= count and active == 0 and queued == 0:
                break
            if active == 0 and queued == 0 and nxt < count:
                time.sleep(max(0.0, min(0.05, arrivals[nxt] - (time.perf_counter() - t0))))
        wall = time.perf_counter() - t0
        sstats = srv.stats()
        lat, same = [], True
        for t, idx in tickets.items():
            res = srv.poll(t)
            same = same and res.best_cut == plain[idx]
            lat.append(srv.latency(t)[1])
        srv.close()
        pl = plain_latencies(arrivals)
        out[mode] = {"attempts_per_s": attempts / wall, "wall_s": wall, "speedup_vs_plain": t_plain / wall,
                     "latency_p50_s": percentile(lat, 0.5), "latency_p99_s": percentile(lat, 0.99),
                     "plain_latency_p50_s": percentile(pl, 0.5), "plain_latency_p99_s": percentile(pl, 0.99),
                     "identical_results": same,
                     "server": {k: sstats[k] for k in ("ticks", "steps", "request_steps", "prep_seconds",
                                                        "admit_seconds", "step_seconds", "peak_active",
                                                        "peak_bytes")}}
        if rate:
            out[mode]["arrival_rate_per_s"] = rate
            out[mode]["load_vs_plain_capacity"] = load
        log(f"served bench: {mode} {wall:.2f} s, p50 {out[mode]['latency_p50_s']:.3f} s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c4p", "c4c"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fields", choices=["auto", "push", "pull"], default="auto")
    ap.add_argument("--batched", default="c1",
                    help="comma-separated workloads for the plain-vs-batched comparison ('' to skip)")
    ap.add_argument("--batch-count", type=int, default=0, help="runs per batched comparison (0: default)")
    ap.add_argument("--served", type=int, default=64,
                    help="requests of the stream for the plain-vs-served comparison (0 to skip)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run an elementwise copy of this many MiB (int32 in, int32 out) five "
                         "times; used to scale the HBM byte counters of rocprofv3")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.arange(n, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "kernel": "neg (elementwise)"}))
        return
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU; sharding the population across GPUs is not "
              "implemented. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_25203_amd import pamc

    w = workload(args.workload)
    fields = None if args.fields == "auto" else args.fields
    if w["kind"] == "csr":
        inst = pamc.Instance.csr(w["graph"], replicas=w["R"], seed=0, fields=fields)
    elif w["kind"] == "max3cut":
        inst = pamc.Instance.max3cut(w["graph"], replicas=w["R"], seed=0, fields=fields)
    elif w["kind"] == "potts":
        inst = pamc.Instance.potts(w["graph"], w["K"], replicas=w["R"], seed=0, potts_rule=w["potts_rule"],
                                   gamma=w["gamma"])
    else:
        inst = pamc.Instance.dense_random(w["n"], 1, replicas=w["R"], seed=0)
    info = inst.info()
    n = info.n
    sched = pamc.schedule(**w["sched"])
    pamc.pamc_profile_enable(inst.h, True)   # warm-up also fills the event pool
    for k in range(args.warmup):
        inst.reset(10_000 + k)
        inst.anneal(sched)
        log(f"warmup {k} done")
    pamc.pamc_profile_enable(inst.h, True)   # zero the counters, keep the pool
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    decoded = []
    for k in range(args.steps):
        inst.reset(k)
        res = inst.anneal(sched)
        tr = inst.trace(w["steps"])
        runs.append((res, tr))
        if w["kind"] == "max3cut":  # the 3-cut of the run's best configuration
            decoded.append(int(inst.max3cut_decode()[0]))
        log(f"run {k}: best cut {res.best_cut}, device time {res.seconds_total:.3f} s")
    inst.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = pamc.pamc_profile_read(inst.h)

    attempts = sum(r.steps_run for r, _ in runs) * w["sweeps"] * n * w["R"]
    finals = [r.best_cut for r, _ in runs]
    finals3 = [c for c in decoded] if decoded else None
    target = int(percentile(finals, 0.5))
    ttt = []
    for res, tr in runs:
        hit = [t for m, t in zip(tr["mstar"], tr["seconds"]) if m >= target]
        if hit:
            ttt.append(float(hit[0]))
    launch_ms = prof["ms"] / max(prof["launches"], 1)
    p_flip = prof["flips"] / max(prof["attempts"], 1)
    if w["kind"] == "dense":
        # One timed unit is a super-block step: the product completing this
        # super-block's fields, then k_dense_step (its sequential pass with
        # the next super-block's product on the other compute units).  Its
        # matrix-core work is one super-block's share of the field products,
        # 2 npad^2 R int8 ops per sweep; the step lasts as long as the
        # sequential pass, so this fraction is that of the whole dense sweep.
        npad = (n + 63) // 64 * 64
        sweeps_done = prof["attempts"] / (n * w["R"])
        ops = 2.0 * npad * npad * w["R"] * sweeps_done / max(prof["launches"], 1)
        achieved = ops / (launch_ms * 1e-3) / 1e12
        roof = {"kernel": "k_dense_step (+ k_dense_gemm)", "bound": "mfma", "achieved": achieved,
                "peak": MFMA_I8_PEAK_TOPS, "unit": "TOP/s (int8)", "frac": achieved / MFMA_I8_PEAK_TOPS,
                "traffic": counters_traffic(w["counters"], "dense.hip"), "launch_ms": launch_ms,
                "launches": prof["launches"], "ops_per_launch": ops, "flip_rate": p_flip}
    else:
        degree = info.nnz / n
        pull = bool(info.pull)
        bpa = sweep_bytes_per_attempt(p_flip, degree, pull)
        apl = prof["attempts"] / max(prof["launches"], 1)
        rate = apl / (launch_ms * 1e-3)
        hbm = bpa * rate / 1e9
        shape = {"tiles_per_wave": info.tiles_per_wave, "quads_per_wave": info.quads_per_wave,
                 "coupling_mode": info.coupling_mode}
        if w["kind"] == "potts":
            slots = potts_slots_per_attempt(degree, info.potts_K, info.X)
            achieved = slots * rate / 1e12
            roof = {"kernel": "k_sweep_potts<3>", "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TSLOTS,
                    "unit": "T int32 lane-op slots/s", "frac": achieved / VALU_PEAK_TSLOTS,
                    "alu_slots_per_attempt": slots, "hbm_algorithmic_gbs": hbm,
                    "hbm_algorithmic_frac": hbm / HBM_PEAK_GBS}
        elif pull:
            # issue-bound: vector ALU slots per attempt (see alu_slots_per_attempt)
            slots = alu_slots_per_attempt(degree, info.coupling_mode)
            achieved = slots * rate / 1e12
            roof = {"kernel": "k_sweep_pull", "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TSLOTS,
                    "unit": "T int32 lane-op slots/s", "frac": achieved / VALU_PEAK_TSLOTS,
                    "alu_slots_per_attempt": slots, "hbm_algorithmic_gbs": hbm,
                    "hbm_algorithmic_frac": hbm / HBM_PEAK_GBS}
        else:
            roof = {"kernel": "k_sweep_push", "bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": hbm / HBM_PEAK_GBS}
        roof.update({"traffic": counters_traffic(w["counters"], "sparse.hip"), "launch_ms": launch_ms,
                     "launches": prof["launches"], "attempts_per_launch": apl, "flip_rate": p_flip,
                     "algorithmic_bytes_per_attempt": bpa, "fields": "pull" if pull else "push",
                     "kernel_shape": shape, "attempts_per_s_in_kernel": rate})
    out = {
        "metric": "spin-flip attempts/s + time-to-target-cut (plain vs batched/served), p50/p99",
        "value": attempts / wall,
        "unit": "flip attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w["desc"], "n": n, "replicas": w["R"], "beta_steps": w["steps"],
                   "sweeps": w["sweeps"], "mode": "plain (one instance per launch sequence)",
                   "parallelism": "1 GPU"},
        "time_to_target": {"target_cut": target, "p50_s": percentile(ttt, 0.5), "p99_s": percentile(ttt, 0.99),
                           "success_fraction": len(ttt) / len(runs), "tts99_s": tts99(ttt, len(runs)),
                           "final_cuts": finals},
        **({"final_3cuts": finals3} if finals3 else {}),
        "roofline": roof,
    }
    inst.close()
    if args.batched:
        out["batched"] = []
        for name in args.batched.split(","):
            log(f"batched comparison on {name} ...")
            out["batched"].append(bench_batched(pamc, torch, name, args.batch_count or None))
    if args.served:
        log("served comparison ...")
        out["served"] = bench_served(pamc, torch, args.served)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        cb = cpu_baseline(w, args.cpu_seconds)
        if cb is not None:
            out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
