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
time-to-target p50/p99 and TTS (Eq. 5) against the workload's recorded
target cut (paper_2606_25203_amd/targets.json; else the median final best
cut of the timed runs),
the dominant kernel's roofline position measured with HIP events around
every launch of it, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2606_25203_amd.tts import recorded_target, scan as tts_scan  # noqa: E402
from paper_2606_25203_amd.workloads import make_instance, workload  # noqa: E402

HBM_PEAK_GBS = 8000.0
MFMA_I8_PEAK_TOPS = 5000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def incremental_field_bytes_per_attempt(p_flip: float, degree: float) -> float:
    """Algorithmic HBM bytes of one (replica, vertex) visit of a sparse sweep
    in the incremental-field layout (the reference model of the method's
    data movement): read the spin (1 B) and the field (4 B); on a flip
    (probability p) write the spin (1 B) and read-modify-write every
    neighbour's int32 field (8 B each); the CSR row (column + coupling,
    8 B per neighbour) is shared by the 64 lanes of a wavefront.  The
    gathered-field kernel computes the same fields from the spins instead,
    so its measured traffic (`traffic`) is below this."""
    return 5.0 + p_flip * (1.0 + 8.0 * degree) + 8.0 * degree / 64.0


def pull_bytes_per_attempt(p_flip: float, degree: float) -> float:
    """Bytes the gathered-field kernel needs at least: read the spin (1 B),
    every spin once more as a neighbour (1 B), write the spin on a flip, and
    the CSR row shared by a wavefront."""
    return 2.0 + p_flip + 8.0 * degree / 64.0


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


def counters(name: str, src: str, kernel: str):
    """Per-dispatch hardware counters of one kernel from a committed
    rocprofv3 summary (profiles/<name>_counters.json, made by
    paper_2606_25203_amd/counters_summary.py): HBM bytes (FETCH_SIZE and
    WRITE_SIZE scaled by a copy kernel of known size), the SQ counters taken
    and, for the sweep kernel, the attempts per dispatch.  None if the
    summary is missing or the kernel sources changed since the counters
    were taken."""
    from paper_2606_25203_amd.profile_kernels import kernel_source_sha256
    path = os.path.join(ROOT, "profiles", f"{name}_counters.json")
    try:
        with open(path) as f:
            c = json.load(f)
        if c.get("facts", {}).get("source_sha256") != kernel_source_sha256(src):
            return None
        return c["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None


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
    tune = insts[0].autotune(w["sched"]["beta0"] + w["sched"]["dbeta"] * w["steps"] / 2, sweeps=2)
    for i in insts[1:]:  # the same shape: the tuner's cached choice
        i.autotune(0.5)
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
            "autotuned_shape": {"tile_sweeps": tune.tile_sweeps, "tiles_per_wave": tune.tiles_per_wave,
                                "quads_per_wave": tune.quads_per_wave},
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
        if len(service) % 250 == 0:
            log(f"served bench: plain {len(service)} of {count} requests")
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
        t_log = 0.0
        while True:
            now = time.perf_counter() - t0
            if now - t_log > 20.0:
                t_log = now
                log(f"served bench: {mode} {nxt} of {count} submitted at {now:.0f} s")
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


def measure(pamc, torch, name, steps, warmup, fields=None):
    """Times `steps` complete runs of a workload on one resident instance
    (after `warmup` untimed runs) and places its sweep kernel on its
    roofline: HIP events bracket each step's sweep launches, the algorithmic
    bytes (or ops) per launch come from the model of the workload's path,
    and the HBM traffic per launch from the committed counter summary."""
    from paper_2606_25203_amd.profile_kernels import sweep_kernel

    w = workload(name)
    inst = make_instance(pamc, w, 0, fields=fields)
    info = inst.info()
    n = info.n
    sched = pamc.schedule(**w["sched"])
    pamc.pamc_profile_enable(inst.h, True)   # warm-up also fills the event pool
    for k in range(warmup):
        inst.reset(10_000 + k)
        inst.anneal(sched)
        log(f"warmup {k} done")
    pamc.pamc_profile_enable(inst.h, True)   # zero the counters, keep the pool
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    decoded = []
    for k in range(steps):
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
    # the workload's recorded target (the plain path's median final M* over
    # fixed seeds, paper_2606_25203_amd/targets.json), else these runs' median
    target = recorded_target(name)
    target_source = "recorded (paper_2606_25203_amd/targets.json)"
    if target is None:
        target, target_source = int(percentile(finals, 0.5)), "median final best cut of the timed runs"
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
                "traffic": None, "launch_ms": launch_ms, "launches": prof["launches"], "ops_per_launch": ops,
                "flip_rate": p_flip}
        step_c = counters(w["counters"], "dense.hip", "k_dense_step<0>")
        gemm_c = counters(w["counters"], "dense.hip", "k_dense_gemm")
        if step_c and gemm_c:
            # one launch unit = one k_dense_step and one k_dense_gemm dispatch
            roof["traffic"] = step_c["hbm_bytes_per_dispatch"] + gemm_c["hbm_bytes_per_dispatch"]
            roof["traffic_gbs"] = roof["traffic"] / (launch_ms * 1e-3) / 1e9
            roof["traffic_frac"] = roof["traffic_gbs"] / HBM_PEAK_GBS
            mops = step_c.get("SQ_INSTS_VALU_MFMA_MOPS_I8", 0.0) + gemm_c.get("SQ_INSTS_VALU_MFMA_MOPS_I8", 0.0)
            roof["counter_mfma_ops_per_launch"] = 512.0 * mops  # the counter counts units of 512 ops
    else:
        degree = info.nnz / n
        pull = bool(info.pull)
        apl = prof["attempts"] / max(prof["launches"], 1)
        rate = apl / (launch_ms * 1e-3)
        shape = {"tiles_per_wave": info.tiles_per_wave, "quads_per_wave": info.quads_per_wave,
                 "coupling_mode": info.coupling_mode, "tile_sweeps": info.tile_sweeps, "hubs": info.hubs}
        kname = sweep_kernel(info, w["kind"] == "potts")
        if w["kind"] == "potts":
            slots = potts_slots_per_attempt(degree, info.potts_K, info.X)
            achieved = slots * rate / 1e12
            roof = {"kernel": kname, "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TSLOTS,
                    "unit": "T int32 lane-op slots/s", "frac": achieved / VALU_PEAK_TSLOTS,
                    "alu_slots_per_attempt": slots}
        elif info.tile_sweeps:
            # one work-group per 64-replica tile holds the tile's spins in
            # LDS for all of a step's sweeps: HBM is idle, and a single
            # instance occupies R/64 compute units; the vector-issue model
            # over the whole chip, with the share of the units it runs on
            # (with matrix-core fields, the vector work is Philox and the
            # decision alone, and the products go to the int8 MFMA peak)
            mma = info.tile_sweeps == 2
            slots = 25.0 + 9.0 if mma else alu_slots_per_attempt(degree, info.coupling_mode)
            # one work-group per 64-replica tile, or per 16-replica group in
            # the matrix-core form of a launch with at most 128 tiles
            cus = w["R"] // 16 if mma and w["R"] // 64 <= 128 else w["R"] // 64
            achieved = slots * rate / 1e12
            roof = {"kernel": kname, "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TSLOTS,
                    "unit": "T int32 lane-op slots/s", "frac": achieved / VALU_PEAK_TSLOTS,
                    "alu_slots_per_attempt": slots, "cus_used": cus,
                    "frac_of_cus_used": achieved / VALU_PEAK_TSLOTS * 256 / cus,
                    "hbm_algorithmic_bytes_per_attempt": incremental_field_bytes_per_attempt(p_flip, degree)}
            if mma:
                ops = 2.0 * degree * rate / 1e12  # the sparse product's multiply-adds, not the zero blocks
                roof["mfma_model"] = {"useful_int8_ops_per_attempt": 2.0 * degree, "achieved_tops": ops,
                                      "peak_tops": MFMA_I8_PEAK_TOPS, "frac": ops / MFMA_I8_PEAK_TOPS}
        else:
            # achieved = the algorithmic bytes of the visits one launch makes
            # (incremental-field layout) over the launch's measured duration
            b_alg = incremental_field_bytes_per_attempt(p_flip, degree)
            achieved = b_alg * rate / 1e9
            roof = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_attempt": b_alg,
                    "algorithmic_model": "5 + p(1 + 8 deg) + 8 deg / 64 bytes per attempt"}
            if pull:
                slots = alu_slots_per_attempt(degree, info.coupling_mode)
                roof["alu_model"] = {"slots_per_attempt": slots, "achieved_tslots": slots * rate / 1e12,
                                     "peak_tslots": VALU_PEAK_TSLOTS,
                                     "frac": slots * rate / 1e12 / VALU_PEAK_TSLOTS,
                                     "kernel_min_bytes_per_attempt": pull_bytes_per_attempt(p_flip, degree)}
        if info.hubs and not pull and not info.tile_sweeps:
            roof["field_forms"] = ("both kept: the launches of the steps below beta 0.8 gather fields "
                                   "(hub fields kept, k_sweep_pull), the rest keep them incrementally "
                                   "(k_sweep_push); launch_ms averages both")
        roof.update({"traffic": None, "launch_ms": launch_ms, "launches": prof["launches"],
                     "attempts_per_launch": apl, "flip_rate": p_flip, "fields": "pull" if pull else "push",
                     "kernel_shape": shape, "attempts_per_s_in_kernel": rate})
        c = counters(w["counters"], "sparse.hip", kname)
        if c and "hbm_bytes_per_dispatch" in c:
            # measured bytes per dispatch of the counted sweeps (at the
            # profiling script's temperature), scaled to this run's launches
            roof["traffic"] = c["hbm_bytes_per_dispatch"] * apl / c.get("attempts_per_dispatch", apl)
            roof["traffic_gbs"] = roof["traffic"] / (launch_ms * 1e-3) / 1e9
            roof["traffic_frac"] = roof["traffic_gbs"] / HBM_PEAK_GBS
            roof["traffic_bytes_per_attempt"] = roof["traffic"] / apl
            if "SQ_INSTS_VALU" in c and c.get("mean_dispatch_ns_under_counters"):
                # VALU wave-instructions per CU and cycle (one per cycle is the
                # issue limit of a CU's four SIMDs for wave64 instructions)
                cyc = c["mean_dispatch_ns_under_counters"] * 1e-9 * 2.4e9
                roof["counter_valu_issue_frac"] = c["SQ_INSTS_VALU"] / (256 * cyc)
                if "cus_used" in roof:
                    roof["counter_valu_issue_frac_of_cus_used"] = c["SQ_INSTS_VALU"] / (roof["cus_used"] * cyc)
            if "SQ_INSTS_VALU_MFMA_MOPS_I8" in c:
                # the matrix-core products as issued (whole 16 x 64 blocks,
                # zeros included; the counter counts units of 512 ops)
                apd = c.get("attempts_per_dispatch", apl)
                roof["counter_mfma_ops_per_attempt"] = 512.0 * c["SQ_INSTS_VALU_MFMA_MOPS_I8"] / apd
                if c.get("mean_dispatch_ns_under_counters"):
                    roof["counter_mfma_busy_frac_of_cus_used"] = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (
                        4 * roof.get("cus_used", 256) * c["mean_dispatch_ns_under_counters"] * 1e-9 * 2.4e9)
    inst.close()
    return {"value": attempts / wall, "wall_s": wall, "ms_per_step": wall / steps * 1e3,
            "config": {"workload": w["desc"], "n": n, "replicas": w["R"], "beta_steps": w["steps"],
                       "sweeps": w["sweeps"], "mode": "plain (one instance per launch sequence)",
                       "parallelism": "1 GPU"},
            "time_to_target": {"target_cut": target, "p50_s": percentile(ttt, 0.5),
                               "p99_s": percentile(ttt, 0.99), "success_fraction": len(ttt) / len(runs),
                               "tts99_s": (tts_scan(ttt, len(runs))[1] or (None, None, None))[2],
                               "target_source": target_source, "final_cuts": finals},
            **({"final_3cuts": finals3} if finals3 else {}),
            # the dense +-1 instance is of the Sherrington-Kirkpatrick kind:
            # its best energy per n^1.5 next to Parisi's ground-state value
            # (context, not a target)
            **({"energy_per_n_1_5": [r.best_energy / n ** 1.5 for r, _ in runs], "parisi_reference": -0.7633}
               if w["kind"] == "dense" else {}),
            "roofline": roof}


def recorded_runs():
    """Key figures of the committed long measurements that a default run
    does not repeat (they take minutes): the full 2,000-request served
    stream and the time-to-solution scans (Eq. 5, 100 runs each)."""
    out = {}
    prof = os.path.join(ROOT, "profiles")
    try:
        with open(os.path.join(prof, "served_c5_2000req_R512.json")) as f:
            s = json.load(f)["served"]
        out["served_c5_2000_requests"] = {
            "command": "python bench.py --steps 1 --warmup 0 --no-cpu-baseline --batched= --served 2000 "
                       "--workload c1",
            "file": "profiles/served_c5_2000req_R512.json", "requests": s["requests"],
            **{m: {k: s[m][k] for k in ("speedup_vs_plain", "latency_p50_s", "latency_p99_s",
                                        "plain_latency_p50_s", "plain_latency_p99_s", "identical_results")}
               for m in ("burst", "poisson", "poisson_overload")}}
    except (OSError, KeyError, ValueError):
        pass
    scans = {}
    for fn in sorted(os.listdir(prof)) if os.path.isdir(prof) else []:
        if fn.startswith("tts_") and fn.endswith("_scan.json"):
            try:
                with open(os.path.join(prof, fn)) as f:
                    d = json.load(f)
                scans[fn[:-len("_scan.json")]] = {k: d[k] for k in ("workload", "mode", "target", "runs",
                                                                     "successes", "tts99_s", "at")}
            except (OSError, KeyError, ValueError):
                pass
    if scans:
        out["tts_scans"] = {"command": "python -m paper_2606_25203_amd.tts scan --workload <c1|c2|c4> "
                                       "[--sa] --runs 100", **scans}
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
    ap.add_argument("--batched", default="c1,c2,c4",
                    help="comma-separated workloads for the plain-vs-batched comparison ('' to skip)")
    ap.add_argument("--batch-count", type=int, default=0, help="runs per batched comparison (0: default)")
    ap.add_argument("--side", default="c1,c3,c4,c4p",
                    help="comma-separated workloads timed once each beside the headline ('' to skip)")
    ap.add_argument("--served", type=int, default=256,
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
    m = measure(pamc, torch, args.workload, args.steps, args.warmup, fields)
    out = {
        "metric": "spin-flip attempts/s + time-to-target-cut (plain vs batched/served), p50/p99",
        "value": m["value"],
        "unit": "flip attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": m["config"],
        "time_to_target": m["time_to_target"],
        **({"final_3cuts": m["final_3cuts"]} if "final_3cuts" in m else {}),
        "roofline": m["roofline"],
    }
    if args.side:
        out["other_workloads"] = {}
        for name in args.side.split(","):
            log(f"workload {name}: one timed run ...")
            out["other_workloads"][name] = measure(pamc, torch, name, 1, 1)
    if args.batched:
        out["batched"] = []
        for name in args.batched.split(","):
            log(f"batched comparison on {name} ...")
            out["batched"].append(bench_batched(pamc, torch, name, args.batch_count or None))
    if args.served:
        log("served comparison ...")
        out["served"] = bench_served(pamc, torch, args.served)
    rec = recorded_runs()
    if rec:
        out["recorded"] = rec
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        cb = cpu_baseline(w, args.cpu_seconds)
        if cb is not None:
            out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
