"""The benchmark workloads: seeded synthetic instances of the shapes the
method is measured on, with the annealing schedule each is run with.

  c1   plain PAMC, random graph n = 800, m = 19,176, w = +1, R = 256,
       50 beta steps 0.1 -> 3.0 x 5 sweeps
  c2   augmented PAMC, 100 x 200 torus with +-1 weights (n = 20,000,
       degree 4), R = 4096, 500 beta steps x 10 sweeps
  c3   plain PAMC, dense +-1 Ising n = 100,000 (int8 J), R = 256,
       200 beta steps 0.1/sqrt(n) -> 3.0/sqrt(n) x 1 sweep
  c4   augmented PAMC, Max-3-Cut one-hot embedding of G(7000, 21000)
       (n = 21,001), R = 2048, 300 beta steps x 10 sweeps
  c4p  the same graph with 3-state Potts labels, softmax-perturbed argmax
  c4c  the same with the cascaded p-bit sampler

`counters` names the committed rocprofv3 counter summary of the workload's
sweep kernel; `cpu` the bounded sample the CPU oracle is timed on.
"""
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def workload(name):
    import synth
    if name == "c2":
        g = synth.torus(100, 200, seed=1)
        return dict(kind="csr", graph=g, R=4096, steps=500, sweeps=10,
                    sched=dict(beta0=0.1, dbeta=0.02, steps=500, sweeps=10, augmented=1, z_rst=400, n_top=128,
                               mis_trials=4, tau=25),
                    desc="augmented PAMC, 100x200 torus +-1 weights (n=20000, degree 4), R=4096, "
                         "500 beta steps x 10 sweeps",
                    counters="k_sweep_pull_torus100x200_R4096", cpu=dict(R=64, step_s=0.4))
    if name == "c1":
        g = synth.random_graph(800, 19176, seed=1)
        return dict(kind="csr", graph=g, R=256, steps=50, sweeps=5,
                    sched=dict(beta0=0.1, dbeta=2.9 / 49, steps=50, sweeps=5),
                    desc="plain PAMC, random graph n=800 m=19176 w=+1, R=256, 50 beta steps 0.1->3.0 x 5 sweeps",
                    counters="k_sweep_tmma_gnm800_R256", cpu=dict(R=256, step_s=0.3))
    if name == "c3":
        n = 100_000
        return dict(kind="dense", n=n, R=256, steps=200, sweeps=1,
                    sched=dict(beta0=0.1 / math.sqrt(n), dbeta=2.9 / math.sqrt(n) / 199, steps=200, sweeps=1),
                    desc="plain PAMC, dense +-1 Ising n=100000 (int8 J, 10 GB), R=256, "
                         "200 beta steps 0.1/sqrt(n)->3.0/sqrt(n) x 1 sweep",
                    counters="k_dense_n100000_R256", cpu=None)
    if name == "c4":
        g = synth.random_graph(7000, 21000, seed=1)
        return dict(kind="max3cut", graph=g, R=2048, steps=300, sweeps=10,
                    sched=dict(beta0=0.1, dbeta=0.02, steps=300, sweeps=10, augmented=1, z_rst=400, n_top=64,
                               mis_trials=4, tau=25),
                    desc="augmented PAMC, Max-3-Cut one-hot embedding of G(7000, 21000) (n=21001), R=2048, "
                         "300 beta steps x 10 sweeps",
                    counters="k_sweep_push_max3cut7000_R2048", cpu=dict(R=64, step_s=1.5))
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
                    counters="k_sweep_potts_potts7000_R2048", cpu=dict(R=64, step_s=0.6))
    raise ValueError(f"unknown workload {name}")


def make_instance(pamc, w, seed, fields=None):
    if w["kind"] == "csr":
        return pamc.Instance.csr(w["graph"], replicas=w["R"], seed=seed, fields=fields)
    if w["kind"] == "max3cut":
        return pamc.Instance.max3cut(w["graph"], replicas=w["R"], seed=seed, fields=fields)
    if w["kind"] == "potts":
        return pamc.Instance.potts(w["graph"], w["K"], replicas=w["R"], seed=seed, potts_rule=w["potts_rule"],
                                   gamma=w["gamma"])
    return pamc.Instance.dense_random(w["n"], 1, replicas=w["R"], seed=seed)
