"""Randomised parity: many small instances drawn from a fixed seed — graph
shapes (random, torus, with a hub, dense-ish with int8 weights), weight
ranges, objectives, Max-3-Cut embeddings and Potts labels, replica counts,
update rules, field forms and schedules (plain, augmented with short
stagnation windows and restarts, SA, stop at target, diversity trace) — each
run through the library and the oracle and compared bit for bit: results,
per-step traces, final populations, best configurations (ln Q sums to 1e-12
relative)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CASES = 96        # the first six kinds, drawn by k % 6
DENSE_CASES = 16  # dense-ish int8 graphs (the matrix-core tile form), after them


@pytest.fixture(scope="module")
def pamc():
    from paper_2606_25203_amd import pamc as m
    return m


def say(*a):
    print(*a, flush=True)


def hub_graph(rng, n, m):
    base = synth.random_graph(n, m, int(rng.integers(1 << 30)))
    us, vs = [], []
    for v in range(n):
        for e in range(base.row_ptr[v], base.row_ptr[v + 1]):
            if base.col[e] > v:
                us.append(v)
                vs.append(int(base.col[e]))
    for v in range(n):
        if rng.random() < 0.6:
            us.append(v)
            vs.append(n)
    w = np.ones(len(us), np.int32)
    return synth.csr_from_edges(n + 1, np.array(us), np.array(vs), w)


def with_weights(rng, g, wmax, positive=False):
    """The graph with symmetric random weights in [-wmax, wmax] \\ {0}
    (in [1, wmax] when positive)."""
    if wmax == 1:
        return g
    us, vs = [], []
    for v in range(g.n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            if g.col[e] > v:
                us.append(v)
                vs.append(int(g.col[e]))
    w = rng.integers(1, wmax + 1, size=len(us))
    if not positive:
        w = w * rng.choice([-1, 1], size=len(us))
    return synth.csr_from_edges(g.n, np.array(us), np.array(vs), w.astype(np.int32))


def int8_mix(rng, g):
    """The graph with weights +-1, +-2 and (one in twenty) +-127."""
    us, vs = [], []
    for v in range(g.n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            if g.col[e] > v:
                us.append(v)
                vs.append(int(g.col[e]))
    w = rng.choice([1, 2, 127], p=[0.5, 0.45, 0.05], size=len(us)) * rng.choice([-1, 1], size=len(us))
    return synth.csr_from_edges(g.n, np.array(us), np.array(vs), w.astype(np.int32))


def draw_dense_case(k):
    rng = np.random.default_rng(9000 + k)
    n = int(rng.integers(24, 420))
    m = min(int(rng.integers(4 * n, 14 * n)), n * (n - 1) // 2)
    g = synth.random_graph(n, m, int(rng.integers(1 << 30)))
    if rng.random() < 0.5:
        g = int8_mix(rng, g)
    R = int(rng.choice([64, 128, 192, 256]))
    steps = int(rng.integers(8, 30))
    sched = dict(beta0=float(rng.uniform(0.02, 0.3)), dbeta=float(rng.uniform(0.01, 0.06)), steps=steps,
                 sweeps=int(rng.integers(1, 4)))
    mode = str(rng.choice(["plain", "augmented", "augmented", "target"]))
    if mode == "augmented":
        sched.update(augmented=1, z_rst=int(rng.integers(steps // 2, steps + 5)), n_top=int(rng.integers(1, R // 8 + 1)),
                     mis_trials=int(rng.integers(1, 5)), win_short=4, win_long=6, max_distinct_short=2,
                     max_distinct_long=3, tau=int(rng.integers(1, 6)))
    elif mode == "target":
        sched.update(target=1, stop_at_target=1)
    return dict(kind="dense_ish", g=g, R=R, rule=int(rng.integers(0, 2)), fields=None,
                objective=int(rng.integers(0, 2)), sched=sched, seed=int(rng.integers(1, 1 << 40)), K=0, prule=0,
                gamma=0.0, mode=mode, wmax=int(np.abs(g.w).max()))


def draw_case(k):
    if k >= CASES:
        return draw_dense_case(k)
    rng = np.random.default_rng(7000 + k)
    kind = ["csr", "csr", "csr", "hub", "max3cut", "potts"][k % 6]
    n = int(rng.integers(24, 420))
    shape = rng.choice(["random", "torus"]) if kind in ("csr", "potts") else "random"
    if kind == "hub":
        g = hub_graph(rng, n, int(rng.integers(n, 3 * n)))
    elif shape == "torus":
        wdt = int(rng.integers(3, 20))
        g = synth.torus(wdt, max(3, n // wdt), int(rng.integers(1 << 30)))
    else:
        g = synth.random_graph(n, int(rng.integers(n // 2, 6 * n)), int(rng.integers(1 << 30)))
    wmax = int(rng.choice([1, 1, 7, 127, 5000])) if kind in ("csr", "hub") else int(rng.choice([1, 3]))
    g = with_weights(rng, g, wmax, positive=kind == "max3cut")
    R = int(rng.choice([64, 128, 192, 256]))
    rule = int(rng.integers(0, 2))
    fields = [None, "push", "pull"][int(rng.integers(0, 3))] if kind != "potts" else None
    objective = int(rng.integers(0, 2)) if kind in ("csr", "hub") else 0
    scale = 1.0 / wmax
    steps = int(rng.integers(8, 36))
    sched = dict(beta0=float(rng.uniform(0.02, 0.4)) * scale, dbeta=float(rng.uniform(0.01, 0.08)) * scale,
                 steps=steps, sweeps=int(rng.integers(1, 4)))
    mode = rng.choice(["plain", "augmented", "augmented", "augmented", "sa", "target"])
    if mode == "augmented":
        ws = int(rng.integers(3, 8))
        sched.update(augmented=1, z_rst=int(rng.integers(steps // 2, steps + 5)),
                     n_top=int(rng.integers(1, R // 8 + 1)), mis_trials=int(rng.integers(1, 5)), win_short=ws,
                     win_long=ws + int(rng.integers(1, 6)), max_distinct_short=2, max_distinct_long=3,
                     tau=int(rng.integers(1, 6)), literal_break=int(rng.random() < 0.2))
    elif mode == "sa":
        sched.update(resample=0)
    elif mode == "target":
        sched.update(target=1, stop_at_target=1)
    if kind != "potts" and rng.random() < 0.4:
        sched.update(dh_every=int(rng.integers(1, 5)))
    seed = int(rng.integers(1, 1 << 40))
    K = int(rng.integers(2, 5)) if kind == "potts" else 0
    prule = int(rng.integers(0, 2)) if K == 3 else 0
    gamma = float(rng.choice([0.0, 0.5, 1.0])) if prule == 0 else 0.0
    return dict(kind=kind, g=g, R=R, rule=rule, fields=fields, objective=objective, sched=sched, seed=seed,
                K=K, prule=prule, gamma=gamma, mode=str(mode), wmax=wmax)


def build(pamc, c):
    g = c["g"]
    if c["kind"] == "max3cut":
        return (pamc.Instance.max3cut(g, replicas=c["R"], seed=c["seed"], rule=c["rule"], fields=c["fields"]),
                oracle.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, c["R"], c["seed"], rule=c["rule"]))
    if c["kind"] == "potts":
        return (pamc.Instance.potts(g, c["K"], replicas=c["R"], seed=c["seed"], potts_rule=c["prule"],
                                    gamma=c["gamma"]),
                oracle.Oracle.potts(g.n, g.row_ptr, g.col, g.w, c["K"], c["R"], c["seed"], rule=c["prule"],
                                    gamma=c["gamma"]))
    obj = pamc.ISING if c["objective"] else pamc.MAXCUT
    oobj = oracle.ISING if c["objective"] else oracle.MAXCUT
    return (pamc.Instance.csr(g, replicas=c["R"], seed=c["seed"], rule=c["rule"], objective=obj,
                              fields=c["fields"]),
            oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, c["R"], c["seed"], rule=c["rule"], objective=oobj))


def close(a, b):
    return abs(a - b) <= 1e-12 * max(1.0, abs(b))


@pytest.mark.parametrize("k", range(CASES + DENSE_CASES))
def test_random_instance_matches_oracle(pamc, k):
    c = draw_case(k)
    say(f"case fuzz {k}: {c['kind']} n={c['g'].n} R={c['R']} rule={c['rule']} fields={c['fields']} "
        f"K={c['K']} mode={c['mode']} wmax={c['wmax']} sched={c['sched']}")
    inst, o = build(pamc, c)
    res = inst.anneal(pamc.schedule(**c["sched"]))
    ores, otr = o.anneal(oracle.default_schedule(**c["sched"]), trace=True)
    for f in ("best_cut", "best_energy", "steps_run", "step_reached", "n_cluster_moves", "n_reheats",
              "n_reversals", "n_restarts"):
        assert getattr(res, f) == getattr(ores, f), (f, getattr(res, f), getattr(ores, f))
    assert close(res.sum_lnq, ores.sum_lnq)
    steps = c["sched"]["steps"]
    tr = inst.trace(steps)
    n = ores.steps_run
    for f in ("mstar", "beta", "events"):
        assert np.array_equal(tr[f], otr[f][:n]), f
    assert all(close(a, b) for a, b in zip(tr["lnq"], otr["lnq"][:n]))
    if c["sched"].get("dh_every"):
        dh = inst.dh_trace(steps)
        want = otr["dh"][:n]
        assert np.array_equal(dh < 0, want < 0)
        assert all(close(a, b) for a, b, w in zip(dh, want, want) if w >= 0)
    s, h, E, fam = inst.state()
    os_, oh, oE, ofam = o.state()
    assert np.array_equal(E, oE) and np.array_equal(s, os_) and np.array_equal(fam, ofam)
    if c["kind"] != "potts":
        assert np.array_equal(h, oh)
    cut, en, sp = inst.best()
    ocut, oen, osp = o.best()
    assert (cut, en) == (ocut, oen) and np.array_equal(sp, osp)
    inst.close()
