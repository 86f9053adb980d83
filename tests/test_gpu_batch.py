"""Batched and served runs: every run's result must be bit-identical to the
same run made alone through pamc_anneal (and hence to the oracle, which the
single-instance path matches in the parity suite).  One direct oracle check
ties the batched path to the oracle itself."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pamc():
    from paper_2606_25203_amd import pamc as p
    return p


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same_result(a, b, tag):
    for f in ("best_cut", "best_energy", "steps_run", "step_reached", "n_cluster_moves", "n_reheats",
              "n_reversals", "n_restarts"):
        assert getattr(a, f) == getattr(b, f), f"{tag}: {f} {getattr(a, f)} != {getattr(b, f)}"
    # the same device kernels sum ln Q in the same order: exact
    assert a.sum_lnq == b.sum_lnq, f"{tag}: sum ln Q differs"


def plain_run(pamc, g, R, seed, sched, fields=None, rule=0):
    inst = pamc.Instance.csr(g, replicas=R, seed=seed, rule=rule, fields=fields)
    res = inst.anneal(sched)
    out = (res, inst.best()[2], inst.state(), inst.trace(sched.steps))
    inst.close()
    return out


def mixed_cases(pamc):
    aug = dict(beta0=0.1, dbeta=0.05, augmented=1, z_rst=60, n_top=8, mis_trials=3, win_short=5,
               win_long=8, tau=4)
    return [
        ("random300_plain", synth.random_graph(301, 2500, 3), 128, 11, pamc.schedule(steps=30, sweeps=3), None),
        ("torus_aug", synth.torus(14, 10, 2), 64, 12, pamc.schedule(steps=70, sweeps=2, **aug), None),
        ("torus_aug_push", synth.torus(16, 12, 5), 192, 13, pamc.schedule(steps=45, sweeps=1, **aug), "push"),
        ("dense_ish_pull", synth.random_graph(90, 2000, 4, weights="pm1"), 64, 14,
         pamc.schedule(steps=25, sweeps=4), "pull"),
        ("random_push", synth.random_graph(500, 9000, 9), 256, 15, pamc.schedule(steps=12, sweeps=2), "push"),
    ]


def test_batch_equals_plain(pamc):
    cases = mixed_cases(pamc)
    say("case batch of", len(cases), "mixed instances")
    insts = [pamc.Instance.csr(g, replicas=R, seed=seed, fields=f) for _, g, R, seed, _, f in cases]
    res = pamc.anneal_batch(insts, [c[4] for c in cases])
    for (name, g, R, seed, sched, f), inst, r in zip(cases, insts, res):
        say("  compare", name)
        pr, pbest, pstate, ptrace = plain_run(pamc, g, R, seed, sched, f)
        same_result(r, pr, name)
        assert np.array_equal(inst.best()[2], pbest), name
        for a, b in zip(inst.state(), pstate):
            assert np.array_equal(a, b), name
        tr = inst.trace(sched.steps)
        for k in ("mstar", "beta", "events"):
            assert np.array_equal(tr[k], ptrace[k]), f"{name}: trace {k}"
        inst.close()


def test_batch_matches_oracle(pamc):
    g = synth.torus(14, 10, 2)
    kw = dict(beta0=0.1, dbeta=0.05, steps=70, sweeps=2, augmented=1, z_rst=60, n_top=8, mis_trials=3,
              win_short=5, win_long=8, tau=4)
    say("case batch vs oracle")
    insts = [pamc.Instance.csr(g, replicas=64, seed=s) for s in (21, 22, 23)]
    res = pamc.anneal_batch(insts, [pamc.schedule(**kw)] * 3)
    for s, inst, r in zip((21, 22, 23), insts, res):
        o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, s)
        ores, otr = o.anneal(oracle.default_schedule(**kw), trace=True)
        assert r.best_cut == ores.best_cut and r.steps_run == ores.steps_run
        assert r.n_cluster_moves == ores.n_cluster_moves and r.n_restarts == ores.n_restarts
        assert abs(r.sum_lnq - ores.sum_lnq) <= 1e-12 * max(1.0, abs(ores.sum_lnq))
        assert np.array_equal(inst.trace(kw["steps"])["mstar"], otr["mstar"])
        inst.close()


def test_batch_many_seeds_one_graph(pamc):
    """The small-graph case batching is for: one graph, many seeds."""
    g = synth.random_graph(200, 4000, 6)
    sched = pamc.schedule(beta0=0.1, dbeta=2.9 / 19, steps=20, sweeps=5)
    seeds = list(range(100, 132))
    say("case 32 seeds")
    insts = [pamc.Instance.csr(g, replicas=64, seed=s) for s in seeds]
    res = pamc.anneal_batch(insts, [sched] * len(seeds))
    for s, r in zip(seeds[::7], res[::7]):
        pr = plain_run(pamc, g, 64, s, sched)[0]
        same_result(r, pr, f"seed {s}")
    for i in insts:
        i.close()


def test_batch_stop_at_target(pamc):
    g = synth.torus(10, 10, 3)
    say("case batch stop at target")
    base = pamc.Instance.csr(g, replicas=64, seed=3)
    full = base.anneal(pamc.schedule(steps=80, sweeps=2))
    base.close()
    target = full.best_cut - 2
    scheds = [pamc.schedule(steps=80, sweeps=2, target=target, stop_at_target=1), pamc.schedule(steps=40, sweeps=1)]
    insts = [pamc.Instance.csr(g, replicas=64, seed=3), pamc.Instance.csr(g, replicas=64, seed=4)]
    res = pamc.anneal_batch(insts, scheds)
    alone = plain_run(pamc, g, 64, 3, scheds[0])[0]
    same_result(res[0], alone, "stopped run")
    assert res[0].best_cut >= target and res[0].steps_run <= 80
    same_result(res[1], plain_run(pamc, g, 64, 4, scheds[1])[0], "full run")
    for i in insts:
        i.close()


def test_batch_rejects_bad_input(pamc):
    g = synth.torus(8, 8, 1)
    a = pamc.Instance.csr(g, replicas=64, seed=1)
    with pytest.raises(pamc.PamcError):
        pamc.anneal_batch([a, a], [pamc.schedule(steps=2)] * 2)
    d = pamc.Instance.dense_random(100, 1, replicas=64, seed=1)
    with pytest.raises(pamc.PamcError):
        pamc.anneal_batch([a, d], [pamc.schedule(steps=2)] * 2)
    a.close()
    d.close()


@pytest.mark.parametrize("slots,budget", [(64, 16 << 30), (2, 16 << 30), (64, 4 << 20)])
def test_server_alone_vs_mix(pamc, slots, budget):
    """Requests served in a mix (continuous batching, admissions and
    retirements between ticks) give the results they give alone."""
    reqs = synth.request_stream(8, 0.0, seed=7, n_min=60, n_max=1500)
    R = 128
    sched = pamc.schedule(beta0=0.1, dbeta=2.9 / 19, steps=20, sweeps=2)
    scheds = [pamc.schedule(beta0=0.1, dbeta=2.9 / (9 + 5 * (i % 3)), steps=10 + 5 * (i % 3), sweeps=1 + i % 2)
              for i in range(len(reqs))]
    say(f"case server slots={slots} budget={budget} requests={len(reqs)}")
    srv = pamc.Server(budget, slots, replicas=R)
    tickets = []
    for q, sc in zip(reqs[:4], scheds):
        tickets.append(srv.submit(q.graph, q.seed, sc))
    # a few ticks, then more arrivals while the first ones run
    srv.tick(3)
    srv.tick(3)
    for q, sc in zip(reqs[4:], scheds[4:]):
        tickets.append(srv.submit(q.graph, q.seed, sc))
    srv.drain()
    for t, q, sc in zip(tickets, reqs, scheds):
        got = srv.poll(t, spins=True)
        assert got is not None
        r, spins = got
        pr, pbest, _, _ = plain_run(pamc, q.graph, R, q.seed, sc)
        same_result(r, pr, f"request {q.index} n={q.graph.n}")
        assert np.array_equal(spins, pbest)
        qs, ts = srv.latency(t)
        assert 0 <= qs <= ts
    srv.close()


def test_server_rejects_oversize(pamc):
    srv = pamc.Server(1 << 20, 4, replicas=512)
    g = synth.torus(100, 100, 1)
    with pytest.raises(pamc.PamcError):
        srv.submit(g, 1, pamc.schedule(steps=5))
    with pytest.raises(pamc.PamcError):
        srv.poll(12345)
    srv.close()


def test_server_reports_bad_request(pamc):
    """A request that fails host preparation finishes with its error and
    does not disturb the others."""
    g = synth.torus(8, 8, 1)
    bad = synth.Graph(g.n, g.row_ptr, g.col, g.w.copy())
    bad.w[0] = 5  # no longer symmetric
    say("case server bad request")
    srv = pamc.Server(1 << 30, 4, replicas=64)
    t_bad = srv.submit(bad, 1, pamc.schedule(steps=3))
    t_ok = srv.submit(g, 2, pamc.schedule(steps=3))
    srv.drain()
    with pytest.raises(pamc.PamcError):
        srv.poll(t_bad)
    r = srv.poll(t_ok)
    assert r is not None and r.steps_run == 3
    st = srv.stats()
    assert st["failed"] == 1 and st["finished"] == 1 and st["submitted"] == 2
    srv.close()


def test_step_graph_replays_match_eager(pamc, monkeypatch):
    """Captured beta steps replayed many times, with eager work and waits
    between replays (stop-flag polls every 16 steps, state reads, a second
    run on the same instance), against the same calls launched eagerly:
    every step's trace entry and the final populations must agree."""
    g = synth.torus(20, 20, 4)
    kw = dict(beta0=0.1, dbeta=0.05, steps=70, sweeps=2, augmented=1, z_rst=50, n_top=4, mis_trials=2,
              win_short=5, win_long=8, tau=3, target=10**9, stop_at_target=1)

    def run():
        inst = pamc.Instance.csr(g, replicas=128, seed=8)
        r1 = inst.anneal(pamc.schedule(**kw))
        t1 = inst.trace(kw["steps"])
        s1 = inst.state()
        r2 = inst.anneal(pamc.schedule(**dict(kw, beta0=0.3)))
        t2 = inst.trace(kw["steps"])
        s2 = inst.state()
        inst.close()
        return (r1, t1, s1), (r2, t2, s2)

    say("case graph vs eager")
    monkeypatch.setenv("PAMC_NO_GRAPH", "1")
    eager = run()
    monkeypatch.delenv("PAMC_NO_GRAPH")
    graph = run()
    for (re_, te, se), (rg, tg, sg) in zip(eager, graph):
        same_result(rg, re_, "graph run")
        for k in ("mstar", "beta", "lnq", "events"):
            assert np.array_equal(tg[k], te[k]), f"trace {k}"
        for a, b in zip(sg, se):
            assert np.array_equal(a, b)


def test_server_budget_with_large_weights(pamc):
    """Admission by device footprint with weighted requests: the threshold
    table has 2X + 1 entries (X = max_v sum_j |w_vj|), so large weights make
    a request large.  The budget is never exceeded, results equal plain runs,
    and a request larger than the whole budget is refused at submission."""
    R = 64
    sched = pamc.schedule(beta0=1e-6, dbeta=2e-6, steps=12, sweeps=2)
    reqs = []
    for i in range(6):
        g = synth.random_graph(200 + 37 * i, 900, 40 + i)
        g.w[:] = 0
        rng = np.random.default_rng(i)
        # symmetric weights up to 2e5: X of a few 1e6, tables of tens of MB
        wmap = {}
        for v in range(g.n):
            for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
                a, b = min(v, g.col[e]), max(v, g.col[e])
                if (a, b) not in wmap:
                    wmap[(a, b)] = int(rng.integers(1, 200_000))
                g.w[e] = wmap[(a, b)]
        reqs.append((g, 500 + i))
    budget = 100 << 20
    srv = pamc.Server(budget, 8, replicas=R)
    say("case server with large weights, budget 100 MiB")
    tickets = [srv.submit(g, seed, sched) for g, seed in reqs]
    peak = 0
    while True:
        active, queued = srv.tick(3)
        st = srv.stats()
        peak = max(peak, st["in_use_bytes"], st["peak_bytes"])
        assert st["in_use_bytes"] <= budget
        if active == 0 and queued == 0:
            break
    assert peak <= budget
    for t, (g, seed) in zip(tickets, reqs):
        res = srv.poll(t)
        inst = pamc.Instance.csr(g, replicas=R, seed=seed)
        pr = inst.anneal(sched)
        same_result(res, pr, f"weighted request {seed}")
        inst.close()
    # one request whose table alone exceeds the budget
    g = synth.random_graph(100, 400, 3)
    g.w[:] = 300_000_000 // 20
    with pytest.raises(pamc.PamcError) as ex:
        srv.submit(g, 1, sched)
    assert ex.value.status == pamc.PAMC_ERR_OUT_OF_MEMORY
    srv.close()


def hub_graph(n, m, seed):
    """A random graph plus one vertex joined to most others (a hub row)."""
    rng = np.random.default_rng(seed)
    base = synth.random_graph(n, m, seed)
    us, vs = [], []
    for v in range(n):
        for e in range(base.row_ptr[v], base.row_ptr[v + 1]):
            if base.col[e] > v:
                us.append(v)
                vs.append(int(base.col[e]))
    for v in range(n):
        if rng.random() < 0.7:
            us.append(v)
            vs.append(n)
    w = rng.integers(1, 3, size=len(us)) * rng.choice([-1, 1], size=len(us))
    return synth.csr_from_edges(n + 1, np.array(us), np.array(vs), w.astype(np.int32))


def test_batch_switches_field_forms_per_instance(pamc, monkeypatch):
    """Hub-graph instances keep both field forms and switch from gathered to
    incremental fields at their own step inside one batched run (the batch
    is rebuilt there); each run against the oracle, bit for bit, next to an
    instance without hubs."""
    monkeypatch.setenv("PAMC_TILE", "0")
    monkeypatch.setenv("PAMC_HUB_SWITCH_BETA", "0.6")
    g1, g2, g3 = hub_graph(280, 600, 1), hub_graph(300, 650, 2), synth.torus(16, 12, 3)
    base = dict(steps=40, sweeps=2, augmented=1, z_rst=35, n_top=8, mis_trials=3, win_short=4, win_long=6,
                max_distinct_short=2, max_distinct_long=3, tau=3)
    cases = [(g1, 128, 5, dict(base, beta0=0.1, dbeta=0.03)),    # switches at step 17
             (g2, 192, 6, dict(base, beta0=0.2, dbeta=0.05)),    # at step 8
             (g1, 64, 7, dict(base, beta0=0.05, dbeta=0.01)),    # never (beta stays below 0.6)
             (g3, 64, 8, dict(base, beta0=0.1, dbeta=0.05))]     # no hubs
    say("case batch with field-form switches")
    insts = [pamc.Instance.csr(g, replicas=R, seed=sd) for g, R, sd, _ in cases]
    assert [i.info().hubs for i in insts] == [1, 1, 1, 0]
    res = pamc.anneal_batch(insts, [pamc.schedule(**kw) for *_, kw in cases])
    for (g, R, sd, kw), inst, r in zip(cases, insts, res):
        o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, sd)
        ores, otr = o.anneal(oracle.default_schedule(**kw), trace=True)
        assert (r.best_cut, r.steps_run, r.n_cluster_moves, r.n_reheats) == \
            (ores.best_cut, ores.steps_run, ores.n_cluster_moves, ores.n_reheats)
        assert np.array_equal(inst.trace(kw["steps"])["mstar"], otr["mstar"])
        s, h, E, f = inst.state()
        os_, oh, oE, of = o.state()
        assert np.array_equal(s, os_) and np.array_equal(h, oh) and np.array_equal(E, oE) and np.array_equal(f, of)
        assert inst.info().pull == 0 or inst.info().hubs == 0
        inst.close()


@pytest.mark.parametrize("count", [40, 130])
def test_batch_of_matrix_core_tiles(pamc, count):
    """Batches of dense-ish int8 instances that take the matrix-core tile
    form: 40 instances of 4 tiles run one 16-wave work-group per tile, 130
    (520 work-groups, two per compute unit) 8-wave ones; a single instance
    runs one work-group per 16-replica group.  Every batched run equals its
    plain run."""
    g = synth.random_graph(301, 2500, 3)
    sched = pamc.schedule(beta0=0.1, dbeta=0.1, steps=10, sweeps=2, augmented=1, z_rst=8, n_top=4, tau=3)
    say(f"case batch of {count} matrix-core tile instances")
    insts = [pamc.Instance.csr(g, replicas=256, seed=100 + k) for k in range(count)]
    assert insts[0].info().tile_sweeps == 2
    res = pamc.anneal_batch(insts, [sched] * count)
    for k in range(0, count, 13 if count > 40 else 3):
        want, wbest, wstate, _ = plain_run(pamc, g, 256, 100 + k, sched)
        same_result(res[k], want, f"instance {k}")
        assert np.array_equal(insts[k].best()[2], wbest)
        for x, y in zip(insts[k].state(), wstate):
            assert np.array_equal(x, y)
    for i in insts:
        i.close()
