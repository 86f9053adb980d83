"""Potts Max-K-Cut labels (Sec. "Max-3-Cut", Eqs. 6-9; the cascaded K = 3
sampler of the Supplement) on the gfx950 library against the CPU oracle,
through the C ABI.  Labels, energies, lineage, best cuts and controller
traces must match bit for bit: every label choice is taken from binary64
values computed by the same sequence of correctly rounded operations on both
sides.  ln Q must agree to 1e-12 relative."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL_LNQ = 1e-12


@pytest.fixture(scope="module")
def pamc():
    from paper_2606_25203_amd import pamc as p
    return p


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same_state(inst, o, tag=""):
    s, h, E, f = inst.state()
    os_, _, oE, of = o.state()
    assert np.array_equal(E, oE), f"{tag}: energies differ at {np.nonzero(E != oE)[0][:8]}"
    assert np.array_equal(s, os_), f"{tag}: labels differ"
    assert not h.any(), f"{tag}: Potts fields should read as 0"
    assert np.array_equal(f, of), f"{tag}: lineage differs"


def close_lnq(a, b):
    return abs(a - b) <= RTOL_LNQ * max(1.0, abs(b))


GRAPHS = {
    "ragged_pm1": lambda: synth.random_graph(301, 1200, 3, weights="pm1"),  # n not a multiple of 4
    "torus": lambda: synth.torus(14, 10, 2),
    "gnm_one": lambda: synth.random_graph(500, 1500, 8),
}
RULES = [(2, 0, 1.0), (3, 0, 1.0), (4, 0, 0.7), (3, 1, 0.0), (3, 0, 0.0)]


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("K,rule,gamma", RULES)
@pytest.mark.parametrize("R", [64, 320])
def test_potts_init_and_sweeps(pamc, gname, K, rule, gamma, R):
    g = GRAPHS[gname]()
    say(f"case potts {gname} K={K} rule={rule} gamma={gamma} R={R}")
    inst = pamc.Instance.potts(g, K, replicas=R, seed=41, potts_rule=rule, gamma=gamma)
    o = oracle.Oracle.potts(g.n, g.row_ptr, g.col, g.w, K, R, 41, rule=rule, gamma=gamma)
    info = inst.info()
    assert info.potts_K == K and info.W == o.W and info.X == o.X and info.num_classes == o.num_classes
    same_state(inst, o, "init")
    for beta, k in [(0.0, 1), (0.3, 2), (1.5, 2), (6.0, 1)]:
        inst.sweep(beta, k)
        o.sweep(beta, k)
        same_state(inst, o, f"beta={beta}")
    inst.close()


@pytest.mark.parametrize("K,rule", [(3, 0), (3, 1), (4, 0)])
def test_potts_resample(pamc, K, rule):
    g = synth.random_graph(200, 700, 5)
    R = 512
    say(f"case potts resample K={K} rule={rule}")
    inst = pamc.Instance.potts(g, K, replicas=R, seed=7, potts_rule=rule)
    o = oracle.Oracle.potts(g.n, g.row_ptr, g.col, g.w, K, R, 7, rule=rule)
    inst.sweep(0.8, 2)
    o.sweep(0.8, 2)
    for delta in (0.0, 0.3, -0.1, 2.0):
        lq = inst.resample(delta)
        olq = o.resample(delta)
        assert close_lnq(lq, olq), (lq, olq)
        same_state(inst, o, f"after resample {delta}")
        inst.sweep(1.0, 1)
        o.sweep(1.0, 1)
        same_state(inst, o, "after sweep")
    inst.close()


def test_potts_weight_table_beyond_lds(pamc):
    # weights up to 900 on degree ~10: max syn - syn_k reaches past the
    # LDS copy of the weight table (1,024 entries) at small beta
    g = synth.random_graph(120, 600, 9)
    rng = np.random.default_rng(1)
    w = np.zeros_like(g.w)
    for i in range(g.n):
        for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = g.col[e]
            if j > i:
                x = int(rng.integers(1, 900))
                w[e] = x
                # mirror entry
                for f in range(g.row_ptr[j], g.row_ptr[j + 1]):
                    if g.col[f] == i:
                        w[f] = x
    g2 = synth.Graph(g.n, g.row_ptr, g.col, w.astype(np.int32))
    say("case potts wide table")
    inst = pamc.Instance.potts(g2, 3, replicas=128, seed=3, potts_rule=1)
    o = oracle.Oracle.potts(g2.n, g2.row_ptr, g2.col, g2.w, 3, 128, 3, rule=1)
    assert 2 * o.X > 4096
    for beta in (0.0005, 0.002, 0.05):
        inst.sweep(beta, 2)
        o.sweep(beta, 2)
        same_state(inst, o, f"beta={beta}")
    inst.close()


def weighted_graph(g, wmax, seed):
    """g with symmetric integer weights drawn from [1, wmax]."""
    rng = np.random.default_rng(seed)
    w = np.zeros_like(g.w)
    for i in range(g.n):
        for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = g.col[e]
            if j > i:
                x = int(rng.integers(1, wmax + 1))
                w[e] = x
                for f in range(g.row_ptr[j], g.row_ptr[j + 1]):
                    if g.col[f] == i:
                        w[f] = x
    return synth.Graph(g.n, g.row_ptr, g.col, w.astype(np.int32))


@pytest.mark.parametrize("K,rule,wmax,packed", [(2, 0, 1500, True), (2, 0, 9000, False), (3, 0, 20, True),
                                                (3, 1, 120, False), (4, 0, 5, True), (4, 0, 40, False)])
def test_potts_weighted_label_sums(pamc, K, rule, wmax, packed):
    # the sweep keeps the K label sums of a vertex as 32/K-bit fields of one
    # integer when max_v sum_j |J_vj| < 2^(32/K - 1), as K integers otherwise;
    # the weights put each case on the side it names
    g = weighted_graph(synth.random_graph(200, 1000, 5), wmax, K)
    say(f"case potts weighted K={K} rule={rule} wmax={wmax}")
    inst = pamc.Instance.potts(g, K, replicas=128, seed=6, potts_rule=rule, gamma=1.0)
    o = oracle.Oracle.potts(g.n, g.row_ptr, g.col, g.w, K, 128, 6, rule=rule, gamma=1.0)
    assert (o.X < (1 << (32 // K - 1))) == packed
    same_state(inst, o, "init")
    for beta in (0.001, 0.02, 0.3):
        inst.sweep(beta, 2)
        o.sweep(beta, 2)
        same_state(inst, o, f"beta={beta}")
    inst.close()


@pytest.mark.parametrize("K,rule,gamma", [(3, 0, 1.0), (3, 1, 0.0), (2, 0, 0.5)])
def test_potts_anneal(pamc, K, rule, gamma):
    g = synth.random_graph(400, 1200, 12)
    say(f"case potts anneal K={K} rule={rule}")
    inst = pamc.Instance.potts(g, K, replicas=256, seed=17, potts_rule=rule, gamma=gamma)
    o = oracle.Oracle.potts(g.n, g.row_ptr, g.col, g.w, K, 256, 17, rule=rule, gamma=gamma)
    kw = dict(beta0=0.2, dbeta=0.05, steps=90, sweeps=3, augmented=1, z_rst=60, n_top=4, mis_trials=2)
    res = inst.anneal(pamc.schedule(**kw))
    ores, otr = o.anneal(oracle.default_schedule(**kw), trace=True)
    for k in ("best_cut", "best_energy", "steps_run", "step_reached", "n_cluster_moves", "n_reheats",
              "n_reversals", "n_restarts"):
        assert getattr(res, k) == getattr(ores, k), (k, getattr(res, k), getattr(ores, k))
    assert res.n_cluster_moves == 0
    assert close_lnq(res.sum_lnq, ores.sum_lnq)
    tr = inst.trace(kw["steps"])
    n = ores.steps_run
    assert np.array_equal(tr["mstar"], otr["mstar"][:n])
    assert np.array_equal(tr["events"], otr["events"][:n])
    c, e, lab = inst.best()
    oc, oe, olab = o.best()
    assert c == oc and e == oe and np.array_equal(lab, olab)
    # the reported cut is the K-cut of the returned labels
    cut = sum(int(g.w[q]) for i in range(g.n) for q in range(g.row_ptr[i], g.row_ptr[i + 1])
              if g.col[q] > i and lab[i] != lab[g.col[q]])
    assert cut == c
    same_state(inst, o, "after anneal")
    inst.close()


def test_potts_batch_equals_plain(pamc):
    # Potts and Ising instances in one batch give their plain results
    gs = [synth.random_graph(300, 900, 2), synth.torus(16, 12, 3), synth.random_graph(150, 500, 4)]
    kw = dict(beta0=0.2, dbeta=0.05, steps=40, sweeps=2)

    def make():
        return [pamc.Instance.potts(gs[0], 3, replicas=128, seed=5, potts_rule=1),
                pamc.Instance.csr(gs[1], replicas=192, seed=6),
                pamc.Instance.potts(gs[2], 4, replicas=64, seed=7, gamma=0.8)]
    plain = []
    for inst in make():
        r = inst.anneal(pamc.schedule(**kw))
        plain.append((r.best_cut, r.steps_run, inst.state()))
        inst.close()
    insts = make()
    res = pamc.anneal_batch(insts, [pamc.schedule(**kw)] * len(insts))
    for inst, r, (c, n, st) in zip(insts, res, plain):
        assert r.best_cut == c and r.steps_run == n
        s2 = inst.state()
        for a, b in zip(s2, st):
            assert np.array_equal(a, b)
        inst.close()


def test_potts_rejects_bad_input(pamc):
    g = synth.random_graph(50, 100, 1)
    for K, rule, gamma in [(1, 0, 1.0), (2, 1, 1.0), (4, 1, 1.0), (3, 2, 1.0), (3, 0, -1.0), (3, 0, float("nan"))]:
        with pytest.raises(pamc.PamcError) as ei:
            pamc.Instance.potts(g, K, replicas=64, seed=1, potts_rule=rule, gamma=gamma)
        assert ei.value.status == 1
    with pytest.raises(pamc.PamcError) as ei:
        pamc.Instance.potts(g, 5, replicas=64, seed=1)
    assert ei.value.status == 5
    inst = pamc.Instance.potts(g, 3, replicas=64, seed=1)
    with pytest.raises(pamc.PamcError) as ei:
        inst.cluster_move(4, 2)
    assert ei.value.status == 5
    with pytest.raises(pamc.PamcError) as ei:
        inst.pair_distance()
    assert ei.value.status == 5
    with pytest.raises(pamc.PamcError):
        inst.sweep(-0.5, 1)
    inst.close()
