"""Dense (fully connected) instances: int8 matrix-core field products and the
block-sequential sweep, against the CPU oracle through the C ABI."""
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


def same_state(inst, o, tag=""):
    s, h, E, f = inst.state()
    os_, oh, oE, of = o.state()
    assert np.array_equal(E, oE), f"{tag}: energies differ at {np.nonzero(E != oE)[0][:8]}"
    assert np.array_equal(s, os_), f"{tag}: spins differ"
    assert np.array_equal(h, oh), f"{tag}: fields differ"
    assert np.array_equal(f, of), f"{tag}: lineage differs"


@pytest.mark.parametrize("n,R", [(300, 64), (1000, 128), (130, 64), (1100, 320)])
@pytest.mark.parametrize("rule", [0, 1])
def test_dense_random_init_and_sweeps(pamc, n, R, rule):
    say(f"case dense random n={n} R={R} rule={rule}")
    inst = pamc.Instance.dense_random(n, 77, replicas=R, seed=5, rule=rule)
    o = oracle.Oracle.dense(oracle.dense_random(n, 77), R, 5, rule=rule)
    assert inst.info().W == o.W and inst.info().X == o.X
    same_state(inst, o, "init")
    for beta, k in [(0.0, 1), (0.05, 2), (0.3, 1)]:
        inst.sweep(beta, k)
        o.sweep(beta, k)
        same_state(inst, o, f"beta={beta}")
    inst.close()


@pytest.mark.parametrize("objective,rule", [(0, 0), (1, 0), (1, 1)])
@pytest.mark.parametrize("n", [200, 1000])
def test_dense_i8_weighted(pamc, objective, rule, n):
    # weights up to 127: at small beta many fields lie beyond the LDS part of
    # the threshold table, so blocks take the exact re-decision path
    rng = np.random.default_rng(3)
    A = rng.integers(-127, 128, size=(n, n)).astype(np.int8)
    J = np.triu(A, 1)
    J = (J + J.T).astype(np.int8)
    say(f"case dense i8 objective={objective} rule={rule} n={n}")
    inst = pamc.Instance.dense(J, replicas=64, seed=9, objective=objective, rule=rule)
    o = oracle.Oracle.dense(J, 64, 9, objective=objective, rule=rule)
    assert inst.info().W == o.W
    for beta in (0.001, 0.01, 0.05):
        inst.sweep(beta, 1)
        o.sweep(beta, 1)
        same_state(inst, o, f"beta={beta}")
    inst.close()


@pytest.mark.parametrize("objective", [0, 1])
@pytest.mark.parametrize("rule", [0, 1])
def test_dense_i4_weighted(pamc, objective, rule):
    # couplings in [-7, 7] take the four-bit sequential pass; n = 1300 spans
    # two super-blocks and a partial last block, and max_v sum_j |J_vj| is
    # above the LDS part of the threshold table, so beta = 0.001 also checks
    # the fields beyond it
    n = 1300
    rng = np.random.default_rng(11)
    A = rng.integers(-7, 8, size=(n, n)).astype(np.int8)
    J = np.triu(A, 1)
    J = (J + J.T).astype(np.int8)
    say(f"case dense i4 objective={objective} rule={rule}")
    inst = pamc.Instance.dense(J, replicas=128, seed=4, objective=objective, rule=rule)
    o = oracle.Oracle.dense(J, 128, 4, objective=objective, rule=rule)
    assert inst.info().W == o.W and o.X > 2047
    for beta in (0.001, 0.05, 0.5):
        inst.sweep(beta, 1)
        o.sweep(beta, 1)
        same_state(inst, o, f"beta={beta}")
    inst.close()


def test_dense_resample_and_anneal(pamc):
    n, R = 400, 128
    J = synth.dense_pm1(n, 8)
    say("case dense anneal")
    inst = pamc.Instance.dense(J, replicas=R, seed=13)
    o = oracle.Oracle.dense(J, R, 13)
    lq = inst.resample(0.01)
    olq = o.resample(0.01)
    assert abs(lq - olq) <= 1e-12 * max(1.0, abs(olq))
    same_state(inst, o, "resample")
    kw = dict(beta0=0.1 / np.sqrt(n), dbeta=2.9 / np.sqrt(n) / 24, steps=25, sweeps=1)
    res = inst.anneal(pamc.schedule(**kw))
    ores, otr = o.anneal(oracle.default_schedule(**kw), trace=True)
    assert res.best_cut == ores.best_cut and res.steps_run == ores.steps_run
    assert abs(res.sum_lnq - ores.sum_lnq) <= 1e-12 * max(1.0, abs(ores.sum_lnq))
    tr = inst.trace(kw["steps"])
    assert np.array_equal(tr["mstar"], otr["mstar"])
    c, e, sp = inst.best()
    oc, oe, osp = o.best()
    assert c == oc and np.array_equal(sp, osp)
    same_state(inst, o, "anneal")
    inst.close()


def test_dense_n4096_one_sweep(pamc):
    """Several matrix-core K slices (2048 columns each) and a full 64-row
    block grid."""
    n, R = 4096, 64
    say("case dense n=4096")
    inst = pamc.Instance.dense_random(n, 1, replicas=R, seed=2)
    o = oracle.Oracle.dense(oracle.dense_random(n, 1), R, 2)
    inst.sweep(0.02, 1)
    o.sweep(0.02, 1)
    same_state(inst, o, "n=4096")
    inst.close()


def test_dense_full_size_sampled(pamc):
    """n = 100,000, R = 256 (10^10 coupling bytes generated on the device):
    after one sweep, sampled fields equal J s with J recomputed from the
    oracle's counter-based definition, and every energy equals -1/2 s.h."""
    n, R, gseed = 100_000, 256, 1
    say("case dense full size")
    inst = pamc.Instance.dense_random(n, gseed, replicas=R, seed=3)
    beta = 0.1 / np.sqrt(n)
    inst.sweep(beta, 1)
    s, h, E, fam = inst.state()
    assert np.array_equal(E, -(s.astype(np.int64) * h).sum(axis=1) // 2)
    rng = np.random.default_rng(0)
    for v in rng.choice(n, 2, replace=False):
        row = np.array([0 if j == v else (1 if oracle.philox([min(v, j), max(v, j), 0, 5],
                                                             [gseed, 0])[0] & 1 else -1)
                        for j in range(n)], dtype=np.int64)
        for r in rng.choice(R, 3, replace=False):
            assert int(row @ s[r].astype(np.int64)) == int(h[r, v])
    inst.close()
