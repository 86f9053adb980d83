"""Checkpoint and resume through the C ABI (Algorithm 1; restart from a
stored population, controller and stream counters).

A run stopped at step k (the forced failure: the process that held it is
gone) is checkpointed; the checkpoint bytes must equal the oracle's after
the same k steps; a new instance (another seed: the checkpoint carries the
key) restored from it and resumed must end bit for bit where the
uninterrupted run ends, and where the oracle ends when it resumes from the
same bytes.  pamc_set_state is checked against the oracle's population
setter, and malformed inputs are refused with nothing changed."""
import math
import struct
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

AUG = dict(beta0=0.1, dbeta=0.05, augmented=1, z_rst=35, n_top=6, mis_trials=3, win_short=5, win_long=8,
           max_distinct_short=3, max_distinct_long=5, tau=4)


@pytest.fixture(scope="module")
def pamc():
    from paper_2606_25203_amd import pamc as p
    return p


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def build(pamc, kind, seed, fields=None):
    """(library instance, oracle instance) of one kind."""
    if kind == "ising":
        g = synth.torus(24, 20, 2)
        return (pamc.Instance.csr(g, replicas=128, seed=seed, fields=fields),
                oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, seed))
    if kind == "potts":
        g = synth.random_graph(300, 900, 3)
        return (pamc.Instance.potts(g, 3, replicas=128, seed=seed, potts_rule=1, gamma=0.0),
                oracle.Oracle.potts(g.n, g.row_ptr, g.col, g.w, 3, 128, seed, rule=1, gamma=0.0))
    if kind == "max3cut":
        g = synth.random_graph(60, 180, 7)
        return (pamc.Instance.max3cut(g, replicas=128, seed=seed, fields=fields),
                oracle.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, 128, seed))
    n = 1100  # two super-blocks, the second ragged
    J = oracle.dense_random(n, 9)
    return (pamc.Instance.dense(J, replicas=128, seed=seed), oracle.Oracle.dense(J, 128, seed))


def schedules(pamc, kind, steps, resume=0):
    if kind == "dense":
        kw = dict(beta0=0.3 / math.sqrt(1100), dbeta=0.2 / math.sqrt(1100), steps=steps, sweeps=1, resume=resume)
    else:
        kw = dict(steps=steps, sweeps=2, resume=resume, **AUG)
    return pamc.schedule(**kw), oracle.default_schedule(**kw)


def same_checkpoint(a, b):
    """Byte for byte, except the sum of ln Q (offset 120), a reported
    binary64 sum whose order of summation differs between the library and
    the oracle: 1e-12 relative."""
    assert len(a) == len(b)
    for lo, hi in ((0, 120), (128, len(a))):
        if a[lo:hi] != b[lo:hi]:
            i = next(i for i in range(lo, hi) if a[i] != b[i])
            raise AssertionError(f"checkpoints differ from byte {i}")
    x, y = struct.unpack_from("<d", a, 120)[0], struct.unpack_from("<d", b, 120)[0]
    assert abs(x - y) <= 1e-12 * max(1.0, abs(y)), (x, y)


RESULT_FIELDS = ("best_cut", "best_energy", "steps_run", "step_reached", "n_cluster_moves", "n_reheats",
                 "n_reversals", "n_restarts")


@pytest.mark.parametrize("kind,fields", [("ising", "pull"), ("ising", "push"), ("potts", None),
                                         ("max3cut", None), ("dense", None)])
def test_checkpoint_resume_bit_identical(pamc, kind, fields):
    N, k = 50, 23
    say(f"case checkpoint/resume kind={kind} fields={fields}")
    # the uninterrupted run
    full, _ = build(pamc, kind, 61, fields)
    rf = full.anneal(schedules(pamc, kind, N)[0])
    tf = full.trace(N)
    # stopped at step k: the library's checkpoint equals the oracle's
    part, opart = build(pamc, kind, 61, fields)
    sk, osk = schedules(pamc, kind, k)
    part.anneal(sk)
    opart.anneal(osk)
    blob = part.checkpoint()
    oblob = opart.checkpoint()
    same_checkpoint(blob, oblob)
    part.close()
    # resumed on a fresh instance built with another seed
    res, ores = build(pamc, kind, 5, fields)
    res.restore(blob)
    assert res.checkpoint() == blob
    ores.restore(blob)
    sN, osN = schedules(pamc, kind, N, resume=1)
    rr = res.anneal(sN)
    orr, otr = ores.anneal(osN, trace=True)
    tr = res.trace(N)
    for f in RESULT_FIELDS:
        assert getattr(rr, f) == getattr(rf, f), (f, getattr(rr, f), getattr(rf, f))
        assert getattr(rr, f) == getattr(orr, f), (f, getattr(rr, f), getattr(orr, f))
    assert abs(rr.sum_lnq - rf.sum_lnq) <= 1e-12 * max(1.0, abs(rf.sum_lnq))
    for key in ("mstar", "beta", "events"):
        assert np.array_equal(tr[key][k:], tf[key][k:]), key
        assert np.array_equal(tr[key][k:], otr[key][k:rr.steps_run]), key
    for a, b, c in zip(res.state(), full.state(), ores.state()):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    assert np.array_equal(res.best()[2], full.best()[2])
    same_checkpoint(res.checkpoint(), ores.checkpoint())
    if kind == "ising":
        assert rf.n_cluster_moves > 0 and rf.n_reheats > 0
    res.close()
    full.close()


@pytest.mark.parametrize("kind", ["ising", "potts", "dense"])
def test_set_state_matches_oracle(pamc, kind):
    say(f"case set_state kind={kind}")
    inst, o = build(pamc, kind, 3)
    rng = np.random.default_rng(4)
    n, R = inst.n, inst.R
    if kind == "potts":
        spins = rng.integers(0, 3, size=(R, n)).astype(np.int8)
    else:
        spins = rng.choice(np.array([-1, 1], np.int8), size=(R, n))
    fam = rng.permutation(R).astype(np.int32)
    inst.set_state(spins, fam, [17, 3, 2])
    o.set_population(spins, fam)
    o.set_counters(17, 3, 2)
    for a, b in zip(inst.state(), o.state()):
        assert np.array_equal(a, b)
    # the stream counters moved with it: the next sweeps agree
    beta = 0.5 if kind != "dense" else 0.5 / math.sqrt(n)
    inst.sweep(beta, 2)
    o.sweep(beta, 2)
    for a, b in zip(inst.state(), o.state()):
        assert np.array_equal(a, b)
    bad = spins.copy()
    bad[1, 2] = 5
    before = inst.state()
    with pytest.raises(pamc.PamcError) as ex:
        inst.set_state(bad)
    assert ex.value.status == pamc.PAMC_ERR_INVALID_ARG
    for a, b in zip(inst.state(), before):
        assert np.array_equal(a, b)
    inst.close()


def test_restore_refuses_mismatch(pamc):
    say("case checkpoint mismatch")
    a, _ = build(pamc, "ising", 3)
    b, _ = build(pamc, "potts", 3)
    blob = a.checkpoint()
    for bad in (blob[:200], b"X" + blob[1:], blob[:640] + bytes(len(blob) - 640)):
        with pytest.raises(pamc.PamcError) as ex:
            a.restore(bad)
        assert ex.value.status == pamc.PAMC_ERR_INVALID_ARG
    with pytest.raises(pamc.PamcError):
        b.restore(blob)
    assert a.checkpoint() == blob
    a.close()
    b.close()
