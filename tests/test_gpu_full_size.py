"""Parity with the oracle at the benchmark configurations' own sizes, on the
paths those configurations take (Algorithm 1; Eqs. 1-4; Scalability
section).  States, best cuts, controller traces (M*, beta, events) and ln Q
are compared after whole runs, not only on sampled replicas.

  C2 graph: the 100 x 200 torus (n = 20,000), R = 256 in the benchmark's
    kernel shape (4 replica tiles per wavefront, 2 quads per wave), with a
    short augmented schedule whose small windows force reheats, a cluster
    move over all 20,000 spins (about 100 KB of LDS per work-group) and a
    restart.
  C4 graph: the full Max-3-Cut embedding of G(7000, 21000) (n = 21,001 with
    the degree-21,000 ancilla), R = 64, 30 steps of 10 sweeps with the same
    forcing, with incremental fields (the default) and with gathered fields
    where the ancilla's field is kept.
  C3 shape: a dense +-1 instance generated on the device with n = 8192 (eight
    1024-row super-blocks), R = 256 (four sequential-pass work-groups and the
    overlapped field product), three plain steps.
The oracle takes 15-30 s per case on one host core."""
import math
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


def close(a, b):
    return abs(a - b) <= RTOL_LNQ * max(1.0, abs(b))


def compare_run(pamc, inst, o, kw):
    res = inst.anneal(pamc.schedule(**kw))
    ores, otr = o.anneal(oracle.default_schedule(**kw), trace=True)
    for k in ("best_cut", "best_energy", "steps_run", "step_reached", "n_cluster_moves", "n_reheats",
              "n_reversals", "n_restarts"):
        assert getattr(res, k) == getattr(ores, k), (k, getattr(res, k), getattr(ores, k))
    assert close(res.sum_lnq, ores.sum_lnq), (res.sum_lnq, ores.sum_lnq)
    tr = inst.trace(kw["steps"])
    k = ores.steps_run
    for key in ("mstar", "beta", "events"):
        assert np.array_equal(tr[key], otr[key][:k]), key
    assert all(close(a, b) for a, b in zip(tr["lnq"], otr["lnq"][:k]))
    c, e, sp = inst.best()
    oc, oe, osp = o.best()
    assert c == oc and e == oe and np.array_equal(sp, osp)
    s, h, E, f = inst.state()
    os_, oh, oE, of = o.state()
    assert np.array_equal(E, oE) and np.array_equal(f, of)
    assert np.array_equal(s, os_)
    assert np.array_equal(h, oh)
    return res, ores


FORCE = dict(win_short=4, win_long=6, max_distinct_short=2, max_distinct_long=3, tau=3, mis_trials=4)


def test_c2_graph_augmented_full_size(pamc, monkeypatch):
    monkeypatch.setenv("PAMC_TPW", "4")
    monkeypatch.setenv("PAMC_QPW", "2")
    g = synth.config_c2_graph()
    R, seed = 256, 77
    say("case c2 graph n=20000 R=256 augmented (forced reheats, cluster move, restart)")
    inst = pamc.Instance.csr(g, replicas=R, seed=seed)
    info = inst.info()
    assert info.pull == 1 and info.tiles_per_wave == 4 and info.quads_per_wave == 2
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, seed)
    kw = dict(beta0=0.1, dbeta=0.1, steps=40, sweeps=2, augmented=1, z_rst=30, n_top=8, **FORCE)
    res, ores = compare_run(pamc, inst, o, kw)
    assert ores.n_cluster_moves >= 1 and ores.n_reheats >= 1 and ores.n_restarts >= 1
    inst.close()


@pytest.mark.parametrize("fields", [None, "pull"])
def test_c4_embedding_augmented_full_size(pamc, fields):
    g = synth.config_c4_graph()
    R, seed = 64, 81  # a seed whose truncated run makes a cluster move and a reheat
    say(f"case c4 embedding n=21001 R=64 augmented, fields={fields or 'incremental'}")
    inst = pamc.Instance.max3cut(g, replicas=R, seed=seed, fields=fields)
    assert inst.info().n == 21001 and inst.info().pull == (1 if fields == "pull" else 0)
    o = oracle.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, R, seed)
    kw = dict(beta0=0.1, dbeta=0.1, steps=30, sweeps=10, augmented=1, z_rst=25, n_top=2, **FORCE)
    res, ores = compare_run(pamc, inst, o, kw)
    assert ores.n_cluster_moves >= 1 and ores.n_reheats >= 1
    cut, labels = inst.max3cut_decode()
    ocut, olabels = o.max3cut_decode(o.best()[2])
    assert cut == ocut and np.array_equal(labels, olabels)
    inst.close()


def test_c3_shape_dense_n8192_r256(pamc):
    n, R, gseed, seed = 8192, 256, 7, 5
    say("case dense n=8192 R=256 (eight super-blocks, four pass work-groups)")
    inst = pamc.Instance.dense_random(n, gseed, replicas=R, seed=seed)
    o = oracle.Oracle.dense(oracle.dense_random(n, gseed), R, seed)
    kw = dict(beta0=1.0 / math.sqrt(n), dbeta=0.5 / math.sqrt(n), steps=3, sweeps=1)
    compare_run(pamc, inst, o, kw)
    inst.close()
