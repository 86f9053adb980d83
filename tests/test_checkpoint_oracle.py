"""Checkpoint and resume on the oracle (CPU), pinned against uninterrupted
runs: Algorithm 1 is a function of the population, the controller
variables and the stream counters, so a run stopped after step k and
resumed from its checkpoint, on the same or on a freshly built instance,
must end bit for bit where the uninterrupted run ends, with the same trace
from step k on.  The checkpoint layout is the library's documented one; a
header field is checked at its stated offset."""
import struct

import numpy as np
import pytest

import synth

AUG = dict(beta0=0.1, dbeta=0.05, augmented=1, z_rst=35, n_top=6, mis_trials=3, win_short=5, win_long=8,
           max_distinct_short=3, max_distinct_long=5, tau=4)


def make(oracle_lib, kind, seed):
    if kind == "ising":
        g = synth.torus(14, 10, 2)
        return oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, seed)
    if kind == "potts":
        g = synth.random_graph(60, 160, 3)
        return oracle_lib.Oracle.potts(g.n, g.row_ptr, g.col, g.w, 3, 64, seed, rule=1)
    if kind == "max3cut":
        g = synth.random_graph(30, 70, 5)
        return oracle_lib.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, 64, seed)
    J = synth.dense_pm1(70, 4)
    return oracle_lib.Oracle.dense(J, 64, seed)


def sched(oracle_lib, kind, steps, resume=0):
    kw = dict(AUG) if kind != "dense" else dict(beta0=0.05, dbeta=0.02)
    return oracle_lib.default_schedule(steps=steps, sweeps=2, resume=resume, **kw)


@pytest.mark.parametrize("kind", ["ising", "potts", "max3cut", "dense"])
@pytest.mark.parametrize("k", [1, 13, 37])
def test_resume_equals_uninterrupted(oracle_lib, kind, k):
    N = 60
    full = make(oracle_lib, kind, 41)
    rf, tf = full.anneal(sched(oracle_lib, kind, N), trace=True)
    part = make(oracle_lib, kind, 41)
    part.anneal(sched(oracle_lib, kind, k))
    blob = part.checkpoint()
    # resumed on a fresh instance with another seed: the checkpoint carries the key
    res = make(oracle_lib, kind, 999)
    res.restore(blob)
    assert res.checkpoint() == blob
    rr, tr = res.anneal(sched(oracle_lib, kind, N, resume=1), trace=True)
    for f in ("best_cut", "steps_run", "step_reached", "n_cluster_moves", "n_reheats", "n_reversals",
              "n_restarts"):
        assert getattr(rr, f) == getattr(rf, f), f
    assert abs(rr.sum_lnq - rf.sum_lnq) <= 1e-12 * max(1.0, abs(rf.sum_lnq))
    for key in ("mstar", "beta", "events"):
        assert np.array_equal(tr[key][k:rf.steps_run], tf[key][k:rf.steps_run]), key
    for a, b in zip(res.state(), full.state()):
        assert np.array_equal(a, b)
    assert res.best()[0] == full.best()[0] and np.array_equal(res.best()[2], full.best()[2])
    if kind == "ising":  # the augmented path really switched states across the cut
        assert rf.n_reheats > 0 and rf.n_cluster_moves > 0


def test_resume_in_place_and_layout(oracle_lib):
    o = make(oracle_lib, "ising", 7)
    r1 = o.anneal(sched(oracle_lib, "ising", 20))
    blob = o.checkpoint()
    assert blob[:8] == b"PAMCCKP1"
    ver, kind, n, R = struct.unpack_from("<IIii", blob, 8)
    assert (ver, kind, n, R) == (1, 0, o.n, 64)
    assert struct.unpack_from("<Q", blob, 24)[0] == 7
    assert list(struct.unpack_from("<III", blob, 32)) == list(o.counters())
    assert struct.unpack_from("<q", blob, 48)[0] == r1.best_cut
    steps_run = struct.unpack_from("<12i", blob, 72)[5]
    assert steps_run == 20
    assert len(blob) == 640 + 64 * o.n + 4 * 64 + o.n
    spins = np.frombuffer(blob, np.int8, 64 * o.n, 640).reshape(64, o.n)
    assert np.array_equal(spins, o.state()[0])
    # resuming in place continues the same run
    o.anneal(sched(oracle_lib, "ising", 45, resume=1))
    full = make(oracle_lib, "ising", 7)
    full.anneal(sched(oracle_lib, "ising", 45))
    for a, b in zip(o.state(), full.state()):
        assert np.array_equal(a, b)


def test_restore_rejects_mismatch(oracle_lib):
    o = make(oracle_lib, "ising", 7)
    blob = o.checkpoint()
    p = make(oracle_lib, "potts", 7)
    with pytest.raises(ValueError):
        p.restore(blob)
    bad = bytearray(blob)
    bad[640] = 3  # spin outside {-1, +1}
    with pytest.raises(ValueError):
        o.restore(bytes(bad))
    with pytest.raises(ValueError):
        o.restore(blob[:100])
