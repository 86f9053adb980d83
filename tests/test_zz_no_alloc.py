"""The batched anneal that allocates no device memory
(pamc_anneal_batch_noalloc) against pamc_anneal_batch through the C ABI:
results and final populations bit for bit, on two calls in a row (the
second smaller, so the fixed scratch holds the first call's contents), and
a batch larger than the fixed scratch refused before any device work."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pamc():
    from paper_2606_25203_amd import pamc as p
    return p


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


FIELDS = ("best_cut", "best_energy", "steps_run", "step_reached", "n_cluster_moves", "n_reheats",
          "n_reversals", "n_restarts")


def build(pamc, cases):
    out = []
    for name, kind, g, R, seed, sched, f in cases:
        if kind == "potts":
            out.append(pamc.Instance.potts(g, 3, replicas=R, seed=seed))
        else:
            out.append(pamc.Instance.csr(g, replicas=R, seed=seed, fields=f))
    return out


def compare(pamc, cases):
    scheds = [c[5] for c in cases]
    ref = build(pamc, cases)
    rr = pamc.anneal_batch(ref, scheds)
    got = build(pamc, cases)
    rg = pamc.anneal_batch_noalloc(got, scheds)
    for c, a, b, ia, ib in zip(cases, rg, rr, got, ref):
        name = c[0]
        for f in FIELDS:
            assert getattr(a, f) == getattr(b, f), f"{name}: {f} {getattr(a, f)} != {getattr(b, f)}"
        assert a.sum_lnq == b.sum_lnq, name
        assert np.array_equal(ia.best()[2], ib.best()[2]), name
        for x, y in zip(ia.state(), ib.state()):
            assert np.array_equal(x, y), name
        assert ia.trace(c[5].steps)["mstar"].size == 0, name  # no trace recorded
    for i in ref + got:
        i.close()


def test_noalloc_batch_equals_batch_twice(pamc):
    aug = dict(beta0=0.1, dbeta=0.05, augmented=1, z_rst=60, n_top=8, mis_trials=3, win_short=5,
               win_long=8, tau=4)
    first = [
        ("random300_plain", "csr", synth.random_graph(301, 2500, 3), 128, 11, pamc.schedule(steps=30, sweeps=3), None),
        ("torus_aug", "csr", synth.torus(14, 10, 2), 64, 12, pamc.schedule(steps=70, sweeps=2, **aug), None),
        ("torus_aug_push", "csr", synth.torus(16, 12, 5), 192, 13, pamc.schedule(steps=45, sweeps=1, **aug), "push"),
        ("c2_graph_aug", "csr", synth.torus(100, 200, 1), 128, 16,
         pamc.schedule(steps=50, sweeps=2, **dict(aug, n_top=16, mis_trials=4)), None),
        ("potts_aug", "potts", synth.random_graph(200, 600, 7), 64, 17, pamc.schedule(steps=40, sweeps=2, **aug), None),
        ("random_push", "csr", synth.random_graph(500, 9000, 9), 256, 15, pamc.schedule(steps=12, sweeps=70), "push"),
    ]
    say("case noalloc batch, first call:", len(first), "instances")
    compare(pamc, first)
    second = [
        ("torus_small_aug", "csr", synth.torus(8, 6, 3), 64, 21, pamc.schedule(steps=60, sweeps=3, **aug), None),
        ("random_small", "csr", synth.random_graph(90, 300, 4), 64, 22, pamc.schedule(steps=20, sweeps=2), None),
    ]
    say("case noalloc batch, second (smaller) call:", len(second), "instances")
    compare(pamc, second)


def test_noalloc_batch_refuses_oversize_scratch(pamc):
    # cluster scratch 512 targets x 8 trials x 20,000 spins = 82 MB > 16 MiB
    g = synth.torus(100, 200, 1)
    say("case noalloc batch larger than the fixed scratch")
    inst = pamc.Instance.csr(g, replicas=512, seed=3)
    before = inst.state()
    sched = pamc.schedule(steps=5, sweeps=1, beta0=0.1, dbeta=0.05, augmented=1, n_top=512, mis_trials=8)
    with pytest.raises(pamc.PamcError) as ex:
        pamc.anneal_batch_noalloc([inst], [sched])
    assert ex.value.status == pamc.PAMC_ERR_UNSUPPORTED and "scratch" in str(ex.value)
    for x, y in zip(inst.state(), before):
        assert np.array_equal(x, y)
    inst.close()
