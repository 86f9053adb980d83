"""The sweep-shape autotuner (tile-resident sweeps on/off, replica tiles
per wavefront, quads per wavefront): it times candidates on a saved copy of
the instance's population and restores it with the stream counters, so a
tuned instance follows exactly the trajectory of an untuned one (and of the
oracle); its choice is cached per instance shape and taken by new
instances of that shape."""
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


CASES = [
    ("small_tile", lambda: synth.random_graph(800, 19176, 1), 256, None),      # tile-resident candidate
    ("torus_pull", lambda: synth.torus(60, 40, 3), 512, None),                  # tiles/quads per wave
    ("random_push", lambda: synth.random_graph(3000, 60000, 2), 256, "push"),   # quads per wave
]


@pytest.mark.parametrize("name,make,R,fields", CASES)
def test_autotune_keeps_the_trajectory(pamc, name, make, R, fields):
    g = make()
    sched = pamc.schedule(beta0=0.1, dbeta=0.05, steps=30, sweeps=3, augmented=1, z_rst=25, n_top=4,
                          mis_trials=2, win_short=4, win_long=6, max_distinct_short=2, max_distinct_long=3, tau=3)
    say(f"case autotune {name}")
    ref = pamc.Instance.csr(g, replicas=R, seed=7, fields=fields)
    ref.sweep(0.4, 2)
    rr = ref.anneal(sched)
    inst = pamc.Instance.csr(g, replicas=R, seed=7, fields=fields)
    inst.sweep(0.4, 2)
    before = inst.state()
    t = inst.autotune(0.8, sweeps=3, force=True)
    assert t.candidates >= 2 and t.cached == 0 and t.best_ms_per_sweep > 0
    assert t.best_ms_per_sweep <= t.default_ms_per_sweep
    info = inst.info()
    assert (info.tile_sweeps, info.tiles_per_wave, info.quads_per_wave) == \
        (t.tile_sweeps, t.tiles_per_wave, t.quads_per_wave)
    for a, b in zip(inst.state(), before):  # population and counters restored
        assert np.array_equal(a, b)
    r = inst.anneal(sched)
    for f in ("best_cut", "steps_run", "n_cluster_moves", "n_reheats", "n_restarts"):
        assert getattr(r, f) == getattr(rr, f), f
    assert r.sum_lnq == rr.sum_lnq
    for a, b in zip(inst.state(), ref.state()):
        assert np.array_equal(a, b)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 7)
    o.sweep(0.4, 2)
    ores = o.anneal(oracle.default_schedule(**{k: getattr(sched, k) for k, _ in sched._fields_}))
    assert ores.best_cut == r.best_cut
    for a, b in zip(inst.state(), o.state()):
        assert np.array_equal(a, b)
    # the choice is cached for this shape: a new instance takes it
    other = pamc.Instance.csr(g, replicas=R, seed=8, fields=fields)
    oi = other.info()
    assert (oi.tile_sweeps, oi.tiles_per_wave, oi.quads_per_wave) == \
        (t.tile_sweeps, t.tiles_per_wave, t.quads_per_wave)
    c = other.autotune(0.8)
    assert c.cached == 1 and c.candidates == 0
    say(f"  chosen tile={t.tile_sweeps} tpw={t.tiles_per_wave} qpw={t.quads_per_wave}: "
        f"{t.best_ms_per_sweep:.4f} ms/sweep vs {t.default_ms_per_sweep:.4f} at creation")
    for i in (ref, inst, other):
        i.close()
