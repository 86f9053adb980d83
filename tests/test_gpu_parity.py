"""Parity of the gfx950 library against the CPU oracle, through the C ABI.

Spins, fields, energies, lineage, best cuts and controller traces must match
bit for bit (integer results and the integer decisions taken from binary64
values computed by the same sequence of IEEE operations on both sides);
ln Q, a reported floating-point sum whose order of summation differs, must
agree to 1e-12 relative.
"""
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
    os_, oh, oE, of = o.state()
    assert np.array_equal(E, oE), f"{tag}: energies differ at {np.nonzero(E != oE)[0][:8]}"
    assert np.array_equal(s, os_), f"{tag}: spins differ"
    assert np.array_equal(h, oh), f"{tag}: fields differ"
    assert np.array_equal(f, of), f"{tag}: lineage differs"


def close_lnq(a, b):
    return abs(a - b) <= RTOL_LNQ * max(1.0, abs(b))


GRAPHS = {
    "c1_shape_small": lambda: synth.random_graph(301, 2500, 3),       # ragged n (not a multiple of 4)
    "torus_pm1": lambda: synth.torus(14, 10, 2),
    "dense_ish": lambda: synth.random_graph(90, 2000, 4, weights="pm1"),
}


FIELDS = ["push", "pull"]


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("R", [64, 512])
@pytest.mark.parametrize("fields", FIELDS)
def test_init_and_sweeps(pamc, gname, rule, R, fields):
    g = GRAPHS[gname]()
    seed = 1234 + R
    say(f"case init/sweeps graph={gname} n={g.n} R={R} rule={rule} fields={fields}")
    inst = pamc.Instance.csr(g, replicas=R, seed=seed, rule=rule, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, seed, rule=rule)
    same_state(inst, o, "init")
    for beta, k in [(0.0, 1), (0.3, 2), (1.7, 3), (5.0, 1)]:
        inst.sweep(beta, k)
        o.sweep(beta, k)
        same_state(inst, o, f"beta={beta}")
    inst.close()


@pytest.mark.parametrize("objective", [0, 1])
def test_objective_and_fixed_order(pamc, objective):
    g = synth.random_graph(200, 900, 8, weights="pm1")
    say(f"case objective={objective}")
    inst = pamc.Instance.csr(g, replicas=128, seed=5, objective=objective, shuffle=False)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, 5, objective=objective, shuffle=False)
    inst.sweep(0.8, 4)
    o.sweep(0.8, 4)
    same_state(inst, o)
    info = inst.info()
    assert info.W == o.W and info.X == o.X and info.num_classes == o.num_classes
    inst.close()


@pytest.mark.parametrize("delta", [0.0, 0.05, -0.03, 2.0])
@pytest.mark.parametrize("fields", FIELDS)
def test_resample(pamc, delta, fields):
    g = synth.random_graph(240, 1500, 6)
    R = 512
    say(f"case resample delta={delta} fields={fields}")
    inst = pamc.Instance.csr(g, replicas=R, seed=77, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 77)
    inst.sweep(0.7, 2)
    o.sweep(0.7, 2)
    for _ in range(3):
        lq = inst.resample(delta)
        olq = o.resample(delta)
        assert close_lnq(lq, olq), (lq, olq)
        same_state(inst, o, "after resample")
        inst.sweep(1.0, 1)
        o.sweep(1.0, 1)
        same_state(inst, o, "after sweep")
    inst.close()


@pytest.mark.parametrize("n_top,trials", [(1, 1), (8, 4), (64, 3)])
@pytest.mark.parametrize("fields", FIELDS)
def test_cluster_move(pamc, n_top, trials, fields):
    g = synth.torus(20, 16, 9)
    R = 128
    say(f"case cluster n_top={n_top} trials={trials} fields={fields}")
    inst = pamc.Instance.csr(g, replicas=R, seed=3, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 3)
    inst.sweep(2.0, 6)
    o.sweep(2.0, 6)
    for _ in range(2):
        f = inst.cluster_move(n_top, trials)
        tot, _ = o.cluster(n_top, trials)
        assert f == tot
        same_state(inst, o, "after cluster")
        inst.sweep(1.5, 1)
        o.sweep(1.5, 1)
    same_state(inst, o, "after cluster + sweep")
    inst.close()


@pytest.mark.parametrize("R,n_top", [(2048, 300), (1216, 1216), (3008, 1)])
def test_cluster_move_large_population(pamc, R, n_top):
    # several slots per thread of the selection, every slot a target, and a
    # population that is not a multiple of the work-group size
    g = synth.torus(12, 10, 4)
    say(f"case cluster R={R} n_top={n_top}")
    inst = pamc.Instance.csr(g, replicas=R, seed=21)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 21)
    inst.sweep(2.5, 4)
    o.sweep(2.5, 4)
    f = inst.cluster_move(n_top, 2)
    tot, _ = o.cluster(n_top, 2)
    assert f == tot
    same_state(inst, o, "after cluster")
    inst.close()


@pytest.mark.parametrize("R", [4096, 16384])
def test_resample_large_population(pamc, R):
    g = synth.random_graph(60, 200, 8)
    say(f"case resample R={R}")
    inst = pamc.Instance.csr(g, replicas=R, seed=5)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 5)
    inst.sweep(0.9, 2)
    o.sweep(0.9, 2)
    for delta in (0.3, -0.1):
        lq = inst.resample(delta)
        olq = o.resample(delta)
        assert close_lnq(lq, olq), (lq, olq)
        same_state(inst, o, "after resample")
    inst.close()


def test_update_best(pamc):
    g = synth.random_graph(150, 700, 2)
    inst = pamc.Instance.csr(g, replicas=64, seed=9)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 9)
    for beta in (0.5, 1.0, 2.0):
        inst.sweep(beta, 2)
        o.sweep(beta, 2)
        inst.update_best()
        o.update_best()
        c, e, sp = inst.best()
        oc, oe, osp = o.best()
        assert (c, e) == (oc, oe) and np.array_equal(sp, osp)
    inst.close()


def compare_anneal(pamc, inst, o, sched_kw):
    res = inst.anneal(pamc.schedule(**sched_kw))
    ores, otr = o.anneal(oracle.default_schedule(**sched_kw), trace=True)
    for k in ("best_cut", "best_energy", "steps_run", "step_reached", "n_cluster_moves", "n_reheats",
              "n_reversals", "n_restarts"):
        assert getattr(res, k) == getattr(ores, k), (k, getattr(res, k), getattr(ores, k))
    assert close_lnq(res.sum_lnq, ores.sum_lnq), (res.sum_lnq, ores.sum_lnq)
    tr = inst.trace(sched_kw["steps"])
    k = ores.steps_run
    assert np.array_equal(tr["mstar"], otr["mstar"][:k])
    assert np.array_equal(tr["beta"], otr["beta"][:k])
    assert np.array_equal(tr["events"], otr["events"][:k])
    assert all(close_lnq(a, b) for a, b in zip(tr["lnq"], otr["lnq"][:k]))
    c, e, sp = inst.best()
    oc, oe, osp = o.best()
    assert c == oc and e == oe and np.array_equal(sp, osp)
    same_state(inst, o, "after anneal")
    return res, ores


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("fields", FIELDS)
def test_plain_anneal_c1_full(pamc, rule, fields):
    """Plain PAMC on the full sparse Max-Cut configuration: n = 800, 19,176
    edges, R = 256, 50 steps linear 0.1 -> 3.0, 5 sweeps per step."""
    g = synth.config_c1_graph()
    say(f"case c1 full rule={rule} fields={fields}")
    inst = pamc.Instance.csr(g, replicas=256, seed=2024, rule=rule, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 256, 2024, rule=rule)
    compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=2.9 / 49, steps=50, sweeps=5))
    inst.close()


@pytest.mark.parametrize("fields", FIELDS)
def test_augmented_anneal_torus(pamc, fields):
    g = synth.torus(24, 20, 5)
    say(f"case augmented torus fields={fields}")
    inst = pamc.Instance.csr(g, replicas=256, seed=99, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 256, 99)
    res, ores = compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=0.02, steps=260, sweeps=3, augmented=1,
                                                   z_rst=120, n_top=8, mis_trials=4, tau=25))
    assert ores.n_cluster_moves > 0 and ores.n_reheats > 0
    inst.close()


def test_augmented_literal_break_and_target(pamc):
    g = synth.torus(12, 10, 1)
    say("case literal break / stop at target")
    inst = pamc.Instance.csr(g, replicas=64, seed=4)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 4)
    compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=0.05, steps=150, sweeps=2, augmented=1, z_rst=0,
                                       n_top=2, literal_break=1))
    inst2 = pamc.Instance.csr(g, replicas=64, seed=4)
    o2 = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 4)
    compare_anneal(pamc, inst2, o2, dict(beta0=0.1, dbeta=0.1, steps=100, sweeps=2, target=100,
                                         stop_at_target=1))
    inst.close()
    inst2.close()


def test_sa_mode_no_resampling(pamc):
    g = synth.random_graph(100, 400, 1)
    inst = pamc.Instance.csr(g, replicas=128, seed=4)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, 4)
    compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=0.1, steps=20, sweeps=2, resample=0))
    inst.close()


@pytest.mark.parametrize("fields", FIELDS)
def test_max3cut_anneal_and_decode(pamc, fields):
    g = synth.random_graph(60, 180, 7)
    R = 128
    say(f"case max3cut fields={fields}")
    inst = pamc.Instance.max3cut(g, replicas=R, seed=21, fields=fields)
    o = oracle.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, R, 21)
    compare_anneal(pamc, inst, o, dict(beta0=0.05, dbeta=0.03, steps=60, sweeps=4, augmented=1, z_rst=0,
                                       n_top=4))
    cut, labels = inst.max3cut_decode()
    _, _, spins = o.best()
    ocut, olabels = o.max3cut_decode(spins)
    assert cut == ocut and np.array_equal(labels, olabels)
    s = inst.state()[0]
    for r in (0, 5, 17):
        c1, l1 = inst.max3cut_decode(s[r])
        c2, l2 = o.max3cut_decode(s[r])
        assert c1 == c2 and np.array_equal(l1, l2)
    inst.close()


def test_tiny_and_edgeless(pamc):
    for g in [synth.csr_from_edges(1, [], [], []), synth.csr_from_edges(5, [], [], []),
              synth.csr_from_edges(2, [0], [1], [3])]:
        say(f"case tiny n={g.n}")
        inst = pamc.Instance.csr(g, replicas=64, seed=1)
        o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 1)
        compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=0.5, steps=6, sweeps=2))
        inst.close()


def test_invalid_inputs(pamc):
    g = synth.random_graph(20, 40, 1)
    with pytest.raises(pamc.PamcError):
        pamc.Instance.csr(g, replicas=100, seed=1)            # not a multiple of 64
    w = g.w.copy()
    w[0] = 7                                                   # breaks symmetry
    with pytest.raises(pamc.PamcError):
        pamc.pamc_create_instance_csr(g.n, g.row_ptr, g.col, w, replicas=64)
    col = g.col.copy()
    col[0] = 0 if g.row_ptr[1] > 0 and col[0] != 0 else col[0]
    with pytest.raises(pamc.PamcError):
        pamc.pamc_create_instance_csr(g.n, g.row_ptr, col, g.w, replicas=64)


@pytest.mark.parametrize("fields", FIELDS)
def test_c2_full_size_subset_parity_and_invariants(pamc, fields):
    """Torus 100 x 200 (n = 20,000) at R = 4096: sweeps of replica r depend
    only on (seed, r), so replicas 0..63 must equal an oracle run with
    R = 64.  Then one augmented step with resampling at full size, checked by
    invariants (h = J s, E = -1/2 s.h) on sampled replicas."""
    g = synth.config_c2_graph()
    say(f"case c2 full size fields={fields}")
    inst = pamc.Instance.csr(g, replicas=4096, seed=31, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 31)
    inst.sweep(0.4, 2)
    o.sweep(0.4, 2)
    s, h, E, fam = inst.state()
    os_, oh, oE, _ = o.state()
    assert np.array_equal(s[:64], os_) and np.array_equal(h[:64], oh) and np.array_equal(E[:64], oE)
    inst.resample(0.02)
    inst.sweep(0.42, 1)
    s, h, E, fam = inst.state()
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    rng = np.random.default_rng(0)
    for r in rng.choice(4096, 16, replace=False):
        sr = s[r].astype(np.int64)
        hr = np.zeros(g.n, np.int64)
        np.add.at(hr, rows, -g.w.astype(np.int64) * sr[g.col])
        assert np.array_equal(hr, h[r])
        assert E[r] == -(sr * hr).sum() // 2
    inst.close()


def weighted_int8_graph(n, m, seed):
    g = synth.random_graph(n, m, seed)
    rng = np.random.default_rng(seed + 1)
    # symmetric weights in [-127, 127] \ {0}: draw per undirected edge
    w = np.zeros_like(g.w)
    for v in range(n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            u = g.col[e]
            if u > v:
                x = int(rng.integers(1, 128)) * (1 if rng.integers(0, 2) else -1)
                w[e] = x
                f = g.row_ptr[u] + int(np.searchsorted(g.col[g.row_ptr[u]:g.row_ptr[u + 1]], v))
                w[f] = x
    return synth.Graph(g.n, g.row_ptr, g.col, w)


@pytest.mark.parametrize("jmode", [0, 1, 2])
@pytest.mark.parametrize("tpw", [1, 2, 4])
@pytest.mark.parametrize("rule", [0, 1])
def test_gathered_field_variants(pamc, monkeypatch, jmode, tpw, rule):
    monkeypatch.setenv("PAMC_TILE", "0")  # the per-class launches, not the tile-resident sweep
    """Every gathered-field kernel variant (coupling mode x tiles per wave)
    on int8 weights, where all three coupling modes apply."""
    g = weighted_int8_graph(203, 1400, 17)
    monkeypatch.setenv("PAMC_JMODE", str(jmode))
    monkeypatch.setenv("PAMC_TPW", str(tpw))
    say(f"case variant jmode={jmode} tpw={tpw} rule={rule}")
    inst = pamc.Instance.csr(g, replicas=256, seed=77, rule=rule, fields="pull")
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 256, 77, rule=rule)
    for beta, k in [(0.01, 1), (0.05, 2), (0.4, 1)]:
        inst.sweep(beta, k)
        o.sweep(beta, k)
        same_state(inst, o, f"beta={beta}")
    inst.close()


@pytest.mark.parametrize("qpw", [1, 2, 4])
@pytest.mark.parametrize("fields", FIELDS)
def test_quads_per_wave(pamc, monkeypatch, qpw, fields):
    """Work-group shapes with 1, 2 and 4 vertex quads per wavefront over
    classes spanning many work-groups with a ragged last one (n = 1,599)."""
    monkeypatch.setenv("PAMC_TILE", "0")
    g = synth.random_graph(1599, 5000, 23, weights="pm1")
    monkeypatch.setenv("PAMC_QPW", str(qpw))
    say(f"case qpw={qpw} fields={fields}")
    inst = pamc.Instance.csr(g, replicas=128, seed=31, fields=fields)
    assert inst.info().quads_per_wave == qpw
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, 31)
    for beta, k in [(0.1, 1), (0.7, 2)]:
        inst.sweep(beta, k)
        o.sweep(beta, k)
        same_state(inst, o, f"beta={beta}")
    inst.close()


@pytest.mark.parametrize("R,wgs", [(256, 4), (256, 12), (512, 24), (512, 80)])
@pytest.mark.parametrize("qpw", [1, 4])
def test_push_work_groups_loop_over_chunks(pamc, monkeypatch, R, wgs, qpw):
    """Incremental-field sweeps with a small work-group budget per instance:
    each of a tile's work-groups takes chunks c, c + stride, ... of the class
    (here 1 to 10 work-groups per tile over classes of up to 20 chunks, with
    4 tiles and with 8, the XCD-aware mapping): the oracle's trajectory
    through an augmented run."""
    monkeypatch.setenv("PAMC_TILE", "0")
    monkeypatch.setenv("PAMC_PUSH_WGS", str(wgs))
    monkeypatch.setenv("PAMC_QPW", str(qpw))
    g = synth.random_graph(1599, 5000, 23, weights="pm1")
    say(f"case push work-groups R={R} budget={wgs} qpw={qpw}")
    inst = pamc.Instance.csr(g, replicas=R, seed=37, fields="push")
    info = inst.info()
    assert info.pull == 0 and info.quads_per_wave == qpw
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 37)
    compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=0.08, steps=25, sweeps=2, augmented=1, z_rst=20, n_top=8,
                                       mis_trials=3, win_short=4, win_long=6, max_distinct_short=2,
                                       max_distinct_long=3, tau=3))
    inst.close()


@pytest.mark.parametrize("fields", FIELDS)
def test_pair_distance_matches_oracle(pamc, fields):
    """Mean normalised pair distance d_H = min(d, 1 - d) (Supplement, Hamming
    distance) of the library against the oracle on the same population:
    after initialisation, sweeps and a resampling (which makes copies, so
    many pairs are at distance 0).  Both sides sum R(R-1)/2 binary64 terms
    in different orders: 1e-12 relative."""
    g = synth.random_graph(301, 2500, 3)
    R = 192
    say(f"case pair distance fields={fields}")
    inst = pamc.Instance.csr(g, replicas=R, seed=8, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 8)
    assert close_lnq(inst.pair_distance(), o.mean_pair_distance())
    inst.sweep(0.8, 3)
    o.sweep(0.8, 3)
    inst.resample(0.3)
    o.resample(0.3)
    inst.sweep(1.2, 2)
    o.sweep(1.2, 2)
    same_state(inst, o, "pair distance")
    a, b = inst.pair_distance(), o.mean_pair_distance()
    assert close_lnq(a, b), (a, b)
    inst.close()


def hub_graph(n, m, hubs, seed, wmax):
    """A random graph plus `hubs` vertices joined to most others (rows far
    longer than a gathered row may be), symmetric weights in [-wmax, wmax]."""
    rng = np.random.default_rng(seed)
    base = synth.random_graph(n, m, seed)
    us, vs = [], []
    for v in range(n):
        for e in range(base.row_ptr[v], base.row_ptr[v + 1]):
            if base.col[e] > v:
                us.append(v)
                vs.append(int(base.col[e]))
    for k in range(hubs):
        h = n + k
        for v in range(n):
            if rng.random() < 0.7:
                us.append(v)
                vs.append(h)
    if hubs == 2:
        us.append(n)
        vs.append(n + 1)
    w = rng.integers(1, wmax + 1, size=len(us)) * rng.choice([-1, 1], size=len(us))
    return synth.csr_from_edges(n + hubs, np.array(us), np.array(vs), w.astype(np.int32))


@pytest.mark.parametrize("hubs", [1, 2])
@pytest.mark.parametrize("wmax,jmode", [(1, 2), (100, 2), (5000, 1), (5000, 0)])
@pytest.mark.parametrize("tpw", [1, 4])
def test_kept_hub_fields(pamc, monkeypatch, hubs, wmax, jmode, tpw):
    """Gathered fields with the hubs' fields kept incrementally (summed per
    work-group before one atomic per replica): sweeps, resampling (hub fields
    gathered with the population), cluster moves (hub fields updated by the
    flipped iso-sites) and the controller, against the oracle."""
    g = hub_graph(300, 700, hubs, 40 + hubs + tpw, wmax)
    monkeypatch.setenv("PAMC_JMODE", str(jmode))
    monkeypatch.setenv("PAMC_TPW", str(tpw))
    monkeypatch.setenv("PAMC_TILE", "0")  # a graph this small would otherwise sweep tile-resident
    R = 256
    say(f"case kept hub fields hubs={hubs} wmax={wmax} jmode={jmode} tpw={tpw}")
    inst = pamc.Instance.csr(g, replicas=R, seed=5, objective=pamc.ISING, fields="pull")
    info = inst.info()
    assert info.pull == 1 and info.tiles_per_wave == tpw and info.hubs == hubs and info.tile_sweeps == 0
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 5, objective=oracle.ISING)
    same_state(inst, o, "init")
    scale = 1.0 / wmax
    compare_anneal(pamc, inst, o, dict(beta0=0.1 * scale, dbeta=0.05 * scale, steps=60, sweeps=2, augmented=1,
                                       z_rst=45, n_top=16, mis_trials=3, win_short=4, win_long=6,
                                       max_distinct_short=2, max_distinct_long=3, tau=3))
    inst.close()


@pytest.mark.parametrize("jmode", [0, 1, 2])
@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("gname,R", [("c1_shape_small", 192), ("torus_pm1", 64), ("dense_ish", 128)])
def test_tile_resident_sweeps(pamc, monkeypatch, jmode, rule, gname, R):
    """Small instances sweep a replica tile per work-group with the tile's
    spins in LDS, all of a step's sweeps in one launch: the same trajectory
    as the oracle (and as the per-class launches), through sweeps,
    resampling, cluster moves and the controller."""
    g = GRAPHS[gname]()
    monkeypatch.setenv("PAMC_JMODE", str(jmode))
    monkeypatch.setenv("PAMC_TILE", "1")  # the gathered form, also where the matrix-core one would be taken
    say(f"case tile-resident sweeps {gname} R={R} jmode={jmode} rule={rule}")
    inst = pamc.Instance.csr(g, replicas=R, seed=17, rule=rule, fields="pull")
    info = inst.info()
    assert info.tile_sweeps == 1
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 17, rule=rule)
    inst.sweep(0.3, 3)
    o.sweep(0.3, 3)
    same_state(inst, o, "sweeps")
    compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=0.05, steps=50, sweeps=3, augmented=1, z_rst=40,
                                       n_top=6, mis_trials=3, win_short=4, win_long=6, max_distinct_short=2,
                                       max_distinct_long=3, tau=3))
    inst.close()


def int8_graph(n, m, seed):
    """A random graph with weights +-1, +-2 and (one in ten) +-127: the
    extremes of int8, with row sums of |w| within the tile forms' table."""
    rng = np.random.default_rng(seed)
    g = synth.random_graph(n, m, seed)
    us, vs = [], []
    for v in range(n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            if g.col[e] > v:
                us.append(v)
                vs.append(int(g.col[e]))
    w = rng.choice([1, 2, 127], p=[0.45, 0.45, 0.1], size=len(us)) * rng.choice([-1, 1], size=len(us))
    return synth.csr_from_edges(n, np.array(us), np.array(vs), w.astype(np.int32))


MMA_GRAPHS = {
    "c1_shape_small": GRAPHS["c1_shape_small"],   # n = 301: a ragged last quad and row tile
    "torus_pm1": GRAPHS["torus_pm1"],             # sparse: most 16 x 64 blocks are zero
    "dense_ish": GRAPHS["dense_ish"],             # one 64-column block
    "int8_weights": lambda: int8_graph(200, 1700, 6),
    "n1024": lambda: synth.random_graph(1024, 12000, 9),  # the largest: 16 column blocks
    "n1021": lambda: synth.random_graph(1021, 9000, 10),
}


MMA_FORMS = {"groups": dict(PAMC_TMMA_GROUPS="1"),                       # a work-group per 16 replicas
             "tile16": dict(PAMC_TMMA_GROUPS="0", PAMC_TMMA_WAVES="16"),  # a 16-wave work-group per tile
             "tile8": dict(PAMC_TMMA_GROUPS="0", PAMC_TMMA_WAVES="8")}    # an 8-wave one (large batches)


@pytest.mark.parametrize("form", list(MMA_FORMS))
@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("gname,R", [("c1_shape_small", 192), ("torus_pm1", 64), ("dense_ish", 128),
                                     ("int8_weights", 64), ("n1024", 128), ("n1021", 64)])
def test_tile_mfma_sweeps(pamc, monkeypatch, form, rule, gname, R):
    """The tile-resident step with each colour class's fields computed on the
    matrix cores (int8 couplings x int8 spins, 16 x 64 blocks), in each of
    its work-group forms: the same trajectory as the oracle through sweeps,
    resampling, cluster moves and the controller."""
    g = MMA_GRAPHS[gname]()
    monkeypatch.setenv("PAMC_TILE", "2")
    for k, v in MMA_FORMS[form].items():
        monkeypatch.setenv(k, v)
    say(f"case tile-resident matrix-core sweeps {gname} n={g.n} R={R} rule={rule} form={form}")
    inst = pamc.Instance.csr(g, replicas=R, seed=23, rule=rule)
    info = inst.info()
    assert info.tile_sweeps == 2 and info.coupling_mode == 2
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 23, rule=rule)
    scale = 1 / 40 if gname == "int8_weights" else 1
    inst.sweep(0.3 * scale, 3)
    o.sweep(0.3 * scale, 3)
    same_state(inst, o, "sweeps")
    compare_anneal(pamc, inst, o, dict(beta0=0.1 * scale, dbeta=0.05 * scale, steps=40, sweeps=3, augmented=1,
                                       z_rst=30, n_top=6, mis_trials=3, win_short=4, win_long=6,
                                       max_distinct_short=2, max_distinct_long=3, tau=3))
    inst.close()


def test_tile_mfma_default_and_mixed_batch(pamc):
    """Dense-ish int8 instances take the matrix-core form by default, sparse
    ones and those with wider couplings the gathered form, and more than
    1024 vertices neither.  A batch mixing both tile forms and per-class launches follows
    the oracle on every instance."""
    dense = synth.random_graph(301, 2500, 3)     # 16.6 entries per row
    sparse = synth.torus(14, 10, 2)              # 4 per row
    t = synth.torus(12, 9, 5)
    wide = synth.Graph(t.n, t.row_ptr, t.col, (200 * t.w).astype(np.int32))  # beyond int8: 24-bit products
    big = synth.random_graph(2052, 3000, 8)
    say("case matrix-core tile form by default, mixed batch")
    insts = [pamc.Instance.csr(g, replicas=128, seed=s) for g, s in ((dense, 1), (sparse, 2), (wide, 3), (big, 4))]
    assert [i.info().tile_sweeps for i in insts] == [2, 1, 1, 0]
    assert insts[2].info().coupling_mode == 1
    sched = pamc.schedule(beta0=0.1, dbeta=0.1, steps=12, sweeps=2, augmented=1, z_rst=10, n_top=4, tau=3)
    res = pamc.anneal_batch(insts, [sched] * 4)
    for inst, g, s, r in zip(insts, (dense, sparse, wide, big), (1, 2, 3, 4), res):
        o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, s)
        ores = o.anneal(oracle.default_schedule(beta0=0.1, dbeta=0.1, steps=12, sweeps=2, augmented=1, z_rst=10,
                                                n_top=4, tau=3))
        assert (r.best_cut, r.n_cluster_moves, r.n_reheats) == (ores.best_cut, ores.n_cluster_moves, ores.n_reheats)
        same_state(inst, o, "mixed tile forms")
        inst.close()


def test_tile_resident_largest_and_mixed_batch(pamc):
    """A large tile-resident instance (1792 vertices: 112 KB of LDS spin
    words beside the table and a class's rows) and a batch mixing
    tile-resident and per-class instances."""
    g = synth.random_graph(1792, 3000, 8)
    say("case tile-resident n=1792")
    inst = pamc.Instance.csr(g, replicas=128, seed=3)
    assert inst.info().tile_sweeps == 1
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, 3)
    compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=0.2, steps=12, sweeps=2))
    inst.close()
    big = synth.random_graph(2052, 3000, 8)
    a = pamc.Instance.csr(big, replicas=128, seed=4)
    assert a.info().tile_sweeps == 0  # 513 quads: per-class launches
    b = pamc.Instance.csr(g, replicas=128, seed=5)
    sched = pamc.schedule(beta0=0.1, dbeta=0.2, steps=10, sweeps=2)
    rb = pamc.anneal_batch([a, b], [sched, sched])
    for inst_, gg, seed, r in ((a, big, 4, rb[0]), (b, g, 5, rb[1])):
        o = oracle.Oracle.sparse(gg.n, gg.row_ptr, gg.col, gg.w, 128, seed)
        ores = o.anneal(oracle.default_schedule(beta0=0.1, dbeta=0.2, steps=10, sweeps=2))
        assert r.best_cut == ores.best_cut
        same_state(inst_, o, "mixed batch")
        inst_.close()


def expected_hist(dists, n, nbins):
    """Bins of d_H = min(d, n - d)/n as the library documents them:
    floor(2 nbins min(d, n - d) / n), the last bin also taking d_H = 1/2."""
    dd = np.rint(np.asarray(dists) * n).astype(np.int64)
    return np.bincount(np.minimum(nbins - 1, (2 * nbins * dd) // n), minlength=nbins).astype(np.int64)


@pytest.mark.parametrize("fields", FIELDS)
@pytest.mark.parametrize("nbins", [1, 7, 64])
def test_pair_distance_histogram(pamc, fields, nbins):
    """Distribution of d_H over all R(R-1)/2 pairs (Supplement, Hamming
    distance): integer bin counts equal to those of the oracle's pair
    distances, on a population with copies (distance 0) after resampling."""
    g = synth.random_graph(333, 2400, 5)
    R = 192
    say(f"case pair distance histogram fields={fields} nbins={nbins}")
    inst = pamc.Instance.csr(g, replicas=R, seed=13, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 13)
    for beta, delta in ((0.6, 0.4), (1.5, 0.5)):
        inst.sweep(beta, 3)
        o.sweep(beta, 3)
        inst.resample(delta)
        o.resample(delta)
    same_state(inst, o, "histogram")
    counts, mean = inst.pair_distance_hist(nbins)
    want = expected_hist(o.pair_distances(), g.n, nbins)
    assert np.array_equal(counts, want), (counts, want)
    assert counts.sum() == R * (R - 1) // 2
    assert close_lnq(mean, o.mean_pair_distance())
    inst.close()


@pytest.mark.parametrize("fields", FIELDS)
def test_diversity_trace_matches_oracle(pamc, fields):
    """Per-step mean d_H of the swept population on every third step of an
    augmented run (reheats, cluster moves and a restart in between), -1 on
    the others, against the oracle's trace; 1e-12 relative."""
    g = synth.torus(24, 20, 5)
    say(f"case diversity trace fields={fields}")
    kw = dict(beta0=0.1, dbeta=0.02, steps=200, sweeps=3, augmented=1, z_rst=120, n_top=8, mis_trials=4,
              tau=25, dh_every=3)
    inst = pamc.Instance.csr(g, replicas=128, seed=99, fields=fields)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, 99)
    res, ores = compare_anneal(pamc, inst, o, kw)
    k = ores.steps_run
    _, otr = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, 99).anneal(
        oracle.default_schedule(**kw), trace=True)
    dh = inst.dh_trace(kw["steps"])
    assert len(dh) == k
    want = otr["dh"][:k]
    assert np.array_equal(dh < 0, want < 0) and np.all(want[::3] >= 0) and np.all(want[1::3] < 0)
    assert all(close_lnq(a, b) for a, b in zip(dh[::3], want[::3]))
    # a run without the trace records none
    inst.anneal(pamc.schedule(beta0=0.1, dbeta=0.02, steps=5, sweeps=1))
    assert len(inst.dh_trace(5)) == 0
    inst.close()


@pytest.mark.parametrize("hubs", [1, 2])
@pytest.mark.parametrize("switch", ["0.5", "0.0", "100"])
def test_hub_graph_switches_field_form(pamc, monkeypatch, hubs, switch):
    """A hub graph with no field form forced keeps both: a run makes the
    steps whose scheduled beta lies below the switch point with gathered
    fields (hub fields kept) and the rest with incremental fields, each
    recomputed from the population at the switch.  Against the oracle,
    across the switch (cluster moves and reheats included), with the switch
    at the start (incremental only) and never (gathered only); the instance
    ends in the incremental form either way."""
    g = hub_graph(300, 700, hubs, 60 + hubs, 3)
    monkeypatch.setenv("PAMC_TILE", "0")
    monkeypatch.setenv("PAMC_HUB_SWITCH_BETA", switch)
    R = 256
    say(f"case field-form switch hubs={hubs} switch beta={switch}")
    inst = pamc.Instance.csr(g, replicas=R, seed=9)
    info = inst.info()
    assert info.pull == 0 and info.hubs == hubs
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 9)
    compare_anneal(pamc, inst, o, dict(beta0=0.05, dbeta=0.03, steps=40, sweeps=2, augmented=1, z_rst=30,
                                       n_top=16, mis_trials=3, win_short=4, win_long=6, max_distinct_short=2,
                                       max_distinct_long=3, tau=3))
    assert inst.info().pull == 0
    # the incremental fields left by the switch back carry on: sweeps and a
    # resampling after the run
    inst.sweep(0.9, 2)
    o.sweep(0.9, 2)
    inst.resample(0.2)
    o.resample(0.2)
    same_state(inst, o, "after the run")
    inst.close()


def test_hub_graph_run_stopping_before_the_switch(pamc, monkeypatch):
    """A run that stops at its target while still in the gathered form
    switches back to incremental fields on the way out."""
    g = hub_graph(300, 700, 1, 71, 2)
    monkeypatch.setenv("PAMC_TILE", "0")
    monkeypatch.setenv("PAMC_HUB_SWITCH_BETA", "100")
    R = 128
    say("case field-form switch, stop at target first")
    inst = pamc.Instance.csr(g, replicas=R, seed=4)
    o = oracle.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 4)
    res, ores = compare_anneal(pamc, inst, o, dict(beta0=0.1, dbeta=0.05, steps=80, sweeps=2, target=1,
                                                   stop_at_target=1))
    assert ores.steps_run < 80 and inst.info().pull == 0
    inst.sweep(1.0, 3)
    o.sweep(1.0, 3)
    same_state(inst, o, "after the stopped run")
    inst.close()
