"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against a fact fixed by the paper or by
mathematics: an independent Philox implementation (rocRAND's, run on the
host), mpmath at high precision, exact enumeration of small Ising models,
closed forms (1-D ring partition function, complete-graph max cut), brute
force over all cuts, and the controller rule's constants as the paper states
them (Sec. "Augmented PAMC": windows of 25 and 40 steps, at most three
distinct values vs more than five, reheat factor 0.8).
"""
import itertools
import math
import os
import shutil
import subprocess
import tempfile

import mpmath
import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------- helpers
def dense_from_graph(g, objective):
    J = np.zeros((g.n, g.n), np.int64)
    for v in range(g.n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            J[v, g.col[e]] = -g.w[e] if objective == 0 else g.w[e]
    return J


def all_states(n):
    return np.array(list(itertools.product([-1, 1], repeat=n)), dtype=np.int64)


def energies_all(J):
    S = all_states(J.shape[0])
    return -0.5 * np.einsum("ki,ij,kj->k", S, J, S), S


def ring(n, w=1):
    u = np.arange(n)
    return synth.csr_from_edges(n, u, (u + 1) % n, np.full(n, w, np.int32))


# ----------------------------------------------------------------- Philox
def test_philox_matches_rocrand_host_engine(oracle_lib, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "kat"
    subprocess.run([hipcc, "-O1", "-w", os.path.join(HERE, "golden", "philox_rocrand_kat.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    rng = np.random.default_rng(123)
    rows = []
    for _ in range(3000):
        seed = int(rng.integers(0, 2**63))
        c = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)),
             int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        rows.append((seed, c))
    rows.append((0, [0, 0, 0, 0]))
    rows.append((2**64 - 1, [2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1]))
    inp = "\n".join(f"{s} {c[0]} {c[1]} {c[2]} {c[3]}" for s, c in rows) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (seed, c), line in zip(rows, out):
        ref = [int(x) for x in line.split()]
        got = oracle_lib.philox(c, [seed & 0xFFFFFFFF, seed >> 32])
        assert list(got) == ref, (seed, c)


def test_philox_bit_balance(oracle_lib):
    words = np.concatenate([oracle_lib.philox([i, 7, 3, 1], [11, 12]) for i in range(4000)])
    bits = np.unpackbits(words.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.01


# ----------------------------------------------------------------- exp
def ulp(x):
    return math.ulp(x) if x != 0 else 5e-324


def test_pexp_within_one_ulp_of_mpmath(oracle_lib):
    mpmath.mp.dps = 40
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.uniform(-740, 705, 6000), rng.uniform(-1, 1, 4000),
                         rng.uniform(-30, 30, 4000), [0.5 * math.log(2), -0.5 * math.log(2), 1e-300, -1e-300]])
    worst = 0.0
    for x in xs:
        got = oracle_lib.pexp(float(x))
        exact = mpmath.exp(mpmath.mpf(float(x)))
        err = abs(mpmath.mpf(got) - exact) / ulp(float(exact))
        worst = max(worst, float(err))
    assert worst <= 1.0, worst
    assert oracle_lib.pexp(0.0) == 1.0
    assert oracle_lib.pexp(-0.0) == 1.0
    assert oracle_lib.pexp(800.0) == math.inf
    assert oracle_lib.pexp(-800.0) == 0.0


def test_pexp_subnormal_range(oracle_lib):
    mpmath.mp.dps = 40
    for x in np.linspace(-745.0, -708.0, 400):
        got = oracle_lib.pexp(float(x))
        exact = float(mpmath.exp(mpmath.mpf(float(x))))  # correctly rounded
        assert abs(got - exact) <= 5e-324, x


# ----------------------------------------------------------------- thresholds
@pytest.mark.parametrize("rule", [0, 1])
def test_thresholds_vs_mpmath(oracle_lib, rule):
    mpmath.mp.dps = 50
    two32 = mpmath.mpf(2) ** 32
    for beta in [0.0, 0.01, 0.1, 0.37, 1.0, 3.0, 10.0]:
        for x in range(-40, 41):
            b = mpmath.mpf(beta)
            if rule == 0:
                p = 1 / (1 + mpmath.exp(2 * b * x))   # Eq. 4 flip probability
            else:
                p = mpmath.mpf(1) if x <= 0 else mpmath.exp(-2 * b * x)
            q = p * two32
            exact = min(int(mpmath.floor(q)), 2**32 - 1)
            got = oracle_lib.threshold(beta, rule, x)
            frac = q - mpmath.floor(q)
            if min(frac, 1 - frac) < mpmath.mpf("1e-5"):
                assert abs(got - exact) <= 1
            else:
                assert got == exact, (beta, x, got, exact)
    assert oracle_lib.threshold(0.7, 0, 0) == 2**31      # h = 0 flips with probability 1/2
    assert all(oracle_lib.threshold(0.0, 0, x) == 2**31 for x in range(-50, 51))


# ----------------------------------------------------------------- colouring
def dsatur(g):
    """Saturation-degree colouring written out plainly: repeatedly the
    uncoloured vertex with the most distinct colours among its coloured
    neighbours (ties: the higher degree, then the lower id) takes the least
    colour none of its neighbours has."""
    col = [-1] * g.n
    deg = [int(g.row_ptr[v + 1] - g.row_ptr[v]) for v in range(g.n)]
    nbrs = [[int(u) for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]] for v in range(g.n)]
    for _ in range(g.n):
        best = None
        for v in range(g.n):
            if col[v] >= 0:
                continue
            key = (len({col[u] for u in nbrs[v] if col[u] >= 0}), deg[v], -v)
            if best is None or key > best[0]:
                best = (key, v)
        v = best[1]
        used = {col[u] for u in nbrs[v]}
        k = 0
        while k in used:
            k += 1
        col[v] = k
    return col


def first_fit(g):
    col = [-1] * g.n
    for v in range(g.n):
        used = {col[u] for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if u < v}
        k = 0
        while k in used:
            k += 1
        col[v] = k
    return col


def test_colouring_is_dsatur_and_valid(oracle_lib):
    for g in [synth.random_graph(300, 2000, 3), synth.torus(10, 8, 1), synth.random_graph(50, 600, 9),
              synth.random_graph(120, 200, 5)]:
        k, col = oracle_lib.colour(g.n, g.row_ptr, g.col)
        assert list(col) == dsatur(g)
        assert k == max(col) + 1
        for v in range(g.n):
            for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]:
                assert col[u] != col[v]
        assert k <= max(first_fit(g)) + 1  # no more colours than first-fit on these graphs
    g = synth.config_c2_graph()
    k, col = oracle_lib.colour(g.n, g.row_ptr, g.col)
    assert k == 2  # even torus is bipartite
    assert list(col) == first_fit(g)  # the same two classes as a first-fit colouring in id order


def test_max3cut_colouring_is_proper_and_balanced(oracle_lib):
    """The embedding's classes: spin (i, a) in (c(i) + a) mod max(k, 3), the
    ancilla alone; a proper colouring of the embedded graph, checked edge by
    edge, and the oracle's instance takes these classes."""
    for g in [synth.random_graph(60, 150, 3), synth.random_graph(7, 13, 4), synth.config_c4_graph()]:
        k, c = oracle_lib.colour(g.n, g.row_ptr, g.col)
        m3k, m3 = oracle_lib.max3cut_colour(g.n, g.row_ptr, g.col)
        m = max(k, 3)
        assert m3k == m + 1 and m3[3 * g.n] == m
        assert all(m3[3 * i + a] == (c[i] + a) % m for i in range(g.n) for a in range(3))
        # the embedding's edges: the three spins of a vertex, the spins of an
        # edge in one layer, the ancilla with every spin
        for i in range(g.n):
            assert len({m3[3 * i], m3[3 * i + 1], m3[3 * i + 2]}) == 3
            for j in g.col[g.row_ptr[i]:g.row_ptr[i + 1]]:
                for a in range(3):
                    assert m3[3 * i + a] != m3[3 * j + a]
        assert np.count_nonzero(m3 == m) == 1
        o = oracle_lib.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, 64, 1)
        assert np.array_equal(np.diff(o.class_ptr()), np.bincount(m3, minlength=m + 1))


def test_internal_order_is_class_major(oracle_lib):
    g = synth.random_graph(120, 700, 4)
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 1)
    _, col = oracle_lib.colour(g.n, g.row_ptr, g.col)
    ids = o.internal_ids()
    order = sorted(range(g.n), key=lambda v: (col[v], v))
    assert [int(ids[v]) for v in order] == list(range(g.n))
    cp = o.class_ptr()
    assert cp[-1] == g.n and len(cp) == max(col) + 2


# ----------------------------------------------------------------- sweep invariants
@pytest.mark.parametrize("rule", [0, 1])
def test_sweep_invariants(oracle_lib, rule):
    g = synth.random_graph(150, 900, 8, weights="pm1")
    for objective in (0, 1):
        o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 3, rule=rule, objective=objective)
        J = dense_from_graph(g, objective)
        W = sum(-J[i, j] for i in range(g.n) for j in range(i + 1, g.n))
        assert o.W == W
        for beta in (0.2, 1.0, 3.0):
            o.sweep(beta, 2)
            s, h, E, _ = o.state()
            s64 = s.astype(np.int64)
            assert np.array_equal(h, s64 @ J.T)                      # Eq. 3
            assert np.array_equal(E, -np.einsum("ri,ij,rj->r", s64, J, s64) // 2)
            cut_direct = np.array([sum(-J[i, j] * (1 - s64[r, i] * s64[r, j]) // 2
                                       for i, j in zip(*np.nonzero(np.triu(J, 1)))) for r in range(4)])
            assert np.array_equal((W - E[:4]) // 2, cut_direct)


def test_beta_zero_heatbath_flips_half(oracle_lib):
    g = synth.random_graph(200, 1000, 2)
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 256, 9)
    s0 = o.state()[0].copy()
    o.sweep(0.0, 1)
    s1 = o.state()[0]
    frac = (s0 != s1).mean()
    assert abs(frac - 0.5) < 0.01


# ----------------------------------------------------------------- Boltzmann
@pytest.mark.parametrize("rule", [0, 1])
def test_boltzmann_histogram_by_enumeration(oracle_lib, rule):
    g = synth.random_graph(9, 16, 21, weights="pm1")
    beta = 0.6
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 512, 17, rule=rule, objective=1)
    o.sweep(beta, 40)
    samples = []
    for _ in range(300):
        o.sweep(beta, 1)
        samples.append(o.state()[2].copy())
    samples = np.concatenate(samples)
    J = dense_from_graph(g, 1)
    Eall, _ = energies_all(J)
    levels = np.unique(Eall)
    wts = np.array([np.exp(-beta * e) * np.sum(Eall == e) for e in levels])
    p_exact = wts / wts.sum()
    p_emp = np.array([np.mean(samples == e) for e in levels])
    tv = 0.5 * np.abs(p_exact - p_emp).sum()
    assert tv < 0.015, tv


# ----------------------------------------------------------------- resampling
def test_resample_counts_follow_weights(oracle_lib):
    # run many independent resamplings of a population with known energies
    g = synth.random_graph(12, 30, 5)
    R = 256
    tot = np.zeros(R)
    expect = np.zeros(R)
    for rep in range(40):
        o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 1000 + rep)
        E = o.state()[2].astype(np.float64)
        delta = 0.15
        lnq, parents = o.resample(delta, return_parents=True)
        assert np.all(np.diff(parents) >= 0)
        tau = np.exp(-delta * (E - E.min()))
        tau = tau / tau.sum() * R                           # Eqs. 1-2: sum tau = R
        cnt = np.bincount(parents, minlength=R)
        # pool by energy level so that expected counts are large
        for e in np.unique(E):
            m = E == e
            tot[int(e - E.min()) % R] += cnt[m].sum()
            expect[int(e - E.min()) % R] += tau[m].sum()
        # ln Q of Eq. 2 to 1e-12 relative, evaluated in mpmath
        mpmath.mp.dps = 40
        Q = sum(mpmath.exp(-mpmath.mpf(delta) * int(x)) for x in E) / R
        assert abs(lnq - float(mpmath.log(Q))) <= 1e-12 * max(1.0, abs(float(mpmath.log(Q))))
    m = expect > 5
    chi2 = float(((tot[m] - expect[m]) ** 2 / expect[m]).sum())
    dof = int(m.sum()) - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof), (chi2, dof)


def test_resample_delta_zero_keeps_multiset_uniform(oracle_lib):
    g = synth.random_graph(12, 30, 5)
    R = 512
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 77)
    s0, h0, E0, f0 = [x.copy() for x in o.state()]
    lnq, parents = o.resample(0.0, return_parents=True)
    assert abs(lnq) < 1e-15
    s1, h1, E1, f1 = o.state()
    assert np.array_equal(s1, s0[parents]) and np.array_equal(E1, E0[parents])
    assert np.array_equal(h1, h0[parents]) and np.array_equal(f1, f0[parents])
    # uniform multinomial: number of distinct parents ~ R(1 - 1/e)
    assert abs(len(np.unique(parents)) / R - (1 - math.exp(-1))) < 0.05


def test_free_energy_ring_closed_form(oracle_lib):
    # ferromagnetic ring: Z = (2 cosh b)^N + (2 sinh b)^N
    n = 12
    g = ring(n)
    o = oracle_lib.Oracle.sparse(n, g.row_ptr, g.col, g.w, 4096, 5, objective=1)
    sched = oracle_lib.default_schedule(beta0=0.0, dbeta=0.05, steps=21, sweeps=2)
    res = o.anneal(sched)
    b = 1.0
    lnz = math.log((2 * math.cosh(b)) ** n + (2 * math.sinh(b)) ** n) - n * math.log(2)
    assert abs(res.sum_lnq - lnz) < 0.05, (res.sum_lnq, lnz)


def test_free_energy_by_enumeration(oracle_lib):
    g = synth.random_graph(12, 24, 33, weights="pm1")
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 4096, 8, objective=1)
    sched = oracle_lib.default_schedule(beta0=0.0, dbeta=0.05, steps=25, sweeps=2)
    res = o.anneal(sched)
    J = dense_from_graph(g, 1)
    Eall, _ = energies_all(J)
    b_end = 24 * 0.05
    lnz = math.log(np.exp(-b_end * Eall).sum()) - g.n * math.log(2)
    assert abs(res.sum_lnq - lnz) < 0.06, (res.sum_lnq, lnz)


# ----------------------------------------------------------------- cluster move
def test_cluster_move_independent_maximal_energy_preserving(oracle_lib):
    g = synth.torus(12, 10, 4)
    R = 64
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 6)
    o.sweep(1.5, 10)
    s0, h0, E0, _ = [x.copy() for x in o.state()]
    n_top = 16
    tot, sizes = o.cluster(n_top, 4)
    s1, h1, E1, _ = o.state()
    assert np.array_equal(E0, E1)                                    # Delta E = 0
    J = dense_from_graph(g, 0)
    assert np.array_equal(h1, s1.astype(np.int64) @ J.T)
    top = sorted(range(R), key=lambda r: (E0[r], r))[:n_top]
    changed = [r for r in range(R) if not np.array_equal(s0[r], s1[r])]
    assert set(changed) <= set(top)
    got = 0
    for r in top:
        F = set(np.nonzero(s0[r] != s1[r])[0])
        got += len(F)
        iso = set(np.nonzero(h0[r] == 0)[0])
        assert F <= iso
        for v in F:                                                  # independent
            assert not (set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]]) & F)
        for v in iso - F:                                            # maximal
            assert set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]]) & F
    assert got == tot


# ----------------------------------------------------------------- controller
def make_ctrl(oracle_lib, hist, beta=0.5, delta=0.02, z=10, cooldown=0):
    c = oracle_lib.Ctrl()
    c.beta, c.delta, c.z, c.cooldown, c.enable = beta, delta, z, cooldown, 0
    for i, v in enumerate(hist):
        c.hist[i] = v
    c.hist_len = len(hist)
    return c


def hist_with(distinct_last25, distinct_last40):
    """A non-decreasing 40-value window with the given numbers of distinct
    values in its last 25 and in all 40 entries.  Returns (first 39 values,
    40th value): the step under test appends the 40th."""
    head_levels = distinct_last40 - distinct_last25
    head = [100 + (k * head_levels) // 15 for k in range(15)]
    tail = [200 + (k * distinct_last25) // 25 for k in range(25)]
    full = head + tail
    return full[:-1], full[-1]


def test_controller_branches(oracle_lib):
    s = oracle_lib.default_schedule(augmented=1, beta0=0.1, dbeta=0.02, z_rst=400)
    # strong stagnation: 1 distinct value in both windows
    c = make_ctrl(oracle_lib, [7] * 39)
    ev = oracle_lib.controller_step(c, s, 7)
    assert ev & 4 and c.enable == 1
    assert c.beta == 0.8 * 0.5 + 0.02 and c.delta == 0.02
    # mild: <=3 distinct in the last 25, >5 in the last 40, beta > beta0
    h, last = hist_with(3, 7)
    c = make_ctrl(oracle_lib, h)
    ev = oracle_lib.controller_step(c, s, last)
    assert ev & 8 and c.delta == -0.02 and c.beta == 0.5 - 0.02 and c.enable == 0
    # mild at beta <= beta0: keep cooling (or stop with the literal reading)
    c = make_ctrl(oracle_lib, h, beta=0.1)
    ev = oracle_lib.controller_step(c, s, last)
    assert not (ev & 12) and c.delta == 0.02
    s2 = oracle_lib.default_schedule(augmented=1, beta0=0.1, dbeta=0.02, z_rst=400, literal_break=1)
    c = make_ctrl(oracle_lib, h, beta=0.1)
    oracle_lib.controller_step(c, s2, last)
    assert c.stop == 1
    # progress: 4 distinct values in the last 25
    h, last = hist_with(4, 9)
    c = make_ctrl(oracle_lib, h, delta=-0.02)
    ev = oracle_lib.controller_step(c, s, last)
    assert not (ev & 12) and c.delta == 0.02
    # history too short: nothing but the advance
    c = make_ctrl(oracle_lib, [7] * 30, delta=-0.02)
    ev = oracle_lib.controller_step(c, s, 7)
    assert ev == 0 and c.beta == 0.5 - 0.02 and c.z == 11
    # cooldown freezes the rule
    c = make_ctrl(oracle_lib, [7] * 39, cooldown=3)
    ev = oracle_lib.controller_step(c, s, 7)
    assert ev == 0 and c.cooldown == 2 and c.enable == 0
    # restart at z >= z_rst
    c = make_ctrl(oracle_lib, [7] * 10, z=400, delta=-0.02, cooldown=5)
    ev = oracle_lib.controller_step(c, s, 7)
    assert ev & 16 and c.z == 1 and c.beta == 0.1 and c.delta == 0.02 and c.hist_len == 0 and c.cooldown == 0


def test_hist_with_helper():
    h, last = hist_with(3, 7)
    full = h + [last]
    assert len(full) == 40
    assert len(set(full[-25:])) == 3 and len(set(full)) == 7


# ----------------------------------------------------------------- anneal vs brute force
def brute_max_cut(g):
    J = dense_from_graph(g, 0)
    E, _ = energies_all(J)
    W = sum(int(x) for x in g.w) // 2
    return int((W - E.min()) // 2)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_plain_anneal_reaches_brute_force_optimum(oracle_lib, seed):
    g = synth.random_graph(16, 40, seed)
    opt = brute_max_cut(g)
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 128, seed)
    sched = oracle_lib.default_schedule(beta0=0.1, dbeta=2.9 / 39, steps=40, sweeps=4)
    res = o.anneal(sched)
    assert res.best_cut == opt
    cut, en, spins = o.best()
    J = dense_from_graph(g, 0)
    s = spins.astype(np.int64)
    assert en == -(s @ J @ s) // 2 and cut == (sum(int(x) for x in g.w) // 2 - en) // 2


def test_augmented_anneal_runs_controller_and_cluster(oracle_lib):
    g = synth.torus(4, 4, 2)
    opt = brute_max_cut(g)
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 5)
    sched = oracle_lib.default_schedule(beta0=0.1, dbeta=0.02, steps=300, sweeps=2, augmented=1,
                                        z_rst=150, n_top=4)
    res, tr = o.anneal(sched, trace=True)
    assert res.best_cut == opt
    assert res.n_cluster_moves > 0 and res.n_reheats > 0 and res.n_restarts == 2
    assert np.all(np.diff(tr["mstar"]) >= 0)


def test_stop_at_target(oracle_lib):
    g = synth.random_graph(16, 40, 1)
    opt = brute_max_cut(g)
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 1)
    sched = oracle_lib.default_schedule(beta0=0.1, dbeta=0.1, steps=200, sweeps=2, target=opt, stop_at_target=1)
    res = o.anneal(sched)
    assert res.best_cut == opt and res.steps_run == res.step_reached + 1


def test_complete_graph_max_cut(oracle_lib):
    n = 14
    J = np.ones((n, n), np.int8) - np.eye(n, dtype=np.int8)
    o = oracle_lib.Oracle.dense(J, 64, 3, objective=0)   # w = +1 on K_n
    res = o.anneal(oracle_lib.default_schedule(beta0=0.1, dbeta=0.1, steps=30, sweeps=3))
    assert res.best_cut == (n // 2) * ((n + 1) // 2)


def test_dense_random_couplings(oracle_lib):
    J = oracle_lib.dense_random(300, 42)
    assert np.array_equal(J, J.T) and np.all(np.diag(J) == 0)
    off = J[~np.eye(300, dtype=bool)]
    assert set(np.unique(off)) == {-1, 1} and abs(off.mean()) < 0.02


def test_dense_matches_sparse_on_same_couplings_and_order(oracle_lib):
    # a dense instance sweeps in vertex order; on a complete graph the
    # DSATUR colouring also gives singleton classes in vertex order.
    J = oracle_lib.dense_random(40, 3)
    g = synth.csr_from_dense(J)
    a = oracle_lib.Oracle.dense(J, 64, 11)
    b = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 11, objective=1, shuffle=False)
    for beta in (0.05, 0.2):
        a.sweep(beta, 2)
        b.sweep(beta, 2)
    sa, ha, Ea, _ = a.state()
    sb, hb, Eb, _ = b.state()
    assert np.array_equal(sa, sb) and np.array_equal(Ea, Eb)


# ----------------------------------------------------------------- Max-3-Cut
def brute_max3cut(g):
    best = -1
    edges = [(i, int(g.col[e]), int(g.w[e])) for i in range(g.n)
             for e in range(g.row_ptr[i], g.row_ptr[i + 1]) if g.col[e] > i]
    for lab in itertools.product(range(3), repeat=g.n):
        c = sum(w for i, j, w in edges if lab[i] != lab[j])
        best = max(best, c)
    return best


def test_max3cut_embedding_energy_identity(oracle_lib):
    g = synth.random_graph(7, 12, 5)
    o = oracle_lib.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, 64, 2)
    o.sweep(2.0, 30)
    s, h, E, _ = o.state()
    d = np.array([g.w[g.row_ptr[i]:g.row_ptr[i + 1]].sum() for i in range(g.n)])
    A = d // 3 + 1
    W = int(g.w.sum()) // 2
    checked = 0
    for r in range(o.R):
        sp = s[r] * (1 if s[r, 3 * g.n] > 0 else -1)
        X = (sp[:3 * g.n].reshape(g.n, 3) > 0)
        if np.all(X.sum(1) == 1):
            lab = X.argmax(1)
            cut3 = o.max3cut_value(lab)
            assert E[r] == W - 4 * cut3 - 4 * int(A.sum())            # H = 4f - (4 sum A + 3W)
            checked += 1
    assert checked > 10


@pytest.mark.parametrize("seed", [1, 2])
def test_max3cut_anneal_reaches_brute_force(oracle_lib, seed):
    g = synth.random_graph(7, 13, seed)
    opt = brute_max3cut(g)
    o = oracle_lib.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, 128, seed)
    res = o.anneal(oracle_lib.default_schedule(beta0=0.05, dbeta=0.03, steps=60, sweeps=4))
    _, _, spins = o.best()
    cut, labels = o.max3cut_decode(spins)
    assert cut == opt


def test_max3cut_decode_one_hot_roundtrip(oracle_lib):
    g = synth.random_graph(9, 20, 3)
    o = oracle_lib.Oracle.max3cut(g.n, g.row_ptr, g.col, g.w, 64, 1)
    rng = np.random.default_rng(0)
    for _ in range(20):
        lab = rng.integers(0, 3, g.n)
        sp = -np.ones(3 * g.n + 1, np.int8)
        sp[3 * np.arange(g.n) + lab] = 1
        sp[-1] = 1
        if rng.random() < 0.5:
            sp = -sp                                                 # gauge
        cut, got = o.max3cut_decode(sp)
        assert np.array_equal(got, lab)
        assert cut == sum(int(g.w[e]) for i in range(g.n) for e in range(g.row_ptr[i], g.row_ptr[i + 1])
                          if g.col[e] > i and lab[i] != lab[g.col[e]])


# Normalised pair distance d_H = min(d, 1 - d) (Supplement, Hamming
# distance), pinned on populations whose distances are known by
# construction, with closed-form sums for the means.
def staircase(R, n):
    # replica r: all +1 with its first r spins flipped, so d(a, b) = |a - b| / n
    s = np.ones((R, n), np.int8)
    for r in range(R):
        s[r, :r] = -1
    return s


def test_pair_distance_known_populations(oracle_lib):
    g = synth.random_graph(64, 150, 2)
    # R = 32 < n/2: every pair is closer than 1/2, d_H = |a - b| / 64;
    # sum_{a<b} (b - a) = sum_d d (R - d) = R D(D+1)/2 - D(D+1)(2D+1)/6, D = R-1
    R, n = 32, 64
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 3)
    o.set_population(staircase(R, n))
    D = R - 1
    total = R * D * (D + 1) // 2 - D * (D + 1) * (2 * D + 1) // 6
    assert total == 5456
    assert o.mean_pair_distance() == pytest.approx(total / n / (R * D // 2), abs=1e-15)
    pd = o.pair_distances()
    k = 0
    for a in range(R):
        for b in range(a + 1, R):
            assert pd[k] == (b - a) / n
            k += 1
    # n = 16, R = 16: distances cross 1/2 and fold back, d_H(k) = min(k, 16-k)/16
    g16 = synth.random_graph(16, 30, 4)
    o = oracle_lib.Oracle.sparse(g16.n, g16.row_ptr, g16.col, g16.w, 16, 3)
    o.set_population(staircase(16, 16))
    want = sum((16 - d) * min(d, 16 - d) for d in range(1, 16)) / 16 / (16 * 15 // 2)
    assert want == pytest.approx(4 / 15)  # sum_d (16-d) min(d, 16-d) = 512
    assert o.mean_pair_distance() == pytest.approx(want, abs=1e-15)


def test_pair_distance_global_flip_symmetry(oracle_lib):
    g = synth.random_graph(40, 100, 5)
    rng = np.random.default_rng(2)
    base = rng.choice(np.array([-1, 1], np.int8), size=40)
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 2, 7)
    for k in range(0, 41):
        pop = np.stack([base, base.copy()])
        pop[1, :k] *= -1
        o.set_population(pop)
        assert o.mean_pair_distance() == pytest.approx(min(k, 40 - k) / 40, abs=1e-15)
        o.set_population(np.stack([base, -pop[1]]))          # complement of the partner
        assert o.mean_pair_distance() == pytest.approx(min(k, 40 - k) / 40, abs=1e-15)
    o.set_population(np.stack([base, -base]))                 # a configuration and its flip: same cut
    assert o.mean_pair_distance() == 0.0


def test_diversity_trace_of_independent_random_chains(oracle_lib):
    """At beta = 0 the heat-bath rule flips each spin with probability 1/2,
    so without resampling every sampled population is R independent uniform
    configurations and E[d_H] = E[min(d, n - d)] / n with d ~ Binomial(n, 1/2),
    summed exactly.  Sampled steps follow dh_every, the others hold -1, and
    the steps' average lies within 6 standard errors (pairs of one step are
    correlated, which the bound over steps allows for)."""
    n, R, steps = 200, 64, 40
    g = synth.random_graph(n, 600, 9)
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 21)
    _, tr = o.anneal(oracle_lib.default_schedule(beta0=0.0, dbeta=0.0, steps=steps, sweeps=2, resample=0,
                                                 dh_every=2), trace=True)
    dh = tr["dh"]
    assert np.all(dh[1::2] == -1.0) and np.all(dh[0::2] >= 0)
    want = sum(math.comb(n, d) * min(d, n - d) for d in range(n + 1)) / 2 ** n / n
    assert want == pytest.approx(0.5 - math.sqrt(n / (2 * math.pi)) / n, abs=2e-3)
    got = dh[0::2]
    se = np.std(got, ddof=1) / math.sqrt(len(got))
    assert abs(got.mean() - want) < max(6 * se, 1e-3), (got.mean(), want, se)
    # a sample is the population right after the step's sweeps: one step
    o1 = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 21)
    _, t1 = o1.anneal(oracle_lib.default_schedule(beta0=0.7, dbeta=0.1, steps=1, sweeps=3, dh_every=1),
                      trace=True)
    o2 = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 21)
    o2.sweep(0.7, 3)
    assert t1["dh"][0] == o2.mean_pair_distance()


def test_invalid_inputs_rejected(oracle_lib):
    g = synth.random_graph(20, 40, 1)
    bad = g.col.copy()
    bad[0] = 0 if g.row_ptr[1] > 0 else bad[0]
    with pytest.raises(ValueError):
        oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col[:-1].copy().tolist() + [g.col[-2]], g.w, 64, 1)
    w = g.w.copy()
    w[0] = 5
    with pytest.raises(ValueError):
        oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, w, 64, 1)


# ----------------------------------------------------------------- Potts labels
# Potts Max-K-Cut (Sec. "Max-3-Cut", Eqs. 6-9; Supplement, cascaded sampler).
def graph_edges(g):
    return [(i, int(g.col[e]), int(g.w[e])) for i in range(g.n)
            for e in range(g.row_ptr[i], g.row_ptr[i + 1]) if g.col[e] > i]


def k_cut(edges, lab):
    return sum(w for i, j, w in edges if lab[i] != lab[j])


@pytest.mark.parametrize("K,rule", [(2, 0), (3, 0), (4, 0), (3, 1)])
def test_potts_energy_and_cut_identities(oracle_lib, K, rule):
    # tracked energy = Eq. 6 recomputed from labels, and (W - E)/2 = the
    # weight of the edges whose ends carry different labels
    g = synth.random_graph(40, 90, 3, weights="pm1")
    o = oracle_lib.Oracle.potts(g.n, g.row_ptr, g.col, g.w, K, 64, 11, rule=rule)
    edges = graph_edges(g)
    for beta, k in [(0.0, 1), (0.7, 3), (2.0, 2)]:
        o.sweep(beta, k)
        o.resample(0.05)
        lab, _, E, _ = o.state()
        assert lab.min() >= 0 and lab.max() < K
        for r in range(0, 64, 7):
            assert E[r] == o.potts_energy(r)
            assert (o.W - E[r]) // 2 == k_cut(edges, lab[r])
            assert (o.W - E[r]) % 2 == 0


def test_potts_cascade_samples_the_gibbs_conditional(oracle_lib):
    # the cascade's two p-bits reproduce P(k) = e^{beta syn_k} / sum_m
    # e^{beta syn_m} (the Supplement's claim), checked against that textbook
    # softmax with independent uniform words
    rng = np.random.default_rng(5)
    for syn, beta in [((3, -1, 2), 0.4), ((0, 0, 0), 1.0), ((-5, 4, 4), 0.3), ((7, -7, 0), 0.05)]:
        p = np.exp(beta * np.array(syn, float))
        p /= p.sum()
        N = 60000
        u = rng.integers(0, 2**32, size=(N, 2), dtype=np.uint64).astype(np.uint32)
        cnt = np.zeros(3)
        for i in range(N):
            cnt[oracle_lib.potts_choose(3, 1, 0.0, beta, syn, u[i])] += 1
        emp = cnt / N
        assert np.all(np.abs(emp - p) < 5 * np.sqrt(p * (1 - p) / N) + 1e-9), (syn, emp, p)


def test_potts_softmax_argmax_two_labels_closed_form(oracle_lib):
    # K = 2: label 1 wins iff U0 - U1 > (P0 - P1)/gamma = c, and U0 - U1 has
    # the triangular density on [-1, 1], so P(1) = (1 - c)^2 / 2 for c >= 0
    # and 1 - (1 + c)^2 / 2 for c < 0
    rng = np.random.default_rng(9)
    for syn, beta, gamma in [((2, -1), 0.3, 1.0), ((-1, 3), 0.2, 0.5), ((0, 0), 1.0, 1.0), ((4, 0), 0.1, 2.0)]:
        e = np.exp(beta * np.array(syn, float))
        P = e / e.sum()
        c = (P[0] - P[1]) / gamma
        p1 = (1 - c) ** 2 / 2 if c >= 0 else 1 - (1 + c) ** 2 / 2
        p1 = min(max(p1, 0.0), 1.0)
        N = 40000
        u = rng.integers(0, 2**32, size=(N, 2), dtype=np.uint64).astype(np.uint32)
        ones = sum(oracle_lib.potts_choose(2, 0, gamma, beta, syn, u[i]) for i in range(N))
        assert abs(ones / N - p1) < 5 * math.sqrt(max(p1 * (1 - p1), 1e-6) / N) + 1e-9, (syn, ones / N, p1)
    # gamma = 0: the most probable label, the lowest on ties
    assert oracle_lib.potts_choose(3, 0, 0.0, 1.0, (1, 5, 5), (7, 8, 9)) == 1
    assert oracle_lib.potts_choose(4, 0, 0.0, 1.0, (2, 2, 2, 2), (9, 1, 5, 3)) == 0


def test_potts_cascade_boltzmann_histogram_by_enumeration(oracle_lib):
    # sweeps of the cascade leave P(labels) ~ e^{beta sum_edges J delta}
    # = e^{-(beta/2) E} (E of Eq. 6) invariant: compare the replica histogram
    # with the exact law over all 3^5 labelings
    g = synth.random_graph(5, 7, 4, weights="pm1")
    beta = 0.8
    o = oracle_lib.Oracle.potts(g.n, g.row_ptr, g.col, g.w, 3, 2048, 23, rule=1)
    o.sweep(beta, 30)
    edges = graph_edges(g)
    states = list(itertools.product(range(3), repeat=g.n))
    index = {s: i for i, s in enumerate(states)}
    logw = np.array([beta * sum(-w for i, j, w in edges if s[i] == s[j]) for s in states])
    p_exact = np.exp(logw - logw.max())
    p_exact /= p_exact.sum()
    cnt = np.zeros(len(states))
    for _ in range(60):
        o.sweep(beta, 1)
        lab = o.state()[0]
        for row in lab:
            cnt[index[tuple(int(x) for x in row)]] += 1
    p_emp = cnt / cnt.sum()
    tv = 0.5 * np.abs(p_exact - p_emp).sum()
    assert tv < 0.03, tv


def test_potts_resample_uses_half_delta(oracle_lib):
    # reading: Eq. 8 at beta samples e^{-(beta/2) E}, so Eq. 2's ln Q uses
    # Delta/2 with the Eq. 6 energy
    g = synth.random_graph(20, 40, 2)
    o = oracle_lib.Oracle.potts(g.n, g.row_ptr, g.col, g.w, 3, 256, 3)
    o.sweep(1.0, 2)
    E = o.state()[2].astype(float)
    for delta in (0.1, -0.04):
        a = -0.5 * delta * E
        lnq = a.max() + math.log(np.exp(a - a.max()).sum()) - math.log(len(E))
        got = o.resample(delta)
        assert abs(got - lnq) <= 1e-12 * max(1.0, abs(lnq))
        E = o.state()[2].astype(float)


@pytest.mark.parametrize("rule", [0, 1])
def test_potts_anneal_reaches_brute_force_max3cut(oracle_lib, rule):
    g = synth.random_graph(8, 16, 6)
    best = brute_max3cut(g)
    o = oracle_lib.Oracle.potts(g.n, g.row_ptr, g.col, g.w, 3, 128, 5, rule=rule)
    res = o.anneal(oracle_lib.default_schedule(beta0=0.2, dbeta=0.1, steps=40, sweeps=4))
    assert res.best_cut == best
    cut, _, lab = o.best()
    assert k_cut(graph_edges(g), lab) == best


def test_potts_invalid_inputs(oracle_lib):
    g = synth.random_graph(10, 20, 1)
    for K, rule in [(1, 0), (5, 0), (2, 1), (4, 1), (3, 2)]:
        with pytest.raises(ValueError):
            oracle_lib.Oracle.potts(g.n, g.row_ptr, g.col, g.w, K, 64, 1, rule=rule)
