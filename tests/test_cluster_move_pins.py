"""Brute-force pins of the oracle's non-local cluster move (Algorithm 1; Sec.
"Augmented PAMC", iso-cluster move).

For every target replica the move is recomputed here from scratch, in plain
Python: the target set (the n_top lowest (E, slot)), the iso-sites (local
field 0), each trial's priority keys drawn from the Philox4x32-10 reference
(itself pinned to rocRAND's engine), the greedy independent set in key order,
and the choice among trials: the largest set, the earliest trial on a tie.
Independence and maximality are also checked over every subset of the
iso-sites.  Cases are searched until trials of different sizes and ties
between different sets of equal size have both been exercised, so an oracle
that kept the last, the smallest or the first trial would fail.
"""
import itertools

import numpy as np

import synth

TAG_CL = 3


def internal_graph(g, to_internal):
    n = g.n
    to_input = np.empty(n, np.int64)
    to_input[to_internal] = np.arange(n)
    nbr = []
    for iv in range(n):
        v = to_input[iv]
        nbr.append(sorted(int(to_internal[g.col[e]]) for e in range(g.row_ptr[v], g.row_ptr[v + 1])))
    return nbr


def greedy(order, nbr):
    taken = set()
    for v in order:
        if not any(u in taken for u in nbr[v]):
            taken.add(v)
    return taken


def expected_move(oracle_lib, seed, g_cl, r, iso, nbr, trials):
    key = (seed & 0xFFFFFFFF, seed >> 32)
    sets = []
    for t in range(trials):
        keyed = sorted((int(oracle_lib.philox((v, g_cl, r, TAG_CL | (t << 8)), key)[0]), v) for v in iso)
        sets.append(greedy([v for _, v in keyed], nbr))
    sizes = [len(s) for s in sets]
    best = sizes.index(max(sizes))  # earliest on ties
    return sets, best


def check_subsets(S, iso, nbr):
    # independent, and no iso-site outside can be added (maximal)
    for v in S:
        assert not (set(nbr[v]) & S)
    for v in set(iso) - S:
        assert set(nbr[v]) & S
    if len(iso) <= 12:  # every independent superset of S within iso is S itself
        for k in range(1, len(iso) + 1):
            for sub in itertools.combinations(sorted(iso), k):
                T = set(sub)
                if S < T:
                    assert any(set(nbr[v]) & T for v in T)


def test_cluster_move_is_largest_greedy_trial_earliest_on_ties(oracle_lib):
    seen_size_diff = seen_tie_diff_sets = seen_not_first = 0
    small_iso_targets = 0
    for gseed in range(1, 40):
        g = synth.torus(4, 4, gseed)  # n = 16, degree 4, +-1 weights: fields in {0, +-2, +-4}
        R, trials, n_top = 64, 6, 16
        o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, R, 100 + gseed)
        o.sweep(0.3 + 0.05 * gseed, 3)
        nbr = internal_graph(g, o.internal_ids())
        to_int = o.internal_ids()
        s0, h0, E0, _ = [x.copy() for x in o.state()]
        g_cl = int(o.counters()[2])
        targets = sorted(range(R), key=lambda r: (int(E0[r]), r))[:n_top]
        tot, sizes = o.cluster(n_top, trials)
        s1, h1, E1, _ = o.state()
        assert np.array_equal(E0, E1)
        want_total = 0
        for i, r in enumerate(targets):
            iso = [int(to_int[v]) for v in range(g.n) if h0[r, v] == 0]
            sets, best = expected_move(oracle_lib, 100 + gseed, g_cl, r, iso, nbr, trials)
            S = sets[best]
            flipped = {int(to_int[v]) for v in np.nonzero(s0[r] != s1[r])[0]}
            assert flipped == S, (gseed, r, sorted(flipped), [sorted(x) for x in sets])
            assert sizes[i] == len(S)
            check_subsets(S, iso, nbr)
            want_total += len(S)
            small_iso_targets += len(iso) <= 7
            szs = [len(x) for x in sets]
            seen_size_diff += len(set(szs)) > 1
            seen_not_first += best > 0
            top = [x for x in sets if len(x) == len(S)]
            seen_tie_diff_sets += any(x != S for x in top)
        assert tot == want_total
        # replicas that are not targets are untouched
        others = [r for r in range(R) if r not in set(targets)]
        assert np.array_equal(s0[others], s1[others])
        if seen_size_diff >= 5 and seen_tie_diff_sets >= 5 and seen_not_first >= 5 and small_iso_targets >= 20:
            break
    assert seen_size_diff >= 5, seen_size_diff
    assert seen_not_first >= 5, seen_not_first
    assert seen_tie_diff_sets >= 5, seen_tie_diff_sets
    assert small_iso_targets >= 20, small_iso_targets


def test_cluster_move_single_iso_site(oracle_lib):
    # on the path 0 - 1 - 2 with couplings (+1, -1) only vertex 1 can have a
    # zero field (when s0 = s2), so every target flips exactly its iso-sites
    g = synth.csr_from_edges(3, np.array([0, 1]), np.array([1, 2]), np.array([1, -1], np.int32))
    o = oracle_lib.Oracle.sparse(g.n, g.row_ptr, g.col, g.w, 64, 9)
    s, h, E, _ = o.state()
    tot, sizes = o.cluster(64, 4)
    s1, _, E1, _ = o.state()
    assert np.array_equal(E, E1)
    for r in range(64):
        iso = [v for v in range(3) if h[r, v] == 0]
        assert iso in ([], [1])
        assert (s1[r] != s[r]).sum() == len(iso)
    assert tot == sum(int((h[r] == 0).sum()) for r in range(64))
