"""Pins of the oracle's Potts label decision against the paper's literal forms.

The oracle (and the library) decide a Potts visit without any division:
  softmax (Eqs. 8-9): the k with the largest omega_k - (gamma U_k) S, where
    omega_k = e^{beta (syn_k - max syn)} and S = sum_m omega_m;
  cascade (Supplement, cascaded p-bits, K = 3): label 0 iff
    omega_0 - s12 > eta_1 (omega_0 + s12), s12 = omega_1 + omega_2, else
    label 1 iff omega_1 - omega_2 > eta_2 s12, else label 2.
The paper writes them as
  softmax: argmax_k [P_k - gamma U_k] with P_k = e^{beta syn_k} / sum_m
    e^{beta syn_m} (lowest k on ties);
  cascade: b = [tanh(Delta) > eta] with Delta_1 = (ln w_0 - ln(w_1 + w_2))/2,
    Delta_2 = (ln w_1 - ln w_2)/2, w_a = e^{beta syn_a}; label 0 if b_1, else
    1 if b_2, else 2 (a zero argument of sgn counts as b = 0).
Both sides are equal in exact arithmetic (multiplying by a positive
denominator keeps an order; tanh(ln(a/b)/2) = (a - b)/(a + b)), but the
oracle evaluates its form in binary64.  Here the literal forms are evaluated
in mpmath at 50 digits on random and on adversarial near-tie inputs, and
every disagreement must lie inside the rounding band derived below.

Rounding band.  omega_k carries at most ~2 ulp of relative error from the
exponential and one more from the product beta (syn_k - m) times its size
|beta (syn_k - m)| (the exponent is off by that many ulp in absolute terms);
S and s12 add at most K ulp; the final products and differences add a few
more.  With A = 1 + max_k |beta (syn_k - m)| and eps = 2^-53, the binary64
score differences are within 32 A (1 + gamma) eps of the exact ones
(normalised by S), so a decision can differ only where the exact margin is
below that.  The inputs' own grids are far coarser: U_k and eta step by
2^-32 and 2^-31, so random inputs put no exact margin that close.
"""
import math
import multiprocessing as mp_pool

import mpmath
import numpy as np
import pytest

EPS = 2.0 ** -53
N_CASES = 100_000  # per decision form


def band(beta, syn, gamma):
    m = max(syn)
    A = 1.0 + max(abs(beta * (s - m)) for s in syn)
    return 32.0 * A * (1.0 + gamma) * EPS


def literal_softmax(K, beta, gamma, syn, u):
    """Eqs. 8-9 at 50 digits: (decision, exact margin between the winner and
    the runner-up, in units of probability)."""
    mpmath.mp.dps = 50
    b = mpmath.mpf(beta)
    w = [mpmath.exp(b * s) for s in syn]
    S = mpmath.fsum(w)
    sc = [w[k] / S - mpmath.mpf(gamma) * (mpmath.mpf(int(u[k])) / 2 ** 32) for k in range(K)]
    best = 0
    for k in range(1, K):
        if sc[k] > sc[best]:
            best = k
    others = [sc[k] for k in range(K) if k != best]
    return best, float(sc[best] - max(others))


def literal_cascade(beta, syn, u):
    """The Supplement's two p-bits at 50 digits: (decision, exact margin of
    the p-bit that decided it)."""
    mpmath.mp.dps = 50
    b = mpmath.mpf(beta)
    w = [mpmath.exp(b * s) for s in syn]
    d1 = (mpmath.log(w[0]) - mpmath.log(w[1] + w[2])) / 2
    eta1 = mpmath.mpf(int(u[0])) / 2 ** 31 - 1
    m1 = mpmath.tanh(d1) - eta1
    if m1 > 0:
        return 0, float(m1)
    d2 = (mpmath.log(w[1]) - mpmath.log(w[2])) / 2
    eta2 = mpmath.mpf(int(u[1])) / 2 ** 31 - 1
    m2 = mpmath.tanh(d2) - eta2
    return (1 if m2 > 0 else 2), float(min(abs(m1), abs(m2)))


def make_cases(form, n, seed):
    """Random (syn, beta, gamma, u) plus a tenth of adversarial cases whose
    words sit on the grid point nearest an exact tie, and exact ties."""
    rng = np.random.default_rng(seed)
    K = 3 if form == "cascade" else int(form[-1])
    cases = []
    for i in range(n):
        spread = rng.choice([2, 10, 60, 400])
        syn = [int(x) for x in rng.integers(-spread, spread + 1, size=K)]
        beta = float(10 ** rng.uniform(-3, 0.7))
        gamma = 0.0 if form == "cascade" else float(rng.choice([0.0, 0.25, 1.0, rng.uniform(0, 3)]))
        u = [int(x) for x in rng.integers(0, 2 ** 32, size=K, dtype=np.uint64)]
        kind = i % 10
        if kind == 0:  # near tie on the words' grid
            P = np.exp(beta * (np.array(syn, float) - max(syn)))
            P /= P.sum()
            if form == "cascade":
                t1 = (P[0] - P[1] - P[2]) / (P[0] + P[1] + P[2])
                u[0] = int(min(2 ** 32 - 1, max(0, round((t1 + 1) * 2 ** 31))))
                if P[1] + P[2] > 0:
                    t2 = (P[1] - P[2]) / (P[1] + P[2])
                    u[1] = int(min(2 ** 32 - 1, max(0, round((t2 + 1) * 2 ** 31))))
            elif gamma > 0:
                j = int(rng.integers(1, K))
                tgt = u[0] / 2 ** 32 + (P[j] - P[0]) / gamma
                u[j] = int(min(2 ** 32 - 1, max(0, round(tgt * 2 ** 32))))
        elif kind == 1:  # exact ties of the fields (and of the words)
            syn[1] = syn[0]
            if form != "cascade":
                u[1] = u[0]
            else:
                syn[2] = syn[1]
                u[1] = 2 ** 31  # eta_2 = 0 = tanh(Delta_2)
        cases.append((syn, beta, gamma, u))
    return K, cases


def _check_chunk(args):
    form, K, cases = args
    import oracle
    rule = 1 if form == "cascade" else 0
    bad, margins = [], []
    for syn, beta, gamma, u in cases:
        got = oracle.potts_choose(K, rule, gamma, beta, syn, u)
        if form == "cascade":
            want, margin = literal_cascade(beta, syn, u)
        else:
            want, margin = literal_softmax(K, beta, gamma, syn, u)
        margins.append(abs(margin))
        if got != want:
            bad.append((syn, beta, gamma, u, got, want, margin, band(beta, syn, gamma)))
    return bad, min(margins)


@pytest.mark.parametrize("form", ["softmax2", "softmax3", "softmax4", "cascade"])
def test_division_free_decision_equals_literal_form(oracle_lib, form):
    K, cases = make_cases(form, N_CASES, {"softmax2": 1, "softmax3": 2, "softmax4": 3, "cascade": 4}[form])
    chunks = [(form, K, cases[i::8]) for i in range(8)]
    with mp_pool.get_context("fork").Pool(8) as pool:
        out = pool.map(_check_chunk, chunks)
    bad = [b for o in out for b in o[0]]
    smallest = min(o[1] for o in out)
    # every disagreement is an exact near-tie inside the rounding band
    for syn, beta, gamma, u, got, want, margin, bnd in bad:
        assert abs(margin) <= bnd, (form, syn, beta, gamma, u, got, want, margin, bnd)
    # the adversarial cases do reach the words' grid (margins of order 2^-32)
    assert smallest < 1e-8, smallest
    print(f"{form}: {len(cases)} cases, {len(bad)} disagreements (all within the band), "
          f"smallest exact margin {smallest:.3g}")


def test_tie_conventions(oracle_lib):
    # softmax: equal scores go to the lowest label (Eq. 9 with a fixed
    # order); cascade: tanh(Delta) = eta gives b = 0 (R19)
    assert oracle_lib.potts_choose(3, 0, 1.0, 0.7, (4, 4, 4), (5, 5, 5)) == 0
    assert oracle_lib.potts_choose(4, 0, 0.5, 0.2, (-3, 1, 1, 0), (9, 7, 7, 2)) == 1
    # Delta_2 = 0 and eta_2 = 0: b_2 = 0 -> label 2 (when b_1 = 0)
    assert oracle_lib.potts_choose(3, 1, 0.0, 1.0, (-50, 2, 2), (2 ** 32 - 1, 2 ** 31)) == 2
    # Delta_1 = 0 exactly is impossible with integer fields unless omega_0 =
    # omega_1 + omega_2; at beta = 0 it is tanh(-ln 2 / 2) = -1/3
    u1 = int(round((-1.0 / 3 + 1) * 2 ** 31))
    for du in (-2, -1, 1, 2):
        eta = (u1 + du) / 2 ** 31 - 1
        want = 0 if -1.0 / 3 > eta else None
        got = oracle_lib.potts_choose(3, 1, 0.0, 0.0, (0, 0, 0), (u1 + du, 0))
        assert (got == 0) == (want == 0), (du, got)


def softmax_law_k3(P, gamma):
    """Probability that label k wins argmax_k [P_k - gamma U_k] with
    independent U_k ~ U(0,1): integrate over U_k the chance that every other
    score is lower, prod_{j != k} Pr[U_j > U_k + (P_j - P_k)/gamma]."""
    out = []
    for k in range(3):
        def f(x, k=k):
            v = mpmath.mpf(1)
            for j in range(3):
                if j != k:
                    v *= min(mpmath.mpf(1), max(mpmath.mpf(0), 1 - x - (P[j] - P[k]) / gamma))
            return v
        # breakpoints where a factor changes form
        pts = sorted({0.0, 1.0} | {float(c) for j in range(3) if j != k
                                   for c in (-(P[j] - P[k]) / gamma, 1 - (P[j] - P[k]) / gamma)
                                   if 0.0 < c < 1.0})
        out.append(float(mpmath.quad(f, pts)))
    return np.array(out)


def test_softmax_k3_law_by_numerical_integration(oracle_lib):
    # the K = 3 softmax-perturbed argmax picks label k with the probability
    # fixed by Eqs. 8-9 and independent uniform noise; compare the oracle's
    # frequencies over random words with that law
    mpmath.mp.dps = 30
    rng = np.random.default_rng(17)
    for syn, beta, gamma in [((3, -1, 2), 0.4, 1.0), ((0, 0, 0), 1.0, 0.3), ((-5, 4, 1), 0.2, 0.5),
                             ((7, 0, -7), 0.05, 2.0), ((2, 2, -1), 0.9, 0.15)]:
        w = np.exp(beta * (np.array(syn, float) - max(syn)))
        P = w / w.sum()
        law = softmax_law_k3(P, gamma)
        assert abs(law.sum() - 1.0) < 1e-9, law
        N = 60000
        u = rng.integers(0, 2 ** 32, size=(N, 3), dtype=np.uint64).astype(np.uint32)
        cnt = np.zeros(3)
        for i in range(N):
            cnt[oracle_lib.potts_choose(3, 0, gamma, beta, syn, u[i])] += 1
        emp = cnt / N
        sig = np.sqrt(np.maximum(law * (1 - law), 1e-8) / N)
        assert np.all(np.abs(emp - law) < 5 * sig + 1e-9), (syn, beta, gamma, emp, law)
