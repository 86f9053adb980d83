"""The dense pass decides a visit by comparing its field x with a critical
field computed from the visit's uniform word u instead of reading the
threshold table.  These checks pin that reformulation on the CPU against the
oracle's own thresholds (Eq. 4 and the Metropolis rule): the table is
non-increasing in x, saturated beyond its half-width, and x < c(u) -- with
the sentinels for words that flip at every or no field and the Metropolis
floor -- gives the oracle's decision for every field, inside the table and
beyond it."""
import math

import numpy as np
import pytest

import oracle

INF = 1 << 30
U32 = 0xFFFFFFFF


def half_width(beta, X):
    # the table half-width: thresholds are saturated beyond ceil(12.5 / beta) + 1
    if beta < 1e-300:
        return min(X, 1)
    return min(X, int(math.ceil(12.5 / beta)) + 1)


def decide(beta, rule, x, u):
    """The oracle's decision for field x (any size) and word u."""
    return u < oracle.threshold(beta, rule, x) or (rule == 1 and x <= 0)


def critical(T, Xl, rule, u):
    """c(u) - Xl with the sentinels, as the critical-field kernel stores it."""
    c = int(np.count_nonzero(T > u))  # T is non-increasing: a prefix exceeds u
    v = -INF if c == 0 else INF if c == len(T) else c - Xl
    return max(v, 1) if rule == 1 else v


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("beta,X", [(0.0, 40), (1e-4, 3000), (0.02, 3000), (0.3, 500), (2.5, 60)])
def test_critical_field_matches_threshold_test(rule, beta, X):
    Xt = half_width(beta, X)
    Xl = min(Xt, 2047)
    T = np.array([oracle.threshold(beta, rule, x) for x in range(-Xl, Xl + 1)], dtype=np.uint64)
    assert np.all(T[:-1] >= T[1:]), "table not monotone"
    # saturation beyond the half-width (what lets fields outside it clamp)
    if Xt < X:
        for x in (Xt + 1, Xt + 7, X):
            assert oracle.threshold(beta, rule, x) == oracle.threshold(beta, rule, Xt)
            assert oracle.threshold(beta, rule, -x) == oracle.threshold(beta, rule, -Xt)
    rng = np.random.default_rng(int(beta * 1e6) + 7 * rule + X)
    words = [0, 1, U32 - 1, U32, 1 << 31, (1 << 31) - 1]
    words += [int(t) + d for t in T[:: max(1, len(T) // 40)] for d in (-1, 0, 1) if 0 <= int(t) + d <= U32]
    words += [int(w) for w in rng.integers(0, 1 << 32, size=200, dtype=np.uint64)]
    # fields inside the LDS table, and (when it is the full table) beyond it
    xs = list(range(-Xl, Xl + 1, max(1, Xl // 50))) + [-Xl, Xl, 0, 1, -1]
    if Xl == Xt:
        xs += [Xl + 1, Xl + 5, -Xl - 1, -Xl - 5, 4 * X + 3, -4 * X - 3]
    for u in words:
        cc = critical(T, Xl, rule, u)
        for x in xs:
            assert (x < cc) == decide(beta, rule, x, u), (beta, rule, u, x, cc)


def test_sign_mask_form():
    """The pass tests x = s h through y = h ^ m (m = 0 for s = +1, -1 for
    s = -1): x < cc is y < cc + m."""
    rng = np.random.default_rng(3)
    for h, cc in rng.integers(-5000, 5000, size=(2000, 2)):
        h, cc = int(h), int(cc)
        for s, m in ((1, 0), (-1, -1)):
            assert ((s * h) < cc) == ((h ^ m) < cc + m)
