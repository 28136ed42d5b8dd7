"""Pins the oracle's temperature levels and Metropolis threshold tables.

The Metropolis acceptance exp(-dE/T) (Sec. III) is decided in integers: a
16-bit draw u stands for U_u = (u + 1/2)/65536 and the move with offset-
shifted cost d is accepted iff d <= thr_T[u] = ceil(-T ln U_u) - 1, which for
integer d is exactly U_u < exp(-d/T).  These tests check the table against
that definition in 50-digit decimal arithmetic, check the acceptance
probability it induces against exp(-d/T), and check the schedule levels.
"""
from decimal import Decimal, getcontext

import numpy as np
import pytest


def _exact_thr(T, u):
    getcontext().prec = 50
    U = (Decimal(u) + Decimal("0.5")) / Decimal(65536)
    y = -Decimal(repr(T)) * U.ln()
    c = int(y.to_integral_value(rounding="ROUND_CEILING")) - 1
    frac_dist = abs(y - y.to_integral_value(rounding="ROUND_HALF_EVEN"))
    return c, frac_dist, y


@pytest.mark.parametrize("T", [0.05, 0.1, 1.0, 3.0, 40.0, 3277.0, 196608.0])
def test_threshold_definition(orc, T):
    thr = orc.threshold_table(T)
    g = np.random.Generator(np.random.PCG64(int(T * 100)))
    us = list(range(0, 64)) + list(range(65536 - 64, 65536)) + list(
        g.integers(0, 65536, size=600))
    for u in us:
        want, dist, y = _exact_thr(T, int(u))
        if dist < Decimal("1e-9") * (1 + abs(y)):
            assert thr[u] in (want, want + 1, want - 1)
        else:
            assert thr[u] == want, (T, u, thr[u], want)


@pytest.mark.parametrize("T", [0.1, 2.0, 7.5, 1e4])
def test_threshold_shape(orc, T):
    thr = orc.threshold_table(T).astype(np.int64)
    assert np.all(np.diff(thr) <= 0), "non-increasing in u"
    assert thr.min() >= 0, "every non-positive d is accepted at T > 0"
    U = (np.arange(65536) + 0.5) / 65536
    assert np.all(np.abs(thr - (-T * np.log(U))) <= 1.0 + 1e-9)


def test_zero_temperature(orc):
    thr = orc.threshold_table(0.0)
    assert np.all(thr == -1)


@pytest.mark.parametrize("T", [0.5, 3.0, 25.0])
def test_acceptance_probability(orc, T):
    # a(d) = #{u : d <= thr[u]} / 65536 is the count of u with U_u < exp(-d/T),
    # which is within half a draw of exp(-d/T); allow one more for double rounding.
    thr = orc.threshold_table(T).astype(np.int64)
    for d in range(-5, int(12 * T) + 3):
        a = np.count_nonzero(thr >= d) / 65536
        p = min(1.0, float(np.exp(-d / T)))
        assert abs(a - p) <= 1.5 / 65536 + 1e-12, (T, d, a, p)


def test_geometric_levels(orc):
    L = 128
    T = np.array([orc.level_temperature(3.0, 0.05, 0, L, l) for l in range(L)])
    assert T[0] == 3.0
    assert abs(T[-1] - 0.05) < 1e-12
    r = T[1:] / T[:-1]
    assert np.allclose(r, r[0], rtol=1e-12)
    assert orc.level_temperature(3.0, 0.05, 0, 1, 0) == 3.0


def test_linear_beta_levels(orc):
    L = 50
    T = np.array([orc.level_temperature(40.0, 4.0, 1, L, l) for l in range(L)])
    beta = 1.0 / T
    assert np.allclose(np.diff(beta), (1 / 4.0 - 1 / 40.0) / (L - 1), rtol=1e-9)
    assert abs(T[0] - 40.0) < 1e-12 and abs(T[-1] - 4.0) < 1e-12


@pytest.mark.parametrize("L,S", [(128, 10_000), (128, 100), (7, 7), (5, 23), (1, 10)])
def test_level_of_step(orc, L, S):
    lv = np.array([orc.level_of_step(s, L, S) for s in range(S)])
    assert lv[0] == 0
    assert np.all(np.diff(lv) >= 0) and np.all(np.diff(lv) <= L)
    assert lv[-1] == (L - 1 if S >= L else ((S - 1) * L) // S)
    if S >= L:
        counts = np.bincount(lv, minlength=L)
        assert counts.min() >= S // L and counts.max() <= -(-S // L)
