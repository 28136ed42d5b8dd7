"""Pins the oracle's stochastic semantics against exact probabilities.

For a tiny instance the one-step law of the parallel-trial scheme (Sec. II.B,
Sec. III) is computable exactly: each variable i is accepted independently
with probability a_i (the fraction of 16-bit draws whose threshold admits its
cost d_i), and one accepted variable is then chosen uniformly.  So

  P(no flip) = prod_i (1 - a_i)                       (Eq. (2): 1 - P_p)
  P(flip k)  = sum_{A contains k} (1/|A|) prod_{i in A} a_i prod_{i not in A} (1 - a_i).

The oracle's empirical frequencies over many independent steps (different step
indices give independent draws) must match these within chi-square bounds.
"""
import numpy as np
import pytest

from paper_1806_08815_amd import instances


def _exact_law(a):
    N = len(a)
    p_flip = np.zeros(N)
    p_none = float(np.prod(1 - a))
    for mask in range(1, 2**N):
        A = [i for i in range(N) if mask >> i & 1]
        w = 1.0
        for i in range(N):
            w *= a[i] if (mask >> i & 1) else (1 - a[i])
        for k in A:
            p_flip[k] += w / len(A)
    return p_none, p_flip


@pytest.mark.parametrize("N,T,seed", [(5, 6.0, 1), (4, 2.5, 2), (6, 20.0, 3)])
def test_one_step_law(orc, N, T, seed):
    Q = instances.random_qubo(N, seed=seed, lo=-12, hi=12)
    thr = orc.threshold_table(T)
    r0 = 3
    probe = orc.Replica(Q, init=1, seed=seed, r=r0).read()
    x, h = probe["x"], probe["h"]
    d = (1 - 2 * x.astype(np.int64)) * h
    a = np.array([np.count_nonzero(thr.astype(np.int64) >= di) / 65536 for di in d])
    p_none, p_flip = _exact_law(a)
    assert abs(p_none + p_flip.sum() - 1.0) < 1e-12
    trials = 60_000
    counts = np.zeros(N + 1, dtype=np.int64)
    for s in range(trials):
        rep = orc.Replica(Q, init=1, seed=seed, r=r0)
        k = rep.step(thr, s, eoff_inc=0)
        counts[N if k < 0 else k] += 1
    expect = np.concatenate([p_flip, [p_none]]) * trials
    keep = expect > 5
    chi2 = float(((counts[keep] - expect[keep]) ** 2 / expect[keep]).sum())
    dof = int(keep.sum()) - 1
    # 99.99th percentile of chi-square is below dof + 8.5 sqrt(2 dof) for these dof
    assert chi2 < dof + 8.5 * np.sqrt(2 * dof), (chi2, dof, counts, expect)
    assert np.all(counts[~keep] <= 20)


def test_parallel_trial_boost_low_temperature(orc):
    # Eq. (3): at low T the parallel-trial acceptance is ~ the sum of the single
    # acceptances, i.e. ~ N times the single-trial acceptance of Eq. (1).
    N = 8
    Q = instances.random_qubo(N, seed=7, lo=1, hi=9)  # all flips from 0 cost > 0
    thr = orc.threshold_table(0.7)
    probe = orc.Replica(Q, init=0, seed=1, r=0).read()
    d = probe["h"].astype(np.int64)
    a = np.array([np.count_nonzero(thr.astype(np.int64) >= di) / 65536 for di in d])
    p_single = a.mean()
    p_parallel = 1 - np.prod(1 - a)
    assert p_parallel == pytest.approx(a.sum(), rel=0.05)
    assert p_parallel / p_single == pytest.approx(N, rel=0.05)
    trials = 40_000
    hits = 0
    for s in range(trials):
        rep = orc.Replica(Q, init=0, seed=1, r=0)
        hits += rep.step(thr, s) >= 0
    sd = np.sqrt(trials * p_parallel * (1 - p_parallel))
    assert abs(hits - trials * p_parallel) < 5 * sd


def test_uniform_choice_among_accepted(orc):
    # At very high T every flip is accepted, so the choice must be uniform on all N.
    N = 16
    Q = instances.random_qubo(N, seed=8, lo=-3, hi=3)
    thr = orc.threshold_table(1e8)
    assert thr.min() >= 3 + 6 * N  # above any |d| = |h| this instance can reach
    trials = 32_000
    counts = np.zeros(N, dtype=np.int64)
    rep = orc.Replica(Q, init=0, seed=4, r=1)
    for s in range(trials):
        k = rep.step(thr, s)
        counts[k] += 1
    exp = trials / N
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 15 + 8.5 * np.sqrt(30)


def test_selection_order_is_ascending(orc):
    # With every flip accepted, j = floor(v m / 2^32) selects index j itself.
    N = 10
    Q = np.zeros((N, N), dtype=np.int32)
    thr = orc.threshold_table(1e3)
    for s in range(200):
        rep = orc.Replica(Q, init=0, seed=12, r=5)
        k = rep.step(thr, s)
        v = orc.select_draw(12, 5, s)
        assert k == (v * N) >> 32
