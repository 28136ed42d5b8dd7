"""Pins the oracle's adaptive temperature ladder (Sec. II.D: the PTDA's
temperatures follow the adaptive scheme of Hukushima et al. -- lowest and
highest fixed, the ones between moved toward equal replica-exchange
acceptance for every adjacent pair).

* Equal acceptances are a fixed point; the ends never move; the ladder stays
  strictly increasing even when a pair accepts nothing.
* On a model where pair p accepts exp(-kappa_p * d_p) (d_p its interval in
  inverse temperature), repeated updates reach the closed-form fixed point
  kappa_p * d_p = const, where every pair accepts alike.
* The full loop (PT runs, measured acceptances, updates) with frozen replicas
  (no DA steps between exchanges, so energies do not depend on temperature):
  a geometric ladder, whose pairs accept anywhere from about 50% to 93%, ends with
  every pair accepting alike within a few percent, and with intervals in 1/T
  nearly equal -- exactly equal would be the answer if every slot saw
  independent energies; the slots at the ends of a chain see slightly more
  extreme ones, so their intervals come out a little narrower.
"""
import numpy as np

from paper_1806_08815_amd import instances


def test_equal_acceptance_is_a_fixed_point(orc):
    temps = np.geomspace(0.5, 9.0, 9)
    out = orc.ladder_update(temps, [400] * 8, 1000)
    assert out[0] == temps[0] and out[-1] == temps[-1]
    np.testing.assert_allclose(out, temps, rtol=1e-13)


def test_ends_fixed_and_order_kept(orc):
    g = np.random.Generator(np.random.PCG64(3))
    for _ in range(200):
        M = int(g.integers(3, 40))
        temps = np.sort(g.uniform(0.1, 50.0, size=M))
        if np.any(np.diff(temps) <= 0):
            continue
        acc = g.integers(0, 1001, size=M - 1)
        acc[g.integers(0, M - 1)] = 0            # a pair that never swapped
        out = orc.ladder_update(temps, acc, 1000)
        assert out[0] == temps[0] and out[-1] == temps[-1]
        assert np.all(np.diff(out) > 0)


def test_more_accepting_pair_gets_wider(orc):
    temps = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    out = orc.ladder_update(temps, [900, 100, 100, 100], 1000)
    d0 = 1 / temps[:-1] - 1 / temps[1:]
    d1 = 1 / out[:-1] - 1 / out[1:]
    assert d1[0] > d0[0] and np.all(d1[1:] < d0[1:])


def test_model_converges_to_closed_form(orc):
    # acceptance exp(-kappa_p d_p): the fixed point has kappa_p d_p equal for all p,
    # i.e. d_p proportional to 1/kappa_p with the span fixed
    M = 12
    g = np.random.Generator(np.random.PCG64(8))
    kappa = g.uniform(2.0, 10.0, size=M - 1)
    temps = np.geomspace(0.4, 4.0, M)
    span = 1 / temps[0] - 1 / temps[-1]
    proposals = 10**12
    for _ in range(80):
        d = 1 / temps[:-1] - 1 / temps[1:]
        acc = np.round(np.exp(-kappa * d) * proposals).astype(np.int64)
        temps = orc.ladder_update(temps, acc, proposals)
    d = 1 / temps[:-1] - 1 / temps[1:]
    want = (1 / kappa) / (1 / kappa).sum() * span
    np.testing.assert_allclose(d, want, rtol=1e-4)
    a = np.exp(-kappa * d)
    assert a.max() / a.min() < 1.0005


def test_frozen_ladder_becomes_linear_in_beta(orc):
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(30, 4))
    temps = np.geomspace(4.0, 60.0, 8)
    d0 = 1 / temps[:-1] - 1 / temps[1:]
    assert d0.max() / d0.min() > 10
    out, acc = orc.pt_adapt(Q, temps, chains=600, iterations=12, rounds=40,
                            steps_per_round=0, seed=3)
    assert out[0] == temps[0] and out[-1] == temps[-1]
    d = 1 / out[:-1] - 1 / out[1:]
    assert d.max() / d.min() < 1.3, d
    # the acceptances of the last iteration are close to equal
    assert acc[-1].max() - acc[-1].min() < 0.05, acc[-1]
    assert acc[0].max() - acc[0].min() > 0.3, acc[0]
