"""Pins the oracle's parallel-tempering variant (Sec. II.D; exchange move of
Algorithm 3).

* With one temperature, PT is exactly a constant-temperature DA run from the
  random start (the DA steps inside PT are the same steps).
* With no DA steps between exchanges, the states are frozen and the exchange
  move alone must satisfy detailed balance: for two replicas of energies
  E_lo < E_hi at inverse temperatures beta_cold > beta_hot, the long-run
  fraction of rounds with the low-energy replica in the cold slot is
  1 / (1 + exp(-(beta_cold - beta_hot)(E_hi - E_lo))).
* Nearly equal temperatures accept (almost) every exchange.
* The slot assignment stays a permutation and reported energies are exact.
"""
import numpy as np
import pytest

from paper_1806_08815_amd import instances


def test_single_temperature_is_plain_da(orc):
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(40, 3))
    T = 6.0
    pt = orc.pt(Q, [T], chains=3, rounds=7, steps_per_round=50, eoff_inc=2, seed=9)
    da = orc.anneal(Q, T_hi=T, T_lo=T, n_levels=1, eoff_inc=2, init=1, replicas=3,
                    steps=350, seed=9)
    for key in ("best_x", "best_E", "final_x", "final_E", "n_accept"):
        np.testing.assert_array_equal(pt[key], da[key])


def _frozen_pair_fraction(orc, Q, temps, rounds, seed):
    # K = 0: energies never change; follow which replica is cold after each round
    # by running the exchange sweep for 1..rounds rounds and reading slots.
    # (Each call replays the same counter-based draws, so round t's decision is
    # the same in every call.)
    cold_low = 0
    out0 = orc.pt(Q, temps, chains=1, rounds=0, steps_per_round=0, seed=seed)
    E = out0["final_E"]
    low = int(np.argmin(E))
    for t in range(1, rounds + 1):
        out = orc.pt(Q, temps, chains=1, rounds=t, steps_per_round=0, seed=seed)
        cold_low += int(out["slot"][low] == 0)
    return cold_low / rounds, E


def test_exchange_detailed_balance(orc):
    N = 30
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(N, 5))
    temps = [4.0, 9.0]
    frac, E = _frozen_pair_fraction(orc, Q, temps, rounds=2500, seed=21)
    assert E[0] != E[1]
    dbeta = 1 / temps[0] - 1 / temps[1]
    want = 1.0 / (1.0 + np.exp(-dbeta * abs(int(E[0]) - int(E[1]))))
    # successive rounds are correlated (a 2-state Markov chain); allow 6 sigma of
    # an effective sample a few times smaller than the round count
    sd = np.sqrt(want * (1 - want) / 500)
    assert abs(frac - want) < 6 * sd, (frac, want)


def test_close_temperatures_always_swap(orc):
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(24, 6))
    temps = [5.0, 5.0 * (1 + 1e-13), 5.0 * (1 + 2e-13)]
    out = orc.pt(Q, temps, chains=2, rounds=40, steps_per_round=10, seed=3)
    # |dbeta * dE| < 1e-9 << -ln U_max ~ 7.6e-6, so every proposal is accepted
    assert np.all(out["n_swaps"] == 40 * 2)


def test_pt_outputs_consistent(orc):
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(48, 7))
    temps = np.geomspace(2.0, 30.0, 6)
    out = orc.pt(Q, temps, chains=3, rounds=12, steps_per_round=64, eoff_inc=0, seed=4)
    for c in range(3):
        slots = sorted(out["slot"][c * 6:(c + 1) * 6])
        assert slots == list(range(6))
    for q in range(18):
        assert orc.energy(Q, out["final_x"][q]) == out["final_E"][q]
        assert orc.energy(Q, out["best_x"][q]) == out["best_E"][q]
        assert out["best_E"][q] <= out["final_E"][q]
    assert out["n_swaps"].sum() > 0


def test_pt_rejects_bad_ladders(orc):
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(8, 1))
    with pytest.raises(ValueError):
        orc.pt(Q, [3.0, 2.0], chains=1, rounds=1, steps_per_round=1)
    with pytest.raises(ValueError):
        orc.pt(Q, [0.0, 2.0], chains=1, rounds=1, steps_per_round=1)
