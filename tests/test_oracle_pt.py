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


# --- the exchange sweep over a ladder of M >= 3 rungs -------------------------
#
# With K = 0 the replicas' energies are frozen at their random starts, and the
# rounds form a Markov chain over the M! assignments of replicas to slots.
# Every pair move of the sweep is a Metropolis swap at (1/T_p - 1/T_{p+1}), so
# the whole sweep leaves the Boltzmann weights
#     P(pi) ~ exp(-sum_p E_{pi(p)} / T_p)     (pi(p): replica in slot p)
# invariant (Sec. II.D; the exchange move of Algorithm 3).  The long-run
# frequencies of the M! assignments must therefore match P, which a sweep that
# decided pair p on the slots held before the earlier swaps of the same sweep
# does not do (checked below with such a sweep written here).

def _perm_counts(slot_trace, M, burn, thin):
    from itertools import permutations
    index = {pm: q for q, pm in enumerate(permutations(range(M)))}
    counts = np.zeros(len(index))
    for slots in slot_trace[burn::thin]:
        # slots[replica] = slot -> replica in each slot
        ris = [0] * M
        for r, p in enumerate(slots):
            ris[p] = r
        counts[index[tuple(ris)]] += 1
    return counts, list(index)


def _boltzmann(E, temps, perms):
    logw = np.array([-sum(E[pm[p]] / temps[p] for p in range(len(temps))) for pm in perms])
    w = np.exp(logw - logw.max())
    return w / w.sum()


def _ladder_for(E, M):
    """Temperatures that make every adjacent exchange a coin flip of moderate
    bias for these frozen energies (so the chain mixes in a few rounds)."""
    spread = max(1.0, float(np.std(E)))
    step = (1.2 if M == 3 else 0.9) / ((M - 1) * spread)
    betas = 0.02 + np.arange(M)[::-1] * step
    return 1.0 / betas


def _chi2_pvalue(counts, probs):
    from scipy import stats
    exp = counts.sum() * probs
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    return stats.chi2.sf(chi2, len(counts) - 1)


@pytest.mark.parametrize("M,N,inst", [(3, 20, 11), (4, 16, 12)])
def test_exchange_sweep_boltzmann_multirung(orc, M, N, inst):
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(N, inst))
    start = orc.pt(Q, [1.0 + p for p in range(M)], chains=1, rounds=0, steps_per_round=0,
                   seed=5)
    E = start["final_E"].astype(np.float64)
    assert len(set(E.tolist())) == M, "frozen energies must differ"
    temps = _ladder_for(E, M)
    rounds = 40_000 if M == 3 else 120_000
    out = orc.pt(Q, temps, chains=1, rounds=rounds, steps_per_round=0, seed=5, slot_trace=True)
    counts, perms = _perm_counts(out["slot_trace"][0], M, burn=100, thin=10)
    probs = _boltzmann(E, temps, perms)
    assert probs.min() > 0.005, probs   # every assignment is visited often
    p = _chi2_pvalue(counts, probs)
    assert p > 1e-4, (p, counts, counts.sum() * probs)
    # the frozen energies are the random starts, untouched by the sweeps
    np.testing.assert_array_equal(out["final_E"], start["final_E"])


def test_stale_slot_sweep_fails_the_boltzmann_check(orc):
    # The same check applied to a sweep that decides pair p on the slots held
    # at the start of the sweep (a stale read) rejects it: the pin has power.
    M, N = 3, 20
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(N, 11))
    E = orc.pt(Q, [1.0, 2.0, 3.0], chains=1, rounds=0, steps_per_round=0,
               seed=5)["final_E"].astype(np.float64)
    temps = _ladder_for(E, M)
    lnU = np.log((np.arange(65536) + 0.5) / 65536.0)
    ris = list(range(M))
    trace = []
    for t in range(40_000):
        held = list(ris)
        for p in range(M - 1):
            a, b = held[p], held[p + 1]
            delta = (1.0 / temps[p] - 1.0 / temps[p + 1]) * (E[a] - E[b])
            if lnU[orc.exchange_draw(5, 0, t, p)] < delta:
                ris[p], ris[p + 1] = ris[p + 1], ris[p]
        slots = [0] * M
        for p, r in enumerate(ris):
            slots[r] = p
        trace.append(slots)
    counts, perms = _perm_counts(np.array(trace), M, burn=100, thin=10)
    assert _chi2_pvalue(counts, _boltzmann(E, temps, perms)) < 1e-6


def test_pair_swaps_add_up(orc):
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(32, 8))
    temps = np.geomspace(2.0, 20.0, 5)
    out = orc.pt(Q, temps, chains=3, rounds=30, steps_per_round=16, seed=2)
    assert out["pair_swaps"].shape == (3, 4)
    np.testing.assert_array_equal(out["pair_swaps"].sum(axis=1), out["n_swaps"])


def test_chain_base_selects_chains(orc):
    # chains are independent: chain c run alone equals chain c of a larger run
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(24, 9))
    temps = np.geomspace(1.5, 12.0, 4)
    full = orc.pt(Q, temps, chains=3, rounds=6, steps_per_round=20, eoff_inc=1, seed=7)
    one = orc.pt(Q, temps, chains=1, rounds=6, steps_per_round=20, eoff_inc=1, seed=7,
                 chain_base=2)
    for k in ("best_x", "best_E", "final_x", "final_E", "n_accept", "slot"):
        np.testing.assert_array_equal(one[k], full[k][8:12])
    np.testing.assert_array_equal(one["n_swaps"], full["n_swaps"][2:])
