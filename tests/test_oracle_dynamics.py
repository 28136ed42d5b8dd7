"""Pins the oracle's DA dynamics (Algorithm 2, Sec. II.B) against facts that do
not depend on the oracle itself.

* The incremental state is exact: at every step h == b + W x and E == E(x),
  recomputed from scratch by numpy on the raw Q.
* The escape offset follows Algorithm 2: reset to 0 when a flip is applied,
  raised by the increment (saturating at 2^30) when none is accepted.
* best_E is the minimum energy along the trajectory, and best_x attains it.
* Replicas are independent and replayable: a replica run alone equals the same
  replica inside a batch (counter-based random numbers).
* A zero-temperature run ends in a one-flip local minimum.
* Long runs reach the exact optimum found by brute-force enumeration, which is
  itself checked against numpy enumeration; planted (Mattis) instances reach
  their known ground-state energy.
"""
import numpy as np
import pytest

from paper_1806_08815_amd import instances

EOFF_MAX = 2**30


def _np_state(Q, x):
    Q = Q.astype(np.int64)
    W = Q + Q.T
    np.fill_diagonal(W, 0)
    b = np.diag(Q).copy()
    xi = x.astype(np.int64)
    return b + W @ xi, int(xi @ Q @ xi)


@pytest.mark.parametrize("init", [0, 1])
def test_incremental_state_every_step(orc, init):
    N = 24
    Q = instances.random_qubo(N, seed=11, lo=-20, hi=20)
    rep = orc.Replica(Q, init=init, seed=3, r=2)
    st = rep.read()
    h, E = _np_state(Q, st["x"])
    np.testing.assert_array_equal(st["h"], h)
    assert st["E"] == E and st["best_E"] == E
    thr_hot = orc.threshold_table(15.0)
    thr_cold = orc.threshold_table(0.3)
    energies = [E]
    prev = st
    for s in range(3000):
        thr = thr_hot if s < 1000 else thr_cold
        k = rep.step(thr, s, eoff_inc=3)
        st = rep.read()
        h, E = _np_state(Q, st["x"])
        np.testing.assert_array_equal(st["h"], h)
        assert st["E"] == E
        if k < 0:
            np.testing.assert_array_equal(st["x"], prev["x"])
            assert st["eoff"] == min(prev["eoff"] + 3, EOFF_MAX)
            assert st["n_accept"] == prev["n_accept"]
        else:
            diff = np.nonzero(st["x"] != prev["x"])[0]
            assert list(diff) == [k]
            assert st["eoff"] == 0
            assert st["n_accept"] == prev["n_accept"] + 1
        energies.append(E)
        assert st["best_E"] == min(energies)
        assert _np_state(Q, st["best_x"])[1] == st["best_E"]
        prev = st


def test_offset_saturates(orc):
    # A state where no flip can be accepted at T = 0 except through the offset.
    N = 4
    Q = np.diag([10, 10, 10, 10]).astype(np.int32)  # every flip from 0 costs +10
    rep = orc.Replica(Q, init=0, seed=1, r=0)
    thr = orc.threshold_table(0.0)  # accept only d <= -1
    ks = [rep.step(thr, s, eoff_inc=4) for s in range(3)]
    assert ks == [-1, -1, -1]
    assert rep.read()["eoff"] == 12
    # d = 10 - 12 = -2 <= -1 now: the next step must flip something
    assert rep.step(thr, 3, eoff_inc=4) >= 0
    assert rep.read()["eoff"] == 0
    # With b = 2^30 no flip is ever accepted at T = 0 (d = 2^30 - eoff >= 0), so
    # the offset climbs by the increment and then stays at its 2^30 ceiling.
    Qb = np.diag([2**30, 2**30]).astype(np.int32)
    big = orc.Replica(Qb, init=0, seed=1, r=0)
    seen = []
    for s in range(4):
        assert big.step(thr, s, eoff_inc=2**29 + 7) == -1
        seen.append(big.read()["eoff"])
    assert seen == [2**29 + 7, EOFF_MAX, EOFF_MAX, EOFF_MAX]


def test_anneal_trace_matches_stepping(orc):
    N = 20
    Q = instances.random_qubo(N, seed=2, lo=-30, hi=30)
    S, L = 400, 8
    out = orc.anneal(Q, T_hi=40.0, T_lo=1.0, n_levels=L, eoff_inc=5, replicas=3,
                     replica_base=7, steps=S, seed=77, trace=True)
    thr = [orc.threshold_table(orc.level_temperature(40.0, 1.0, 0, L, l)) for l in range(L)]
    for rr in range(3):
        rep = orc.Replica(Q, init=0, seed=77, r=7 + rr)
        for s in range(S):
            k = rep.step(thr[orc.level_of_step(s, L, S)], s, eoff_inc=5)
            st = rep.read()
            assert out["trace_k"][rr, s] == k
            assert out["trace_E"][rr, s] == st["E"]
            assert out["trace_eoff"][rr, s] == st["eoff"]
        st = rep.read()
        np.testing.assert_array_equal(out["final_x"][rr], st["x"])
        np.testing.assert_array_equal(out["best_x"][rr], st["best_x"])
        assert out["final_E"][rr] == st["E"] and out["best_E"][rr] == st["best_E"]
        assert out["n_accept"][rr] == st["n_accept"]


def test_replicas_replay_alone(orc):
    Qq, _ = instances.ising_to_qubo(instances.sk_bimodal(32, 4))
    batch = orc.anneal(Qq, T_hi=8.0, T_lo=0.5, replicas=6, steps=500, seed=5, eoff_inc=1)
    for rr in (0, 3, 5):
        one = orc.anneal(Qq, T_hi=8.0, T_lo=0.5, replicas=1, replica_base=rr, steps=500,
                         seed=5, eoff_inc=1)
        for key in ("best_x", "final_x", "best_E", "final_E", "n_accept"):
            np.testing.assert_array_equal(one[key][0], batch[key][rr])


def test_zero_steps_and_zero_temperature(orc):
    Q, _ = instances.ising_to_qubo(instances.sk_bimodal(40, 8))
    out = orc.anneal(Q, T_hi=5.0, T_lo=1.0, replicas=2, steps=0, seed=1, init=1)
    for rr in range(2):
        x0 = np.array([orc.init_bit(1, rr, i) for i in range(40)], dtype=np.uint8)
        np.testing.assert_array_equal(out["final_x"][rr], x0)
        assert out["final_E"][rr] == orc.energy(Q, x0) == out["best_E"][rr]
    # T = 0, no offset: greedy descent; it ends in a one-flip local minimum and
    # its energy never rises.
    out = orc.anneal(Q, T_hi=0.0, T_lo=0.0, n_levels=1, replicas=4, steps=400, seed=3,
                     init=1, trace=True)
    for rr in range(4):
        x = out["final_x"][rr]
        h = orc.fields(Q, x)
        dE = (1 - 2 * x.astype(np.int64)) * h
        assert dE.min() >= 0
        assert np.all(np.diff(out["trace_E"][rr]) <= 0)
        assert out["best_E"][rr] == out["final_E"][rr]


def _numpy_bruteforce(Q):
    N = Q.shape[0]
    X = ((np.arange(2**N)[:, None] >> np.arange(N)[None, :]) & 1).astype(np.int64)
    E = np.einsum("si,ij,sj->s", X, Q.astype(np.int64), X)
    return int(E.min()), int(np.count_nonzero(E == E.min()))


@pytest.mark.parametrize("N,seed", [(1, 1), (2, 2), (7, 3), (12, 4), (14, 5)])
def test_bruteforce_matches_numpy(orc, N, seed):
    Q = instances.random_qubo(N, seed=seed, lo=-9, hi=9)
    e, n, x = orc.bruteforce(Q)
    assert (e, n) == _numpy_bruteforce(Q)
    assert orc.energy(Q, x) == e


@pytest.mark.parametrize("kind,N", [("sk-bimodal", 16), ("sk-bimodal", 20),
                                    ("sk-gaussian", 18), ("random", 12)])
def test_anneal_reaches_exact_optimum(orc, kind, N):
    if kind == "sk-bimodal":
        Q, _ = instances.ising_to_qubo(instances.sk_bimodal(N, 21))
        T_hi, T_lo, inc = 6.0, 0.2, 1
    elif kind == "sk-gaussian":
        Q, _ = instances.ising_to_qubo(instances.sk_gaussian(N, 22, scale=2**16))
        T_hi, T_lo, inc = 2.0 * 2**16, 0.05 * 2**16, 2**14
    else:
        Q = instances.random_qubo(N, seed=23, lo=-50, hi=50)
        T_hi, T_lo, inc = 200.0, 1.0, 5
    e_min, n_min, _ = orc.bruteforce(Q)
    out = orc.anneal(Q, T_hi=T_hi, T_lo=T_lo, eoff_inc=inc, replicas=16, steps=4000, seed=9)
    assert out["best_E"].min() == e_min
    assert np.all(out["best_E"] >= e_min)
    hits = int(np.count_nonzero(out["best_E"] == e_min))
    assert hits >= 4, hits
    for rr in range(16):
        assert orc.energy(Q, out["best_x"][rr]) == out["best_E"][rr]


def test_mattis_sk_ground_state(orc):
    N = 48
    J, eps = instances.mattis(N, 31, "sk")
    Q, c = instances.ising_to_qubo(J)
    Hmin = -N * (N - 1) // 2
    out = orc.anneal(Q, T_hi=30.0, T_lo=0.5, eoff_inc=1, replicas=8, steps=3000, seed=2)
    assert out["best_E"].min() + c == Hmin
    assert np.all(out["best_E"] + c >= Hmin)
    k = int(np.argmin(out["best_E"]))
    s = out["best_x"][k].astype(np.int64) * 2 - 1
    assert abs(int(s @ eps)) == N


def test_mattis_torus_ground_state(orc):
    L = 6
    N = L * L
    J, eps = instances.mattis(N, 32, "torus2d", L=L)
    Q, c = instances.ising_to_qubo(J)
    out = orc.anneal(Q, T_hi=3.0, T_lo=0.1, eoff_inc=1, replicas=8, steps=6000, seed=4)
    assert out["best_E"].min() + c == -2 * N
    assert np.all(out["best_E"] + c >= -2 * N)


def test_mattis_small_bruteforce(orc):
    J, _ = instances.mattis(16, 33, "sk")
    Q, c = instances.ising_to_qubo(J)
    e, n, _ = orc.bruteforce(Q)
    assert e + c == -16 * 15 // 2 and n == 2


@pytest.mark.parametrize("kind", [0, 1])
def test_per_step_schedule_is_one_level_per_step(orc, kind):
    """n_levels = 0 (a new temperature every step, App. A) runs step s at level s of an
    S-level schedule: the per-draw thresholds give the same run as S level tables."""
    from paper_1806_08815_amd import instances
    Q = instances.ising_to_qubo(instances.sk_bimodal(40, 8))[0]
    S = 300
    a = orc.anneal(Q, T_hi=12.0, T_lo=0.2, kind=kind, n_levels=0, eoff_inc=1, replicas=3,
                   steps=S, seed=5, trace=True)
    b = orc.anneal(Q, T_hi=12.0, T_lo=0.2, kind=kind, n_levels=S, eoff_inc=1, replicas=3,
                   steps=S, seed=5, trace=True)
    for k in ("best_x", "best_E", "final_x", "final_E", "n_accept", "trace_k", "trace_E"):
        assert np.array_equal(a[k], b[k]), k
    # and it is a different run from a coarse schedule
    c = orc.anneal(Q, T_hi=12.0, T_lo=0.2, kind=kind, n_levels=4, eoff_inc=1, replicas=3,
                   steps=S, seed=5, trace=True)
    assert not np.array_equal(a["trace_k"], c["trace_k"])


def test_single_trial_sweeps_in_order(orc):
    """Single-trial mode: at step s only variable s mod N may flip (sequential sweeps)."""
    Q = instances.ising_to_qubo(instances.sk_bimodal(30, 4))[0]
    out = orc.anneal(Q, T_hi=5.0, T_lo=5.0, n_levels=1, replicas=4, steps=600, seed=2,
                     trace=True, trial=1, init=1)
    k = out["trace_k"]
    s = np.arange(600)[None, :].repeat(4, 0)
    assert np.all((k == -1) | (k == s % 30))
    assert (k >= 0).sum() > 100


def test_single_trial_acceptance_is_metropolis(orc):
    """One single-trial step from many random states: variable 0 flips with
    probability min(1, exp(-dE/T)) (Sec. III), dE computed here from Q by numpy."""
    Q = instances.random_qubo(10, 7, lo=-6, hi=6)
    N, T, R = 10, 4.0, 40_000
    out = orc.anneal(Q, T_hi=T, T_lo=T, n_levels=1, replicas=R, steps=1, seed=11, init=1,
                     trial=1)
    x0 = np.array([[orc.init_bit(11, r, i) for i in range(N)] for r in range(R)], np.int64)
    W = Q + Q.T
    np.fill_diagonal(W, 0)
    b = np.diag(Q).astype(np.int64)
    h0 = b[0] + x0 @ W[0].astype(np.int64)
    dE = (1 - 2 * x0[:, 0]) * h0
    flipped = out["final_x"][:, 0].astype(np.int64) != x0[:, 0]
    assert np.all(out["final_x"][:, 1:] == x0[:, 1:])          # nothing else moves
    for d in np.unique(dE):
        sel = dE == d
        n = int(sel.sum())
        if n < 500:
            continue
        p = min(1.0, float(np.exp(-d / T)))
        f = flipped[sel].mean()
        tol = 4.5 * np.sqrt(max(p * (1 - p), 1e-4) / n) + 2.0 ** -15
        assert abs(f - p) < tol, (d, f, p, n)


def test_single_trial_zero_temperature_is_greedy_descent(orc):
    """T = 0, no offset: a variable flips only when that lowers the energy; after
    enough sweeps the state is a one-flip local minimum (checked with numpy)."""
    Q = instances.random_qubo(25, 3, lo=-20, hi=20)
    out = orc.anneal(Q, T_hi=0.0, T_lo=0.0, n_levels=1, replicas=3, steps=25 * 30, seed=1,
                     init=1, trial=1, trace=True)
    W = Q + Q.T
    np.fill_diagonal(W, 0)
    b = np.diag(Q).astype(np.int64)
    for r in range(3):
        x = out["final_x"][r].astype(np.int64)
        h = b + W.astype(np.int64) @ x
        assert np.all((1 - 2 * x) * h >= 0)
        E = out["trace_E"][r]
        assert np.all(np.diff(E) <= 0)
