"""Parallel tempering and the full-size workloads on the GPU against the oracle.

PT (Sec. II.D, exchange move of Algorithm 3) runs its exchanges on the device;
the per-replica outputs, final temperature slots and swap counts must equal
the oracle's.  At full workload sizes the oracle replays sampled replicas one
by one (the counter-based random numbers make any replica replayable alone);
the GPU runs the whole workload in the launch shape the benchmark times.
"""
import numpy as np
import pytest

import oracle
from paper_1806_08815_amd import instances, workloads

pytestmark = pytest.mark.gpu

KEYS = ("best_x", "best_E", "final_x", "final_E", "n_accept")


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1806_08815_amd import api as a
    a.lib()
    return a


@pytest.mark.parametrize("N,M,chains,rounds,K,inc", [
    (64, 8, 3, 10, 64, 0), (200, 5, 2, 70, 16, 1), (700, 4, 1, 6, 100, 3), (1024, 32, 2, 3, 1024, 0),
])
def test_pt_parity(api, N, M, chains, rounds, K, inc):
    Q = instances.ising_to_qubo(instances.sk_bimodal(N, N))[0]
    temps = workloads.pt_temperatures(M, 0.1, 3.0, scale=N ** 0.5)
    ctx = api.da_create(Q)
    gpu = api.da_pt(ctx, temps, chains, rounds, K, inc, 5)
    ref = oracle.pt(Q, temps, chains=chains, rounds=rounds, steps_per_round=K, eoff_inc=inc,
                    seed=5)
    for k in KEYS + ("slot", "n_swaps"):
        assert np.array_equal(gpu[k], ref[k]), k
    if M >= 5:
        assert ref["n_swaps"].sum() > 0   # the exchange path was exercised


def test_pt_gaussian_parity(api):
    N, M = 300, 6
    Q = instances.ising_to_qubo(instances.sk_gaussian(N, 3, scale=2**16))[0]
    temps = workloads.pt_temperatures(M, 0.1, 3.0, scale=2**16)
    ctx = api.da_create(Q)
    gpu = api.da_pt(ctx, temps, 2, 8, 200, 2**16, 9)
    ref = oracle.pt(Q, temps, chains=2, rounds=8, steps_per_round=200, eoff_inc=2**16, seed=9)
    for k in KEYS + ("slot", "n_swaps"):
        assert np.array_equal(gpu[k], ref[k]), k


@pytest.mark.parametrize("chains", [2, 40])
def test_pt_gaussian_estimates_parity(api, chains):
    """Gaussian PT takes per-draw estimates: with few replicas the
    random-number waves hand them over (the estimate ring in LDS), with many
    (40 chains x 16 temperatures: lazy draws) the compute lanes evaluate them;
    one sampled chain against the oracle either way."""
    N, M, K, rounds = 700, 16, 300, 6
    Q = instances.ising_to_qubo(instances.sk_gaussian(N, 4, scale=2**16))[0]
    temps = workloads.pt_temperatures(M, 0.1, 3.0, scale=2**16)
    ctx = api.da_create(Q)
    gpu = api.da_pt(ctx, temps, chains, rounds, K, 2**16, 11)
    assert api.da_last_kernel_stats(ctx)["draw_estimates"] == 1
    c = chains - 1
    ref = oracle.pt(Q, temps, chains=1, rounds=rounds, steps_per_round=K, eoff_inc=2**16,
                    seed=11, chain_base=c)
    rows = slice(c * M, (c + 1) * M)
    for k in KEYS + ("slot",):
        assert np.array_equal(gpu[k][rows], ref[k]), k


def _sampled(api, name, rows, dtype=None, launch=None):
    w = workloads.WORKLOADS[name]
    Q, _ = w.instance()
    ctx = api.da_create(Q, w.dtype_hint if dtype is None else dtype)
    sch = api.schedule(w.T_hi, w.T_lo, w.schedule, w.n_levels, w.eoff_inc, w.init)
    gpu = api.da_anneal_ex(ctx, sch, 0, w.replicas, w.steps, w.seed, launch)
    for r in rows:
        ref = oracle.anneal(Q, T_hi=w.T_hi, T_lo=w.T_lo, n_levels=w.n_levels,
                            eoff_inc=w.eoff_inc, init=0 if w.init == "zeros" else 1,
                            replica_base=r, replicas=1, steps=w.steps, seed=w.seed)
        for k in KEYS:
            assert np.array_equal(gpu[k][r], ref[k][0]), (name, r, k)
    return gpu


def test_torus2d_bimodal_1024_sampled(api):
    """128 replicas x 10^5 steps, int16 storage, the benchmark's launch."""
    gpu = _sampled(api, "torus2d-bimodal-1024", rows=(0, 127))
    assert gpu["n_accept"].min() > 0


def test_sk_gaussian_1024_sampled(api):
    """1024 replicas x 10^5 steps of the fixed-point Gaussian SK instance."""
    _sampled(api, "sk-gaussian-1024", rows=(0, 1023))


def test_sk_gaussian_1024_int32_storage(api):
    """Same workload with couplings forced to int32 storage: identical results."""
    w = workloads.WORKLOADS["sk-gaussian-1024"]
    Q, _ = w.instance()
    sch = api.schedule(w.T_hi, w.T_lo, w.schedule, w.n_levels, w.eoff_inc, w.init)
    a = api.da_anneal_ex(api.da_create(Q, 0), sch, 0, 64, 20_000, w.seed)
    b = api.da_anneal_ex(api.da_create(Q, 4), sch, 0, 64, 20_000, w.seed)
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


def test_sk_bimodal_1024_random_start_sampled(api):
    """The +-1 variant with a random start (int8 MFMA initial fields)."""
    w = workloads.WORKLOADS["sk-bimodal-1024-random"]
    Q, _ = w.instance()
    ctx = api.da_create(Q)
    assert ctx.info()["dtype"] == 1
    sch = api.schedule(w.T_hi, w.T_lo, w.schedule, w.n_levels, w.eoff_inc, w.init)
    gpu = api.da_anneal_ex(ctx, sch, 0, 1024, 2000, w.seed)
    ref = oracle.anneal(Q, T_hi=w.T_hi, T_lo=w.T_lo, n_levels=w.n_levels, eoff_inc=w.eoff_inc,
                        init=1, replica_base=1000, replicas=24, steps=2000, seed=w.seed)
    for k in KEYS:
        assert np.array_equal(gpu[k][1000:1024], ref[k]), k


def test_argument_errors(api):
    Q = instances.random_qubo(10, 1)
    with pytest.raises(api.DaError) as e:
        api.da_create(np.zeros((0, 0), np.int32))
    assert e.value.code == api.DA_EINVAL
    big = np.full((4, 4), 2**29, np.int32)
    with pytest.raises(api.DaError) as e:
        api.da_create(big)
    assert e.value.code == api.DA_ERANGE
    with pytest.raises(api.DaError) as e:
        api.da_create(instances.random_qubo(8, 2, lo=-1000, hi=1000), api.DA_DTYPE_I8)
    assert e.value.code == api.DA_ERANGE
    ctx = api.da_create(Q)
    with pytest.raises(api.DaError) as e:
        api.da_anneal(ctx, api.schedule(1.0, 0.5), 0, 10, 1)
    assert e.value.code == api.DA_EINVAL
    with pytest.raises(api.DaError) as e:
        api.da_anneal(ctx, api.schedule(-1.0, 0.5), 2, 10, 1)
    assert e.value.code == api.DA_EINVAL
    with pytest.raises(api.DaError) as e:
        api.da_pt(ctx, [2.0, 1.0], 1, 1, 1, 0, 1)
    assert e.value.code == api.DA_EINVAL
    assert "ok" in api.da_strerror(0)


def test_random_start_tiled_mfma_fields(api):
    """Random start of many replicas of a +-1 instance: the LDS-tiled int8 MFMA
    field kernel (R x ld large enough, ragged in both) gives the exact energies of
    every start state and the oracle's trajectories."""
    N, R = 1000, 4200
    Q = instances.ising_to_qubo(instances.sk_bimodal(N, 31))[0]
    ctx = api.da_create(Q)
    assert ctx.info()["dtype"] == 1
    sch = api.schedule(3.0 * N ** 0.5, 0.1, "geometric", 16, 1, "random")
    g0 = api.da_anneal_ex(ctx, sch, 0, R, 0, 13)
    X = g0["final_x"].astype(np.int64)
    Qi = Q.astype(np.int64)
    E = np.einsum("ri,ij,rj->r", X, Qi, X)
    assert np.array_equal(g0["final_E"], E)
    gpu = api.da_anneal_ex(ctx, sch, 0, R, 60, 13)
    for r in (0, 2047, R - 1):
        ref = oracle.anneal(Q, T_hi=3.0 * N ** 0.5, T_lo=0.1, n_levels=16, eoff_inc=1, init=1,
                            replica_base=r, replicas=1, steps=60, seed=13)
        for k in KEYS:
            assert np.array_equal(gpu[k][r], ref[k][0]), (r, k)

def test_random_start_large_mfma_fields(api):
    """A larger random start on the LDS-tiled MFMA field kernel (ragged in both
    directions, many blocks per CU): exact energies of every random start state,
    and the oracle's trajectories for sampled replicas."""
    N, R = 1950, 4500
    Q = instances.ising_to_qubo(instances.sk_bimodal(N, 37))[0]
    ctx = api.da_create(Q)
    assert ctx.info()["dtype"] == 1
    sch = api.schedule(3.0 * N ** 0.5, 0.1, "geometric", 16, 1, "random")
    g0 = api.da_anneal_ex(ctx, sch, 0, R, 0, 19)
    X = g0["final_x"].astype(np.float64)
    E = ((X @ Q.astype(np.float64)) * X).sum(axis=1)   # exact: integers below 2^53
    assert np.array_equal(g0["final_E"], E.astype(np.int64))
    gpu = api.da_anneal_ex(ctx, sch, 0, R, 40, 19)
    for r in (0, 2303, R - 1):
        ref = oracle.anneal(Q, T_hi=3.0 * N ** 0.5, T_lo=0.1, n_levels=16, eoff_inc=1, init=1,
                            replica_base=r, replicas=1, steps=40, seed=19)
        for k in KEYS:
            assert np.array_equal(gpu[k][r], ref[k][0]), (r, k)


@pytest.mark.timeout(600)
def test_pt_full_size_sampled_chain(api):
    """The PT workload at full chain count: 64 chains x 32 temperatures of the
    N = 1024 +-1 instance, K = 1024 steps per round, 100 rounds on the device;
    one sampled chain (its 32 replicas, slots and swaps) replayed by the oracle."""
    p = workloads.PT_WORKLOAD
    Q, _ = workloads.make_instance(p["kind"], p["N"], p["instance_seed"])
    temps = workloads.pt_temperatures(p["M"], p["T_lo"], p["T_hi"], p["temp_scale"])
    M, C, rounds = p["M"], p["chains"], 100
    ctx = api.da_create(Q)
    gpu = api.da_pt(ctx, temps, C, rounds, p["steps_per_round"], p["eoff_inc"], p["seed"])
    c = 37
    ref = oracle.pt(Q, temps, chains=1, rounds=rounds, steps_per_round=p["steps_per_round"],
                    eoff_inc=p["eoff_inc"], seed=p["seed"], chain_base=c)
    rows = slice(c * M, (c + 1) * M)
    for k in KEYS + ("slot",):
        assert np.array_equal(gpu[k][rows], ref[k]), k
    assert gpu["n_swaps"][c] == ref["n_swaps"][0] > 0
    # every chain's slots are a permutation of the ladder
    for q in range(C):
        assert sorted(gpu["slot"][q * M:(q + 1) * M]) == list(range(M))


@pytest.mark.parametrize("N,M,chains,iters,rounds,K", [
    (64, 8, 4, 3, 20, 64), (300, 12, 3, 4, 10, 128), (1024, 16, 2, 2, 4, 1024),
])
def test_pt_adapt_parity(api, N, M, chains, iters, rounds, K):
    """Adaptive ladder (Sec. II.D): PT runs on the device, per-pair acceptance
    counts, ladder updates -- the final ladder and every iteration's measured
    acceptances equal the oracle's."""
    Q = instances.ising_to_qubo(instances.sk_bimodal(N, N + 1))[0]
    temps = workloads.pt_temperatures(M, 0.1, 3.0, scale=N ** 0.5)
    ctx = api.da_create(Q)
    got, acc = api.da_pt_adapt(ctx, temps, chains, iters, rounds, K, 0, 3)
    want, wacc = oracle.pt_adapt(Q, temps, chains=chains, iterations=iters, rounds=rounds,
                                 steps_per_round=K, seed=3)
    assert np.array_equal(got, want)
    assert np.array_equal(acc, wacc)
    assert got[0] == temps[0] and got[-1] == temps[-1]


def test_pt_pair_swaps_parity(api):
    N, M = 200, 9
    Q = instances.ising_to_qubo(instances.sk_bimodal(N, 4))[0]
    temps = workloads.pt_temperatures(M, 0.1, 3.0, scale=N ** 0.5)
    ctx = api.da_create(Q)
    gpu = api.da_pt(ctx, temps, 5, 70, 32, 1, 8)
    ref = oracle.pt(Q, temps, chains=5, rounds=70, steps_per_round=32, eoff_inc=1, seed=8)
    assert np.array_equal(gpu["pair_swaps"], ref["pair_swaps"])
    assert np.array_equal(gpu["pair_swaps"].sum(axis=1), gpu["n_swaps"])
