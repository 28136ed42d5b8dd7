"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Everything here is integer work, so the bar is bit-exact: per-step traces
(flipped variable, energy, offset), final and best states and energies, and
accepted-step counts.  Cases span several tiles and ragged tails (N not a
multiple of 8 or 64, replica counts not a multiple of the workgroup shape),
every coupling storage type, every launch shape, zero and random starts,
both schedule kinds, zero temperature and the offset ceiling.
"""
import numpy as np
import pytest

import oracle
from paper_1806_08815_amd import instances

pytestmark = pytest.mark.gpu

KEYS = ("best_x", "best_E", "final_x", "final_E", "n_accept")


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1806_08815_amd import api as a
    a.lib()
    return a


def _same(gpu, ref, keys=KEYS, rows=None):
    for k in keys:
        g = gpu[k] if rows is None else gpu[k][rows]
        if not np.array_equal(g, ref[k]):
            bad = np.argwhere(np.asarray(g) != np.asarray(ref[k]))[:5]
            raise AssertionError(f"{k} differs at {bad.tolist()}")


def _q(kind, N, seed):
    if kind == "sk":
        return instances.ising_to_qubo(instances.sk_bimodal(N, seed))[0]
    if kind == "gauss":
        return instances.ising_to_qubo(instances.sk_gaussian(N, seed, scale=2**16))[0]
    if kind == "random":
        return instances.random_qubo(N, seed, lo=-300, hi=300)
    if kind == "random_big":
        return instances.random_qubo(N, seed, lo=-40000, hi=40000)
    if kind == "sk_huge":
        # common factor 2^24 >= 2^23: 8/16-bit storage takes the full-width
        # multiply in the field update
        return instances.ising_to_qubo(instances.sk_bimodal(N, seed))[0] * 2**22
    raise ValueError(kind)


@pytest.mark.parametrize("kind,N,dtype", [
    ("sk", 1, 0), ("sk", 5, 0), ("sk", 64, 0), ("sk", 100, 0), ("sk", 1000, 0),
    ("random", 77, 0), ("random", 300, 2), ("random_big", 130, 0), ("gauss", 513, 4),
    ("sk", 200, 4), ("sk", 129, 2),
])
def test_energy(api, kind, N, dtype):
    Q = _q(kind, N, 3)
    ctx = api.da_create(Q, dtype)
    g = np.random.Generator(np.random.PCG64(N))
    X = g.integers(0, 2, size=(37, N)).astype(np.uint8)
    E = api.da_energy(ctx, X)
    want = [oracle.energy(Q, X[r]) for r in range(37)]
    assert E.tolist() == want


@pytest.mark.parametrize("rng", [1, -1])
@pytest.mark.parametrize("kind,N,dtype,F,rpw", [
    ("sk", 20, 0, 8, 1), ("sk", 64, 0, 8, 1), ("sk", 64, 2, 4, 2), ("sk", 100, 4, 8, 3),
    ("random", 70, 0, 8, 2), ("random", 257, 2, 8, 1), ("gauss", 300, 0, 4, 1),
    ("sk", 513, 0, 8, 1), ("sk", 1000, 2, 8, 2), ("gauss", 1024, 4, 8, 1),
    ("random_big", 600, 4, 4, 1), ("sk", 1536, 1, 8, 1), ("sk", 1024, 2, 4, 1),
    ("gauss", 2048, 0, 4, 1), ("sk_huge", 40, 0, 8, 1), ("sk_huge", 40, 2, 4, 1),
])
def test_trace_parity(api, kind, N, dtype, F, rpw, rng):
    Q = _q(kind, N, 5)
    if kind == "gauss":
        T_hi, T_lo, inc = 3.0 * 2**16, 0.05 * 2**16, 2**16
    elif kind == "sk_huge":
        T_hi, T_lo, inc = 3.0 * N ** 0.5 * 2**22, 0.1 * 2**22, 2**22
    elif kind.startswith("random"):
        T_hi, T_lo, inc = 4000.0, 10.0, 50
    else:
        T_hi, T_lo, inc = 3.0 * max(1.0, N ** 0.5), 0.1, 1
    R, S, L = 5, 700, 16
    ctx = api.da_create(Q, dtype)
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc)
    gpu = api.da_anneal_ex(ctx, sch, 3, R, S, 11, api.launch(F, rpw, 0, rng), trace=True)
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, replica_base=3,
                        replicas=R, steps=S, seed=11, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


@pytest.mark.parametrize("rng", [1, -1])
@pytest.mark.parametrize("kind,N,dtype,F,rpw", [
    ("sk", 64, 0, 4, 1), ("sk", 100, 4, 8, 3), ("sk", 300, 2, 4, 1), ("sk", 1024, 2, 4, 1),
    ("sk", 1000, 1, 8, 2), ("gauss", 1024, 0, 8, 1), ("gauss", 513, 4, 4, 2),
])
def test_direct_table_trace_parity(api, kind, N, dtype, F, rpw, rng):
    """Levels of at least 256 steps: the narrow-band levels (tmax - tmin <= 255)
    decide in-band flips by their direct tables, read a step ahead; wider bands
    (the hottest +-1 level, every Gaussian level) take the brackets, so runs
    cross both kinds of level change."""
    Q = _q(kind, N, 7)
    if kind == "gauss":
        T_hi, T_lo, inc = 3.0 * 2**16, 0.05 * 2**16, 2**16
    else:
        T_hi, T_lo, inc = 3.0 * max(1.0, N ** 0.5), 0.1, 1
    R, S, L = 4, 1600, 4
    ctx = api.da_create(Q, dtype)
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc)
    gpu = api.da_anneal_ex(ctx, sch, 1, R, S, 23, api.launch(F, rpw, 0, rng), trace=True)
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, replica_base=1,
                        replicas=R, steps=S, seed=23, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


@pytest.mark.parametrize("N,dtype,F,rpw", [
    (1024, 0, 8, 1), (1000, 0, 8, 1), (300, 4, 4, 2), (513, 0, 8, 1), (2048, 0, 8, 1), (64, 0, 4, 1),
])
def test_wide_band_trace_parity(api, N, dtype, F, rpw):
    """Gaussian couplings with random-number waves and no per-draw estimates:
    every level's band is wide (buckets of 2^sh costs), so full waves decide
    each flip by one bracket read (costs past the buckets meet the reject-all
    entry) and waves holding ghost flips take the band tests; N = 1000, 300 and
    513 mix both in one replica."""
    Q = _q("gauss", N, 5)
    T_hi, T_lo, inc = 3.0 * 2**16, 0.05 * 2**16, 2**16
    R, S, L = 5, 1200, 6
    ctx = api.da_create(Q, dtype)
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc)
    gpu = api.da_anneal_ex(ctx, sch, 3, R, S, 11, api.launch(F, rpw, 0, 1, -1), trace=True)
    assert api.da_last_kernel_stats(ctx)["draw_estimates"] == 0
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, replica_base=3,
                        replicas=R, steps=S, seed=11, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


@pytest.mark.parametrize("kind,N,dtype,F,rpw,init", [
    ("gauss", 1024, 0, 8, 1, 0), ("gauss", 1024, 0, 4, 1, 1), ("gauss", 1000, 0, 8, 1, 0),
    ("gauss", 300, 4, 4, 2, 1), ("gauss", 513, 0, 8, 1, 0), ("gauss", 2048, 0, 8, 1, 0),
    ("gauss", 4096, 2, 8, 1, 1), ("sk", 1024, 0, 8, 1, 0), ("sk", 1000, 1, 4, 2, 1),
    ("sk", 300, 0, 4, 4, 0), ("random", 777, 0, 4, 1, 1),
])
@pytest.mark.parametrize("rng", [1, -1])
def test_draw_estimate_trace_parity(api, kind, N, dtype, F, rpw, init, rng):
    """Per-draw estimates: the random-number waves hand over G(u) ~ -thr[u]
    (rng = 1; with rng = -1 each compute lane draws its block and evaluates
    them itself) and full waves decide each flip by the sign of
    d - glo + G(u) - 1, reading thr[u] only inside the measured window.  Gaussian levels are wide; the
    +-1 and small-integer instances have levels of a few units, so costs sit
    inside the window often and the exact reads run many times per step.
    Short levels keep the direct tables off, so every level takes the
    estimates; ragged N mixes full waves with band-test waves."""
    Q = _q(kind, N, 13)
    if kind == "gauss":
        T_hi, T_lo, inc = 3.0 * 2**16, 0.05 * 2**16, 2**16
    else:
        T_hi, T_lo, inc = 3.0 * max(1.0, N ** 0.5), 0.1, 1
    R, S, L = 4, 1500, 12   # levels of 125 steps: no direct tables
    ctx = api.da_create(Q, dtype)
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc, init=init)
    gpu = api.da_anneal_ex(ctx, sch, 2, R, S, 29, api.launch(F, rpw, 0, rng, 1), trace=True)
    st = api.da_last_kernel_stats(ctx)
    assert st["draw_estimates"] == 1 and (st["rng_waves"] > 0) == (rng > 0)
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, init=init,
                        replica_base=2, replicas=R, steps=S, seed=29, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


@pytest.mark.parametrize("over", [False, True])
def test_draw_estimate_field_bound(api, over):
    """Fields at the estimate path's bound: row 0's |b_0| + sum_j |W_0j| is
    exactly 2^30 - 2^22 - 256 (one more with over), random starts put fields
    near it at once, tmax sits just under 2^22 and the offset saturates at 2^30,
    so d - glo + G(u) - 1 reaches the int32 ends.  Over the bound the host keeps
    the path off."""
    N, bound = 512, 2**30 - 2**22 - 256
    rng = np.random.default_rng(41)
    q = (bound - 2000) // (N - 1)
    mag = q - rng.integers(0, 4, size=(N, N))
    Q = np.triu(mag * rng.choice([-1, 1], size=(N, N)), 1).astype(np.int64)
    W = np.abs(Q + Q.T)
    b = rng.integers(-900, 901, size=N)
    b[0] = bound - W[0].sum() + (1 if over else 0)
    Q[np.arange(N), np.arange(N)] = b
    hb = (W.sum(axis=1) + np.abs(b)).max()
    assert hb == bound + (1 if over else 0)
    Q = Q.astype(np.int32)
    T_hi, T_lo, inc = 3.5e5, 1.0e4, 2**28
    R, S, L = 4, 800, 8
    ctx = api.da_create(Q, 4)
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc, init=1)
    gpu = api.da_anneal_ex(ctx, sch, 0, R, S, 5, api.launch(4, 1, 0, 1, 1), trace=True)
    assert api.da_last_kernel_stats(ctx)["draw_estimates"] == (0 if over else 1)
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, init=1,
                        replicas=R, steps=S, seed=5, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


@pytest.mark.parametrize("N,S,L", [(70, 100, 128), (90, 65, 128), (110, 300, 64), (130, 575, 128)])
def test_tuned_short_schedules(api, N, S, L):
    """Schedules of fewer than 576 steps: the tuner's timing window must stay
    inside the schedule (past its last step the level index would leave the
    level tables).  Each N is new to the process, so the tuner runs."""
    Q = _q("random", N, 31)
    ctx = api.da_create(Q)
    sch = api.schedule(20.0, 1.0, "geometric", L, eoff_inc=2)
    gpu = api.da_anneal(ctx, sch, 3, S, 9)
    ref = oracle.anneal(Q, T_hi=20.0, T_lo=1.0, n_levels=L, eoff_inc=2, replicas=3, steps=S,
                        seed=9)
    _same(gpu, ref)


@pytest.mark.parametrize("w_lds", [1, -1])
def test_sk_bimodal_64_full(api, w_lds):
    """16 replicas x 10^4 steps of an N = 64 +-1 SK instance, escape offset on."""
    Q = _q("sk", 64, 1)
    ctx = api.da_create(Q)
    sch = api.schedule(3.0, 0.05, "geometric", 128, eoff_inc=1)
    gpu = api.da_anneal_ex(ctx, sch, 0, 16, 10_000, 1, api.launch(0, 0, w_lds))
    ref = oracle.anneal(Q, T_hi=3.0, T_lo=0.05, n_levels=128, eoff_inc=1, replicas=16,
                        steps=10_000, seed=1)
    _same(gpu, ref)


@pytest.mark.parametrize("kind,N", [("sk", 1000), ("random", 130), ("gauss", 1024)])
def test_random_start(api, kind, N):
    Q = _q(kind, N, 9)
    ctx = api.da_create(Q)
    T = 2.0 * 2**16 if kind == "gauss" else 50.0
    sch = api.schedule(T, T / 20, "linear_beta", 8, eoff_inc=3, init="random")
    R = 37
    gpu = api.da_anneal_ex(ctx, sch, 0, R, 0, 7)
    X0 = np.array([[oracle.init_bit(7, r, i) for i in range(N)] for r in range(R)], np.uint8)
    assert np.array_equal(gpu["final_x"], X0)
    assert gpu["final_E"].tolist() == [oracle.energy(Q, X0[r]) for r in range(R)]
    gpu = api.da_anneal_ex(ctx, sch, 0, R, 300, 7)
    ref = oracle.anneal(Q, T_hi=T, T_lo=T / 20, kind=1, n_levels=8, eoff_inc=3, init=1,
                        replicas=R, steps=300, seed=7)
    _same(gpu, ref)


def test_edge_cases(api):
    # N = 1, zero steps, zero temperature, a single level, S < L
    Q1 = np.array([[-3]], np.int32)
    ctx = api.da_create(Q1)
    out = api.da_anneal(ctx, api.schedule(1.0, 1.0, n_levels=1), 3, 5, 1)
    ref = oracle.anneal(Q1, T_hi=1.0, T_lo=1.0, n_levels=1, replicas=3, steps=5, seed=1)
    _same(out, ref)
    Q = _q("sk", 40, 2)
    ctx = api.da_create(Q)
    out = api.da_anneal(ctx, api.schedule(2.0, 1.0), 4, 0, 1)
    assert np.all(out["final_x"] == 0) and np.all(out["final_E"] == 0)
    for sch_args in [dict(T_hi=0.0, T_lo=0.0, n_levels=1), dict(T_hi=9.0, T_lo=0.5, n_levels=500)]:
        sch = api.schedule(sch_args["T_hi"], sch_args["T_lo"], "geometric", sch_args["n_levels"],
                           eoff_inc=2, init="random")
        out = api.da_anneal_ex(ctx, sch, 0, 6, 333, 4, trace=True)
        ref = oracle.anneal(Q, T_hi=sch_args["T_hi"], T_lo=sch_args["T_lo"],
                            n_levels=sch_args["n_levels"], eoff_inc=2, init=1, replicas=6,
                            steps=333, seed=4, trace=True)
        _same(out, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


def test_offset_ceiling(api):
    Qb = np.diag([2**30, 2**30, 2**30]).astype(np.int32)
    ctx = api.da_create(Qb)
    sch = api.schedule(0.0, 0.0, n_levels=1, eoff_inc=2**29 + 7)
    out = api.da_anneal_ex(ctx, sch, 0, 2, 4, 1, trace=True)
    assert out["trace_eoff"].tolist() == [[2**29 + 7, 2**30, 2**30, 2**30]] * 2
    assert np.all(out["trace_k"] == -1)


def test_replica_base_replay(api):
    Q = _q("sk", 300, 4)
    ctx = api.da_create(Q)
    sch = api.schedule(20.0, 0.5, eoff_inc=1)
    batch = api.da_anneal_ex(ctx, sch, 0, 24, 2000, 3, api.launch(8, 4, 0, -1))
    for r in (0, 13, 23):
        one = api.da_anneal_ex(ctx, sch, r, 1, 2000, 3, api.launch(4, 1, 0, 1))
        for k in KEYS:
            assert np.array_equal(one[k][0], batch[k][r])


@pytest.mark.parametrize("kind,N,dtype,launch", [
    ("sk", 8192, 0, None), ("gauss", 8192, 4, None), ("sk", 4096, 2, None),
    ("sk", 4096, 0, (8, 1, 0, 1)), ("gauss", 5000, 0, None), ("sk", 3001, 0, (4, 1, 0, -1)),
])
def test_large_n_trace_parity(api, kind, N, dtype, launch):
    """The largest sizes: 16 compute waves per replica, ragged last wave."""
    Q = _q(kind, N, 6)
    if kind == "gauss":
        T_hi, T_lo, inc = 3.0 * 2**16, 0.05 * 2**16, 2**16
    else:
        T_hi, T_lo, inc = 3.0 * N ** 0.5, 0.1, 1
    R, S, L = 3, 400, 8
    ctx = api.da_create(Q, dtype)
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc)
    opts = api.launch(*launch) if launch else None
    gpu = api.da_anneal_ex(ctx, sch, 1, R, S, 2, opts, trace=True)
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, replica_base=1,
                        replicas=R, steps=S, seed=2, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


@pytest.mark.parametrize("rng", [1, -1])
@pytest.mark.parametrize("kind,N,dtype,F,sk", [
    ("sk", 64, 0, 4, 0), ("sk", 300, 2, 8, 1), ("gauss", 1024, 0, 4, 1), ("random", 130, 4, 4, 0),
    ("sk", 1000, 0, 8, 1),
])
def test_per_step_schedule_parity(api, kind, N, dtype, F, sk, rng):
    """A new temperature every step (App. A): thresholds decided as d < T G[u]."""
    Q = _q(kind, N, 12)
    if kind == "gauss":
        T_hi, T_lo, inc = 3.0 * 2**16, 0.05 * 2**16, 2**16
    elif kind == "random":
        T_hi, T_lo, inc = 4000.0, 10.0, 50
    else:
        T_hi, T_lo, inc = 3.0 * N ** 0.5, 0.1, 1
    R, S = 4, 900
    kinds = ("geometric", "linear_beta")
    ctx = api.da_create(Q, dtype)
    sch = api.schedule(T_hi, T_lo, kinds[sk], 0, eoff_inc=inc)
    gpu = api.da_anneal_ex(ctx, sch, 2, R, S, 9, api.launch(F, 1, 0, rng), trace=True)
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, kind=sk, n_levels=0, eoff_inc=inc,
                        replica_base=2, replicas=R, steps=S, seed=9, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


def test_per_step_batch_and_resume(api):
    import torch
    Q = _q("sk", 500, 3)
    sch = api.schedule(60.0, 0.1, "linear_beta", 0, eoff_inc=1)
    ctx = api.da_create(Q)
    whole = api.da_anneal_ex(ctx, sch, 0, 6, 2000, 4)
    ref = oracle.anneal(Q, T_hi=60.0, T_lo=0.1, kind=1, n_levels=0, eoff_inc=1, replicas=6,
                        steps=2000, seed=4)
    _same(whole, ref)
    for a, b in [(0, 700), (700, 701), (701, 2000)]:
        part = api.da_anneal_steps(ctx, sch, 0, 6, 2000, a, b, 4)
    _same(part, whole)
    c2 = api.da_create(Q)
    item = dict(ctx=c2, schedule=sch, replica_base=0, replicas=6, steps=2000, seed=4,
                out_dev=api.device_outputs(6, 500))
    api.da_anneal_batch([item])
    torch.cuda.synchronize()
    for k in KEYS:
        assert np.array_equal(item["out_dev"][k].cpu().numpy(), whole[k]), k
    srv = api.da_server_create(1 << 30)
    with pytest.raises(api.DaError) as e:
        api.da_submit(srv, Q, sch, 6, 2000, 4)
    assert e.value.code == api.DA_EINVAL
    srv.close()


@pytest.mark.parametrize("rng", [1, -1])
@pytest.mark.parametrize("kind,N,dtype,F,L", [
    ("sk", 64, 0, 4, 16), ("sk", 1000, 2, 8, 16), ("gauss", 513, 0, 4, 8), ("random", 130, 4, 8, 0),
])
def test_single_trial_parity(api, kind, N, dtype, F, L, rng):
    """Single-trial Metropolis in sequential sweeps (the SA baseline, Sec. III) on the
    same kernels: variable s mod N alone proposes at step s."""
    Q = _q(kind, N, 14)
    if kind == "gauss":
        T_hi, T_lo, inc = 3.0 * 2**16, 0.05 * 2**16, 0
    elif kind == "random":
        T_hi, T_lo, inc = 4000.0, 10.0, 0
    else:
        T_hi, T_lo, inc = 3.0 * N ** 0.5, 0.1, 0
    R, S = 3, 2 * N + 37
    ctx = api.da_create(Q, dtype)
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc, init="random", trial="single")
    gpu = api.da_anneal_ex(ctx, sch, 1, R, S, 6, api.launch(F, 1, 0, rng), trace=True)
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, init=1, trial=1,
                        replica_base=1, replicas=R, steps=S, seed=6, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)
    assert (gpu["trace_k"] >= 0).sum() > 0


def test_single_trial_resume_and_serve(api):
    Q = _q("sk", 300, 8)
    sch = api.schedule(50.0, 0.5, "geometric", 32, init="random", trial="single")
    ctx = api.da_create(Q)
    whole = api.da_anneal_ex(ctx, sch, 0, 5, 3001, 2)
    api.da_anneal_steps(ctx, sch, 0, 5, 3001, 0, 1111, 2)
    part = api.da_anneal_steps(ctx, sch, 0, 5, 3001, 1111, 3001, 2)
    _same(part, whole)
    srv = api.da_server_create(1 << 30, epoch_steps=700)
    got = api.da_wait(srv, api.da_submit(srv, Q, sch, 5, 3001, 2))
    srv.close()
    _same(got, whole)


@pytest.mark.parametrize("rng", [1, -1])
@pytest.mark.parametrize("N,F,rpw", [(128, 4, 1), (200, 4, 2), (200, 8, 1), (256, 4, 1),
                                     (256, 8, 2)])
def test_w_in_lds_trace_parity(api, N, F, rpw, rng):
    """16-bit couplings staged in LDS for N up to 256 (128 KiB of W at N = 256):
    every accepted step reads row k from LDS instead of L2."""
    Q = _q("random", N, 21)
    T_hi, T_lo, inc = 4000.0, 10.0, 50
    R, S, L = 5, 700, 16
    ctx = api.da_create(Q, 2)
    assert ctx.info()["dtype"] == 2
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc)
    gpu = api.da_anneal_ex(ctx, sch, 2, R, S, 17, api.launch(F, rpw, 1, rng), trace=True)
    assert api.da_last_kernel_stats(ctx)["w_in_lds"] == 1
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, replica_base=2,
                        replicas=R, steps=S, seed=17, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


@pytest.mark.parametrize("inc", [2**30, 2**31 - 1])
def test_offset_increment_extremes(api, inc):
    """Offset increments at and above the 2^30 ceiling (R7): the offset
    saturates at 2^30 after one rejected step, and the step after accepts every
    flip; the kernel's update must not leave int32 on the way."""
    Q = _q("random", 90, 22)
    ctx = api.da_create(Q)
    sch = api.schedule(30.0, 2.0, "geometric", 8, eoff_inc=inc)
    for rng in (1, -1):
        gpu = api.da_anneal_ex(ctx, sch, 0, 4, 3000, 5, api.launch(4, 1, 0, rng), trace=True)
        ref = oracle.anneal(Q, T_hi=30.0, T_lo=2.0, n_levels=8, eoff_inc=inc, replicas=4,
                            steps=3000, seed=5, trace=True)
        _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)
        assert (ref["trace_eoff"] == 2**30).any()


def test_snapshot_offset_out_of_range_rejected(api):
    Q = _q("sk", 64, 3)
    ctx = api.da_create(Q)
    sch = api.schedule(3.0, 0.05, eoff_inc=1)
    api.da_anneal_steps(ctx, sch, 0, 2, 1000, 0, 500, 1)
    snap = api.da_state_save(ctx, 2)
    bad = snap.copy()
    tail = 32 + 2 * 6 * 64 + 2 * 24          # header, x/best x/h, E/best E/accepted
    bad[tail:tail + 4] = np.frombuffer(np.int32(2**30 + 1).tobytes(), np.uint8)
    with pytest.raises(api.DaError) as e:
        api.da_state_load(ctx, bad)
    assert e.value.code == api.DA_EINVAL
    api.da_state_load(ctx, snap)


@pytest.mark.parametrize("rng", [1, -1])
@pytest.mark.parametrize("kind,N,dtype,L,S,extra", [
    ("sk", 1024, 2, 16, 700, {}), ("sk", 1000, 0, 4, 1600, {}),       # narrow bands, direct tables
    ("gauss", 1024, 0, 16, 700, {}), ("random", 257, 2, 16, 700, {}),  # wide bands, ragged N
    ("sk", 2000, 0, 8, 400, {}),                                       # 16 compute waves
    ("random", 200, 2, 16, 700, {"w_lds": 1}),                         # W in LDS
    ("sk", 300, 0, 16, 637, {"trial": "single"}),                      # single trial
    ("sk", 500, 2, 0, 600, {}),                                        # a new temperature every step
])
def test_two_flips_per_lane_trace_parity(api, kind, N, dtype, L, S, extra, rng):
    """Two variables per lane (8- and 16-bit couplings): twice the compute waves
    of four per lane, selection over up to 16 waves."""
    Q = _q(kind, N, 33)
    if kind == "gauss":
        T_hi, T_lo, inc = 3.0 * 2**16, 0.05 * 2**16, 2**16
    elif kind == "random":
        T_hi, T_lo, inc = 4000.0, 10.0, 50
    else:
        T_hi, T_lo, inc = 3.0 * N ** 0.5, 0.1, 1
    trial = extra.get("trial", "parallel")
    if trial == "single":
        inc = 0
    R = 4
    ctx = api.da_create(Q, dtype)
    sch = api.schedule(T_hi, T_lo, "geometric", L, eoff_inc=inc, trial=trial)
    gpu = api.da_anneal_ex(ctx, sch, 2, R, S, 41, api.launch(2, 1, extra.get("w_lds", 0), rng),
                           trace=True)
    assert api.da_last_kernel_stats(ctx)["flips_per_lane"] == 2
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=L, eoff_inc=inc, replica_base=2,
                        replicas=R, steps=S, seed=41, trace=True,
                        trial=1 if trial == "single" else 0)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)


def test_two_flips_per_lane_falls_back_for_int32(api):
    Q = _q("gauss", 300, 3)
    ctx = api.da_create(Q, 4)
    sch = api.schedule(3.0 * 2**16, 0.05 * 2**16, "geometric", 8, eoff_inc=2**16)
    gpu = api.da_anneal_ex(ctx, sch, 0, 3, 500, 2, api.launch(2, 1, 0, 1))
    assert api.da_last_kernel_stats(ctx)["flips_per_lane"] == 4
    ref = oracle.anneal(Q, T_hi=3.0 * 2**16, T_lo=0.05 * 2**16, n_levels=8, eoff_inc=2**16,
                        replicas=3, steps=500, seed=2)
    _same(gpu, ref)
