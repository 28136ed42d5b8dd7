"""Batched persistent launches and the continuous-batching server on the GPU.

A job's results must not depend on what it is batched or served with: every
random number is keyed by (seed, job-local replica, step) and the step kernel
resumes exactly at epoch boundaries.  So each job here is compared bit-exactly
with the same job run alone through da_anneal, and small jobs with the oracle.
"""
import time

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


def _job(kind, N, seed):
    if kind == "sk":
        Q = instances.ising_to_qubo(instances.sk_bimodal(N, seed))[0]
        sc = max(1.0, N ** 0.5)
        return Q, dict(T_hi=3.0 * sc, T_lo=0.05 * sc, eoff_inc=1)
    Q = instances.ising_to_qubo(instances.sk_gaussian(N, seed, scale=2**16))[0]
    return Q, dict(T_hi=3.0 * 2**16, T_lo=0.05 * 2**16, eoff_inc=2**16)


SPECS = [  # kind, N, replicas, steps, init, dtype hint, n_levels
    ("sk", 64, 16, 3000, "zeros", 0, 128),
    ("gauss", 100, 7, 2500, "random", 0, 64),
    ("sk", 300, 33, 1500, "zeros", 2, 128),
    ("gauss", 1000, 5, 1200, "zeros", 4, 32),
    ("sk", 1024, 20, 900, "random", 0, 128),
    ("sk", 2000, 3, 700, "zeros", 0, 16),
    ("gauss", 513, 17, 1000, "random", 0, 50),
]


def test_batch_matches_alone(api):
    import torch
    ctxs, items, alone = [], [], []
    for a, (kind, N, R, S, init, hint, L) in enumerate(SPECS):
        Q, t = _job(kind, N, 10 + a)
        ctx = api.da_create(Q, hint)
        sch = api.schedule(t["T_hi"], t["T_lo"], "geometric", L, t["eoff_inc"], init)
        alone.append(api.da_anneal(ctx, sch, R, S, 100 + a))
        ctxs.append(ctx)
        items.append(dict(ctx=ctx, schedule=sch, replica_base=0, replicas=R, steps=S,
                          seed=100 + a, out_dev=api.device_outputs(R, N)))
    api.da_anneal_batch(items)
    torch.cuda.synchronize()
    for a, it in enumerate(items):
        for k in KEYS:
            got = it["out_dev"][k].cpu().numpy()
            assert np.array_equal(got, alone[a][k]), (SPECS[a], k)
    # and the oracle for the small ones
    for a in (0, 1):
        kind, N, R, S, init, hint, L = SPECS[a]
        Q, t = _job(kind, N, 10 + a)
        ref = oracle.anneal(Q, T_hi=t["T_hi"], T_lo=t["T_lo"], n_levels=L,
                            eoff_inc=t["eoff_inc"], init=0 if init == "zeros" else 1,
                            replicas=R, steps=S, seed=100 + a)
        for k in KEYS:
            assert np.array_equal(items[a]["out_dev"][k].cpu().numpy(), ref[k]), (a, k)


def test_batch_large_n(api):
    """Batches holding the largest sizes (one replica per workgroup) beside small jobs;
    N = 6000 and N = 1500 leave surplus waves in their workgroups (12 and 3 x 5 of 16),
    the last block of N = 1500 also holds empty replica slots."""
    import torch
    specs = [("sk", 8192, 3, 300, "zeros", 0, 8), ("gauss", 4096, 5, 500, "random", 0, 16),
             ("sk", 64, 40, 800, "zeros", 0, 16), ("gauss", 6000, 2, 200, "zeros", 4, 4),
             ("sk", 1500, 7, 300, "zeros", 0, 8)]
    items, alone = [], []
    for a, (kind, N, R, S, init, hint, L) in enumerate(specs):
        Q, t = _job(kind, N, 70 + a)
        ctx = api.da_create(Q, hint)
        sch = api.schedule(t["T_hi"], t["T_lo"], "geometric", L, t["eoff_inc"], init)
        alone.append(api.da_anneal(ctx, sch, R, S, 3 + a))
        items.append(dict(ctx=ctx, schedule=sch, replica_base=0, replicas=R, steps=S,
                          seed=3 + a, out_dev=api.device_outputs(R, N)))
    api.da_anneal_batch(items)
    torch.cuda.synchronize()
    for a, it in enumerate(items):
        for k in KEYS:
            assert np.array_equal(it["out_dev"][k].cpu().numpy(), alone[a][k]), (specs[a], k)
    kind, N, R, S, init, hint, L = specs[0]
    Q, t = _job(kind, N, 70)
    ref = oracle.anneal(Q, T_hi=t["T_hi"], T_lo=t["T_lo"], n_levels=L, eoff_inc=t["eoff_inc"],
                        replica_base=2, replicas=1, steps=S, seed=3)
    for k in KEYS:
        assert np.array_equal(items[0]["out_dev"][k].cpu().numpy()[2:3], ref[k]), k


def test_server_results_equal_alone(api):
    # a budget that holds only some jobs at once forces queueing and admission
    # as memory frees up; an epoch that does not divide the step counts forces
    # resumption at arbitrary steps
    specs = SPECS + [("sk", 128, 40, 2000, "zeros", 0, 128), ("gauss", 64, 9, 3100, "zeros", 0, 8)]
    foot = [api.da_job_footprint(N, 4, R, L) for (_, N, R, _, _, _, L) in specs]
    srv = api.da_server_create(int(max(foot) * 2.2), epoch_steps=777)
    tickets, want = [], []
    for a, (kind, N, R, S, init, hint, L) in enumerate(specs):
        Q, t = _job(kind, N, 40 + a)
        sch = api.schedule(t["T_hi"], t["T_lo"], "geometric", L, t["eoff_inc"], init)
        ctx = api.da_create(Q, hint)
        want.append(api.da_anneal(ctx, sch, R, S, 7 + a))
        ctx.close()
        tickets.append(api.da_submit(srv, Q, sch, R, S, 7 + a, hint))
    got = [api.da_wait(srv, t) for t in tickets]
    for a in range(len(specs)):
        for k in KEYS:
            assert np.array_equal(got[a][k], want[a][k]), (specs[a], k)
        st = got[a]["stats"]
        assert st["t_submit"] <= st["t_admit"] <= st["t_done"]
        assert st["epochs"] == -(-specs[a][3] // 777)
    # somebody had to wait for memory
    assert max(g["stats"]["t_admit"] - g["stats"]["t_submit"] for g in got) > 0
    srv.close()
    # and the oracle: one sampled replica of every served job, replayed alone
    for a, (kind, N, R, S, init, hint, L) in enumerate(specs):
        _oracle_replica(kind, N, 40 + a, R - 1 - a % R, S, init, L, 7 + a, got[a])


def _oracle_replica(kind, N, inst, r, S, init, L, seed, got):
    Q, t = _job(kind, N, inst)
    ref = oracle.anneal(Q, T_hi=t["T_hi"], T_lo=t["T_lo"], n_levels=L, eoff_inc=t["eoff_inc"],
                        init=0 if init == "zeros" else 1, replica_base=r, replicas=1, steps=S,
                        seed=seed)
    for k in KEYS:
        assert np.array_equal(np.asarray(got[k])[r], ref[k][0]), (kind, N, r, k)


def test_server_large_jobs_vs_oracle(api):
    """The largest served sizes: an N = 8192 +-1 job and int32-stored Gaussian
    jobs (N = 4096 and 2048) beside small ones, under a budget that holds the
    big jobs one at a time, so they queue; every result equals the job alone
    and, for one sampled replica per job, the oracle."""
    specs = [("sk", 8192, 3, 400, "zeros", 0, 8), ("gauss", 4096, 4, 500, "random", 4, 16),
             ("gauss", 2048, 6, 900, "zeros", 4, 32), ("sk", 256, 24, 1500, "zeros", 0, 64),
             ("gauss", 77, 11, 2000, "random", 4, 16)]
    jobs, want, foot = [], [], []
    for a, (kind, N, R, S, init, hint, L) in enumerate(specs):
        Q, t = _job(kind, N, 90 + a)
        sch = api.schedule(t["T_hi"], t["T_lo"], "geometric", L, t["eoff_inc"], init)
        ctx = api.da_create(Q, hint)
        want.append(api.da_anneal(ctx, sch, R, S, 50 + a))
        foot.append(api.da_job_footprint(N, ctx.info()["dtype"], R, L))
        ctx.close()
        jobs.append((Q, sch, R, S, 50 + a, hint))
    # room for either big job plus all the small ones, never both big jobs
    budget = max(foot[:2]) + sum(foot[2:]) + (1 << 20)
    assert budget < foot[0] + foot[1]
    srv = api.da_server_create(budget, epoch_steps=333)
    tickets = [api.da_submit(srv, *j) for j in jobs]
    got = [api.da_wait(srv, t) for t in tickets]
    srv.close()
    for a, (kind, N, R, S, init, hint, L) in enumerate(specs):
        for k in KEYS:
            assert np.array_equal(got[a][k], want[a][k]), (specs[a], k)
    assert got[1]["stats"]["t_admit"] >= got[0]["stats"]["t_done"] - 1e-6
    for a, (kind, N, R, S, init, hint, L) in enumerate(specs):
        _oracle_replica(kind, N, 90 + a, R - 1, S, init, L, 50 + a, got[a])


def test_server_tickets_and_admission(api):
    Q, t = _job("sk", 256, 3)
    sch = api.schedule(t["T_hi"], t["T_lo"], "geometric", 16, 1)
    fp = api.da_job_footprint(256, 1, 64, 16)
    assert fp > 256 * 256
    assert api.da_job_footprint(512, 1, 64, 16) > fp
    assert api.da_job_footprint(256, 4, 64, 16) > fp
    srv = api.da_server_create(fp + 1024, epoch_steps=500)
    with pytest.raises(api.DaError) as e:
        api.da_submit(srv, Q, sch, 65_000, 10, 1)
    assert e.value.code == api.DA_ENOMEM
    t1 = api.da_submit(srv, Q, sch, 64, 20_000, 1)
    t2 = api.da_submit(srv, Q, sch, 64, 1_000, 2)   # waits for t1's memory
    r2 = api.da_wait(srv, t2)
    r1 = api.da_wait(srv, t1)
    assert r2["stats"]["t_admit"] >= r1["stats"]["t_done"] - 1e-6
    with pytest.raises(api.DaError) as e:
        api.da_wait(srv, t1)
    assert e.value.code == api.DA_ENOTFOUND
    srv.close()


def test_server_poll_not_ready(api):
    Q, t = _job("sk", 1024, 5)
    sch = api.schedule(t["T_hi"], t["T_lo"], "geometric", 16, 1)
    srv = api.da_server_create(1 << 34, epoch_steps=2000)
    tk = api.da_submit(srv, Q, sch, 256, 40_000, 1)
    assert api.da_poll(srv, tk) is None
    t0 = time.time()
    while api.da_poll(srv, tk) is None:
        assert time.time() - t0 < 120
        time.sleep(0.01)
    srv.close()


def test_server_preemption(api):
    """A high-priority job that does not fit preempts a running low-priority
    one: the low job is snapshotted to host memory between epochs, released,
    re-admitted after the high job, and resumes from its snapshot.  Both
    results equal the jobs run alone, and a sampled replica of the preempted
    job equals the oracle's."""
    low = ("sk", 512, 16, 200_000, "zeros", 0, 64)
    high = ("gauss", 384, 12, 3000, "random", 0, 32)
    jobs, want, foot = [], [], []
    for a, (kind, N, R, S, init, hint, L) in enumerate((low, high)):
        Q, t = _job(kind, N, 120 + a)
        sch = api.schedule(t["T_hi"], t["T_lo"], "geometric", L, t["eoff_inc"], init)
        ctx = api.da_create(Q, hint)
        want.append(api.da_anneal(ctx, sch, R, S, 60 + a))
        foot.append(api.da_job_footprint(N, ctx.info()["dtype"], R, L))
        ctx.close()
        jobs.append((Q, sch, R, S, 60 + a, hint))
    srv = api.da_server_create(max(foot) + min(foot) // 2, epoch_steps=500)
    t_low = api.da_submit(srv, *jobs[0], priority=0)
    t0 = time.time()
    while True:   # wait until the low job is resident and has run an epoch
        state, done = api.da_job_status(srv, t_low)
        assert state != 2, "low-priority job finished before the high one arrived"
        if state == 1 and done > 0:
            break
        assert time.time() - t0 < 60
        time.sleep(0.001)
    t_high = api.da_submit(srv, *jobs[1], priority=5)
    r_high = api.da_wait(srv, t_high)
    r_low = api.da_wait(srv, t_low)
    with pytest.raises(api.DaError) as e:   # collected tickets are gone
        api.da_job_status(srv, t_low)
    assert e.value.code == api.DA_ENOTFOUND
    srv.close()
    for k in KEYS:
        assert np.array_equal(r_high[k], want[1][k]), k
        assert np.array_equal(r_low[k], want[0][k]), k
    assert r_low["stats"]["preemptions"] >= 1
    assert r_high["stats"]["preemptions"] == 0
    assert r_low["stats"]["t_done"] > r_high["stats"]["t_done"]
    kind, N, R, S, init, hint, L = low
    _oracle_replica(kind, N, 120, 5, S, init, L, 60, r_low)


def test_server_priority_order_without_preemption(api):
    """A budget for one job at a time: waiting jobs are admitted by priority,
    then submission order, and a waiting job whose priority is not above the
    running job's preempts nothing."""
    Q, t = _job("sk", 256, 9)
    sch = api.schedule(t["T_hi"], t["T_lo"], "geometric", 16, 1)
    fp = api.da_job_footprint(256, 1, 32, 16)
    srv = api.da_server_create(fp + fp // 2, epoch_steps=400)
    t1 = api.da_submit(srv, Q, sch, 32, 6000, 1, priority=1)
    t2 = api.da_submit(srv, Q, sch, 32, 1000, 2, priority=0)
    t3 = api.da_submit(srv, Q, sch, 32, 1000, 3, priority=1)
    r = {k: api.da_wait(srv, k) for k in (t1, t2, t3)}
    srv.close()
    assert all(v["stats"]["preemptions"] == 0 for v in r.values())
    assert r[t1]["stats"]["t_admit"] <= r[t3]["stats"]["t_admit"] <= r[t2]["stats"]["t_admit"]
    assert r[t3]["stats"]["t_admit"] >= r[t1]["stats"]["t_done"] - 1e-6
