"""Sparse row lists (DA_STORE_SPARSE) on the GPU.

An accepted step reads the neighbours of the flipped variable from a padded
row list (in LDS when it fits) and updates only their fields; results must be
bit-identical to the dense path and to the oracle, for every launch shape,
feature mode and batch path.
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


def _same(a, b, keys=KEYS):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k


def _inst(kind, seed):
    if kind == "torus":
        return instances.ising_to_qubo(instances.torus2d(32, seed, "bimodal"))[0], 3.0, 0.1, 1
    if kind == "torus-gauss":
        # 2^12 fixed point: the torus couplings are not normalised, and a row
        # list holds 16-bit values
        return (instances.ising_to_qubo(instances.torus2d(20, seed, "gaussian", scale=2**12))[0],
                3.0 * 2**12, 0.05 * 2**12, 2**12)
    if kind == "er":
        return instances.ising_to_qubo(instances.erdos_renyi(500, 0.05, seed))[0], 8.0, 0.1, 1
    if kind == "sk":
        return instances.ising_to_qubo(instances.sk_bimodal(64, seed))[0], 24.0, 0.4, 1
    raise ValueError(kind)


@pytest.mark.parametrize("kind,F,rng,w_lds", [
    ("torus", 4, 1, 0), ("torus", 8, -1, -1), ("torus-gauss", 4, -1, 0), ("er", 8, 1, 0),
    ("er", 4, -1, -1), ("sk", 4, 1, 0),
])
def test_sparse_trace_parity(api, kind, F, rng, w_lds):
    Q, T_hi, T_lo, inc = _inst(kind, 3)
    N = Q.shape[0]
    ctx = api.da_create(Q, api.DA_STORE_SPARSE)
    assert ctx.info()["sparse_degree"] >= 4
    sch = api.schedule(T_hi, T_lo, "geometric", 16, inc)
    R, S = 4, 1200
    gpu = api.da_anneal_ex(ctx, sch, 5, R, S, 3, api.launch(F, 1, w_lds, rng), trace=True)
    ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, n_levels=16, eoff_inc=inc, replica_base=5,
                        replicas=R, steps=S, seed=3, trace=True)
    _same(gpu, ref, ("trace_k", "trace_E", "trace_eoff") + KEYS)
    assert N == ctx.N


def test_sparse_equals_dense_full_run(api):
    """The bench's 2D torus, 128 replicas x 20000 steps: sparse == dense."""
    Q, T_hi, T_lo, inc = _inst("torus", 1)
    sch = api.schedule(T_hi, T_lo, "geometric", 128, inc)
    dense = api.da_anneal(api.da_create(Q, api.DA_DTYPE_I16), sch, 128, 20_000, 1)
    sp = api.da_anneal(api.da_create(Q, api.DA_DTYPE_I16 | api.DA_STORE_SPARSE), sch, 128,
                       20_000, 1)
    _same(sp, dense)


def test_sparse_modes_batch_and_errors(api):
    import torch
    Q, T_hi, T_lo, inc = _inst("er", 9)
    ctx = api.da_create(Q, api.DA_STORE_SPARSE)
    for trial, L in (("single", 8), ("parallel", 0), ("single", 0)):
        sch = api.schedule(T_hi, T_lo, "linear_beta", L, inc, "random", trial)
        gpu = api.da_anneal_ex(ctx, sch, 0, 3, 900, 2)
        ref = oracle.anneal(Q, T_hi=T_hi, T_lo=T_lo, kind=1, n_levels=L, eoff_inc=inc, init=1,
                            trial=1 if trial == "single" else 0, replicas=3, steps=900, seed=2)
        _same(gpu, ref)
    # batched: a sparse job beside a dense one
    sch = api.schedule(T_hi, T_lo, "geometric", 32, inc)
    alone = api.da_anneal(ctx, sch, 6, 1500, 4)
    Qd = instances.ising_to_qubo(instances.sk_bimodal(100, 2))[0]
    cd = api.da_create(Qd)
    schd = api.schedule(30.0, 0.5, "geometric", 16, 1)
    alone_d = api.da_anneal(cd, schd, 5, 1500, 4)
    c2 = api.da_create(Q, api.DA_STORE_SPARSE)
    items = [dict(ctx=c2, schedule=sch, replicas=6, steps=1500, seed=4,
                  out_dev=api.device_outputs(6, Q.shape[0])),
             dict(ctx=cd, schedule=schd, replicas=5, steps=1500, seed=4,
                  out_dev=api.device_outputs(5, 100))]
    api.da_anneal_batch(items)
    torch.cuda.synchronize()
    for it, want in zip(items, (alone, alone_d)):
        for k in KEYS:
            assert np.array_equal(it["out_dev"][k].cpu().numpy(), want[k]), k
    # values beyond 16 bits cannot go in a row list
    big = instances.random_qubo(50, 1, lo=-90000, hi=90000)
    with pytest.raises(api.DaError) as e:
        api.da_create(big, api.DA_STORE_SPARSE)
    assert e.value.code == api.DA_ERANGE
