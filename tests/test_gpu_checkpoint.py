"""Checkpoint / resume on the GPU.

A run cut into pieces -- continued in the same context, or saved to host
memory and resumed in a fresh context -- must end exactly where the
uninterrupted run ends (counter-based draws keyed by the global step), and
both must equal the oracle.
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


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("N,R,S,L,cuts,init", [
    (200, 7, 3000, 16, [1, 1500, 2999], "zeros"),       # mid-level cuts, one-step pieces
    (1024, 5, 2048, 8, [256, 512, 1024], "random"),    # cuts on level boundaries
    (64, 33, 1000, 128, [333, 777], "zeros"),
    # >= 256 steps per level: narrow-band levels decide by direct tables; cuts
    # mid-level and one step before a level change
    (300, 5, 2400, 4, [1, 700, 1199, 2399], "zeros"),
])
def test_split_equals_one_shot(api, N, R, S, L, cuts, init):
    Q = instances.ising_to_qubo(instances.sk_bimodal(N, 21))[0]
    sc = max(1.0, N ** 0.5)
    sch = api.schedule(3.0 * sc, 0.1, "geometric", L, 1, init)
    ctx = api.da_create(Q)
    whole = api.da_anneal_ex(ctx, sch, 4, R, S, 17)
    edges = [0] + cuts + [S]
    for a, b in zip(edges[:-1], edges[1:]):
        part = api.da_anneal_steps(ctx, sch, 4, R, S, a, b, 17)
    _same(part, whole)
    ref = oracle.anneal(Q, T_hi=3.0 * sc, T_lo=0.1, n_levels=L, eoff_inc=1,
                        init=0 if init == "zeros" else 1, replica_base=4, replicas=R, steps=S,
                        seed=17)
    _same(whole, ref)


def test_save_load_resume_in_fresh_context(api):
    N, R, S = 1000, 9, 4000
    Q = instances.ising_to_qubo(instances.sk_gaussian(N, 5, scale=2**16))[0]
    sch = api.schedule(3.0 * 2**16, 0.05 * 2**16, "geometric", 64, 2**16)
    a = api.da_create(Q)
    whole = api.da_anneal_ex(a, sch, 0, R, S, 3)
    api.da_anneal_steps(a, sch, 0, R, S, 0, 1234, 3)
    snap = api.da_state_save(a, R)
    assert snap.nbytes == api.da_state_bytes(N, R)
    a.close()
    b = api.da_create(Q)
    api.da_state_load(b, snap)
    rest = api.da_anneal_steps(b, sch, 0, R, S, 1234, S, 3)
    _same(rest, whole)
    # a snapshot of fewer replicas resumes just those
    c = api.da_create(Q)
    api.da_anneal_steps(c, sch, 0, R, S, 0, 2000, 3)
    snap3 = api.da_state_save(c, 3)
    d = api.da_create(Q)
    api.da_state_load(d, snap3)
    part = api.da_anneal_steps(d, sch, 0, 3, S, 2000, S, 3)
    for k in KEYS:
        assert np.array_equal(part[k], whole[k][:3]), k


def test_resume_errors(api):
    Q = instances.random_qubo(50, 2)
    sch = api.schedule(20.0, 1.0)
    ctx = api.da_create(Q)
    with pytest.raises(api.DaError) as e:          # nothing to resume
        api.da_anneal_steps(ctx, sch, 0, 4, 100, 10, 20, 1)
    assert e.value.code == api.DA_EINVAL
    api.da_anneal_steps(ctx, sch, 0, 4, 100, 0, 10, 1)
    with pytest.raises(api.DaError):                # wrong resume step
        api.da_anneal_steps(ctx, sch, 0, 4, 100, 11, 20, 1)
    with pytest.raises(api.DaError):                # other replica ids
        api.da_anneal_steps(ctx, sch, 1, 4, 100, 10, 20, 1)
    with pytest.raises(api.DaError):                # more replicas than held
        api.da_anneal_steps(ctx, sch, 0, 5, 100, 10, 20, 1)
    with pytest.raises(api.DaError):                # range outside the run
        api.da_anneal_steps(ctx, sch, 0, 4, 100, 10, 101, 1)
    api.da_anneal_steps(ctx, sch, 0, 4, 100, 10, 100, 1)
    snap = api.da_state_save(ctx, 4)
    other = api.da_create(instances.random_qubo(51, 2))
    with pytest.raises(api.DaError):                # different N
        api.da_state_load(other, snap)
    bad = snap.copy()
    bad[0] ^= 0xFF
    with pytest.raises(api.DaError):                # not a snapshot
        api.da_state_load(ctx, bad)
    with pytest.raises(api.DaError):                # truncated
        api.da_state_load(ctx, snap[:-1])
