"""The allocation-free energy entry point (da_energy_noalloc) against
da_energy: same states, same energies, bit-exact (integer work), on two calls
in a row on one device, the second with fewer states; the count limit of its
fixed scratch is enforced before any work."""
import numpy as np
import pytest

from paper_1806_08815_amd import instances

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1806_08815_amd import api as a
    a.lib()
    return a


def _cap(N):
    ld = -(-N // 64) * 64
    c = 0
    while -(-(c + 1) * ld // 256) * 256 + 4 * (c + 1) * ld <= 2**25:
        c += 1
    return c


@pytest.mark.parametrize("kind,N,hint,counts", [
    ("sk", 1000, 0, (5000, 37)),       # int8: tiled matrix-core fields, then the small kernel
    ("random", 300, 2, (900, 11)),     # int16 row kernel, ragged N
    ("gauss", 513, 4, (400, 3)),       # int32 couplings
    ("sk", 8192, 0, (819, 64)),        # the largest N at its count limit
])
def test_noalloc_energy_matches_da_energy(api, kind, N, hint, counts):
    import torch
    if kind == "sk":
        Q = instances.ising_to_qubo(instances.sk_bimodal(N, 5))[0]
    elif kind == "gauss":
        Q = instances.ising_to_qubo(instances.sk_gaussian(N, 5, scale=2**16))[0]
    else:
        Q = instances.random_qubo(N, 5, lo=-300, hi=300)
    ctx = api.da_create(Q, hint)
    assert counts[0] <= _cap(N)
    g = np.random.Generator(np.random.PCG64(N))
    stream = torch.cuda.current_stream()
    for count in counts:
        X = g.integers(0, 2, size=(count, N)).astype(np.uint8)
        X[0] = 0
        X[-1] = 1
        xd = torch.from_numpy(X).cuda()
        Ed = torch.full((count,), -7, dtype=torch.int64, device="cuda")
        api.da_energy_noalloc(ctx, xd, Ed, stream)
        torch.cuda.synchronize()
        want = api.da_energy(ctx, X)
        assert np.array_equal(Ed.cpu().numpy(), want), (kind, N, count)
        assert int(want[0]) == 0 and int(want[-1]) == int(Q.astype(np.int64).sum())


def test_noalloc_energy_rejects_counts_beyond_scratch(api):
    import torch
    N = 1024
    Q = instances.ising_to_qubo(instances.sk_bimodal(N, 2))[0]
    ctx = api.da_create(Q)
    cap = _cap(N)
    assert cap == 6553
    xd = torch.zeros((cap + 1, N), dtype=torch.uint8, device="cuda")
    Ed = torch.zeros(cap + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(api.DaError) as e:
        api.da_energy_noalloc(ctx, xd, Ed)
    assert e.value.code == api.DA_EINVAL
    api.da_energy_noalloc(ctx, xd[:cap], Ed[:cap])
    torch.cuda.synchronize()
    assert int(Ed[:cap].abs().max().item()) == 0
