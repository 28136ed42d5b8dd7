"""Pins the oracle's problem arithmetic: W/b derivation, energy, local fields.

* Energy against x^T Q x evaluated directly by numpy on the raw Q.
* The flip identity E(x xor e_i) - E(x) = (1 - 2 x_i) h_i, exhaustively over
  all states of small random (non-symmetric) Q.
* The Ising encoding of Sec. V: H(s) computed directly from J equals the
  QUBO energy plus the constant, on every instance class.
"""
import itertools

import numpy as np
import pytest

from paper_1806_08815_amd import instances


def test_energy_is_xQx(orc):
    g = np.random.Generator(np.random.PCG64(1))
    for N in (1, 2, 5, 17, 40):
        Q = instances.random_qubo(N, seed=N, lo=-1000, hi=1000)
        for _ in range(20):
            x = g.integers(0, 2, size=N).astype(np.uint8)
            xi = x.astype(np.int64)
            want = int(xi @ Q.astype(np.int64) @ xi)
            assert orc.energy(Q, x) == want


@pytest.mark.parametrize("N", [1, 3, 6, 10])
def test_flip_identity_exhaustive(orc, N):
    Q = instances.random_qubo(N, seed=100 + N, lo=-50, hi=50)
    for bits in itertools.product((0, 1), repeat=N):
        x = np.array(bits, dtype=np.uint8)
        E = orc.energy(Q, x)
        h = orc.fields(Q, x)
        for i in range(N):
            y = x.copy()
            y[i] ^= 1
            assert orc.energy(Q, y) - E == (1 - 2 * int(x[i])) * int(h[i])


def test_fields_definition(orc):
    # h_i = Q_ii + sum_{j != i} (Q_ij + Q_ji) x_j, directly from Q
    N = 23
    Q = instances.random_qubo(N, seed=5).astype(np.int64)
    x = np.random.Generator(np.random.PCG64(3)).integers(0, 2, size=N).astype(np.uint8)
    S = Q + Q.T
    np.fill_diagonal(S, 0)
    want = np.diag(Q) + S @ x.astype(np.int64)
    np.testing.assert_array_equal(orc.fields(Q, x), want)


@pytest.mark.parametrize("maker", [
    lambda: instances.sk_bimodal(30, 1),
    lambda: instances.sk_gaussian(30, 2, scale=2**16),
    lambda: instances.torus2d(5, 3, "bimodal"),
    lambda: instances.torus2d(4, 4, "gaussian", scale=1000),
    lambda: instances.erdos_renyi(25, 0.3, 5),
    lambda: instances.mattis(20, 6)[0],
])
def test_ising_encoding(orc, maker):
    J = maker()
    N = J.shape[0]
    g = np.random.Generator(np.random.PCG64(N))
    hfield = g.integers(-3, 4, size=N)
    for h in (None, hfield):
        Q, c = instances.ising_to_qubo(J, h)
        for _ in range(25):
            s = g.integers(0, 2, size=N) * 2 - 1
            x = ((s + 1) // 2).astype(np.uint8)
            assert instances.ising_energy(J, h, s) == orc.energy(Q, x) + c


def test_delta_e_equals_delta_h(orc):
    # In QUBO units a flip changes the energy exactly as the Ising spin flip does.
    J = instances.sk_bimodal(16, 9)
    Q, c = instances.ising_to_qubo(J)
    g = np.random.Generator(np.random.PCG64(9))
    s = g.integers(0, 2, size=16) * 2 - 1
    x = ((s + 1) // 2).astype(np.uint8)
    h = orc.fields(Q, x)
    for i in range(16):
        s2 = s.copy()
        s2[i] = -s2[i]
        dH = instances.ising_energy(J, None, s2) - instances.ising_energy(J, None, s)
        assert dH == (1 - 2 * int(x[i])) * int(h[i])
        # and the textbook spin-glass form 2 s_i sum_j J_ij s_j
        assert dH == 2 * int(s[i]) * int(J[i] @ s)
