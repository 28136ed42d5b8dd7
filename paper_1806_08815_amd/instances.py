"""Seeded synthetic problem instances shaped like the paper's benchmark classes.

Sec. V of Aramon et al. (arXiv:1806.08815) benchmarks spin glasses with zero
biases on two graphs (a 2D torus and the complete graph, "SK") with bimodal
(+-1) or Gaussian couplings, and Sec. VI.C adds Erdos-Renyi graphs of varying
density.  The paper's own instances (Spin Glass Server, Biq Mac) are not
available, so these generators produce stand-ins of the same shapes from a
numpy PCG64 stream.  Gaussian couplings are quantised to integers by a fixed
scale, as the DA hardware requires integer coefficients (Sec. V).

This module only produces inputs.  It holds none of the annealer's arithmetic;
the one formula in it is the problem encoding itself: an Ising Hamiltonian
H(s) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i (Sec. V, eq:ising) becomes a
QUBO over x in {0,1}^N through s = 2x - 1.
"""
from __future__ import annotations

import hashlib

import numpy as np

INT32_MAX = 2**31 - 1


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _sym(J: np.ndarray) -> np.ndarray:
    J = np.triu(J, 1)
    return J + J.T


def sk_bimodal(N: int, seed: int) -> np.ndarray:
    """Complete graph, J_ij = +-1 with equal probability (Sec. V, SK-bimodal)."""
    g = _rng(seed)
    J = g.integers(0, 2, size=(N, N), dtype=np.int64) * 2 - 1
    return _sym(J)


def sk_gaussian(N: int, seed: int, scale: float = 2.0**16) -> np.ndarray:
    """Complete graph, J_ij ~ N(0,1)/sqrt(N), quantised as rint(J * scale)."""
    g = _rng(seed)
    J = g.standard_normal(size=(N, N)) / np.sqrt(N)
    return _sym(np.rint(J * scale).astype(np.int64))


def torus2d(L: int, seed: int, dist: str = "bimodal", scale: float = 2.0**16) -> np.ndarray:
    """L x L torus (periodic boundaries), right and down neighbours, N = L*L.

    dist='bimodal': J = +-1; dist='gaussian': rint(N(0,1) * scale).
    Site (r, c) is variable r*L + c.  For L = 2 the two bonds between a pair
    of neighbours add up.
    """
    g = _rng(seed)
    N = L * L
    J = np.zeros((N, N), dtype=np.int64)
    for r in range(L):
        for c in range(L):
            i = r * L + c
            for (rr, cc) in (((r, (c + 1) % L)), (((r + 1) % L, c))):
                j = rr * L + cc
                if dist == "bimodal":
                    v = int(g.integers(0, 2)) * 2 - 1
                elif dist == "gaussian":
                    v = int(np.rint(g.standard_normal() * scale))
                else:
                    raise ValueError(dist)
                if i != j:
                    J[i, j] += v
                    J[j, i] += v
    return J


def erdos_renyi(N: int, density: float, seed: int) -> np.ndarray:
    """G(N, p) graph with +-1 couplings on present edges (Sec. VI.C)."""
    g = _rng(seed)
    present = g.random(size=(N, N)) < density
    J = g.integers(0, 2, size=(N, N), dtype=np.int64) * 2 - 1
    return _sym(np.where(present, J, 0))


def mattis(N: int, seed: int, graph: str = "sk", L: int | None = None):
    """Planted (Mattis) instance J_ij = eps_i eps_j on the chosen graph.

    Its ground states are s = eps and s = -eps, with H_min = -(number of
    edges).  Returns (J, eps).
    """
    g = _rng(seed)
    if graph == "sk":
        eps = g.integers(0, 2, size=N, dtype=np.int64) * 2 - 1
        J = _sym(np.outer(eps, eps))
    elif graph == "torus2d":
        assert L is not None and L * L == N
        eps = g.integers(0, 2, size=N, dtype=np.int64) * 2 - 1
        mask = torus2d(L, seed=0) != 0
        J = np.where(mask, np.outer(eps, eps), 0)
    else:
        raise ValueError(graph)
    return J, eps


def ising_to_qubo(J: np.ndarray, h: np.ndarray | None = None):
    """Upper-triangular int32 Q and constant c with H(s) = x^T Q x + c, s = 2x - 1.

    Expanding s_i s_j = 4 x_i x_j - 2 x_i - 2 x_j + 1 gives
      Q_ij = -4 J_ij (i < j),  Q_ii = 2 sum_{j != i} J_ij - 2 h_i,
      c = -sum_{i<j} J_ij + sum_i h_i.
    """
    J = np.asarray(J, dtype=np.int64)
    N = J.shape[0]
    if h is None:
        h = np.zeros(N, dtype=np.int64)
    h = np.asarray(h, dtype=np.int64)
    Ju = np.triu(J, 1)
    Q = -4 * Ju
    row = J.sum(axis=1) - np.diag(J)
    Q[np.arange(N), np.arange(N)] = 2 * row - 2 * h
    c = -int(Ju.sum()) + int(h.sum())
    if np.abs(Q).max(initial=0) > INT32_MAX:
        raise OverflowError("QUBO coefficients do not fit int32")
    return Q.astype(np.int32), c


def ising_energy(J: np.ndarray, h: np.ndarray | None, s: np.ndarray) -> int:
    """H(s) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i, computed directly."""
    J = np.asarray(J, dtype=np.int64)
    s = np.asarray(s, dtype=np.int64)
    e = -int(s @ np.triu(J, 1) @ s)
    if h is not None:
        e -= int(np.asarray(h, dtype=np.int64) @ s)
    return e


def random_qubo(N: int, seed: int, lo: int = -100, hi: int = 100) -> np.ndarray:
    """Dense, non-symmetric integer Q (exercises the general x^T Q x convention)."""
    g = _rng(seed)
    return g.integers(lo, hi + 1, size=(N, N), dtype=np.int64).astype(np.int32)


def digest(Q: np.ndarray) -> str:
    """SHA-256 of the int32 bytes of Q (identifies an instance across runs)."""
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.int32))
    return hashlib.sha256(Q.tobytes()).hexdigest()
