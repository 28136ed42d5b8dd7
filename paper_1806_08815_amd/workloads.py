"""Named synthetic workloads: instance recipe plus run parameters.

Each workload fixes the instance (class, size, seed) and the run (replicas,
steps, temperature schedule, escape-offset increment, random seed).  Shapes
follow the paper's benchmark classes (Sec. V) at the sizes the DA hardware
handles (up to 1024 variables now, 8192 for the next generation, Sec. I and
Sec. II.D).  Only parameters live here; see ``instances`` for the generators.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import instances

GAUSS_SCALE = 2**16


@dataclass(frozen=True)
class Workload:
    name: str
    kind: str            # 'sk-bimodal' | 'sk-gaussian' | 'torus2d-bimodal' | ...
    N: int
    instance_seed: int
    replicas: int
    steps: int
    T_hi: float
    T_lo: float
    eoff_inc: int
    seed: int = 1
    schedule: str = "geometric"
    n_levels: int = 128
    dtype_hint: int = 0   # 0 = smallest exact storage
    init: str = "zeros"
    extra: dict = field(default_factory=dict)

    def instance(self) -> tuple[np.ndarray, int]:
        """(Q, const) for this workload."""
        return make_instance(self.kind, self.N, self.instance_seed)


def make_instance(kind: str, N: int, seed: int) -> tuple[np.ndarray, int]:
    if kind == "sk-bimodal":
        J = instances.sk_bimodal(N, seed)
    elif kind == "sk-gaussian":
        J = instances.sk_gaussian(N, seed, scale=GAUSS_SCALE)
    elif kind == "torus2d-bimodal":
        L = int(round(N ** 0.5))
        assert L * L == N
        J = instances.torus2d(L, seed, "bimodal")
    elif kind == "torus2d-gaussian":
        L = int(round(N ** 0.5))
        assert L * L == N
        J = instances.torus2d(L, seed, "gaussian", scale=GAUSS_SCALE)
    else:
        raise ValueError(kind)
    return instances.ising_to_qubo(J)


# Temperatures of Gaussian instances are in units of the unquantised couplings
# (J ~ N(0,1)/sqrt(N)), so they are multiplied by the quantisation scale, and so
# is the escape-offset increment.
WORKLOADS = {
    # Plain DA on a fully connected +-1 instance, N = 64, 16 replicas.
    "sk-bimodal-64": Workload(
        name="sk-bimodal-64", kind="sk-bimodal", N=64, instance_seed=1, replicas=16,
        steps=10_000, T_hi=3.0, T_lo=0.05, eoff_inc=1, seed=1),
    # 2D torus L = 32 (N = 1024), +-1 couplings embedded in a dense int16 matrix.
    "torus2d-bimodal-1024": Workload(
        name="torus2d-bimodal-1024", kind="torus2d-bimodal", N=1024, instance_seed=1,
        replicas=128, steps=100_000, T_hi=3.0, T_lo=0.1, eoff_inc=1, seed=1, dtype_hint=2),
    # Fully connected N = 1024, Gaussian couplings at fixed point 2^16, 1024 replicas.
    "sk-gaussian-1024": Workload(
        name="sk-gaussian-1024", kind="sk-gaussian", N=1024, instance_seed=1, replicas=1024,
        steps=100_000, T_hi=3.0 * GAUSS_SCALE, T_lo=0.05 * GAUSS_SCALE, eoff_inc=GAUSS_SCALE,
        seed=1),
    # The +-1 variant of the same run, random start (initial fields by int8 MFMA).
    "sk-bimodal-1024-random": Workload(
        name="sk-bimodal-1024-random", kind="sk-bimodal", N=1024, instance_seed=1,
        replicas=1024, steps=100_000, T_hi=3.0 * 32, T_lo=0.05 * 32, eoff_inc=1, seed=1,
        init="random"),
}

# Parallel tempering with DA steps: N = 1024 +-1, 32 temperatures geometric
# 0.1 -> 3.0 (in units of the coupling scale sqrt(N) for an SK +-1 instance),
# exchange every 1024 steps, 64 chains, 10^4 rounds.
PT_WORKLOAD = dict(name="pt-sk-bimodal-1024", kind="sk-bimodal", N=1024, instance_seed=1,
                   M=32, T_lo=0.1, T_hi=3.0, steps_per_round=1024, chains=64,
                   rounds=10_000, eoff_inc=0, seed=1, temp_scale=32.0)


def pt_temperatures(M: int, T_lo: float, T_hi: float, scale: float = 1.0) -> np.ndarray:
    """Geometric ladder T_p = T_lo (T_hi/T_lo)^(p/(M-1)), times `scale`."""
    if M == 1:
        return np.array([T_lo * scale])
    p = np.arange(M) / (M - 1)
    return (T_lo * (T_hi / T_lo) ** p) * scale


# Served request stream: Poisson arrivals; N uniform on {64, ..., 8192}; half +-1
# and half quantised Gaussian couplings; 16-256 replicas; 10^4-10^5 steps.
SERVE_SIZES = (64, 128, 256, 512, 1024, 2048, 4096, 8192)


def serve_stream(n_jobs: int, seed: int, rate_hz: float, sizes=SERVE_SIZES,
                 steps_range=(10_000, 100_000), replica_choices=(16, 32, 64, 128, 256)):
    """List of job dicts with arrival times (seconds from stream start)."""
    g = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += float(g.exponential(1.0 / rate_hz))
        N = int(g.choice(sizes))
        kind = "sk-bimodal" if j % 2 == 0 else "sk-gaussian"
        R = int(g.choice(replica_choices))
        lo, hi = np.log(steps_range[0]), np.log(steps_range[1])
        S = int(round(float(np.exp(g.uniform(lo, hi)))))
        if kind == "sk-bimodal":
            scale = float(np.sqrt(N))
            T_hi, T_lo, inc = 3.0 * scale, 0.05 * scale, 1
        else:
            T_hi, T_lo, inc = 3.0 * GAUSS_SCALE, 0.05 * GAUSS_SCALE, GAUSS_SCALE
        jobs.append(dict(job=j, arrival=t, kind=kind, N=N, instance_seed=1000 + j, replicas=R,
                         steps=S, T_hi=T_hi, T_lo=T_lo, eoff_inc=inc, seed=1 + j))
    return jobs
