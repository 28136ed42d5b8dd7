"""Acceptance boost of the parallel trial (Sec. III, Figs. 1-2), measured on the GPU.

For a class of instances at N = 64 and a fixed temperature T, replicas are
thermalised and then measured in two modes of the same step kernel:

* single trial (one variable proposes per step, sequential sweeps): P_s is the
  fraction of proposals accepted -- the acceptance probability of standard
  single-flip Metropolis (Eq. (1));
* parallel trial (every variable proposes, the DA): P_p is the fraction of
  steps that accept a flip (Eq. (2)).

Also reported is 1 - (1 - P_s)^N, the value Eq. (2) would give if every
variable were accepted with the mean single-flip probability independently.
The instances are the synthetic stand-ins of `instances.py` (SK and 2D torus,
+-1 and Gaussian couplings); temperatures are in Ising units of the
unquantised couplings, and for +-1 SK in units of sqrt(N) (T_c = 1 for SK).
Run: python -m paper_1806_08815_amd.acceptance [temperature|size]
"""
from __future__ import annotations

import json
import sys

import numpy as np

from . import api, instances

CLASSES = {
    "sk-bimodal": lambda seed: instances.sk_bimodal(64, seed),
    "sk-gaussian": lambda seed: instances.sk_gaussian(64, seed, scale=2**16),
    "2d-bimodal": lambda seed: instances.torus2d(8, seed, "bimodal"),
    "2d-gaussian": lambda seed: instances.torus2d(8, seed, "gaussian", scale=2**16),
}


def acceptance(Q, T: float, trial: str, replicas: int, therm: int, meas: int, seed: int) -> float:
    ctx = api.da_create(Q)
    sch = api.schedule(T, T, "geometric", 1, 0, "random", trial)
    total = therm + meas
    a = api.da_anneal_steps(ctx, sch, 0, replicas, total, 0, therm, seed)["n_accept"]
    b = api.da_anneal_steps(ctx, sch, 0, replicas, total, therm, total, seed)["n_accept"]
    ctx.close()
    return float((b - a).sum()) / (replicas * meas)


def _concurrently(tasks):
    """Run acceptance() calls at once: each has its own context, hence its own
    stream, and the library releases the interpreter lock, so the GPU runs them
    side by side (each alone fills a small part of the chip)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=len(tasks)) as ex:
        return list(ex.map(lambda t: acceptance(*t), tasks))


def run(temps=None, replicas=256, therm_sweeps=100_000, meas_sweeps=5_000, seed=1) -> dict:
    """P_s and P_p against T for the four N = 64 classes (Figs. 1-2), with the
    paper's 10^5 thermalisation and 5 x 10^3 measured sweeps by default."""
    temps = list(np.geomspace(0.2, 3.0, 8)) if temps is None else temps
    cls = []
    for name, make in CLASSES.items():
        Q = instances.ising_to_qubo(make(seed))[0]
        N = Q.shape[0]
        # Gaussian couplings are quantised at 2^16; +-1 SK couplings are not
        # normalised by sqrt(N), so their temperature unit is sqrt(N)
        unit = 2.0**16 if "gaussian" in name else (N ** 0.5 if name.startswith("sk") else 1.0)
        cls.append((name, Q, N, unit))
    out = {name: [] for name, _, _, _ in cls}
    for T in temps:
        tasks = []
        for name, Q, N, unit in cls:
            for trial in ("single", "parallel"):
                tasks.append((Q, T * unit, trial, replicas, therm_sweeps * N, meas_sweeps * N,
                              seed))
        res = _concurrently(tasks)
        for q, (name, Q, N, unit) in enumerate(cls):
            ps, pp = res[2 * q], res[2 * q + 1]
            out[name].append({"T": float(T), "P_s": ps, "P_p": pp,
                              "independent_trials": 1.0 - (1.0 - ps) ** N,
                              "boost": pp / ps if ps > 0 else None})
    return out


def boost_vs_size(sizes=(64, 256, 1024), temps=(0.05, 0.1, 0.2), replicas=256, sweeps=None,
                  seed=1) -> list:
    """P_p / P_s against N at low temperatures on +-1 SK instances (T in units
    of sqrt(N), T_c = 1): the parallel trial's advantage grows with N, and
    P_p / P_s approaches N where N P_s << 1 (Eq. (2) expanded for small P_s);
    where N P_s is not small, P_p saturates at 1 and the ratio at 1 / P_s.
    Sweeps (thermalisation, measured) per size default to (10^5, 5 x 10^3) at
    N = 64 and fewer at larger N, where a sweep costs N times more steps."""
    sweeps = sweeps or {64: (100_000, 5_000), 256: (10_000, 2_000), 1024: (2_000, 500)}
    rows, tasks, keys = [], [], []
    for N in sizes:
        Q = instances.ising_to_qubo(instances.sk_bimodal(N, seed))[0]
        th, me = sweeps[N]
        for T in temps:
            keys.append((N, T))
            for trial in ("single", "parallel"):
                tasks.append((Q, T * N ** 0.5, trial, replicas, th * N, me * N, seed))
    res = _concurrently(tasks)
    for q, (N, T) in enumerate(keys):
        th, me = sweeps[N]
        ps, pp = res[2 * q], res[2 * q + 1]
        rows.append({"N": N, "T": T, "therm_sweeps": th, "meas_sweeps": me, "P_s": ps,
                     "P_p": pp, "ratio": pp / ps if ps > 0 else None,
                     "ratio_over_N": (pp / ps / N) if ps > 0 else None,
                     "independent_trials": 1.0 - (1.0 - ps) ** N})
    return rows


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "temperature"
    res = run() if which == "temperature" else boost_vs_size()
    json.dump(res, sys.stdout, indent=1)
    print()
