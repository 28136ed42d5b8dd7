"""CPU oracle for the Digital Annealer step -- TEST INFRASTRUCTURE ONLY.

This package wraps ``oracle.c``, a plain single-threaded C implementation of
the DA parallel-trial Monte Carlo step (Algorithm 2, Sec. II.B of Aramon et
al., arXiv:1806.08815) and of its parallel-tempering variant (Sec. II.D, with
the exchange move of Algorithm 3).  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product library
never does.  It shares no code with the GPU path.

Pinned by ``tests/test_oracle_*.py`` (brute-force optima, per-step field and
energy invariants, planted ground states, exact one-step transition
probabilities, threshold-table definition, Philox against an independent
implementation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCHED_GEOMETRIC = 0
SCHED_LINEAR_BETA = 1
INIT_ZEROS = 0
INIT_RANDOM = 1


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    with _lib_lock:   # callers on several threads build and bind it once
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32, u64, dbl = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        L.orc_philox4x32_10.argtypes = [P, u64, P]
        L.orc_philox4x32_10.restype = None
        L.orc_metropolis_draw.argtypes = [u64, u32, u32, u32]
        L.orc_metropolis_draw.restype = u32
        L.orc_select_draw.argtypes = [u64, u32, u32]
        L.orc_select_draw.restype = u32
        L.orc_exchange_draw.argtypes = [u64, u32, u32, u32]
        L.orc_exchange_draw.restype = u32
        L.orc_init_bit.argtypes = [u64, u32, u32]
        L.orc_init_bit.restype = u32
        L.orc_derive.argtypes = [ctypes.c_int, P, P, P]
        L.orc_derive.restype = None
        L.orc_energy.argtypes = [ctypes.c_int, P, P, P]
        L.orc_energy.restype = i64
        L.orc_fields.argtypes = [ctypes.c_int, P, P, P, P]
        L.orc_fields.restype = None
        L.orc_level_temperature.argtypes = [dbl, dbl, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_level_temperature.restype = dbl
        L.orc_level_of_step.argtypes = [i64, ctypes.c_int, i64]
        L.orc_level_of_step.restype = ctypes.c_int
        L.orc_threshold_table.argtypes = [dbl, P]
        L.orc_threshold_table.restype = None
        L.orc_anneal.argtypes = [ctypes.c_int, P, dbl, dbl, ctypes.c_int, ctypes.c_int, i64,
                                 ctypes.c_int, ctypes.c_int, i64, ctypes.c_int, i64, u64,
                                 P, P, P, P, P, P, P, P]
        L.orc_anneal.restype = ctypes.c_int
        L.orc_pt.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, i64, ctypes.c_int,
                             i64, u64, P, P, P, P, P, P, P]
        L.orc_pt.restype = ctypes.c_int
        L.orc_pt_ex.argtypes = [ctypes.c_int, P, P, ctypes.c_int, i64, ctypes.c_int, i64,
                                ctypes.c_int, i64, u64, P, P, P, P, P, P, P, P, P]
        L.orc_pt_ex.restype = ctypes.c_int
        L.orc_pt_sweep.argtypes = [ctypes.c_int, P, P, P, P, u64, u32, u32, P]
        L.orc_pt_sweep.restype = i64
        L.orc_ladder_update.argtypes = [ctypes.c_int, P, P, i64, P]
        L.orc_ladder_update.restype = None
        L.orc_pt_adapt.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   i64, ctypes.c_int, i64, u64, P]
        L.orc_pt_adapt.restype = ctypes.c_int
        L.orc_rep_new.argtypes = [ctypes.c_int, P, ctypes.c_int, u64, u32]
        L.orc_rep_new.restype = P
        L.orc_rep_step.argtypes = [P, P, u64, u32, u32, i64]
        L.orc_rep_step.restype = ctypes.c_int
        L.orc_rep_read.argtypes = [P, P, P, P, P]
        L.orc_rep_read.restype = None
        L.orc_rep_free.argtypes = [P]
        L.orc_rep_free.restype = None
        L.orc_bruteforce.argtypes = [ctypes.c_int, P, P, P, P]
        L.orc_bruteforce.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _q(Q) -> np.ndarray:
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.int32))
    assert Q.ndim == 2 and Q.shape[0] == Q.shape[1]
    return Q


def philox(ctr, seed: int) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), ctypes.c_uint64(seed), _p(out))
    return out


def metropolis_draw(seed: int, r: int, s: int, i: int) -> int:
    return int(lib().orc_metropolis_draw(seed, r, s, i))


def select_draw(seed: int, r: int, s: int) -> int:
    return int(lib().orc_select_draw(seed, r, s))


def exchange_draw(seed: int, c: int, t: int, p: int) -> int:
    return int(lib().orc_exchange_draw(seed, c, t, p))


def init_bit(seed: int, r: int, i: int) -> int:
    return int(lib().orc_init_bit(seed, r, i))


def derive(Q):
    Q = _q(Q)
    N = Q.shape[0]
    W = np.zeros((N, N), dtype=np.int64)
    b = np.zeros(N, dtype=np.int64)
    lib().orc_derive(N, _p(Q), _p(W), _p(b))
    return W, b


def energy(Q, x) -> int:
    W, b = derive(Q)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    return int(lib().orc_energy(W.shape[0], _p(W), _p(b), _p(x)))


def fields(Q, x) -> np.ndarray:
    W, b = derive(Q)
    N = W.shape[0]
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    h = np.zeros(N, dtype=np.int64)
    lib().orc_fields(N, _p(W), _p(b), _p(x), _p(h))
    return h


def level_temperature(T_hi: float, T_lo: float, kind: int, L: int, l: int) -> float:
    return float(lib().orc_level_temperature(T_hi, T_lo, kind, L, l))


def level_of_step(s: int, L: int, S: int) -> int:
    return int(lib().orc_level_of_step(s, L, S))


def threshold_table(T: float) -> np.ndarray:
    thr = np.zeros(65536, dtype=np.int32)
    lib().orc_threshold_table(float(T), _p(thr))
    return thr


def anneal(Q, *, T_hi: float, T_lo: float, kind: int = SCHED_GEOMETRIC, n_levels: int = 128,
           eoff_inc: int = 0, init: int = INIT_ZEROS, replica_base: int = 0, replicas: int = 1,
           steps: int = 1000, seed: int = 1, trace: bool = False, trial: int = 0) -> dict:
    """Run the oracle DA for `replicas` replicas; returns numpy outputs.  trial = 1:
    single-trial Metropolis (variable s mod N proposes at step s) instead of the
    DA's parallel trial."""
    Q = _q(Q)
    N = Q.shape[0]
    R, S = int(replicas), int(steps)
    out = {
        "best_x": np.zeros((R, N), np.uint8), "best_E": np.zeros(R, np.int64),
        "final_x": np.zeros((R, N), np.uint8), "final_E": np.zeros(R, np.int64),
        "n_accept": np.zeros(R, np.int64),
    }
    tk = tE = to = None
    if trace:
        tk = np.zeros((R, S), np.int32)
        tE = np.zeros((R, S), np.int64)
        to = np.zeros((R, S), np.int64)
    rc = lib().orc_anneal(N, _p(Q), float(T_hi), float(T_lo), int(kind), int(n_levels),
                          int(eoff_inc), int(init), int(trial), int(replica_base), R, S,
                          ctypes.c_uint64(seed),
                          _p(out["best_x"]), _p(out["best_E"]), _p(out["final_x"]),
                          _p(out["final_E"]), _p(out["n_accept"]), _p(tk), _p(tE), _p(to))
    if rc != 0:
        raise ValueError("oracle anneal rejected its arguments")
    if trace:
        out["trace_k"], out["trace_E"], out["trace_eoff"] = tk, tE, to
    return out


def pt(Q, temps, *, chains: int, rounds: int, steps_per_round: int, eoff_inc: int = 0,
       seed: int = 1, chain_base: int = 0, slot_trace: bool = False) -> dict:
    """Parallel tempering of chains chain_base .. chain_base+chains-1 (outputs
    indexed from the first of them).  pair_swaps [chains][M-1] are the accepted
    exchanges per pair; with slot_trace, slot_trace [chains][rounds][M] holds
    every replica's slot after each round's exchange sweep."""
    Q = _q(Q)
    N = Q.shape[0]
    t = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    M = t.shape[0]
    C = int(chains)
    R = M * C
    out = {
        "best_x": np.zeros((R, N), np.uint8), "best_E": np.zeros(R, np.int64),
        "final_x": np.zeros((R, N), np.uint8), "final_E": np.zeros(R, np.int64),
        "n_accept": np.zeros(R, np.int64), "slot": np.zeros(R, np.int32),
        "n_swaps": np.zeros(C, np.int64),
        "pair_swaps": np.zeros((C, max(M - 1, 1)), np.int64),
    }
    tr = np.zeros((C, int(rounds), M), np.int32) if slot_trace else None
    rc = lib().orc_pt_ex(N, _p(Q), _p(t), M, int(chain_base), C, int(rounds),
                         int(steps_per_round), int(eoff_inc), ctypes.c_uint64(seed),
                         _p(out["best_x"]), _p(out["best_E"]), _p(out["final_x"]),
                         _p(out["final_E"]), _p(out["n_accept"]), _p(out["slot"]),
                         _p(out["n_swaps"]), _p(tr), _p(out["pair_swaps"]))
    if rc != 0:
        raise ValueError("oracle pt rejected its arguments")
    out["pair_swaps"] = out["pair_swaps"][:, :max(M - 1, 0)]
    if slot_trace:
        out["slot_trace"] = tr
    return out


_lnU = None


def pt_sweep(E, temps, replica_in_slot, seed: int, chain: int, round_: int):
    """One exchange sweep over the ladder (frozen energies E of the chain's
    replicas); returns (new replica_in_slot, accepted swaps per pair)."""
    global _lnU
    E = np.ascontiguousarray(np.asarray(E, dtype=np.int64))
    t = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    M = t.shape[0]
    if _lnU is None:
        _lnU = np.log((np.arange(65536, dtype=np.float64) + 0.5) / 65536.0)
    lnU = _lnU
    ris = np.ascontiguousarray(np.asarray(replica_in_slot, dtype=np.int32)).copy()
    ps = np.zeros(max(M - 1, 1), np.int64)
    lib().orc_pt_sweep(M, _p(E), _p(t), _p(lnU), _p(ris), ctypes.c_uint64(seed), int(chain),
                       int(round_), _p(ps))
    return ris, ps[:max(M - 1, 0)]


def ladder_update(temps, accepted, proposals: int) -> np.ndarray:
    """One adaptive-ladder update (ends fixed, intervals toward equal acceptance)."""
    t = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    a = np.ascontiguousarray(np.asarray(accepted, dtype=np.int64))
    out = np.zeros_like(t)
    lib().orc_ladder_update(t.shape[0], _p(t), _p(a), int(proposals), _p(out))
    return out


def pt_adapt(Q, temps, *, chains: int, iterations: int, rounds: int, steps_per_round: int,
             eoff_inc: int = 0, seed: int = 1):
    """Adapted ladder and the acceptances [iterations][M-1] measured on the way."""
    Q = _q(Q)
    t = np.ascontiguousarray(np.asarray(temps, dtype=np.float64)).copy()
    M = t.shape[0]
    acc = np.zeros((int(iterations), max(M - 1, 1)))
    rc = lib().orc_pt_adapt(Q.shape[0], _p(Q), _p(t), M, int(chains), int(iterations),
                            int(rounds), int(steps_per_round), int(eoff_inc),
                            ctypes.c_uint64(seed), _p(acc))
    if rc != 0:
        raise ValueError("oracle pt_adapt rejected its arguments")
    return t, acc[:, :max(M - 1, 0)]


class Replica:
    """One oracle replica driven step by step (for invariant tests)."""

    def __init__(self, Q, init: int = INIT_ZEROS, seed: int = 1, r: int = 0):
        self.Q = _q(Q)
        self.N = self.Q.shape[0]
        self.seed, self.r = int(seed), int(r)
        self._h = lib().orc_rep_new(self.N, _p(self.Q), int(init), ctypes.c_uint64(seed), r)
        if not self._h:
            raise MemoryError("oracle replica allocation failed")

    def step(self, thr: np.ndarray, s: int, eoff_inc: int = 0) -> int:
        thr = np.ascontiguousarray(thr, dtype=np.int32)
        return int(lib().orc_rep_step(self._h, _p(thr), ctypes.c_uint64(self.seed), self.r, s,
                                      int(eoff_inc)))

    def read(self) -> dict:
        x = np.zeros(self.N, np.uint8)
        h = np.zeros(self.N, np.int64)
        bx = np.zeros(self.N, np.uint8)
        sc = np.zeros(4, np.int64)
        lib().orc_rep_read(self._h, _p(x), _p(h), _p(bx), _p(sc))
        return {"x": x, "h": h, "best_x": bx, "E": int(sc[0]), "eoff": int(sc[1]),
                "best_E": int(sc[2]), "n_accept": int(sc[3])}

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_rep_free(self._h)
            self._h = None


def bruteforce(Q):
    """Exact (E_min, number of minimisers, one minimiser) for N <= 24."""
    Q = _q(Q)
    N = Q.shape[0]
    e = np.zeros(1, np.int64)
    n = np.zeros(1, np.int64)
    x = np.zeros(N, np.uint8)
    rc = lib().orc_bruteforce(N, _p(Q), _p(e), _p(n), _p(x))
    if rc != 0:
        raise ValueError("bruteforce needs 1 <= N <= 24")
    return int(e[0]), int(n[0]), x
