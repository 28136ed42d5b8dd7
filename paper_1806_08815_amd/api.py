"""Python binding of the C ABI in include/da.h (argument marshalling only).

Every step of the anneal runs in the HIP kernels of ``libdapt.so``; this module
converts numpy arrays and torch device tensors to pointers and back.  It never
computes anything itself and has no fallback: importing it without the built
library raises.  Function names are those of the C ABI.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdapt.so")

DA_OK, DA_EINVAL, DA_ERANGE, DA_ENOMEM, DA_EDEVICE, DA_ENOTREADY, DA_ENOTFOUND = (
    0, -1, -2, -3, -4, -5, -6)
DA_DTYPE_AUTO, DA_DTYPE_I8, DA_DTYPE_I16, DA_DTYPE_I32 = 0, 1, 2, 4
DA_STORE_SPARSE = 0x100
DA_SCHED_GEOMETRIC, DA_SCHED_LINEAR_BETA = 0, 1
DA_INIT_ZEROS, DA_INIT_RANDOM = 0, 1
DA_TRIAL_PARALLEL, DA_TRIAL_SINGLE = 0, 1

_P = ctypes.c_void_p
_i32, _i64, _u64, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double


class DaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class da_schedule(ctypes.Structure):
    _fields_ = [("T_hi", _dbl), ("T_lo", _dbl), ("kind", _i32), ("n_levels", _i32),
                ("eoff_inc", _i32), ("init", _i32), ("trial", _i32), ("reserved", _i32)]


class da_result(ctypes.Structure):
    _fields_ = [("best_x", _P), ("best_E", _P), ("final_x", _P), ("final_E", _P),
                ("n_accept", _P)]


class da_trace(ctypes.Structure):
    _fields_ = [("k", _P), ("E", _P), ("eoff", _P)]


class da_launch(ctypes.Structure):
    _fields_ = [("flips_per_lane", _i32), ("replicas_per_block", _i32), ("w_in_lds", _i32),
                ("rng_waves", _i32), ("draw_estimates", _i32)]


class da_kernel_stats(ctypes.Structure):
    _fields_ = [("kernel_ms", _dbl), ("total_ms", _dbl), ("launches", _i64), ("blocks", _i32),
                ("threads", _i32),
                ("flips_per_lane", _i32), ("replicas_per_block", _i32), ("w_in_lds", _i32),
                ("rng_waves", _i32), ("dtype", _i32), ("draw_estimates", _i32)]


class da_info(ctypes.Structure):
    _fields_ = [("N", _i32), ("ld", _i32), ("dtype", _i32), ("wscale", _i32),
                ("device_bytes", _i64), ("sparse_degree", _i32), ("reserved", _i32)]


class da_batch_item(ctypes.Structure):
    _fields_ = [("ctx", _P), ("schedule", da_schedule), ("replica_base", _i64),
                ("replicas", _i32), ("reserved", _i32), ("steps", _i64), ("seed", _u64),
                ("out_dev", da_result)]


class da_pt_result(ctypes.Structure):
    _fields_ = [("best_x", _P), ("best_E", _P), ("final_x", _P), ("final_E", _P),
                ("n_accept", _P), ("slot", _P), ("n_swaps", _P), ("pair_swaps", _P)]


class da_job(ctypes.Structure):
    _fields_ = [("Q", _P), ("N", _i32), ("dtype_hint", _i32), ("schedule", da_schedule),
                ("replicas", _i32), ("priority", _i32), ("steps", _i64), ("seed", _u64)]


class da_job_stats(ctypes.Structure):
    _fields_ = [("t_submit", _dbl), ("t_admit", _dbl), ("t_done", _dbl),
                ("device_bytes", _i64), ("epochs", _i32), ("preemptions", _i32)]


class da_server_opts(ctypes.Structure):
    _fields_ = [("epoch_steps", _i64), ("max_resident", _i32), ("reserved", _i32)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libdapt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1806_08815_amd.build` (or __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes libdapt.so bind to that one copy instead of a second runtime.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    # a library built from other sources than these is refused, not run
    from . import build as _build
    L.da_build_id.restype = ctypes.c_char_p
    L.da_build_id.argtypes = []
    built, here = L.da_build_id().decode(), _build.source_hash()
    if built != here:
        raise ImportError(f"{LIB_PATH} was built from other sources (build id {built[:12]}, "
                          f"sources {here[:12]}): rebuild it with "
                          "`python -m paper_1806_08815_amd.build`")
    sig = {
        "da_create": (_i32, [_P, _i32, _i32, ctypes.POINTER(_P)]),
        "da_destroy": (None, [_P]),
        "da_get_info": (_i32, [_P, ctypes.POINTER(da_info)]),
        "da_anneal": (_i32, [_P, ctypes.POINTER(da_schedule), _i32, _i64, _u64,
                             ctypes.POINTER(da_result)]),
        "da_anneal_ex": (_i32, [_P, ctypes.POINTER(da_schedule), _i64, _i32, _i64, _u64,
                                ctypes.POINTER(da_launch), ctypes.POINTER(da_result),
                                ctypes.POINTER(da_trace)]),
        "da_anneal_async": (_i32, [_P, ctypes.POINTER(da_schedule), _i64, _i32, _i64, _u64,
                                   ctypes.POINTER(da_launch), ctypes.POINTER(da_result), _P]),
        "da_anneal_batch": (_i32, [ctypes.POINTER(da_batch_item), _i32, _P]),
        "da_pt": (_i32, [_P, _P, _i32, _i32, _i64, _i32, _i32, _u64,
                         ctypes.POINTER(da_pt_result)]),
        "da_energy": (_i32, [_P, _P, _i32, _P]),
        "da_energy_noalloc": (_i32, [_P, _P, _i32, _P, _P]),
        "da_pt_ladder_update": (_i32, [_i32, _P, _P, _i64, _P]),
        "da_pt_adapt": (_i32, [_P, _P, _i32, _i32, _i32, _i64, _i32, _i32, _u64, _P]),
        "da_last_kernel_stats": (_i32, [_P, ctypes.POINTER(da_kernel_stats)]),
        "da_reset_kernel_stats": (_i32, [_P]),
        "da_last_error": (ctypes.c_char_p, [_P]),
        "da_strerror": (ctypes.c_char_p, [_i32]),
        "da_threshold_table": (_i32, [_dbl, _P]),
        "da_level_temperature": (_dbl, [ctypes.POINTER(da_schedule), _i32]),
        "da_server_create": (_i32, [ctypes.c_size_t, ctypes.POINTER(da_server_opts),
                                    ctypes.POINTER(_P)]),
        "da_submit": (_i32, [_P, ctypes.POINTER(da_job), ctypes.POINTER(ctypes.c_uint64)]),
        "da_poll": (_i32, [_P, ctypes.c_uint64, ctypes.POINTER(da_result),
                           ctypes.POINTER(da_job_stats)]),
        "da_wait": (_i32, [_P, ctypes.c_uint64, ctypes.POINTER(da_result),
                           ctypes.POINTER(da_job_stats)]),
        "da_job_footprint": (_i64, [_i32, _i32, _i32, _i32]),
        "da_job_status": (_i32, [_P, ctypes.c_uint64, ctypes.POINTER(_i32),
                                 ctypes.POINTER(_i64)]),
        "da_server_destroy": (None, [_P]),
        "da_probe_row_stream": (_i32, [_i32, _i32, _i32, _i32, _i32, _i64,
                                       ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]),
        "da_anneal_steps": (_i32, [_P, ctypes.POINTER(da_schedule), _i64, _i32, _i64, _i64, _i64,
                                   _u64, ctypes.POINTER(da_result)]),
        "da_state_bytes": (_i64, [_i32, _i32]),
        "da_state_save": (_i32, [_P, _i32, _P, ctypes.c_size_t]),
        "da_state_load": (_i32, [_P, _P, ctypes.c_size_t]),
        "da_probe_fields_mfma": (_i32, [_i32, _i32, _i32, ctypes.POINTER(_dbl),
                                        ctypes.POINTER(_dbl)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int, ctx_ptr=None):
    if rc != DA_OK:
        msg = lib().da_last_error(ctx_ptr)
        raise DaError(rc, msg.decode() if msg else "error")


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(_P)


def schedule(T_hi: float, T_lo: float, kind: str | int = "geometric", n_levels: int = 128,
             eoff_inc: int = 0, init: str | int = "zeros",
             trial: str | int = "parallel") -> da_schedule:
    k = {"geometric": DA_SCHED_GEOMETRIC, "linear_beta": DA_SCHED_LINEAR_BETA}.get(kind, kind)
    i = {"zeros": DA_INIT_ZEROS, "random": DA_INIT_RANDOM}.get(init, init)
    t = {"parallel": DA_TRIAL_PARALLEL, "single": DA_TRIAL_SINGLE}.get(trial, trial)
    return da_schedule(float(T_hi), float(T_lo), int(k), int(n_levels), int(eoff_inc), int(i),
                       int(t), 0)


def launch(flips_per_lane: int = 0, replicas_per_block: int = 0, w_in_lds: int = 0,
           rng_waves: int = 0, draw_estimates: int = 0) -> da_launch:
    return da_launch(int(flips_per_lane), int(replicas_per_block), int(w_in_lds), int(rng_waves),
                     int(draw_estimates))


class Ctx:
    """Owns a da_ctx*."""

    def __init__(self, ptr, N: int):
        self.ptr = ptr
        self.N = N

    @property
    def _as_parameter_(self):
        return self.ptr

    def info(self) -> dict:
        inf = da_info()
        _check(lib().da_get_info(self.ptr, ctypes.byref(inf)), self.ptr)
        return {f: getattr(inf, f) for f, _ in da_info._fields_}

    def close(self):
        if self.ptr:
            lib().da_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def da_create(Q, dtype_hint: int = DA_DTYPE_AUTO) -> Ctx:
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.int32))
    if Q.ndim != 2 or Q.shape[0] != Q.shape[1]:
        raise ValueError("Q must be square")
    out = _P()
    _check(lib().da_create(_ptr(Q), Q.shape[0], int(dtype_hint), ctypes.byref(out)))
    return Ctx(out.value, Q.shape[0])


def da_destroy(ctx: Ctx) -> None:
    ctx.close()


def _host_outputs(R: int, N: int) -> dict:
    return {"best_x": np.zeros((R, N), np.uint8), "best_E": np.zeros(R, np.int64),
            "final_x": np.zeros((R, N), np.uint8), "final_E": np.zeros(R, np.int64),
            "n_accept": np.zeros(R, np.int64)}


def _result_struct(o: dict) -> da_result:
    return da_result(*[_ptr(o.get(k)) for k in ("best_x", "best_E", "final_x", "final_E",
                                                "n_accept")])


def da_anneal(ctx: Ctx, sched: da_schedule, replicas: int, steps: int, seed: int) -> dict:
    out = _host_outputs(int(replicas), ctx.N)
    res = _result_struct(out)
    _check(lib().da_anneal(ctx.ptr, ctypes.byref(sched), int(replicas), int(steps),
                           ctypes.c_uint64(seed), ctypes.byref(res)), ctx.ptr)
    return out


def da_anneal_ex(ctx: Ctx, sched: da_schedule, replica_base: int, replicas: int, steps: int,
                 seed: int, launch_opts: da_launch | None = None, trace: bool = False) -> dict:
    R, S = int(replicas), int(steps)
    out = _host_outputs(R, ctx.N)
    res = _result_struct(out)
    tr = None
    if trace:
        out["trace_k"] = np.zeros((R, S), np.int32)
        out["trace_E"] = np.zeros((R, S), np.int64)
        out["trace_eoff"] = np.zeros((R, S), np.int64)
        tr = da_trace(_ptr(out["trace_k"]), _ptr(out["trace_E"]), _ptr(out["trace_eoff"]))
    _check(lib().da_anneal_ex(ctx.ptr, ctypes.byref(sched), int(replica_base), R, S,
                              ctypes.c_uint64(seed),
                              ctypes.byref(launch_opts) if launch_opts is not None else None,
                              ctypes.byref(res), ctypes.byref(tr) if tr is not None else None),
           ctx.ptr)
    return out


def da_anneal_steps(ctx: Ctx, sched: da_schedule, replica_base: int, replicas: int,
                    total_steps: int, step_begin: int, step_end: int, seed: int) -> dict:
    """Steps [step_begin, step_end) of a total_steps-step anneal (see da.h)."""
    R = int(replicas)
    out = _host_outputs(R, ctx.N)
    res = _result_struct(out)
    _check(lib().da_anneal_steps(ctx.ptr, ctypes.byref(sched), int(replica_base), R,
                                 int(total_steps), int(step_begin), int(step_end),
                                 ctypes.c_uint64(seed), ctypes.byref(res)), ctx.ptr)
    return out


def da_state_bytes(N: int, replicas: int) -> int:
    return int(lib().da_state_bytes(int(N), int(replicas)))


def da_state_save(ctx: Ctx, replicas: int) -> np.ndarray:
    """Snapshot of the first `replicas` replicas of the context's state (uint8 array)."""
    n = da_state_bytes(ctx.N, replicas)
    if n < 0:
        raise DaError(DA_EINVAL, "bad arguments")
    buf = np.zeros(n, np.uint8)
    _check(lib().da_state_save(ctx.ptr, int(replicas), _ptr(buf), n), ctx.ptr)
    return buf


def da_state_load(ctx: Ctx, buf) -> None:
    b = np.ascontiguousarray(np.asarray(buf, dtype=np.uint8))
    _check(lib().da_state_load(ctx.ptr, _ptr(b), b.nbytes), ctx.ptr)


def device_outputs(R: int, N: int, device="cuda"):
    """torch device buffers for da_anneal_async / da_anneal_batch outputs."""
    import torch
    return {"best_x": torch.zeros((R, N), dtype=torch.uint8, device=device),
            "best_E": torch.zeros(R, dtype=torch.int64, device=device),
            "final_x": torch.zeros((R, N), dtype=torch.uint8, device=device),
            "final_E": torch.zeros(R, dtype=torch.int64, device=device),
            "n_accept": torch.zeros(R, dtype=torch.int64, device=device)}


def _dev_result(o: dict | None) -> da_result:
    if o is None:
        return da_result()
    return da_result(*[(o[k].data_ptr() if o.get(k) is not None else None)
                       for k in ("best_x", "best_E", "final_x", "final_E", "n_accept")])


def da_anneal_async(ctx: Ctx, sched: da_schedule, replica_base: int, replicas: int, steps: int,
                    seed: int, launch_opts: da_launch | None, out_dev: dict | None,
                    stream=None) -> None:
    res = _dev_result(out_dev)
    _check(lib().da_anneal_async(ctx.ptr, ctypes.byref(sched), int(replica_base), int(replicas),
                                 int(steps), ctypes.c_uint64(seed),
                                 ctypes.byref(launch_opts) if launch_opts is not None else None,
                                 ctypes.byref(res) if out_dev is not None else None,
                                 _stream_ptr(stream)), ctx.ptr)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def da_anneal_batch(items: list[dict], stream=None) -> None:
    """items: dicts with ctx, schedule, replica_base, replicas, steps, seed, out_dev."""
    arr = (da_batch_item * len(items))()
    for a, it in enumerate(items):
        arr[a] = da_batch_item(it["ctx"].ptr, it["schedule"], int(it.get("replica_base", 0)),
                               int(it["replicas"]), 0, int(it["steps"]),
                               ctypes.c_uint64(it["seed"]).value, _dev_result(it.get("out_dev")))
    _check(lib().da_anneal_batch(arr, len(items), _stream_ptr(stream)))


def da_pt(ctx: Ctx, temps, chains: int, rounds: int, steps_per_round: int, eoff_inc: int,
          seed: int) -> dict:
    t = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    M = t.shape[0]
    R = M * int(chains)
    out = _host_outputs(R, ctx.N)
    out["slot"] = np.zeros(R, np.int32)
    out["n_swaps"] = np.zeros(int(chains), np.int64)
    out["pair_swaps"] = np.zeros((int(chains), max(M - 1, 1)), np.int64)
    res = da_pt_result(*[_ptr(out[k]) for k in ("best_x", "best_E", "final_x", "final_E",
                                                "n_accept", "slot", "n_swaps", "pair_swaps")])
    _check(lib().da_pt(ctx.ptr, _ptr(t), M, int(chains), int(rounds), int(steps_per_round),
                       int(eoff_inc), ctypes.c_uint64(seed), ctypes.byref(res)), ctx.ptr)
    out["pair_swaps"] = out["pair_swaps"][:, :max(M - 1, 0)]
    return out


def da_pt_ladder_update(temps, accepted, proposals: int) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    a = np.ascontiguousarray(np.asarray(accepted, dtype=np.int64))
    out = np.zeros_like(t)
    _check(lib().da_pt_ladder_update(t.shape[0], _ptr(t), _ptr(a), int(proposals), _ptr(out)))
    return out


def da_pt_adapt(ctx: Ctx, temps, chains: int, iterations: int, rounds: int,
                steps_per_round: int, eoff_inc: int, seed: int):
    """(adapted ladder, acceptances [iterations][M-1])."""
    t = np.ascontiguousarray(np.asarray(temps, dtype=np.float64)).copy()
    M = t.shape[0]
    acc = np.zeros((int(iterations), max(M - 1, 1)))
    _check(lib().da_pt_adapt(ctx.ptr, _ptr(t), M, int(chains), int(iterations), int(rounds),
                             int(steps_per_round), int(eoff_inc), ctypes.c_uint64(seed),
                             _ptr(acc)), ctx.ptr)
    return t, acc[:, :max(M - 1, 0)]


def da_energy(ctx: Ctx, x) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    if x.ndim == 1:
        x = x[None, :]
    E = np.zeros(x.shape[0], np.int64)
    _check(lib().da_energy(ctx.ptr, _ptr(x), x.shape[0], _ptr(E)), ctx.ptr)
    return E


def da_energy_noalloc(ctx: Ctx, x_dev, E_dev, stream=None) -> None:
    """Energies of the device states x_dev [count][N] (torch uint8) into E_dev
    [count] (torch int64), enqueued on `stream`; allocates nothing."""
    count = int(x_dev.shape[0])
    assert x_dev.dtype.itemsize == 1 and x_dev.is_contiguous() and x_dev.shape[1] == ctx.N
    assert E_dev.dtype.itemsize == 8 and E_dev.is_contiguous() and E_dev.shape[0] >= count
    _check(lib().da_energy_noalloc(ctx.ptr, x_dev.data_ptr(), count, E_dev.data_ptr(),
                                   _stream_ptr(stream)), ctx.ptr)


def da_last_kernel_stats(ctx: Ctx) -> dict:
    st = da_kernel_stats()
    _check(lib().da_last_kernel_stats(ctx.ptr, ctypes.byref(st)), ctx.ptr)
    return {f: getattr(st, f) for f, _ in da_kernel_stats._fields_}


def da_reset_kernel_stats(ctx: Ctx) -> None:
    _check(lib().da_reset_kernel_stats(ctx.ptr), ctx.ptr)


def da_threshold_table(T: float) -> np.ndarray:
    thr = np.zeros(65536, np.int32)
    _check(lib().da_threshold_table(float(T), _ptr(thr)))
    return thr


def da_level_temperature(sched: da_schedule, level: int) -> float:
    return float(lib().da_level_temperature(ctypes.byref(sched), int(level)))


def da_strerror(code: int) -> str:
    return lib().da_strerror(int(code)).decode()


def da_probe_row_stream(n_rows: int, row_elems: int, dtype_bytes: int, chains: int,
                        waves_per_chain: int, steps: int) -> dict:
    ns = _dbl()
    gbs = _dbl()
    _check(lib().da_probe_row_stream(int(n_rows), int(row_elems), int(dtype_bytes), int(chains),
                                     int(waves_per_chain), int(steps), ctypes.byref(ns),
                                     ctypes.byref(gbs)))
    return {"ns_per_step": ns.value, "GBps": gbs.value}


def da_probe_fields_mfma(N: int, R: int, iters: int) -> dict:
    ms = _dbl()
    tops = _dbl()
    _check(lib().da_probe_fields_mfma(int(N), int(R), int(iters), ctypes.byref(ms),
                                      ctypes.byref(tops)))
    return {"ms_per_call": ms.value, "tera_ops": tops.value}


# ---- server -----------------------------------------------------------------
class Server:
    def __init__(self, ptr):
        self.ptr = ptr
        self._jobs = {}

    def close(self):
        if self.ptr:
            lib().da_server_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def da_server_create(hbm_budget: int, epoch_steps: int = 0, max_resident: int = 0) -> Server:
    out = _P()
    opts = da_server_opts(int(epoch_steps), int(max_resident), 0)
    _check(lib().da_server_create(int(hbm_budget), ctypes.byref(opts), ctypes.byref(out)))
    return Server(out.value)


def da_submit(srv: Server, Q, sched: da_schedule, replicas: int, steps: int, seed: int,
              dtype_hint: int = DA_DTYPE_AUTO, priority: int = 0) -> int:
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.int32))
    job = da_job(_ptr(Q), Q.shape[0], int(dtype_hint), sched, int(replicas), int(priority),
                 int(steps), ctypes.c_uint64(seed).value)
    t = ctypes.c_uint64()
    _check(lib().da_submit(srv.ptr, ctypes.byref(job), ctypes.byref(t)))
    srv._jobs[t.value] = (int(replicas), Q.shape[0])
    return t.value


def _collect(fn, srv: Server, ticket: int):
    if ticket not in srv._jobs:   # unknown here: let the library report it
        _check(fn(srv.ptr, ctypes.c_uint64(ticket), None, None))
    R, N = srv._jobs[ticket]
    out = _host_outputs(R, N)
    res = _result_struct(out)
    st = da_job_stats()
    rc = fn(srv.ptr, ctypes.c_uint64(ticket), ctypes.byref(res), ctypes.byref(st))
    if rc == DA_ENOTREADY:
        return None
    _check(rc)
    del srv._jobs[ticket]
    out["stats"] = {f: getattr(st, f) for f, _ in da_job_stats._fields_}
    return out


def da_poll(srv: Server, ticket: int):
    """Outputs of a finished job, or None while it runs."""
    return _collect(lib().da_poll, srv, ticket)


def da_wait(srv: Server, ticket: int) -> dict:
    return _collect(lib().da_wait, srv, ticket)


def da_job_status(srv: Server, ticket: int) -> tuple[int, int]:
    """(state, done_steps): state 0 waiting, 1 resident, 2 finished."""
    st = _i32()
    done = _i64()
    _check(lib().da_job_status(srv.ptr, ctypes.c_uint64(ticket), ctypes.byref(st),
                               ctypes.byref(done)))
    return int(st.value), int(done.value)


def da_job_footprint(N: int, dtype_bytes: int, replicas: int, n_levels: int) -> int:
    return int(lib().da_job_footprint(int(N), int(dtype_bytes), int(replicas), int(n_levels)))


def da_server_destroy(srv: Server) -> None:
    srv.close()
