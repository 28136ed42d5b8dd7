#!/usr/bin/env python3
"""Benchmark of the Digital Annealer parallel-trial step on one MI355X.

One "step" of this benchmark is one whole anneal of the headline workload --
the fully connected Gaussian SK instance, N = 1024, 1024 replicas x 10^5
Monte Carlo steps (Algorithm 2 of arXiv:1806.08815) in one persistent launch
of the HIP step kernel, from the common zero state.  Inputs (coupling matrix,
tables, state buffers) are resident in HBM before timing starts; the timed
region covers K anneals bracketed by device synchronisation.

Prints ONE JSON line:
  value        flip evaluations per second = replicas * MC steps * N * K / time
  roofline     row-stream bytes of the step kernel (accepted steps * N * bytes
               per coupling) / its event-timed duration, against the
               achievable rate of the same access pattern (a dependent random
               row gather at the same chain count, measured in the same run),
               with the HBM fraction beside it
  cpu_baseline the CPU oracle on 8 spread replicas of the same workload
Side legs (skipped with --skip-extras): the N = 64 SK workload (ns per step),
the 2D torus batched against per-replica launches, TTS99 measured the paper's
way (Sec. IV) against an independent parallel-tempering reference energy,
parallel tempering at full size, ladder adaptation, the served request stream
(p50/p99 latency, alone-vs-mix identity of every job), checkpointing, per-step
schedules, the matrix-core initial fields and the sparse-row density sweep.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "parallel-trial flip evaluations/s; TTS99 at 1 GPU; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
KEYS = ("best_x", "best_E", "final_x", "final_E", "n_accept")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


KERNEL_SOURCES = ("paper_1806_08815_amd/csrc/da_kernels.hip", "paper_1806_08815_amd/csrc/da_internal.h")


def measured_traffic(workload: str, launch: dict):
    """HBM bytes per launch of the step kernel from the committed memory-counter
    summary of this workload, or None when the kernel source or the launch
    shape differs from the one the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_k_run_{workload}.md")
    try:
        with open(path) as f:
            recs = [json.loads(l.split(":", 1)[1]) for l in f if l.startswith("machine-readable:")]
    except OSError:
        return None
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    # one record per launch shape the counters were taken on
    for rec in recs:
        if rec.get("kernel_source_sha256") != h.hexdigest():
            continue
        if any(launch.get(k) != v for k, v in rec["launch"].items()):
            continue
        return float(rec["traffic_bytes_per_launch"])
    return None


def describe(w):
    return (f"{w.name}: {w.kind} N={w.N}, {w.replicas} replicas x {w.steps} MC steps, "
            f"{w.schedule} T {w.T_hi:g}->{w.T_lo:g} ({w.n_levels} levels), "
            f"E_off increment {w.eoff_inc}, {w.init} start, Philox seed {w.seed}")


def sched_of(api, w, kind=None, n_levels=None):
    return api.schedule(w.T_hi, w.T_lo, w.schedule if kind is None else kind,
                        w.n_levels if n_levels is None else n_levels, w.eoff_inc, w.init)


def oracle_replicas(oracle, Q, w, rows, threads):
    """The oracle on the given replicas of a workload, one replica per thread
    (the C loop releases the interpreter lock); returns (outputs by row, wall
    seconds, per-replica seconds)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(r):
        t = time.perf_counter()
        o = oracle.anneal(Q, T_hi=w.T_hi, T_lo=w.T_lo,
                          kind=0 if w.schedule == "geometric" else 1,
                          n_levels=w.n_levels, eoff_inc=w.eoff_inc,
                          init=0 if w.init == "zeros" else 1, replicas=1, replica_base=r,
                          steps=w.steps, seed=w.seed)
        return o, time.perf_counter() - t

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        outs = list(ex.map(one, rows))
    return {r: o for r, (o, _) in zip(rows, outs)}, time.perf_counter() - t0, \
        [dt for _, dt in outs]


def same_rows(gpu: dict, ref: dict) -> bool:
    """Every output of the oracle's replicas (ref: row -> one-replica outputs)
    equals the GPU's row."""
    import numpy as np
    return all(np.array_equal(ref[r][k][0], gpu[k][r]) for r in ref for k in KEYS)


def to_host(out: dict) -> dict:
    return {k: out[k].cpu().numpy() for k in KEYS}


def row_stream_peak(api, N, dtype, chains):
    """Achievable rate of the step's access pattern: `chains` dependent chains
    each fetching one random row of an N x N matrix of this element type per
    step (no flip work), with the step kernel's waves per chain."""
    waves = max(1, -(-N // 512))
    return api.da_probe_row_stream(N, N, dtype, chains, waves, 20_000)


def anneal_timed(api, ctx, sch, R, S, seed, out, stream, launch=None, reps=1):
    """Kernel time of `reps` anneals (HIP events on the launch stream) and wall time."""
    import torch
    api.da_reset_kernel_stats(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        api.da_anneal_async(ctx, sch, 0, R, S, seed, launch, out, stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    ks = api.da_last_kernel_stats(ctx)
    return ks, ks["total_ms"] / 1e3 / ks["launches"], wall


# --------------------------------------------------------------------------
# side legs
# --------------------------------------------------------------------------

def small_sk_leg(api, oracle, workloads):
    """The N = 64 +-1 SK workload: 16 replicas x 10^4 steps, W in LDS; a chain of
    10^4 dependent steps per replica, so it is latency-bound: ns per step."""
    import torch
    w = workloads.WORKLOADS["sk-bimodal-64"]
    Q, _ = w.instance()
    ctx = api.da_create(Q)
    sch = sched_of(api, w)
    out = api.device_outputs(w.replicas, w.N)
    stream = torch.cuda.current_stream()
    api.da_anneal_async(ctx, sch, 0, w.replicas, w.steps, w.seed, None, out, stream)
    ks, kern, wall = anneal_timed(api, ctx, sch, w.replicas, w.steps, w.seed, out, stream, reps=5)
    gpu = to_host(out)
    rows = list(range(w.replicas))
    ref, t_cpu, per = oracle_replicas(oracle, Q, w, rows, min(16, os.cpu_count() or 1))
    return {
        "workload": describe(w), "kernel_ms": kern * 1e3, "ns_per_mc_step": kern / w.steps * 1e9,
        "wall_ms_per_anneal": wall * 1e3,
        "flip_evals_per_s": w.replicas * w.steps * w.N / wall,
        "launch": {k: ks[k] for k in ("blocks", "threads", "flips_per_lane",
                                      "replicas_per_block", "w_in_lds", "rng_waves",
                                      "draw_estimates")},
        "oracle_all_replicas_equal": same_rows(gpu, ref),
        "oracle_single_core_flip_evals_per_s": w.steps * w.N / (sum(per) / len(per)),
    }


def torus_leg(api, workloads):
    """The 2D torus (+-1, N = 1024, dense int16): one batched launch of 128
    replicas against 128 one-replica launches on the same stream."""
    import torch
    w = workloads.WORKLOADS["torus2d-bimodal-1024"]
    Q, _ = w.instance()
    ctx = api.da_create(Q, w.dtype_hint)
    info = ctx.info()
    sch = sched_of(api, w)
    R, S, N = w.replicas, w.steps, w.N
    out = api.device_outputs(R, N)
    stream = torch.cuda.current_stream()
    api.da_anneal_async(ctx, sch, 0, R, S, w.seed, None, out, stream)
    ks, kern, wall = anneal_timed(api, ctx, sch, R, S, w.seed, out, stream, reps=3)
    n_acc = out["n_accept"].cpu().numpy()
    row_bytes = float(n_acc.sum()) * N * info["dtype"]
    peak = row_stream_peak(api, N, info["dtype"], R)
    achieved = row_bytes / kern / 1e9
    one = api.device_outputs(1, N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(R):
        api.da_anneal_async(ctx, sch, r, 1, S, w.seed, None, one, stream)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    return {
        "workload": describe(w),
        "batched": {"seconds": wall, "flip_evals_per_s": R * S * N / wall, "kernel_ms": kern * 1e3,
                    "ns_per_mc_step": kern / S * 1e9,
                    "launch": {k: ks[k] for k in ("blocks", "threads", "flips_per_lane",
                                                  "replicas_per_block", "rng_waves")}},
        "plain": {"form": f"{R} launches of 1 replica each", "seconds": t_plain,
                  "flip_evals_per_s": R * S * N / t_plain},
        "batched_speedup": t_plain / wall,
        "same_result_as_batched": int(one["best_E"][0].item()) == int(out["best_E"][R - 1].item()),
        "row_stream": {"achieved_GBps": achieved, "achievable_GBps_at_128_chains": peak["GBps"],
                       "frac": achieved / peak["GBps"],
                       "dependent_fetch_ns": peak["ns_per_step"],
                       "fetch_over_step": peak["ns_per_step"] / (kern / S * 1e9)},
        "out": to_host(out), "ctx": ctx, "sched": sch, "Q": Q, "w": w,
    }


def pt_reference(api, Q, temps, chains, rounds, K, seed):
    """Best energy of an independent parallel-tempering run (an upper bound on
    the optimum, used as the TTS reference instead of the runs it scores)."""
    ctx = api.da_create(Q)
    t0 = time.perf_counter()
    o = api.da_pt(ctx, temps, chains, rounds, K, 0, seed)
    dt = time.perf_counter() - t0
    ctx.close()
    return int(o["best_E"].min()), dt


def tts_leg(api, tts, ctx, sch, w, best_E, E_ref, E_ref_kind, const, cap=32768):
    """TTS99 the paper's way for the DA (Sec. IV): the wall time of one launch
    with ceil(R99) replicas, R99 from the Jeffreys posterior median of the
    success probability; beside it the plain per-instance form tau * R99, tau
    the wall time of a one-replica launch.  Launches above `cap` replicas are
    timed at `cap` and scaled (flagged)."""
    import torch
    N, S = w.N, w.steps
    stream = torch.cuda.current_stream()
    y = tts.success_count(best_E, E_ref)
    runs = len(best_E)

    def time_launch(reps):
        reps_t = min(reps, cap)
        o = api.device_outputs(reps_t, N)
        api.da_anneal_async(ctx, sch, 0, reps_t, S, w.seed, None, o, stream)   # tuner, warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        api.da_anneal_async(ctx, sch, 0, reps_t, S, w.seed, None, o, stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * reps / reps_t

    t99 = tts.tts99_measured(y, runs, time_launch)
    one = api.device_outputs(1, N)
    api.da_anneal_async(ctx, sch, 0, 1, S, w.seed, None, one, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(3):
        api.da_anneal_async(ctx, sch, r, 1, S, w.seed, None, one, stream)
        torch.cuda.synchronize()
    tau = (time.perf_counter() - t0) / 3
    r99 = t99["r99"]
    return {
        "E_ref": E_ref + int(const), "E_ref_kind": E_ref_kind,
        "best_of_runs": int(min(best_E)) + int(const),
        "successes": y, "runs": runs, "theta_median": t99["theta"], "r99": r99,
        "batched": {"replicas_launched": t99["replicas"], "seconds": t99["tts_s"],
                    "timed_at_cap": bool(t99["replicas"] and t99["replicas"] > cap)},
        "plain": {"tau_one_replica_s": tau,
                  "seconds": tau * r99 if math.isfinite(r99) else math.inf},
        "batched_speedup_over_plain": (tau * r99 / t99["tts_s"]) if math.isfinite(r99) else None,
    }


def pt_leg(api, workloads, rounds: int):
    """Parallel tempering at the full ladder and chain count (32 temperatures x
    64 chains of the N = 1024 +-1 SK instance, 1024 steps per round)."""
    import numpy as np
    p = workloads.PT_WORKLOAD
    Q, _ = workloads.make_instance(p["kind"], p["N"], p["instance_seed"])
    temps = workloads.pt_temperatures(p["M"], p["T_lo"], p["T_hi"], p["temp_scale"])
    ctx = api.da_create(Q)
    api.da_pt(ctx, temps, p["chains"], 2, p["steps_per_round"], p["eoff_inc"], p["seed"])
    api.da_reset_kernel_stats(ctx)
    t0 = time.perf_counter()
    out = api.da_pt(ctx, temps, p["chains"], rounds, p["steps_per_round"], p["eoff_inc"],
                    p["seed"])
    dt = time.perf_counter() - t0
    ks = api.da_last_kernel_stats(ctx)
    R = p["M"] * p["chains"]
    steps = rounds * p["steps_per_round"]
    fe = R * steps * p["N"]
    acc = float(out["n_accept"].sum()) / (R * steps)
    pair = out["pair_swaps"].sum(axis=0) / (p["chains"] * rounds)
    dtype = ctx.info()["dtype"]
    stream_gbps = acc * R * steps * p["N"] * dtype / (ks["kernel_ms"] / 1e3) / 1e9
    # the same gather at the same chain count: rows of N * dtype bytes (int8 rows
    # are probed as int16 rows of half the elements, the same bytes)
    elems = p["N"] * dtype // 2
    probe = api.da_probe_row_stream(p["N"], elems, 2, R, max(1, -(-p["N"] // 512)), 20_000)
    return {
        "workload": f"{p['name']}: {p['kind']} N={p['N']}, {p['chains']} chains x M={p['M']} "
                    f"temperatures, K={p['steps_per_round']} steps per round, random start",
        "rounds": rounds, "rounds_full": p["rounds"], "seconds": dt,
        "flip_evals_per_s": fe / dt, "ns_per_round_step": ks["kernel_ms"] / steps * 1e6,
        "accepted_step_fraction": acc,
        "row_stream_GBps": stream_gbps,
        "row_stream_achievable_GBps": probe["GBps"],
        "row_stream_frac": stream_gbps / probe["GBps"],
        "hbm_frac": stream_gbps / HBM_PEAK_GBS,
        "exchange_decisions": int(rounds * p["chains"] * (p["M"] - 1)),
        "swaps_accepted": int(np.asarray(out["n_swaps"]).sum()),
        "pair_acceptance_min_max": [float(pair.min()), float(pair.max())],
        "best_E": int(out["best_E"].min()),
    }


def ladder_leg(api, workloads, iterations=6, rounds=40):
    """The adaptive ladder (Sec. II.D) on the PT workload's instance: the
    spread of the adjacent-pair exchange acceptances before and after."""
    p = workloads.PT_WORKLOAD
    Q, _ = workloads.make_instance(p["kind"], p["N"], p["instance_seed"])
    temps = workloads.pt_temperatures(p["M"], p["T_lo"], p["T_hi"], p["temp_scale"])
    ctx = api.da_create(Q)
    t0 = time.perf_counter()
    adapted, acc = api.da_pt_adapt(ctx, temps, p["chains"], iterations, rounds,
                                   p["steps_per_round"], p["eoff_inc"], p["seed"])
    dt = time.perf_counter() - t0
    return {"iterations": iterations, "rounds_per_iteration": rounds, "seconds": dt,
            "acceptance_first": [float(a) for a in acc[0]],
            "acceptance_last": [float(a) for a in acc[-1]],
            "spread_first": float(acc[0].max() - acc[0].min()),
            "spread_last": float(acc[-1].max() - acc[-1].min()),
            "ladder": [float(t) for t in adapted]}


def sparse_sweep_leg(api, R=128, S=20_000):
    """Step time of dense rows vs sparse row lists over coupling density (the
    paper's density study, Sec. VI.C, at N = 1024), and on a large 2D torus."""
    import torch
    from paper_1806_08815_amd import instances
    cases = [("torus L=32", instances.torus2d(32, 1, "bimodal"))]
    for p in (0.01, 0.02, 0.05, 0.1, 0.2, 0.5):
        cases.append((f"G(1024, {p})", instances.erdos_renyi(1024, p, 1)))
    cases.append(("torus L=90 (N=8100)", instances.torus2d(90, 1, "bimodal")))
    out = []
    stream = torch.cuda.current_stream()
    for name, J in cases:
        Q = instances.ising_to_qubo(J)[0]
        N = Q.shape[0]
        deg = float((J != 0).sum(axis=1).mean())
        T_hi = 3.0 * max(1.0, deg ** 0.5)
        sch = api.schedule(T_hi, 0.05 * T_hi, "geometric", 128, 1)
        row = {"instance": name, "N": N, "mean_degree": deg}
        same = []
        for label, hint in (("dense", 0), ("sparse", api.DA_STORE_SPARSE)):
            try:
                ctx = api.da_create(Q, hint)
            except api.DaError as e:
                row[label] = str(e)
                continue
            o = api.device_outputs(R, N)
            api.da_anneal_async(ctx, sch, 0, R, S, 1, None, o, stream)
            torch.cuda.synchronize()
            api.da_reset_kernel_stats(ctx)
            api.da_anneal_async(ctx, sch, 0, R, S, 1, None, o, stream)
            torch.cuda.synchronize()
            ks = api.da_last_kernel_stats(ctx)
            row[label] = {"ns_per_step": ks["kernel_ms"] / S * 1e6,
                          "row_list_in_lds": bool(ks["w_in_lds"]) if label == "sparse" else None,
                          "degree_slots": ctx.info()["sparse_degree"]}
            same.append(o["best_E"].cpu().numpy().tolist())
            ctx.close()
        row["sparse_equals_dense"] = len(same) == 2 and same[0] == same[1]
        out.append(row)
    return out


def checkpoint_leg(api, w, cut_frac: float = 0.5):
    """Stop an anneal part-way, snapshot it to host memory, resume in a fresh
    context, and compare with the uninterrupted run."""
    import numpy as np
    Q, _ = w.instance()
    sch = sched_of(api, w)
    R, S = w.replicas, w.steps
    cut = int(S * cut_frac)
    a = api.da_create(Q, w.dtype_hint)
    whole = api.da_anneal_ex(a, sch, 0, R, S, w.seed)
    api.da_anneal_steps(a, sch, 0, R, S, 0, cut, w.seed)
    t0 = time.perf_counter()
    snap = api.da_state_save(a, R)
    t_save = time.perf_counter() - t0
    a.close()
    b = api.da_create(Q, w.dtype_hint)
    t0 = time.perf_counter()
    api.da_state_load(b, snap)
    t_load = time.perf_counter() - t0
    rest = api.da_anneal_steps(b, sch, 0, R, S, cut, S, w.seed)
    same = all(np.array_equal(rest[k], whole[k]) for k in KEYS)
    return {"workload": w.name, "cut_step": cut, "snapshot_bytes": int(snap.nbytes),
            "save_ms": t_save * 1e3, "load_ms": t_load * 1e3, "resumed_equals_whole": bool(same)}


def per_step_leg(api, w, S=100_000):
    """The workload with the paper's DA setting: linear in 1/T, a new temperature
    every step (App. A)."""
    import torch
    Q, _ = w.instance()
    ctx = api.da_create(Q, w.dtype_hint)
    sch = sched_of(api, w, kind="linear_beta", n_levels=0)
    out = api.device_outputs(w.replicas, w.N)
    stream = torch.cuda.current_stream()
    api.da_anneal_async(ctx, sch, 0, w.replicas, S, w.seed, None, out, stream)
    ks, kern, wall = anneal_timed(api, ctx, sch, w.replicas, S, w.seed, out, stream)
    return {"workload": w.name, "schedule": "linear_beta, a new temperature every step",
            "mc_steps": S, "flip_evals_per_s": w.replicas * S * w.N / wall,
            "ns_per_mc_step": kern / S * 1e9}


def serve_bench(api, workloads, n_jobs: int, seed: int, budget_gb: float, epoch_steps: int,
                steps_range=(10_000, 100_000)):
    """Served stream against plain service of the same jobs.

    A job's latency runs from the moment it arrives with its Q on the host to
    the moment its results are on the host.  Served: every job goes through
    the continuous-batching server (da_submit / da_wait).  Plain: one
    da_create + da_anneal (one launch) + free per job, first come first
    served; its latencies under the same arrivals follow from the measured
    service times.  Every served job's outputs are compared with the same job
    run alone (the plain service run)."""
    import numpy as np
    import torch

    jobs = workloads.serve_stream(n_jobs, seed, rate_hz=1.0, steps_range=steps_range)
    Qs = [workloads.make_instance(j["kind"], j["N"], j["instance_seed"])[0] for j in jobs]
    scheds = [api.schedule(j["T_hi"], j["T_lo"], "geometric", 128, j["eoff_inc"]) for j in jobs]
    work = float(sum(j["replicas"] * j["steps"] * j["N"] for j in jobs))

    def plain(j, Q, sch, steps):
        t = time.perf_counter()
        ctx = api.da_create(Q)
        o = api.da_anneal(ctx, sch, j["replicas"], steps, j["seed"])
        ctx.close()
        return time.perf_counter() - t, o

    # the launch-shape tuner runs once per (N, coupling type, replica-count
    # bucket): let it run here, untimed, for every combination in the stream
    seen = set()
    for j, Q, sch in zip(jobs, Qs, scheds):
        key = (j["N"], j["kind"], 1 << (int(j["replicas"]) - 1).bit_length())
        if key not in seen:
            seen.add(key)
            plain(j, Q, sch, min(j["steps"], 1000))
    torch.cuda.synchronize()
    service, alone = [], []
    for j, Q, sch in zip(jobs, Qs, scheds):
        dt, o = plain(j, Q, sch, j["steps"])
        service.append(dt)
        alone.append(o)
    busy = sum(service)
    log(f"serve: plain service of {n_jobs} jobs {busy:.1f} s")

    def run_stream(arrivals):
        srv = api.da_server_create(int(budget_gb * 2**30), epoch_steps=epoch_steps)
        t0 = time.perf_counter()
        tickets, late = [], []
        for j, Q, sch, ta in zip(jobs, Qs, scheds, arrivals):
            delay = ta - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            late.append(max(0.0, (time.perf_counter() - t0) - ta))
            tickets.append(api.da_submit(srv, Q, sch, j["replicas"], j["steps"], j["seed"]))
        outs = [api.da_wait(srv, t) for t in tickets]
        makespan = time.perf_counter() - t0
        srv.close()
        # submission can lag the arrival (the submitting thread was busy): count it
        lat = np.array([o["stats"]["t_done"] - o["stats"]["t_submit"] + lt
                        for o, lt in zip(outs, late)])
        return outs, lat, makespan

    outs0, _, makespan0 = run_stream([0.0] * n_jobs)
    same = [all(np.array_equal(o[k], a[k]) for k in KEYS) for o, a in zip(outs0, alone)]
    log(f"serve: capacity run {makespan0:.1f} s, {sum(same)}/{n_jobs} jobs equal alone")

    def at_rate(rate):
        g = np.random.Generator(np.random.PCG64(seed + 1))
        arrivals = list(np.cumsum(g.exponential(1.0 / rate, size=n_jobs)))
        outs, lat, _ = run_stream(arrivals)
        t_free, plain_lat = 0.0, []
        for ta, sv in zip(arrivals, service):
            start = max(ta, t_free)
            t_free = start + sv
            plain_lat.append(t_free - ta)
        pct = lambda v, q: float(np.percentile(v, q))
        eq = sum(all(np.array_equal(o[k], a[k]) for k in KEYS) for o, a in zip(outs, alone))
        return {"arrival_rate_jobs_per_s": rate,
                "served_p50_s": pct(lat, 50), "served_p99_s": pct(lat, 99),
                "plain_p50_s": pct(plain_lat, 50), "plain_p99_s": pct(plain_lat, 99),
                "jobs_equal_alone": int(eq)}

    r_served = at_rate(0.8 * n_jobs / makespan0)
    log(f"serve: at 80% of served capacity {json.dumps(r_served)}")
    r_plain = at_rate(0.8 * n_jobs / busy)
    return {
        "jobs": n_jobs,
        "sizes": sorted({j["N"] for j in jobs}),
        "replicas_range": [min(j["replicas"] for j in jobs), max(j["replicas"] for j in jobs)],
        "steps_range": [min(j["steps"] for j in jobs), max(j["steps"] for j in jobs)],
        "flip_evals": work,
        "served_capacity_jobs_per_s": n_jobs / makespan0,
        "plain_capacity_jobs_per_s": n_jobs / busy,
        "served_flip_evals_per_s": work / makespan0,
        "plain_flip_evals_per_s": work / busy,
        "jobs_equal_alone_in_mix": int(sum(same)),
        "latency_at_80pct_of_served_capacity": r_served,
        "latency_at_80pct_of_plain_capacity": r_plain,
        "epoch_steps": epoch_steps, "budget_gb": budget_gb,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sk-gaussian-1024")
    ap.add_argument("--dtype", type=int, default=None, help="force coupling storage bytes")
    ap.add_argument("--launch", default=None,
                    help="fixed step-kernel shape F:RPW:RNG[:EST] (flips per lane, replicas per "
                         "workgroup, random-number waves: 1 on, -1 off, per-draw estimates: 1 "
                         "on, -1 off) instead of the tuned one")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-extras", action="store_true")
    ap.add_argument("--legs", default="small,torus,tts,pt,ladder,serve,checkpoint,perstep,mfma,sparse",
                    help="side legs to run (comma separated)")
    ap.add_argument("--serve-jobs", type=int, default=256)
    ap.add_argument("--pt-rounds", type=int, default=10_000)
    ap.add_argument("--ref-rounds", type=int, default=1500,
                    help="rounds of the parallel-tempering runs that set the TTS reference energies")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, one plain device copy of this many MiB "
                         "(the known-size reference for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(replicas would shard across GPUs with no per-step communication; that path is "
              "designed, not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1806_08815_amd import api, tts, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = workloads.WORKLOADS[args.workload]
    Q, const = w.instance()
    N, R, S = w.N, w.replicas, w.steps
    dtype_hint = args.dtype if args.dtype is not None else w.dtype_hint
    ctx = api.da_create(Q, dtype_hint)
    info = ctx.info()
    sch = sched_of(api, w)
    stream = torch.cuda.current_stream()
    out = api.device_outputs(R, N)

    fixed = None
    if args.launch:
        parts = [int(v) for v in args.launch.split(":")]
        F_, rpw_, rng_ = parts[:3]
        est_ = parts[3] if len(parts) > 3 else 0
        fixed = api.launch(F_, rpw_, 0, rng_, est_)

    def anneal():
        api.da_anneal_async(ctx, sch, 0, R, S, w.seed, fixed, out, stream)

    log(f"{describe(w)}; storage int{8 * info['dtype']} x{info['wscale']}")
    for _ in range(args.warmup):
        anneal()
    torch.cuda.synchronize()
    api.da_reset_kernel_stats(ctx)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        anneal()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ks = api.da_last_kernel_stats(ctx)
    kernel_s = ks["total_ms"] / 1e3 / ks["launches"]
    gpu = to_host(out)
    n_acc = gpu["n_accept"]
    flip_evals = float(R) * S * N * args.steps
    value = flip_evals / elapsed
    row_bytes = float(n_acc.sum()) * N * info["dtype"]
    achieved = row_bytes / kernel_s / 1e9
    log(f"{args.steps} anneals in {elapsed:.3f} s; step kernel {kernel_s * 1e3:.3f} ms per launch; "
        f"{value:.4g} flip-evals/s; {achieved:.1f} GB/s row stream")

    # the achievable rate of the same access pattern at the same chain count
    peak = row_stream_peak(api, N, info["dtype"], R) if info["dtype"] in (2, 4) else None
    launch = {k: ks[k] for k in ("blocks", "threads", "flips_per_lane", "replicas_per_block",
                                 "w_in_lds", "rng_waves", "draw_estimates")}
    traffic = measured_traffic(args.workload, launch)
    ns_step = kernel_s / S * 1e9
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "flip-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": describe(w),
            "N": N, "replicas": R, "mc_steps": S,
            "coupling_storage": f"int{8 * info['dtype']}",
            "wscale": info["wscale"],
            "launch": launch,
        },
        "roofline": {
            "bound": "l2",
            "achieved": achieved,
            "peak": peak["GBps"] if peak else None,
            "unit": "GB/s",
            "frac": achieved / peak["GBps"] if peak else None,
            "traffic": traffic,
            "peak_kind": (f"measured in this run: {R} dependent chains, one random row of the "
                          f"same {N} x {N} int{8 * info['dtype']} matrix per chain per step "
                          "(the step kernel's access pattern without its flip work; the matrix "
                          "is L2-resident)"),
            "hbm_peak": HBM_PEAK_GBS,
            "hbm_frac": achieved / HBM_PEAK_GBS,
            "kernel": "k_run (step kernel)",
            "kernel_ms": kernel_s * 1e3,
            "bytes_per_launch": row_bytes,
            "accepted_step_fraction": float(n_acc.sum()) / (R * S),
            "ns_per_mc_step": ns_step,
            "dependent_fetch_ns": peak["ns_per_step"] if peak else None,
            "fetch_over_step": (peak["ns_per_step"] / ns_step) if peak else None,
        },
    }

    if args.copy_probe_mb > 0:
        nbytes = args.copy_probe_mb << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if not args.skip_cpu:
        import oracle
        model, ncpu = cpu_info()
        rows = sorted({int(round(q)) for q in np.linspace(0, R - 1, 8)})
        threads = max(1, min(ncpu or 1, len(rows)))
        ref, t_all, per = oracle_replicas(oracle, Q, w, rows, threads)
        result["cpu_baseline"] = {
            "value": len(rows) * S * N / t_all,
            "unit": "flip-evals/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"replicas {rows} of {R} (spread over the launch), all {S} MC steps of "
                      f"the same schedule, one replica per thread on {threads} threads, "
                      f"{t_all:.1f} s wall on {model} ({ncpu} host CPUs)",
            "single_core": {"value": S * N / (sum(per) / len(per)),
                            "seconds_per_replica": sum(per) / len(per)},
            "matches_gpu_replicas": bool(same_rows(gpu, ref)),
        }
        log(f"oracle: {len(rows)} replicas on {threads} threads {t_all:.1f} s, parity with GPU: "
            f"{result['cpu_baseline']['matches_gpu_replicas']}")

    legs = set() if args.skip_extras else set(args.legs.split(","))
    if "small" in legs:
        import oracle
        result["sk_bimodal_64"] = small_sk_leg(api, oracle, workloads)
        log(f"N=64 leg: {json.dumps(result['sk_bimodal_64'])}")
    torus = None
    if "torus" in legs or "tts" in legs:
        torus = torus_leg(api, workloads)
        result["torus2d_bimodal_1024"] = {k: v for k, v in torus.items()
                                          if k not in ("out", "ctx", "sched", "Q", "w")}
        log(f"torus leg: {json.dumps(result['torus2d_bimodal_1024'])}")
    if "tts" in legs:
        p = workloads.PT_WORKLOAD
        tt = {}
        # 2D torus: ladder over the annealing range in units of J
        tq = workloads.pt_temperatures(32, 0.1, 3.0, 1.0)
        E_t, dt_t = pt_reference(api, torus["Q"], tq, p["chains"], args.ref_rounds, 1024, 77)
        kind = (f"best energy of an independent PT run ({p['chains']} chains x 32 temperatures "
                f"0.1..3, {args.ref_rounds} rounds x 1024 steps, {dt_t:.1f} s): an upper bound "
                "on the optimum")
        tt["torus2d_bimodal_1024"] = tts_leg(api, tts, torus["ctx"], torus["sched"], torus["w"],
                                             torus["out"]["best_E"], E_t, kind,
                                             torus["w"].instance()[1])
        # Gaussian SK: ladder in units of the unquantised couplings (x 2^16)
        gq = workloads.pt_temperatures(32, 0.1, 3.0, float(workloads.GAUSS_SCALE))
        wg = workloads.WORKLOADS["sk-gaussian-1024"]
        Qg, cg = wg.instance()
        E_g, dt_g = pt_reference(api, Qg, gq, p["chains"], args.ref_rounds, 1024, 77)
        kind = (f"best energy of an independent PT run ({p['chains']} chains x 32 temperatures "
                f"(0.1..3) x 2^16, {args.ref_rounds} rounds x 1024 steps, {dt_g:.1f} s): an "
                "upper bound on the optimum")
        if args.workload == "sk-gaussian-1024":
            c_g, s_g, best_g = ctx, sch, gpu["best_E"]
        else:
            c_g = api.da_create(Qg)
            s_g = sched_of(api, wg)
            o_g = api.device_outputs(wg.replicas, wg.N)
            api.da_anneal_async(c_g, s_g, 0, wg.replicas, wg.steps, wg.seed, None, o_g, stream)
            torch.cuda.synchronize()
            best_g = o_g["best_E"].cpu().numpy()
        tt["sk_gaussian_1024"] = tts_leg(api, tts, c_g, s_g, wg, best_g, E_g, kind, cg)
        result["tts99"] = tt
        log(f"TTS legs: {json.dumps(tt)}")
    if "pt" in legs and args.pt_rounds > 0:
        t0 = time.perf_counter()
        result["pt"] = pt_leg(api, workloads, args.pt_rounds)
        log(f"PT leg ({time.perf_counter() - t0:.1f} s): {json.dumps(result['pt'])}")
    if "ladder" in legs:
        result["pt_ladder_adaptation"] = ladder_leg(api, workloads)
        log(f"ladder leg: {json.dumps(result['pt_ladder_adaptation'])}")
    if "checkpoint" in legs:
        result["checkpoint"] = checkpoint_leg(api, workloads.WORKLOADS["torus2d-bimodal-1024"])
    if "perstep" in legs:
        result["per_step_schedule"] = per_step_leg(api, workloads.WORKLOADS["torus2d-bimodal-1024"])
    if "mfma" in legs:
        INT8_PEAK_TOPS = 5000.0
        fm = {}
        for n, r in ((1024, 1024), (1024, 2048), (8192, 8192)):
            p_ = api.da_probe_fields_mfma(n, r, 10)
            fm[f"N{n}_R{r}"] = {**p_, "frac_of_int8_peak": p_["tera_ops"] / INT8_PEAK_TOPS}
        result["initial_fields_mfma"] = fm
    if "sparse" in legs:
        result["sparse_rows"] = sparse_sweep_leg(api)
    if legs & {"checkpoint", "perstep", "mfma", "sparse"}:
        log(f"other legs: " + json.dumps({k: result.get(k) for k in (
            "checkpoint", "per_step_schedule", "initial_fields_mfma", "sparse_rows")}))
    if "serve" in legs and args.serve_jobs > 0:
        t0 = time.perf_counter()
        result["serve"] = serve_bench(api, workloads, args.serve_jobs, seed=1, budget_gb=16.0,
                                      epoch_steps=4096)
        log(f"served stream: {time.perf_counter() - t0:.1f} s; {json.dumps(result['serve'])}")

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
