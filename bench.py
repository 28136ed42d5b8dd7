#!/usr/bin/env python3
"""Benchmark of the Digital Annealer parallel-trial step on one MI355X.

One "step" of this benchmark is one whole anneal of the workload: every
replica runs all its Monte Carlo steps (Algorithm 2 of arXiv:1806.08815) in
the HIP step kernel, starting from the common zero state.  Inputs (coupling
matrix, tables, state buffers) are resident in HBM before timing starts; the
timed region covers K anneals bracketed by device synchronisation.

Prints ONE JSON line:
  value        flip evaluations per second = replicas * MC steps * N * K / time
  roofline     row-stream bytes of the step kernel (accepted steps * N *
               bytes per coupling) / its event-timed duration, against HBM peak
  cpu_baseline the CPU oracle on one full-length replica of the same workload
  tts99        time to solution at 99% (Sec. IV), measured the paper's way for
               the DA: the wall time of one launch with ceil(R99) replicas
  plain        the same replicas run one launch per replica, beside the
               single batched launch
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
            line = next(l for l in f if l.startswith("machine-readable:"))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line.split(":", 1)[1])
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    if rec.get("kernel_source_sha256") != h.hexdigest():
        return None
    if any(launch.get(k) != v for k, v in rec["launch"].items()):
        return None
    return float(rec["traffic_bytes_per_launch"])


def describe(w):
    return (f"{w.name}: {w.kind} N={w.N}, {w.replicas} replicas x {w.steps} MC steps, "
            f"{w.schedule} T {w.T_hi:g}->{w.T_lo:g} ({w.n_levels} levels), "
            f"E_off increment {w.eoff_inc}, {w.init} start, Philox seed {w.seed}")


def throughput_leg(api, workloads, name: str, steps=None, kind=None, n_levels=None):
    """One full anneal of a workload in its autotuned launch (after one warm-up
    anneal): flip-evals/s, ns per step and row-stream bytes.  kind / n_levels
    override the workload's schedule (n_levels = 0: a new temperature every step)."""
    import torch
    w = workloads.WORKLOADS[name]
    Q, _ = w.instance()
    ctx = api.da_create(Q, w.dtype_hint)
    info = ctx.info()
    kind = w.schedule if kind is None else kind
    n_levels = w.n_levels if n_levels is None else n_levels
    sch = api.schedule(w.T_hi, w.T_lo, kind, n_levels, w.eoff_inc, w.init)
    S = w.steps if steps is None else steps
    out = api.device_outputs(w.replicas, w.N)
    stream = torch.cuda.current_stream()
    api.da_anneal_async(ctx, sch, 0, w.replicas, S, w.seed, None, out, stream)
    torch.cuda.synchronize()
    api.da_reset_kernel_stats(ctx)
    t0 = time.perf_counter()
    api.da_anneal_async(ctx, sch, 0, w.replicas, S, w.seed, None, out, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ks = api.da_last_kernel_stats(ctx)
    kern = ks["kernel_ms"] / 1e3
    acc = float(out["n_accept"].sum().item())
    row_bytes = acc * w.N * info["dtype"]
    return {
        "workload": describe(w), "schedule": f"{kind}, "
        + ("a new temperature every step" if n_levels == 0 else f"{n_levels} levels"),
        "replicas": w.replicas, "mc_steps": S,
        "coupling_storage": f"int{8 * info['dtype']}",
        "flip_evals_per_s": w.replicas * S * w.N / wall,
        "kernel_ms": kern * 1e3, "ns_per_mc_step": kern / S * 1e9,
        "accepted_step_fraction": acc / (w.replicas * S),
        "row_stream_GBps": row_bytes / kern / 1e9,
        "launch": {k: ks[k] for k in ("blocks", "threads", "flips_per_lane",
                                      "replicas_per_block", "rng_waves")},
    }


def pt_leg(api, workloads, rounds: int):
    """Parallel tempering at the full ladder and chain count, a bounded number
    of rounds (the rate is per round, so the full 10^4 rounds scale linearly)."""
    import numpy as np
    p = workloads.PT_WORKLOAD
    Q, _ = workloads.make_instance(p["kind"], p["N"], p["instance_seed"])
    temps = workloads.pt_temperatures(p["M"], p["T_lo"], p["T_hi"], p["temp_scale"])
    ctx = api.da_create(Q)
    api.da_pt(ctx, temps, p["chains"], 2, p["steps_per_round"], p["eoff_inc"], p["seed"])
    t0 = time.perf_counter()
    out = api.da_pt(ctx, temps, p["chains"], rounds, p["steps_per_round"], p["eoff_inc"],
                    p["seed"])
    dt = time.perf_counter() - t0
    R = p["M"] * p["chains"]
    fe = R * rounds * p["steps_per_round"] * p["N"]
    return {
        "workload": f"{p['name']}: {p['kind']} N={p['N']}, {p['chains']} chains x M={p['M']} "
                    f"temperatures, K={p['steps_per_round']} steps per round, random start",
        "rounds_timed": rounds, "rounds_full": p["rounds"], "seconds": dt,
        "flip_evals_per_s": fe / dt, "exchange_decisions": int(rounds * p["chains"] * (p["M"] - 1)),
        "swaps_accepted": int(np.asarray(out["n_swaps"]).sum()),
        "full_run_estimate_s": dt / rounds * p["rounds"],
    }


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
            row.setdefault("same_results", []).append(o["best_E"].cpu().numpy().tolist())
            ctx.close()
        same = row.pop("same_results", [])
        row["sparse_equals_dense"] = len(same) == 2 and same[0] == same[1]
        out.append(row)
    return out


def checkpoint_leg(api, workloads, name: str, cut_frac: float = 0.5):
    """Stop the workload's anneal part-way, snapshot it to host memory, resume in a
    fresh context, and compare with the uninterrupted run."""
    import numpy as np
    w = workloads.WORKLOADS[name]
    Q, _ = w.instance()
    sch = api.schedule(w.T_hi, w.T_lo, w.schedule, w.n_levels, w.eoff_inc, w.init)
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
    same = all(np.array_equal(rest[k], whole[k])
               for k in ("best_x", "best_E", "final_x", "final_E", "n_accept"))
    return {"workload": name, "cut_step": cut, "snapshot_bytes": int(snap.nbytes),
            "save_ms": t_save * 1e3, "load_ms": t_load * 1e3, "resumed_equals_whole": bool(same)}


def cpu_all_cores(oracle, Q, w, threads: int):
    """The oracle on `threads` replicas at once (one replica per thread; the C
    loop releases the interpreter lock), the same schedule as the GPU run."""
    from concurrent.futures import ThreadPoolExecutor

    def one(r):
        return oracle.anneal(Q, T_hi=w.T_hi, T_lo=w.T_lo,
                             kind=0 if w.schedule == "geometric" else 1,
                             n_levels=w.n_levels, eoff_inc=w.eoff_inc,
                             init=0 if w.init == "zeros" else 1, replicas=1, replica_base=r,
                             steps=w.steps, seed=w.seed)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        outs = list(ex.map(one, range(threads)))
    dt = time.perf_counter() - t0
    return threads * w.steps * w.N / dt, dt, outs


def serve_bench(api, workloads, n_jobs: int, seed: int, budget_gb: float, epoch_steps: int,
                steps_range=(10_000, 50_000)):
    """Served stream against plain service of the same jobs.

    A job's latency runs from the moment it arrives with its Q on the host to
    the moment its results are on the host.  Served: every job goes through
    the continuous-batching server (da_submit / da_wait).  Plain: one
    da_create + da_anneal (one launch) + free per job, first come first
    served; its latencies under the same arrivals follow from the measured
    service times.  Arrivals are Poisson at 80% of the server's measured
    capacity (all jobs submitted at once)."""
    import numpy as np
    import torch

    jobs = workloads.serve_stream(n_jobs, seed, rate_hz=1.0, steps_range=steps_range)
    Qs = [workloads.make_instance(j["kind"], j["N"], j["instance_seed"])[0] for j in jobs]
    scheds = [api.schedule(j["T_hi"], j["T_lo"], "geometric", 128, j["eoff_inc"]) for j in jobs]
    work = float(sum(j["replicas"] * j["steps"] * j["N"] for j in jobs))

    def plain(j, Q, sch, steps):
        t = time.perf_counter()
        ctx = api.da_create(Q)
        api.da_anneal(ctx, sch, j["replicas"], steps, j["seed"])
        ctx.close()
        return time.perf_counter() - t

    for j, Q, sch in zip(jobs, Qs, scheds):   # launch-shape tuner, untimed
        plain(j, Q, sch, min(j["steps"], 1000))
    torch.cuda.synchronize()
    service = [plain(j, Q, sch, j["steps"]) for j, Q, sch in zip(jobs, Qs, scheds)]
    busy = sum(service)

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

    _, _, makespan0 = run_stream([0.0] * n_jobs)

    def at_rate(rate):
        g = np.random.Generator(np.random.PCG64(seed + 1))
        arrivals = list(np.cumsum(g.exponential(1.0 / rate, size=n_jobs)))
        _, lat, _ = run_stream(arrivals)
        t_free, plain_lat = 0.0, []
        for ta, sv in zip(arrivals, service):
            start = max(ta, t_free)
            t_free = start + sv
            plain_lat.append(t_free - ta)
        pct = lambda v, q: float(np.percentile(v, q))
        return {"arrival_rate_jobs_per_s": rate,
                "served_p50_s": pct(lat, 50), "served_p99_s": pct(lat, 99),
                "plain_p50_s": pct(plain_lat, 50), "plain_p99_s": pct(plain_lat, 99)}

    return {
        "jobs": n_jobs,
        "sizes": sorted({j["N"] for j in jobs}),
        "flip_evals": work,
        "served_capacity_jobs_per_s": n_jobs / makespan0,
        "plain_capacity_jobs_per_s": n_jobs / busy,
        "served_flip_evals_per_s": work / makespan0,
        "plain_flip_evals_per_s": work / busy,
        "latency_at_80pct_of_served_capacity": at_rate(0.8 * n_jobs / makespan0),
        "latency_at_80pct_of_plain_capacity": at_rate(0.8 * n_jobs / busy),
        "epoch_steps": epoch_steps, "budget_gb": budget_gb,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="torus2d-bimodal-1024")
    ap.add_argument("--dtype", type=int, default=None, help="force coupling storage bytes")
    ap.add_argument("--launch", default=None,
                    help="fixed step-kernel shape F:RPW:RNG (flips per lane, replicas per "
                         "workgroup, random-number waves: 1 on, -1 off) instead of the tuned one")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-extras", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=24,
                    help="jobs in the served-stream leg (0 skips it)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, one plain device copy of this many MiB "
                         "(the known-size reference for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(replicas shard across GPUs with no per-step communication, see DESIGN.md)",
              file=sys.stderr)
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
    sch = api.schedule(w.T_hi, w.T_lo, w.schedule, w.n_levels, w.eoff_inc, w.init)
    stream = torch.cuda.current_stream()
    out = api.device_outputs(R, N)

    fixed = None
    if args.launch:
        F_, rpw_, rng_ = (int(v) for v in args.launch.split(":"))
        fixed = api.launch(F_, rpw_, 0, rng_)

    def anneal():
        api.da_anneal_async(ctx, sch, 0, R, S, w.seed, fixed, out, stream)

    print(f"[bench] {describe(w)}; storage int{8 * info['dtype']} x{info['wscale']}",
          file=sys.stderr, flush=True)
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
    n_acc = out["n_accept"].cpu().numpy()
    best_E = out["best_E"].cpu().numpy()
    best_x0 = out["best_x"][0].cpu().numpy()
    final_x0 = out["final_x"][0].cpu().numpy()
    flip_evals = float(R) * S * N * args.steps
    value = flip_evals / elapsed
    row_bytes = float(n_acc.sum()) * N * info["dtype"]
    achieved = row_bytes / kernel_s / 1e9
    print(f"[bench] {args.steps} anneals in {elapsed:.3f} s; step kernel {kernel_s * 1e3:.3f} ms "
          f"per launch; {value:.4g} flip-evals/s; {achieved:.1f} GB/s row stream",
          file=sys.stderr, flush=True)

    # latency floor: a dependent chain of row fetches alone, same matrix size and
    # element type, one chain per replica (no flip work)
    floor_ns = None
    if info["dtype"] in (2, 4):
        waves = max(1, -(-N // 512))
        floor_ns = api.da_probe_row_stream(N, N, info["dtype"], R, waves, 20_000)["ns_per_step"]

    launch = {k: ks[k] for k in ("blocks", "threads", "flips_per_lane", "replicas_per_block",
                                 "w_in_lds", "rng_waves")}
    traffic = measured_traffic(args.workload, launch)
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
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_run (step kernel)",
            "kernel_ms": kernel_s * 1e3,
            "bytes_per_launch": row_bytes,
            "accepted_step_fraction": float(n_acc.sum()) / (R * S),
            "ns_per_mc_step": kernel_s / S * 1e9,
            "row_fetch_chain_ns": floor_ns,
            "fetch_chain_over_step": (floor_ns / (kernel_s / S * 1e9)) if floor_ns else None,
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
        t0 = time.perf_counter()
        ref = oracle.anneal(Q, T_hi=w.T_hi, T_lo=w.T_lo,
                            kind=0 if w.schedule == "geometric" else 1,
                            n_levels=w.n_levels, eoff_inc=w.eoff_inc,
                            init=0 if w.init == "zeros" else 1, replicas=1, replica_base=0,
                            steps=S, seed=w.seed)
        t_cpu = time.perf_counter() - t0
        same = (int(ref["best_E"][0]) == int(best_E[0]) and int(ref["n_accept"][0]) == int(n_acc[0])
                and np.array_equal(ref["best_x"][0], best_x0)
                and np.array_equal(ref["final_x"][0], final_x0))
        threads = max(1, min(ncpu or 1, 16, R))
        v_all, t_all, outs = cpu_all_cores(oracle, Q, w, threads)
        same_all = all(int(o["best_E"][0]) == int(best_E[r]) for r, o in enumerate(outs))
        result["cpu_baseline"] = {
            "value": v_all,
            "unit": "flip-evals/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"replicas 0..{threads - 1} of {R}, all {S} MC steps of the same schedule, "
                      f"one replica per thread on {threads} threads, {t_all:.1f} s wall on "
                      f"{model} ({ncpu} host CPUs)",
            "single_core": {"value": S * N / t_cpu, "seconds": t_cpu, "replica": 0},
            "matches_gpu_replicas": bool(same and same_all),
        }
        print(f"[bench] oracle: 1 core {t_cpu:.1f} s, {threads} threads {t_all:.1f} s, parity "
              f"with GPU replicas: {same and same_all}", file=sys.stderr, flush=True)

    if not args.skip_extras:
        # one launch per replica, on the same stream, same outputs per replica
        one = api.device_outputs(1, N)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(R):
            api.da_anneal_async(ctx, sch, r, 1, S, w.seed, None, one, stream)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        same_last = int(one["best_E"][0].item()) == int(best_E[R - 1])
        result["plain"] = {
            "form": f"{R} launches of 1 replica each",
            "seconds": t_plain,
            "flip_evals_per_s": float(R) * S * N / t_plain,
            "batched_speedup": t_plain / (elapsed / args.steps),
            "same_result_as_batched": bool(same_last),
        }
        print(f"[bench] plain per-replica launches: {t_plain:.2f} s", file=sys.stderr, flush=True)

        E_ref = int(best_E.min())
        y = tts.success_count(best_E, E_ref)

        def time_launch(reps):
            o = api.device_outputs(reps, N)
            torch.cuda.synchronize()
            t = time.perf_counter()
            api.da_anneal_async(ctx, sch, 0, reps, S, w.seed, None, o, stream)
            torch.cuda.synchronize()
            return time.perf_counter() - t

        t99 = tts.tts99_measured(y, R, time_launch)
        result["tts99"] = {
            "E_ref": E_ref + int(const),
            "E_ref_kind": f"best over {R} replicas (upper bound on the optimum)",
            "successes": y, "runs": R, "theta_median": t99["theta"], "r99": t99["r99"],
            "replicas_launched": t99["replicas"], "seconds": t99["tts_s"],
        }

    if not args.skip_extras:
        t0 = time.perf_counter()
        result["sk_gaussian_1024"] = throughput_leg(api, workloads, "sk-gaussian-1024")
        result["pt"] = pt_leg(api, workloads, rounds=20)
        result["checkpoint"] = checkpoint_leg(api, workloads, args.workload)
        result["per_step_schedule"] = throughput_leg(api, workloads, args.workload,
                                                     kind="linear_beta", n_levels=0)
        INT8_PEAK_TOPS = 5000.0
        fm = {}
        for n, r in ((1024, 1024), (1024, 2048), (8192, 8192)):
            p = api.da_probe_fields_mfma(n, r, 10)
            fm[f"N{n}_R{r}"] = {**p, "frac_of_int8_peak": p["tera_ops"] / INT8_PEAK_TOPS}
        result["initial_fields_mfma"] = fm
        result["sparse_rows"] = sparse_sweep_leg(api)
        print(f"[bench] gaussian and PT legs: {time.perf_counter() - t0:.1f} s; "
              f"{json.dumps(result['sk_gaussian_1024'])} {json.dumps(result['pt'])} "
              f"{json.dumps(result['checkpoint'])} {json.dumps(result['per_step_schedule'])} "
              f"{json.dumps(result['initial_fields_mfma'])} {json.dumps(result['sparse_rows'])}",
              file=sys.stderr, flush=True)

    if not args.skip_extras and args.serve_jobs > 0:
        t0 = time.perf_counter()
        result["serve"] = serve_bench(api, workloads, args.serve_jobs, seed=1, budget_gb=16.0,
                                      epoch_steps=4096)
        print(f"[bench] served stream: {time.perf_counter() - t0:.1f} s; "
              f"{json.dumps(result['serve'])}", file=sys.stderr, flush=True)

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
