/*
 * da.h -- C ABI of dapt, the Digital Annealer's parallel-trial Monte Carlo
 * step for fully connected QUBO problems on AMD MI355X (gfx950).
 *
 * Method: Aramon et al., "Physics-Inspired Optimization for Quadratic
 * Unconstrained Problems Using a Digital Annealer", arXiv:1806.08815.
 *   - Algorithm 2 (Sec. II.B): every Monte Carlo step tests a flip of each of
 *     the N variables in parallel against dE_j - E_offset, applies one of the
 *     accepted flips chosen uniformly at random, updates all local fields,
 *     and raises the dynamic offset E_offset when nothing was accepted.
 *   - Sec. II.D: parallel tempering whose replicas run those steps
 *     (exchange move of Algorithm 3).
 *   - Sec. V: the problem is a QUBO, minimise x^T Q x over x in {0,1}^N.
 *
 * Conventions shared by every call:
 *   - E(x) = x^T Q x for any int32 Q (not necessarily symmetric).  Internally
 *     W_ij = Q_ij + Q_ji (i != j), W_ii = 0, b_i = Q_ii, local field
 *     h = b + W x, and flipping x_i changes E by (1 - 2 x_i) h_i.
 *   - Temperatures are in the energy units of Q.  The Metropolis test
 *     exp(-dE/T) (Sec. III) is decided exactly in integers: a 16-bit draw u
 *     accepts offset-shifted cost d iff d <= ceil(-T ln((u + 1/2)/65536)) - 1.
 *   - Random numbers are Philox4x32-10 keyed by the 64-bit seed, with
 *     counters (variable block, step, replica id, use), so results depend only
 *     on (instance, schedule, replica id, steps, seed) -- never on batching,
 *     launch shape or what else runs on the GPU.
 *   - Energies are int64.  Fields and offsets are int32; da_create rejects
 *     instances whose fields could leave [-2^30, 2^30].
 *   - All calls return DA_OK (0) or a negative status; none throws.  A
 *     da_ctx may be used by one thread at a time; distinct contexts are
 *     independent.  The last error message of a context is kept for
 *     da_last_error(ctx); calls without a context keep theirs per thread,
 *     read with da_last_error(NULL).
 *   - Host buffers are owned by the caller.  Device buffers passed to the
 *     *_async calls are owned by the caller and must stay valid until the
 *     work enqueued on the given stream completes.
 */
#ifndef DAPT_DA_H
#define DAPT_DA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DA_OK 0
#define DA_EINVAL (-1)      /* bad argument (null, out of range, inconsistent)  */
#define DA_ERANGE (-2)      /* coefficients too large for exact int32 fields    */
#define DA_ENOMEM (-3)      /* device or host allocation failed / over budget   */
#define DA_EDEVICE (-4)     /* HIP runtime error or no usable gfx950 device     */
#define DA_ENOTREADY (-5)   /* da_poll: the job has not finished yet            */
#define DA_ENOTFOUND (-6)   /* da_poll/da_wait: unknown or already-taken ticket */

/* ---- coupling storage types -------------------------------------------- */
#define DA_DTYPE_AUTO 0     /* smallest exact storage (after a common factor)  */
#define DA_DTYPE_I8 1
#define DA_DTYPE_I16 2
#define DA_DTYPE_I32 4

/* ---- schedules and starts ------------------------------------------------ */
#define DA_SCHED_GEOMETRIC 0    /* T_l = T_hi (T_lo/T_hi)^(l/(L-1))            */
#define DA_SCHED_LINEAR_BETA 1  /* 1/T_l linear from 1/T_hi to 1/T_lo (App. A) */
#define DA_INIT_ZEROS 0         /* common all-zero start (Algorithm 2, App. A) */
#define DA_INIT_RANDOM 1        /* Philox random start, per replica            */

/* Proposals per step (da_schedule.trial). */
#define DA_TRIAL_PARALLEL 0     /* every variable proposes (Algorithm 2)       */
#define DA_TRIAL_SINGLE 1       /* variable s mod N alone proposes at step s:
                                   single-flip Metropolis in sequential sweeps
                                   (the SA baseline of Sec. III), same tables,
                                   draws and offset rule                       */

#define DA_MAX_N 8192           /* next-generation DA size (Sec. II.D)         */
#define DA_EOFF_MAX (1 << 30)   /* saturation of the dynamic offset            */

typedef struct da_ctx da_ctx;

/* Temperature schedule of an anneal (Algorithm 2 lowers the temperature at
 * intervals during the run).  An S-step run is cut into n_levels equal
 * parts; step s uses level floor(s * n_levels / S).  T_hi and T_lo must be
 * > 0 for DA_SCHED_GEOMETRIC and DA_SCHED_LINEAR_BETA alike, except that
 * T_hi = T_lo = 0 selects a zero-temperature run (only strictly improving
 * flips, d < 0).  eoff_inc >= 0 is Algorithm 2's rate of offset increase
 * (0 switches the dynamic offset off, as in the paper's final runs, App. A).
 * 1 <= n_levels <= 4096, or n_levels = 0: a new temperature every step, as
 * in the paper's DA runs (App. A) -- step s runs at level s of an S-level
 * schedule, S <= 2^24; its flips are decided as d < T_s * (-ln U_u), which
 * equals the table test d <= thr[u] of that temperature.  Per-step schedules
 * are run by da_anneal* and da_anneal_batch, not by the server.  trial is
 * DA_TRIAL_PARALLEL (the DA) or DA_TRIAL_SINGLE; reserved must be 0. */
typedef struct da_schedule {
    double T_hi;
    double T_lo;
    int32_t kind;
    int32_t n_levels;
    int32_t eoff_inc;
    int32_t init;
    int32_t trial;
    int32_t reserved;
} da_schedule;

/* Outputs of an anneal for R replicas; every field may be NULL (skipped).
 * Layouts: best_x/final_x [R][N] uint8 0/1; best_E/final_E/n_accept [R].
 * best_* is the lowest-energy state seen (initial state included, first one
 * kept on ties); n_accept counts the steps that applied a flip.
 * In da_anneal/da_anneal_ex they are host pointers; in the *_async calls
 * they are device pointers. */
typedef struct da_result {
    uint8_t *best_x;
    int64_t *best_E;
    uint8_t *final_x;
    int64_t *final_E;
    int64_t *n_accept;
} da_result;

/* Optional per-step trace of an anneal (host pointers, [R][S] each, any may be
 * NULL): the flipped variable or -1, and E and E_offset after the step.  A
 * traced run takes a slower kernel variant and exists for verification. */
typedef struct da_trace {
    int32_t *k;
    int64_t *E;
    int64_t *eoff;
} da_trace;

/* Launch-shape knobs; zero fields mean "choose automatically" (autotuned
 * table).  Results never depend on them.
 *   flips_per_lane      2, 4 or 8 variables per GPU lane (2: 8/16-bit
 *                       couplings only, else 4)
 *   replicas_per_block  replicas sharing one workgroup (1..16)
 *   w_in_lds            1: stage W in LDS when it fits; -1: never; 0: auto
 *   rng_waves           1: dedicated random-number waves generate each
 *                       step's draws one step ahead, off the critical path;
 *                       -1: the compute waves draw lazily, only for undecided
 *                       flips; 0: auto
 *   draw_estimates      wide bands, several compute waves per replica and at
 *                       least 4 flips per lane: 1 decides flips against an
 *                       fp32 estimate of each draw's threshold (handed over by
 *                       the random-number waves, or evaluated by the compute
 *                       lanes under lazy draws), so most flips take one sign
 *                       test and only those inside the estimate's measured
 *                       window read the exact table; -1: never; 0: auto */
typedef struct da_launch {
    int32_t flips_per_lane;
    int32_t replicas_per_block;
    int32_t w_in_lds;
    int32_t rng_waves;
    int32_t draw_estimates;
} da_launch;

/* What the step-kernel launches of a context looked like and how long they
 * took: HIP events recorded on the launch stream right around every step
 * kernel launch (one anneal = one launch; a PT call = all its rounds). */
typedef struct da_kernel_stats {
    double kernel_ms;          /* duration of the last anneal / PT call's kernels */
    double total_ms;           /* summed over calls since da_reset_kernel_stats   */
    int64_t launches;          /* calls summed in total_ms                        */
    int32_t blocks;            /* grid size of the step kernel               */
    int32_t threads;           /* workgroup size                             */
    int32_t flips_per_lane;
    int32_t replicas_per_block;
    int32_t w_in_lds;
    int32_t rng_waves;         /* random-number waves per replica (0: lazy)  */
    int32_t dtype;             /* bytes per stored coupling                  */
    int32_t draw_estimates;    /* 1: the step kernel took per-draw estimates */
} da_kernel_stats;

/* Static facts about a context. */
typedef struct da_info {
    int32_t N;
    int32_t ld;                /* padded row stride of W on the device       */
    int32_t dtype;             /* bytes per stored coupling (1, 2, 4)        */
    int32_t wscale;            /* W = wscale * stored W (common factor)      */
    int64_t device_bytes;      /* device memory held by the context now     */
    int32_t sparse_degree;     /* entries per row of the sparse copy, 0: none */
    int32_t reserved;
} da_info;

/* OR-ed into da_create's dtype_hint: besides dense W, keep every row's
 * nonzero couplings as a padded list (the row's largest degree D, rounded up
 * to a multiple of 4, of 32-bit entries column | (W_ij / wscale) << 16), and
 * run anneals on it: an accepted step then reads D entries of row k (from LDS
 * when the list fits there) instead of the whole dense row, and updates only
 * the fields of k's neighbours.  Needs |W_ij / wscale| <= 32767 and D <= 1024;
 * results are identical to the dense path.  Parallel tempering uses the
 * dense copy. */
#define DA_STORE_SPARSE 0x100

/* Build a context for E(x) = x^T Q x.  Q is N x N int32, row-major, host;
 * it is copied (the caller keeps its buffer).  Derives W and b (Sec. V),
 * takes out the greatest common divisor of W as wscale, stores W/wscale in
 * dtype_hint (or the smallest exact type for DA_DTYPE_AUTO) and uploads W and
 * b to the current HIP device; with DA_STORE_SPARSE also the sparse row lists.
 * Errors: DA_EINVAL (null, N < 1, N > DA_MAX_N, bad hint), DA_ERANGE
 * (max_i |b_i| + sum_j |W_ij| > 2^30, W/wscale does not fit the forced type,
 * or a sparse list out of range), DA_ENOMEM, DA_EDEVICE (no gfx950 device). */
int da_create(const int32_t *Q, int32_t N, int32_t dtype_hint, da_ctx **out);

/* Frees the context and its device memory; NULL is a no-op. */
void da_destroy(da_ctx *ctx);

int da_get_info(const da_ctx *ctx, da_info *info);

/* Anneal `replicas` independent runs (Algorithm 2) of `steps` steps each and
 * copy the outputs to host buffers; synchronous.  Replica ids are
 * 0..replicas-1.  Same (ctx instance, schedule, replicas, steps, seed) gives
 * identical outputs.  Errors: DA_EINVAL (null ctx/schedule, replicas < 1,
 * steps < 0 or >= 2^31, bad schedule), DA_ENOMEM, DA_EDEVICE. */
int da_anneal(da_ctx *ctx, const da_schedule *schedule, int32_t replicas, int64_t steps,
              uint64_t seed, da_result *out);

/* As da_anneal, for replica ids replica_base .. replica_base+replicas-1
 * (replica_base + replicas <= 2^31), with optional launch knobs (NULL = auto)
 * and an optional per-step trace (NULL = none).  Replica r's outputs are the
 * same whichever call, batch or launch shape produced them. */
int da_anneal_ex(da_ctx *ctx, const da_schedule *schedule, int64_t replica_base,
                 int32_t replicas, int64_t steps, uint64_t seed, const da_launch *launch,
                 da_result *out, const da_trace *trace);

/* Asynchronous form: enqueue the whole anneal on `stream` (a hipStream_t;
 * NULL = the null stream) and write outputs to DEVICE buffers in `out_dev`.
 * Returns once the work is enqueued; the caller synchronises the stream.
 * Kernel timing for da_last_kernel_stats is recorded with events on the same
 * stream.  Device scratch (replica state) is owned by the context and reused
 * by later calls on it, which therefore must be ordered on one stream. */
int da_anneal_async(da_ctx *ctx, const da_schedule *schedule, int64_t replica_base,
                    int32_t replicas, int64_t steps, uint64_t seed, const da_launch *launch,
                    const da_result *out_dev, void *stream);

/* One anneal of a batch (see da_anneal_batch). */
typedef struct da_batch_item {
    da_ctx *ctx;
    da_schedule schedule;
    int64_t replica_base;
    int32_t replicas;
    int32_t reserved;
    int64_t steps;
    uint64_t seed;
    da_result out_dev;         /* device output buffers, as in da_anneal_async */
} da_batch_item;

/* Run several anneals -- different instances, sizes, coupling types,
 * schedules and replica counts -- in ONE persistent kernel launch on
 * `stream`, each with exactly the outputs it would have alone.  Contexts must
 * be distinct and live on the current device.  Errors as da_anneal_async. */
int da_anneal_batch(const da_batch_item *items, int32_t count, void *stream);

/* ---- checkpoint / resume ------------------------------------------------
 * A DA step (Algorithm 2, Sec. II.B) is a function of the replica state, the
 * step index, the replica id and the seed alone (counter-based draws), so a
 * run may stop after any step and continue later -- in another context, on
 * another device, after the process restarted -- with results identical to an
 * uninterrupted run. */

/* Runs steps [step_begin, step_end) of a total_steps-step anneal of replicas
 * replica_base .. replica_base+replicas-1.  step_begin = 0 starts from the
 * schedule's initial state; step_begin > 0 continues from the state the
 * context holds, which must be that of the same replicas after exactly
 * step_begin steps (left by the previous da_anneal_steps call on the context,
 * or by da_state_load).  The level of step s is floor(s L / total_steps), so
 * pieces of one run must all pass the same total_steps, schedule and seed.
 * `out` (nullable) receives best/final states, energies and accepted counts as
 * of step_end.  Synchronous.  Errors: DA_EINVAL (ranges, 0 <= step_begin <=
 * step_end <= total_steps < 2^31, state not at step_begin), DA_ENOMEM,
 * DA_EDEVICE. */
int da_anneal_steps(da_ctx *ctx, const da_schedule *schedule, int64_t replica_base,
                    int32_t replicas, int64_t total_steps, int64_t step_begin,
                    int64_t step_end, uint64_t seed, da_result *out);

/* Snapshot layout (host memory, little-endian):
 *   da_state_header, then for replicas r = 0..R-1 in order: x (N bytes, 0/1),
 *   best x (N bytes), local fields h = b + W x (N int32, true units), then
 *   E[R], best E[R], accepted steps[R] (int64 each), E_offset[R] (int32). */
typedef struct da_state_header {
    uint32_t magic;            /* 0x54534144 "DAST"                            */
    uint32_t version;          /* 1                                            */
    int32_t N;
    int32_t replicas;
    int64_t step;              /* steps completed                              */
    uint64_t replica_base;
} da_state_header;

/* Bytes of a snapshot of `replicas` replicas of an N-variable instance
 * (host-only); -1 for bad arguments. */
int64_t da_state_bytes(int32_t N, int32_t replicas);

/* Copies the first `replicas` replicas of the context's state (as left by the
 * last da_anneal_steps) to `buf` (host, `bytes` >= da_state_bytes).  Errors:
 * DA_EINVAL (no state for that many replicas, short buffer), DA_EDEVICE. */
int da_state_save(da_ctx *ctx, int32_t replicas, void *buf, size_t bytes);

/* Makes a snapshot the context's state, so the next da_anneal_steps may
 * continue at header.step.  The snapshot must be of an instance with the same
 * N (the caller is responsible for it being the same instance: fields are
 * not recomputed).  Errors: DA_EINVAL (bad magic/version, N mismatch, short
 * buffer), DA_ENOMEM, DA_EDEVICE. */
int da_state_load(da_ctx *ctx, const void *buf, size_t bytes);

/* Outputs of parallel tempering, indexed by replica id c*M + m (chain c,
 * replica m); any field may be NULL.  slot: temperature index of each replica
 * at the end; n_swaps [chains]: accepted exchanges per chain; pair_swaps
 * [chains][M-1]: accepted exchanges of each adjacent pair (p, p+1). */
typedef struct da_pt_result {
    uint8_t *best_x;
    int64_t *best_E;
    uint8_t *final_x;
    int64_t *final_E;
    int64_t *n_accept;
    int32_t *slot;
    int64_t *n_swaps;
    int64_t *pair_swaps;
} da_pt_result;

/* Parallel tempering with DA steps (Sec. II.D, exchange move of Algorithm 3),
 * replica exchange on the device.  `chains` independent chains of M replicas
 * at temperatures temps[0] < ... < temps[M-1] (all > 0); replica m of chain c
 * has id c*M + m, a random start, and starts at temps[m].  Each of `rounds`
 * rounds runs steps_per_round DA steps in every replica at its current
 * temperature (global step t*steps_per_round + q), then for p = 0..M-2 in
 * order proposes to swap the temperatures of the replicas at temps[p] and
 * temps[p+1], accepted with probability min(1, exp((1/T_p - 1/T_{p+1})
 * (E_a - E_b))).  eoff_inc as in da_schedule.  Host outputs; synchronous.
 * Errors: DA_EINVAL (ladder not strictly increasing or not positive, M < 1,
 * chains < 1, rounds * steps_per_round >= 2^31), DA_ENOMEM, DA_EDEVICE. */
int da_pt(da_ctx *ctx, const double *temps, int32_t M, int32_t chains, int64_t rounds,
          int32_t steps_per_round, int32_t eoff_inc, uint64_t seed, da_pt_result *out);

/* Adaptive temperature ladder (Sec. II.D: the PTDA sets its temperatures by
 * the adaptive scheme of Hukushima et al., keeping the lowest and highest
 * fixed and moving the others toward equal replica-exchange acceptance for
 * every adjacent pair).  One update, host-only: in inverse temperatures
 * beta_p = 1/temps[p], pair p's new interval is proportional to its old
 * interval times its acceptance accepted[p] / proposals (floored at half a
 * swap so no interval collapses), scaled to fill beta_0 - beta_{M-1};
 * out[0] = temps[0], out[M-1] = temps[M-1], out strictly increasing.
 * accepted [M-1] (may be NULL for M = 1); out [M] may alias nothing.  Errors:
 * DA_EINVAL (nulls, M < 1, proposals < 0). */
int da_pt_ladder_update(int32_t M, const double *temps, const int64_t *accepted,
                        int64_t proposals, double *out);

/* Adapts a PT ladder on the device: each of `iterations` iterations runs
 * da_pt's parallel tempering (`chains` chains, `rounds` rounds of
 * steps_per_round DA steps, random starts, seed + iteration) on the current
 * ladder, counts every pair's accepted exchanges over all chains and rounds,
 * and applies da_pt_ladder_update with proposals = chains * rounds.  temps
 * [M] (host, strictly increasing, > 0) is replaced by the adapted ladder;
 * acceptance [iterations][M-1] (host, nullable) receives each iteration's
 * measured acceptances.  Errors: as da_pt, and DA_EINVAL for M < 2 or
 * rounds < 1. */
int da_pt_adapt(da_ctx *ctx, double *temps, int32_t M, int32_t chains, int32_t iterations,
                int64_t rounds, int32_t steps_per_round, int32_t eoff_inc, uint64_t seed,
                double *acceptance);

/* Exact E(x) = x^T Q x (int64) of `count` host states x [count][N] (uint8,
 * nonzero = 1), computed on the device.  Errors: DA_EINVAL, DA_ENOMEM,
 * DA_EDEVICE. */
int da_energy(da_ctx *ctx, const uint8_t *x, int32_t count, int64_t *E);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): da_energy
 * on device buffers, with no allocation.  x_dev [count][N] uint8 (nonzero =
 * 1) and E_dev [count] int64 are device buffers owned by the caller; the work
 * is enqueued on `stream` (a hipStream_t; NULL = the null stream) and the
 * call returns without waiting.  The intermediates (padded states, local
 * fields) live in a fixed 32 MiB scratch array the library holds on each
 * device until the process ends, so count is limited by
 *   ceil(count * ld / 256) * 256 + 4 * count * ld <= 2^25,  ld = N rounded up to 64
 * (6553 states at N = 1024, 819 at N = 8192); a larger count is rejected
 * with DA_EINVAL before any work.  Every call on a device shares that
 * device's scratch and the last call's contents stay there: calls that
 * overlap on one GPU (other streams, threads or contexts) race, and the
 * caller must order them.  Errors: DA_EINVAL (nulls, count < 1 or too large,
 * context on another device), DA_EDEVICE. */
int da_energy_noalloc(da_ctx *ctx, const uint8_t *x_dev, int32_t count, int64_t *E_dev,
                      void *stream);

/* Stats of the context's step kernels (synchronises with the last end event;
 * call it outside timed regions). */
int da_last_kernel_stats(da_ctx *ctx, da_kernel_stats *stats);

/* Starts a new accumulation window for total_ms / launches. */
int da_reset_kernel_stats(da_ctx *ctx);

/* Last error message of ctx, or of the calling thread when ctx is NULL. */
const char *da_last_error(const da_ctx *ctx);

/* Static description of a status code. */
const char *da_strerror(int status);

/* Identity of this build: the SHA-256 (hex) of the library sources it was
 * compiled from, so a caller can refuse a binary older than its sources. */
const char *da_build_id(void);

/* Host-only: the 65536-entry Metropolis threshold table at temperature T
 * (thr[u] = ceil(-T ln((u + 1/2)/65536)) - 1 clamped to [-1, 2^30]; all -1
 * for T <= 0) and the temperature of level l of a schedule.  These are what
 * the device kernels decide against; exposed for verification. */
int da_threshold_table(double T, int32_t *thr);
double da_level_temperature(const da_schedule *schedule, int32_t level);

/* Roofline probe of the row stream (measurement only; allocates its own
 * matrix).  `chains` workgroups of `waves_per_chain` waves each walk a random
 * cycle through the rows of an n_rows x row_elems matrix of dtype_bytes (2 or
 * 4) integers, one dependent row fetch per step -- the access pattern of the
 * step kernel without its arithmetic.  Reports the time per dependent step
 * (fetch latency at that working-set size) and the row bytes per second over
 * all chains.  Errors: DA_EINVAL (sizes; int16 needs n_rows < 32768,
 * row_elems <= 512 * waves_per_chain), DA_ENOMEM, DA_EDEVICE. */
int da_probe_row_stream(int32_t n_rows, int32_t row_elems, int32_t dtype_bytes, int32_t chains,
                        int32_t waves_per_chain, int64_t steps, double *ns_per_step,
                        double *gbytes_per_s);

/* Matrix-core probe of the random start's initial fields H = X W^T + b
 * (Sec. II.D random starts; int8 couplings, v_mfma_i32_32x32x32_i8): times
 * `iters` launches of the field kernel alone on R random states of a random
 * +-1 N-variable instance and reports ms per launch and int8 tera-ops/s
 * (2 ld^2 R per launch, ld = N rounded up to 64).  Allocates and frees its own
 * device buffers.  Errors: DA_EINVAL (32 <= N <= 8192, R >= 1, iters >= 1),
 * DA_ENOMEM, DA_EDEVICE. */
int da_probe_fields_mfma(int32_t N, int32_t R, int32_t iters, double *ms_per_call,
                         double *tera_ops);

/* ---- continuous-batching server ----------------------------------------- */
typedef struct da_server da_server;

/* One solve request.  Q is copied at submit time.  priority: higher values
 * are admitted first; a waiting job that does not fit the free budget may
 * preempt resident jobs of strictly lower priority (0 for all jobs: plain
 * first-fit admission in submission order, never any preemption). */
typedef struct da_job {
    const int32_t *Q;
    int32_t N;
    int32_t dtype_hint;
    da_schedule schedule;
    int32_t replicas;
    int32_t priority;
    int64_t steps;
    uint64_t seed;
} da_job;

/* Per-job accounting, seconds on the server's monotonic clock. */
typedef struct da_job_stats {
    double t_submit;
    double t_admit;            /* when its device memory was reserved        */
    double t_done;             /* when its results were on the host          */
    int64_t device_bytes;      /* footprint it was admitted with             */
    int32_t epochs;            /* device epochs it took part in              */
    int32_t preemptions;       /* times it was preempted and re-admitted     */
} da_job_stats;

/* Server knobs (zero = default). */
typedef struct da_server_opts {
    int64_t epoch_steps;       /* steps each resident job advances per epoch  */
    int32_t max_resident;      /* cap on concurrently resident jobs           */
    int32_t reserved;
} da_server_opts;

/* Start a server that keeps job state resident on the current device and
 * runs every resident job in shared persistent-kernel epochs.  hbm_budget is
 * the device memory (bytes) jobs may hold at once.  opts may be NULL. */
int da_server_create(size_t hbm_budget, const da_server_opts *opts, da_server **out);

/* Queue a job; never blocks on the GPU.  A job that does not fit the free
 * budget waits and is admitted as memory frees up (higher priority first,
 * then submission order).  When the highest-priority waiting job does not
 * fit, resident jobs of strictly lower priority are preempted at the next
 * epoch boundary -- lowest priority, latest admitted first, as many as it
 * takes -- their state (x, best x, fields, energies, offsets, counts, step)
 * and coupling matrix copied to host memory and their device memory freed;
 * a preempted job waits again and, re-admitted, continues from its snapshot.
 * Results equal those of da_anneal on the same (Q, schedule, replicas, steps,
 * seed), whatever else is running and however often the job was preempted.
 * Errors: DA_EINVAL, DA_ERANGE, DA_ENOMEM (the job alone exceeds the budget). */
int da_submit(da_server *srv, const da_job *job, uint64_t *ticket);

/* Where a job is: state 0 = waiting (being prepared, queued, or preempted),
 * 1 = resident on the device, 2 = finished (results not yet collected);
 * done_steps = Monte Carlo steps completed so far (nullable outputs).
 * Errors: DA_ENOTFOUND (unknown or already collected ticket). */
int da_job_status(da_server *srv, uint64_t ticket, int32_t *state, int64_t *done_steps);

/* Collect a finished job into host buffers (layouts as da_result, R x N),
 * releasing its ticket.  DA_ENOTREADY if it is still queued or running.
 * stats may be NULL. */
int da_poll(da_server *srv, uint64_t ticket, da_result *out, da_job_stats *stats);

/* As da_poll, but waits for the job. */
int da_wait(da_server *srv, uint64_t ticket, da_result *out, da_job_stats *stats);

/* Device bytes a job would hold while resident (coupling matrix, fields,
 * tables, state).  Host-only; the admission policy uses exactly this. */
int64_t da_job_footprint(int32_t N, int32_t dtype_bytes, int32_t replicas, int32_t n_levels);

/* Drains running jobs, then frees everything; NULL is a no-op. */
void da_server_destroy(da_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* DAPT_DA_H */
