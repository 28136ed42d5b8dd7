// da_internal.h -- structures shared by the host runtime and the gfx950 kernels.
//
// Device data layout (all in HBM, one context per instance):
//   W    [ld rows][ld] int8/int16/int32, row-major, symmetric, zero diagonal,
//        zero padding beyond N; stores W / wscale.
//   b    [ld] int32, zero beyond N.
//   Replica state, [R] replicas, row stride ld:
//     h [R][ld] int32 local fields, x / bx [R][ld] uint8 current / best state,
//     E, bE, nacc [R] int64, eoff [R] int32.
//   Level tables (one level per temperature in force):
//     thr [L][65536] int32 Metropolis thresholds,
//     hdr [L] LevelHdr, brk [...] uint32 acceptance brackets (see below).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dapt {

// The band of a level: with thr non-increasing in u, every d <= tmin = thr[65535]
// is accepted for all draws and every d > tmax = thr[0] is rejected for all
// draws, so only tmin < d <= tmax needs a random draw.  Inside the band the
// accepting draws of d form a prefix u < ucut(d) = #{u : thr[u] >= d}, with
// ucut non-increasing in d.  The band is cut into buckets of 2^sh values of d;
// bucket D holds (lo, hi) = (ucut(last d of the bucket), ucut(first d)) packed
// as lo | hi << 16, so u < lo accepts, u >= hi rejects, and only lo <= u < hi
// needs the table entry thr[u].  With sh = 0 the bracket is exact (lo == hi).
// The last bucket's lo is taken at its true end (0 once past tmax), and a
// reject-all entry 0 follows the buckets of every level.
//
// Narrow bands (tmax - tmin <= kDirectSpan) also get a direct table of the
// decision by draw: q[u] = thr[u] - tmin in [0, tmax - tmin], one byte per
// draw, so an in-band flip with ub = d - tmin - 1 is accepted iff ub < q[u].
// The table depends on the draw only, so it can be read before the flip's
// cost is known.  Such levels also have |tmin| <= kDirectTmin (always true of
// a narrow band, as thr >= -1; stated so that tmin + 1 + E_off + q fits int32).
//
// Wide bands can also be decided from a per-draw estimate computed by the
// random-number waves (kernel variant kModeGen): G(u) = bits(fma(log2(u + 1/2),
// ga, gb)) - kGenMagic in fp32 with ga = T ln 2 and gb = 1.5 2^23 - 16 T ln 2:
// the sum lands in [2^23, 2^24), where the float's bits minus those of 1.5 2^23
// are the rounded integer, so -G(u) is within a few units of thr[u] (levels with
// tmax < 2^22 only).  A device pass over all 65536 draws measures, with the
// kernel's own instructions, off(u) = thr[u] + G(u) and keeps its range
// [glo, ghi], so thr[u] lies in [glo - G(u), ghi - G(u)] for every draw:
// d <= glo - G(u) accepts, d > ghi - G(u) rejects, and only the rare d in
// between (a window of ghi - glo values) reads thr[u].  gth = 1 marks a level
// whose window was measured and is at most kGenWindow wide.
struct LevelHdr {
    int32_t tmin;
    int32_t tmax;
    int32_t sh;
    int32_t off;   // first bucket of this level in brk
    int32_t q8;    // index of this level's direct table, or -1
    int32_t gth;   // per-draw estimate usable (set by the measuring pass)
    float ga, gb;  // estimate coefficients (T ln 2, -16 T ln 2)
    int32_t glo, ghi;   // range of thr[u] + G(u) over all draws
    int32_t pad[2];
};
constexpr int kGenWindow = 64;      // widest measured window a level may use
constexpr int kGenOffMax = 64;      // and |glo|, |ghi| at most this
constexpr int32_t kGenTmax = 1 << 22;            // levels with tmax below this only
constexpr uint32_t kGenMagic = 0x4B400000u;      // bits of 1.5 2^23
// the estimate path's d - glo + G(u) - 1 stays in int32 when |h| stays below
// this bound (E_off <= 2^30, tmax < 2^22)
constexpr int64_t kGenFieldMax = (int64_t(1) << 30) - (int64_t(1) << 22) - 256;
constexpr int kDirectSpan = 255;
constexpr int kDirectTmin = 256;
constexpr int kMaxDirectLevels = 512;   // schedules with more levels use brackets only

constexpr int kMaxBuckets = 4096;   // bracket entries per level (reject-all included)
constexpr int kMaxLevels = 4096;
constexpr int kMaxN = 8192;
constexpr int32_t kEoffMax = 1 << 30;

// One anneal segment (or one parallel-tempering round) of one instance.
// Per-step schedule (temperature changed every step, App. A): the step's
// temperature and band [tmin, tmax] (= thr[65535], thr[0] at that
// temperature); an in-band flip is accepted iff d < T * G[u], G[u] = -ln U_u,
// which equals d <= thr[u] for integer d.
struct StepT {
    double T;
    int32_t tmin, tmax;
};

// Compile-time feature sets of the step kernel (see run_block).
constexpr int kModePlain = 0, kModeSingle = 1, kModePerStep = 2, kModeDynamic = 4,
              kModeSparse = 8, kModeWide = 16, kModeDirect = 32, kModeGen = 64,
              kModeNW4 = 128;

struct JobDesc {
    const void *W;
    const int32_t *b;
    int32_t N, ld, dtype, wscale;
    int32_t *h;
    uint8_t *x;
    uint8_t *bx;
    int64_t *E;
    int64_t *bE;
    int32_t *eoff;
    int64_t *nacc;
    int32_t R;             // replicas of this job (state rows 0..R-1)
    uint32_t rid_base;     // random-number replica id of state row 0
    uint64_t seed;
    int64_t s0, s1, S;     // run steps [s0, s1) of an S-step schedule
    int32_t L;             // schedule levels (anneal mode)
    int32_t eoff_inc;
    const int32_t *lvl_of_rep;   // PT mode: level of each replica, else null
    const uint32_t *round_ptr;   // PT mode: device round counter, else null
    int32_t K;                   // PT mode: steps per round
    int32_t NW;                  // compute waves per replica
    int32_t NH;                  // random-number waves per replica (0: lazy draws)
    int32_t RPW;                 // replicas per workgroup
    int32_t w_lds;               // W staged in LDS
    const LevelHdr *hdr;
    const uint32_t *brk;
    const int32_t *thr;
    const StepT *stepT;          // per-step schedule, else null
    const double *G;             // -ln U_u, with stepT
    const uint8_t *q8;           // direct tables staged in LDS (anneal mode), or null
    int32_t single;              // 1: only variable s mod N proposes at step s
    int32_t ell_D;               // sparse row lists: entries per row (0: dense)
    const uint32_t *ell;         // [N][ell_D] column | value << 16, or null
    int32_t gth;                 // 1: random-number waves hand over per-draw estimates
};

constexpr int64_t kMaxPerStepSteps = int64_t(1) << 24;

// Host guard of every step-kernel launch.  Anneal mode: the step range
// [s0, s1) lies inside the S-step schedule, so the level index
// floor(s L / S) of every step it runs stays below L; the offset increment is
// in [0, 2^30] (the kernel saturates the offset as min(E_off, 2^30 - inc) +
// inc, which equals min(E_off + inc, 2^30) only there); a per-step schedule
// has at most 2^24 steps.  Parallel-tempering mode (round counter on the
// device): a level per replica and a non-negative round length.  Returns
// nullptr when the job may be launched, else what is wrong.
inline const char *job_range_error(const JobDesc &J) {
    if (J.R < 1 || J.N < 1 || J.N > kMaxN || J.ld < J.N || (J.ld & 63) != 0)
        return "job has no replicas or an inconsistent size";
    if (J.NW < 1 || J.NH < 0 || J.RPW < 1 || J.NW * J.RPW + J.NH * J.RPW > 16)
        return "launch shape exceeds one workgroup";
    if (J.eoff_inc < 0 || J.eoff_inc > kEoffMax) return "offset increment outside [0, 2^30]";
    if (J.L < 1 || !J.hdr) return "job has no temperature levels";
    if (J.round_ptr) {
        if (!J.lvl_of_rep || J.K < 0) return "parallel-tempering job without levels or round";
        return nullptr;
    }
    if (J.s0 < 0 || J.s0 > J.s1 || J.s1 > J.S)
        return "step range [s0, s1) leaves the schedule's [0, S)";
    if (J.stepT && J.S > kMaxPerStepSteps) return "per-step schedule longer than 2^24 steps";
    return nullptr;
}
struct TraceDesc {
    int32_t *k;
    int64_t *E;
    int64_t *eoff;
    int64_t stride;        // steps per replica row
};

// Work item of the batched persistent kernel: the replicas of job `job` that
// one workgroup runs, starting at state row `r0` (RPW of them).
struct BatchItem {
    int32_t job;
    int32_t r0;
};

// Host-side launch wrappers implemented in da_kernels.hip.  All enqueue on
// `stream` and return a hipError_t value as int.
int launch_state_zero(const JobDesc &J, void *stream);
int launch_rand_bits(uint8_t *X, int32_t R, int32_t N, int32_t ld, uint32_t rid_base,
                     uint64_t seed, void *stream);
int launch_fields(const JobDesc &J, const uint8_t *X, int32_t R, int32_t *H, void *stream);
int launch_energy_from_fields(const JobDesc &J, const uint8_t *X, const int32_t *H, int32_t R,
                              int64_t *E_out, bool finish_state, void *stream);
int launch_run(const JobDesc &J, int F, bool help, const TraceDesc *trace, int blocks,
               int threads, size_t lds_bytes, void *stream);
// Persistent batched step kernel; the item count is read from device memory so
// one captured graph can serve batches of any size.
// dynamic: the kernel variant that reads each job's optional features
// (single-trial, per-step schedule) instead of the plain DA step.
int launch_batch(const JobDesc *jobs_dev, const BatchItem *items_dev, const int32_t *n_items_dev,
                 int32_t *counter_dev, int blocks, int threads, size_t lds_bytes, void *stream,
                 bool dynamic);
// Exchange sweep of every chain (one workgroup per chain, M <= 4096); round
// points to two words: the round index and a count of the workgroups that
// have read it.  pair_swaps [chains][M-1] counts accepted exchanges per pair.
int launch_pt_exchange(int64_t *E, int32_t *slot2rep, int32_t *lvl_of_rep, const double *dbeta,
                       const double *lnU, int32_t M, int32_t chains, uint64_t seed,
                       uint32_t *round_ptr, int64_t *n_swaps, int64_t *pair_swaps,
                       void *stream);
int launch_pt_setup(int32_t *slot2rep, int32_t *lvl_of_rep, int64_t *n_swaps,
                    int64_t *pair_swaps, uint32_t *round_ptr, int32_t M, int32_t chains,
                    void *stream);
int launch_extract(const JobDesc &J, const uint8_t *src_x, uint8_t *dst_x, int32_t R,
                   void *stream);
int launch_copy_i64(const int64_t *src, int64_t *dst, int32_t n, void *stream);
int launch_fill_i32(int32_t *dst, int32_t value, int64_t n, void *stream);

// Dynamic LDS a workgroup may use on the current device (bytes).
int device_lds_limit();

// LDS of one replica slot of a workgroup (byte offsets): the selection
// exchange of multi-wave replicas (lane records, the energy hand-off) and, with random-number waves, the selection-draw ring and the
// double-buffered Philox blocks; with sparse row lists (dhF = flips per lane)
// one field-delta buffer of 64 * dhF int32 per compute wave.
struct SlotLayout {
    int rec, dEs, vring, draws, dh, est, bytes;
};
__host__ __device__ inline SlotLayout slot_layout(int NW, int NH, int dhF = 0, bool gen = false) {
    SlotLayout L{0, 0, 0, 0, 0, 0, 0};
    int off = 0;
    if (NW > 1 || NH > 0) {
        // lane records [2][max(NW, 4) * 64]: four waves' records can always be
        // read at fixed offsets (the entries past NW are never selected)
        L.rec = off;
        off += 2 * (NW > 4 ? NW : 4) * 64 * 4;
        L.dEs = off;
        off += 8;
    }
    if (NH > 0) {
        // selection draws of 128 steps: the random-number waves write 64 at a
        // time, one step per lane
        L.vring = off;
        off += 128 * 4;
        off = (off + 15) & ~15;
        // Philox blocks of two steps, [2][NH * 64] int4; with per-draw
        // estimates each block is followed by its draws' estimates G(u)
        // (draws 0..3, then 4..7), [2][NH * 64][3] int4, so one address and
        // fixed offsets reach all three
        L.draws = off;
        L.est = off;
        off += 2 * NH * 64 * 16 * (gen ? 3 : 1);
    }
    if (dhF > 0) {
        off = (off + 15) & ~15;
        L.dh = off;
        off += NW * 64 * dhF * 4;
    }
    L.bytes = (off + 15) & ~15;
    return L;
}

// Workgroup LDS bytes the run kernel needs for a launch shape (stage_brk: the
// level's bracket table is staged in LDS, anneal mode; direct: so is a direct
// table of 65536 bytes).
size_t run_lds_bytes(int NW, int RPW, int F, int w_lds_bytes, int stage_brk, int NH,
                     bool sparse = false, bool direct = false, bool gen = false);
// Measures glo/ghi of every level marked gth in hdr (device, [L]) against the
// threshold tables thr [L][65536], and clears gth where the window is too wide.
int launch_gen_calibrate(LevelHdr *hdr, const int32_t *thr, int32_t L, void *stream);

}  // namespace dapt
