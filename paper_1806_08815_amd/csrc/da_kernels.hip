// da_kernels.hip -- gfx950 kernels of the Digital Annealer parallel-trial step.
//
// Method: Algorithm 2 (Sec. II.B) of Aramon et al., arXiv:1806.08815, and its
// parallel-tempering variant (Sec. II.D, exchange move of Algorithm 3).
//
// Mapping of one DA step onto CDNA4:
//   * A replica is NW wavefronts; lane g of the replica owns the F consecutive
//     variables i0 = g*F .. g*F+F-1 and keeps their fields h (int32) and bits
//     of x in registers for the whole run.
//   * Each lane scores its F flips, d = (1 - 2 x_i) h_i - E_offset.  The level's
//     band decides most of them with no random draw: d <= tmin accepts,
//     d > tmax rejects.  Only in-band flips pay for a Philox4x32-10 block (one
//     block per 8 variables, so F <= 8 costs one call per lane) and an
//     acceptance bracket; a global table read is needed only inside a
//     non-exact bracket.  This reproduces d <= thr[u] exactly.  When draws
//     come from generator waves, narrow bands take one compare per flip
//     against a direct decision table, and wide bands one bracket read per
//     flip with no band tests.
//   * The accepted count and the rank of the chosen flip come from wave
//     ballots plus mbcnt (an exclusive prefix sum without data movement).
//     With NW > 1, lanes publish their accepted masks, x bits and in-wave
//     prefixes to LDS (double-buffered by step parity) and one workgroup
//     barrier per step lets every wave find the chosen flip k on its own;
//     nothing else is shared.
//   * The only bulk traffic of a step is row k of W (N * dtype bytes), streamed
//     once: every lane loads its F contiguous couplings with vector loads and
//     updates its fields.  W stays in L2 / MALL / HBM, or in LDS when small.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "da_internal.h"

namespace dapt {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

enum : uint32_t { kTagMetropolis = 0, kTagSelect = 1, kTagExchange = 2, kTagInit = 3 };

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// with the key advanced by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)c0;   // v_mad_u64_u32
        const uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)c2;
        c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        c1 = (uint32_t)p1;
        c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c3 = (uint32_t)p0;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Word 0 of Philox4x32-10 for a counter and key that are the same in every
// lane of the wave (the selection draw): written with 32-bit high and low
// products of wave-uniform operands, so the ten rounds run on the scalar
// unit instead of taking vector issue slots.  Same function as philox().x.
__device__ __forceinline__ uint32_t philox_x_uniform(uint32_t c0, uint32_t c1, uint32_t c2,
                                                     uint32_t c3, uint32_t k0, uint32_t k1) {
    c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c0);
    c1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c1);
    c2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c2);
    c3 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c3);
    k0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)k0);
    k1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)k1);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint32_t hi0 = __umulhi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint32_t hi1 = __umulhi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    return c0;
}

// Per-draw estimate of a level (coefficients ga = T ln 2, gb = 1.5 2^23 -
// 16 T ln 2): T ln((u + 1/2) / 65536) + 1.5 2^23 evaluated as an fp32 base-2
// logarithm and one fused multiply-add, returned as the float's bits.  For
// tmax < 2^22 the sum lies in [2^23, 2^24), so the bits are kGenMagic plus the
// rounded value: G(u) = draw_estimate - kGenMagic ~ -thr[u], with the offset
// folded into the step's constants.  Any deterministic function would do: the
// window pass below measures thr[u] + G(u) over every draw with these same
// instructions, and decisions only use G inside that measured bracket.
__device__ __forceinline__ int draw_estimate(uint32_t u, float ga, float gb) {
    const float x = (float)u + 0.5f;                 // exact for u < 2^16
    const float lg = __builtin_amdgcn_logf(x);       // v_log_f32
    return __float_as_int(__builtin_fmaf(lg, ga, gb));
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, int w) {
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ int mbcnt64(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int readlane(int v, int lane) {
    return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
// a wave-uniform 64-bit value kept in scalar registers (the 64-bit division
// of the level arithmetic leaves its results in vector registers)
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Exclusive prefix sum over the wave of c (0 <= c < 32) and the wave total,
// from ballots of the bits of c.
template <int BITS>
__device__ __forceinline__ void wave_prefix(int c, int &excl, int &total) {
    excl = 0;
    total = 0;
#pragma unroll
    for (int q = 0; q < BITS; ++q) {
        const uint64_t bq = ballot((c >> q) & 1);
        excl += mbcnt64(bq) << q;
        total += __popcll(bq) << q;
    }
}

// The same from a DPP scan: inclusive sums within rows of 16 lanes (shifts 1,
// 2, 4, 8), then each row's predecessors added by the row broadcasts of lanes
// 15 and 31; six dependent adds instead of a ballot and two mbcnt per bit.
__device__ __forceinline__ void wave_scan(int c, int &excl, int &total) {
    int v = c;
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
    excl = v - c;
    total = __builtin_amdgcn_readlane(v, 63);
}

// Position of the r-th (0-based) set bit of a 4-bit mask m, for every (m, r):
// entry 4 (m & 7) + r of half m >> 3, two bits each.
constexpr uint64_t select4_half(int half) {
    uint64_t t = 0;
    for (int m = 8 * half; m < 8 * half + 8; ++m)
        for (int r = 0; r < 4; ++r) {
            int cnt = 0, pos = 0;
            for (int q = 0; q < 4; ++q)
                if ((m >> q) & 1) {
                    if (cnt == r) pos = q;
                    ++cnt;
                }
            t |= (uint64_t)pos << (2 * ((m - 8 * half) * 4 + r));
        }
    return t;
}

__device__ __forceinline__ int select_bit4(uint32_t m, int r) {
    constexpr uint64_t lo = select4_half(0), hi = select4_half(1);
    const uint64_t t = (m & 8u) ? hi : lo;
    return (int)((t >> (2 * (((m & 7u) << 2) + (uint32_t)r))) & 3u);
}

// Position of the r-th (0-based) set bit of the F-bit mask m, r < popc(m)
// (table lookups, no loop over bits).
template <int F>
__device__ __forceinline__ int select_bit(uint32_t m, int r) {
    static_assert(F == 2 || F == 4 || F == 8, "2, 4 or 8 flips per lane");
    if (F == 2) return (r == 0 && (m & 1u)) ? 0 : 1;
    if (F == 4) return select_bit4(m, r);
    const uint32_t low = m & 15u;
    const int c = __popc(low);
    return r < c ? select_bit4(low, r) : 4 + select_bit4(m >> 4, r - c);
}

// h[bit] for a wave-uniform bit: a select tree on the bits of `bit` (F - 1
// selects, log2 F uniform conditions)
// (explicit selects: written as plain conditionals the compiler turns the
// tree back into an indexed read, a compare chain per level)
template <int F>
__device__ __forceinline__ int pick_field(const int (&h)[F], int bit) {
    const int ub = __builtin_amdgcn_readfirstlane(bit);
    int v[F];
#pragma unroll
    for (int f = 0; f < F; ++f) v[f] = h[f];
#pragma unroll
    for (int w = 1; w < F; w <<= 1) {
        const uint64_t up = (ub & w) ? ~0ull : 0ull;   // wave-uniform lane mask
#pragma unroll
        for (int q = 0; q < F; q += 2 * w)
            asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(v[q]) : "v"(v[q]), "v"(v[q + w]), "s"(up));
    }
    return v[0];
}

template <int F>
struct CountBits {
    static constexpr int value = F >= 8 ? 4 : (F >= 4 ? 3 : (F >= 2 ? 2 : 1));
};

template <typename T, int F>
struct VecOf {
    typedef T type __attribute__((ext_vector_type(F)));
};

// Sign-extended load of F consecutive couplings.
template <typename WT, int F>
__device__ __forceinline__ void load_row(const WT *p, int (&w)[F]) {
    typedef typename VecOf<WT, F>::type V;
    const V v = *reinterpret_cast<const V *>(p);
#pragma unroll
    for (int f = 0; f < F; ++f) w[f] = (int)v[f];
}

// h[f] += raw[f] * dw for 16-bit couplings and |dw| < 2^15: one 16 x 16 -> 32
// bit multiply-add per field, which takes the coupling in place from its half
// of the loaded dword (op_sel selects the high half).
template <typename WT, int F>
__device__ __forceinline__ void update_i16(const typename VecOf<WT, F>::type &raw, int dw,
                                           int (&h)[F]) {
    if constexpr (sizeof(WT) == 2 && F == 2) {
        const int pr = __builtin_bit_cast(int, raw);
        asm("v_mad_i32_i16 %0, %1, %2, %0" : "+v"(h[0]) : "v"(pr), "s"(dw));
        asm("v_mad_i32_i16 %0, %1, %2, %0 op_sel:[1,0,0,0]" : "+v"(h[1]) : "v"(pr), "s"(dw));
    } else if constexpr (sizeof(WT) == 2) {
        typedef typename VecOf<int, F / 2>::type PairV;
        const PairV pr = __builtin_bit_cast(PairV, raw);
#pragma unroll
        for (int q = 0; q < F / 2; ++q) {
            asm("v_mad_i32_i16 %0, %1, %2, %0" : "+v"(h[2 * q]) : "v"(pr[q]), "s"(dw));
            asm("v_mad_i32_i16 %0, %1, %2, %0 op_sel:[1,0,0,0]" : "+v"(h[2 * q + 1]) : "v"(pr[q]), "s"(dw));
        }
    }
}

// Level in force at step s of an S-step, L-level schedule: floor(s L / S),
// clamped to the last level (the host never launches steps s >= S; the clamp
// keeps a level-table read in range whatever it is given).
__device__ __forceinline__ int level_of(int64_t s, int32_t L, int64_t S) {
    return S > 0 ? min((int)((s * (int64_t)L) / S), L - 1) : 0;
}

// First step whose level exceeds `lvl`.
__device__ __forceinline__ int64_t next_level_step(int lvl, int32_t L, int64_t S) {
    if (lvl + 1 >= L) return INT64_MAX;
    return ((int64_t)(lvl + 1) * S + L - 1) / L;
}

// DPP inclusive prefix sum within each row of 16 lanes.
__device__ __forceinline__ int row16_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    return v;
}

}  // namespace

size_t run_lds_bytes(int NW, int RPW, int F, int w_lds_bytes, int stage_brk, int NH,
                     bool sparse, bool direct, bool gen) {
    const SlotLayout SL = slot_layout(NW, NH, sparse ? F : 0, gen);
    size_t w = (size_t)((w_lds_bytes + 15) & ~15);
    size_t b = stage_brk ? (size_t)kMaxBuckets * 4 + (direct ? 65536 : 0) : 0;
    return w + b + (size_t)SL.bytes * RPW;
}

// Runs steps [s0, s1) for the replicas of one workgroup.  `blk` selects which
// replicas of the job (rows blk*RPW ..).  All waves of the workgroup execute
// the same number of loop iterations and barriers.
//
// HELP: besides the NW compute waves, each replica has NH random-number
// waves.  They only run Philox: during step s they write step s+1's 16-bit
// draws and selection draw into a double-buffered LDS ring, and the per-step
// barrier hands them over, so the compute waves' critical path (fetch, update,
// test, select) carries no generator work at all; the generator waves run on
// issue slots the compute waves leave idle while they wait on memory.
// Without HELP, draws are generated lazily by the compute waves, only for
// lanes with in-band flips (least total work when the chip is full).
// STAGE: one level per workgroup (anneal), its brackets live in LDS; else
// (parallel tempering) every replica has its own level, read through L1/L2.
//
// Multi-wave replicas (NW > 1) exchange, once per step, each lane's accepted
// mask, x bits and in-wave prefix (the last lane's is the wave's count)
// through LDS, double-buffered by step parity, around one workgroup barrier.  The energy change of the
// chosen flip is handed to the other waves one step later through the same
// buffers (the owning lane writes it after the selection), so it never adds
// an LDS round trip to the critical path; the energy and the best-state check
// of step s therefore complete after barrier s+1, before step s+1 flips.
// MODE selects optional features at compile time, so the plain DA step carries
// none of their code: kModeSingle (single-trial proposals), kModePerStep (a new
// temperature every step), both, or kModeDynamic (read from the job; used by
// the batched kernel when a batch mixes them).  kModeWide states that every
// replica spans several compute waves, W is read from global memory and
// 16-bit couplings have a common factor below 2^15, so the single-wave,
// LDS-resident and 24-bit update paths drop out of the step loop.
// kModeDirect carries the direct-table decisions of narrow-band levels;
// kModeGen the per-draw threshold estimates of wide bands (for jobs that set
// gth, on levels whose window was measured narrow); kModeNW4 states that a
// replica has at most 4 compute waves (the selection's wave records are all
// read before the search).
// BATCH: the persistent batched kernel, whose workgroups may hold more waves
// than the job's replica slots.
template <typename WT, int F, bool TRACE, bool HELP, bool STAGE, int MODE, bool BATCH = false>
__device__ __forceinline__ void run_block(const JobDesc &J, int blk, uint8_t *smem,
                                          const TraceDesc &T) {
    const bool single = MODE == kModeDynamic ? J.single != 0 : (MODE & kModeSingle) != 0;
    const bool perstep = MODE == kModeDynamic ? J.stepT != nullptr : (MODE & kModePerStep) != 0;
    const bool sparse = MODE == kModeDynamic ? J.ell != nullptr : (MODE & kModeSparse) != 0;
    static_assert(F == 2 || F == 4 || F == 8, "a lane's record holds at most 8 flips");
    constexpr int NB = (F + 7) / 8;   // Philox blocks per lane
    typedef typename VecOf<WT, F>::type RowV;
    const int lane = threadIdx.x & 63;
    // lanes 0..F-1: the flips at or above position `lane` of a lane's mask
    const uint32_t ge_mask = lane < F ? ((0xFFu << lane) & ((1u << F) - 1u)) : 0u;
    // wave-level quantities are uniform: keep them in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    constexpr bool wide = (MODE & kModeWide) != 0;
    constexpr bool nw4 = (MODE & kModeNW4) != 0;
    static_assert(!nw4 || !BATCH, "the batched kernel mixes wave counts");
    const int NW = wide ? max(J.NW, 2) : J.NW;
    const int w_lds = wide ? 0 : J.w_lds;
    const int NH = HELP ? J.NH : 0;
    const int ncomp = J.RPW * NW;
    const bool helper = HELP && wave >= ncomp;
    // compute waves first: the random-number waves share SIMDs with some of
    // them and must not delay the step's critical path
    if (HELP && !helper) __builtin_amdgcn_s_setprio(2);
    const int slot = helper ? (wave - ncomp) / NH : wave / NW;
    const int wr = helper ? (wave - ncomp) - slot * NH : wave - slot * NW;
    const int g = wr * 64 + lane;
    const int i0 = g * F;
    const int rr = blk * J.RPW + slot;
    // waves beyond the replica slots (the batched kernel always runs 16) hold
    // no replica and only keep the barrier count: their slot has fewer than NW
    // waves, so its exchange data would never be complete
    const bool idle = BATCH && !helper && slot >= J.RPW;
    const bool active = (slot < J.RPW) && (rr < J.R);
    const bool lane_has = !helper && active && (i0 < J.ld);
    // every flip of this wave is a variable of an active replica
    const bool full = active && !helper && (wr + 1) * 64 * F <= J.N;
    const int col0 = lane_has ? i0 : 0;     // row column this lane reads (ghost lanes: 0)
    const uint32_t rid = J.rid_base + (uint32_t)rr;
    const uint32_t k0 = (uint32_t)J.seed;
    const uint32_t k1 = (uint32_t)(J.seed >> 32);
    const int ld = J.ld;
    const int wscale = J.wscale;
    // the wide variants run 16-bit couplings only with a factor below 2^15
    const bool mul16 =
        sizeof(WT) == 2 && (wide || (wscale < (1 << 15) && wscale > -(1 << 15)));
    const bool mul24 = sizeof(WT) < 4 && wscale < (1 << 23) && wscale > -(1 << 23);
    constexpr bool stage = STAGE;
    const bool sync = HELP || NW > 1;       // a workgroup barrier every step
    const int nblk = (J.N + 7) >> 3;        // Philox blocks per replica-step
    const int eoff_cap = kEoffMax - J.eoff_inc;   // the host keeps inc in [0, 2^30]

    int64_t s0 = J.s0, s1 = J.s1;
    if (J.round_ptr) {
        const uint32_t t = *J.round_ptr;
        s0 = (int64_t)t * J.K;
        s1 = s0 + J.K;
    }

    // --- LDS carve-up: [W][brackets][direct table][per replica slot] ----------
    // LDS may hold dense W, or with sparse rows the row lists instead
    const int w_src = sparse ? J.N * J.ell_D * 4 : J.N * ld * (int)sizeof(WT);
    const int w_bytes = w_lds ? ((w_src + 15) & ~15) : 0;
    const WT *Wl = reinterpret_cast<const WT *>(smem);
    uint32_t *brk_l = reinterpret_cast<uint32_t *>(smem + w_bytes);
    // direct tables (narrow bands, anneal mode): the level's 65536 decisions
    constexpr bool dq = (MODE & kModeDirect) != 0;
    const bool has_q = dq && stage && !perstep && J.q8 != nullptr;
    const uint8_t *q_l = smem + w_bytes + kMaxBuckets * 4;
    // per-draw estimates handed over by the random-number waves (wide bands)
    constexpr bool gen = (MODE & kModeGen) != 0;
    // (with random-number waves they hand the estimates over; without, each
    // compute lane draws its block and evaluates them itself)
    static_assert(!gen || F >= 4, "estimates: 4 or 8 flips per lane");
    const SlotLayout SL = slot_layout(NW, NH, sparse ? F : 0, gen);
    uint8_t *sel = smem + w_bytes + (stage ? kMaxBuckets * 4 + (has_q ? 65536 : 0) : 0) +
                   (size_t)SL.bytes * slot;
    // lane records by step parity; a wave's total is its last lane's prefix
    const int RS = max(NW, 4) * 64;
    uint32_t *rec = reinterpret_cast<uint32_t *>(sel + SL.rec);    // [2][RS]
    int *dEs = reinterpret_cast<int *>(sel + SL.dEs);              // [2]
    uint32_t *vring = reinterpret_cast<uint32_t *>(sel + SL.vring);  // [128] selection draws
    // Philox blocks by step parity, each followed by its two int4 of estimates
    // in the estimate variants: block b of parity p at draws[p * PB + b * BS]
    uint4 *draws = reinterpret_cast<uint4 *>(sel + SL.draws);
    constexpr int BS = ((MODE & kModeGen) != 0) ? 3 : 1;
    const int PB = NH * 64 * BS;
    // sparse rows: this wave's field-delta buffer [64 * F], kept all zero between steps
    int *dh = reinterpret_cast<int *>(sel + SL.dh) + (helper ? 0 : wr) * 64 * F;
    if (sparse && !helper) {
#pragma unroll
        for (int f = 0; f < F; ++f) dh[lane * F + f] = 0;
    }

    if (w_lds) {
        const uint4 *src = reinterpret_cast<const uint4 *>(sparse ? (const void *)J.ell : J.W);
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        const int n16 = w_src / 16;
        for (int q = threadIdx.x; q < n16; q += blockDim.x) dst[q] = src[q];
        __syncthreads();
    }

    // --- replica state into registers --------------------------------------
    int h[F];
    uint32_t xb = 0, bxb = 0, vmask = 0;
#pragma unroll
    for (int f = 0; f < F; ++f) h[f] = 0;
    if (lane_has) {
        const size_t base = (size_t)rr * ld + i0;
        typedef typename VecOf<int, F>::type IV;
        typedef typename VecOf<uint8_t, F>::type BV;
        const IV hv = *reinterpret_cast<const IV *>(J.h + base);
        const BV xv = *reinterpret_cast<const BV *>(J.x + base);
        const BV bv = *reinterpret_cast<const BV *>(J.bx + base);
#pragma unroll
        for (int f = 0; f < F; ++f) {
            h[f] = hv[f];
            xb |= (uint32_t)(xv[f] & 1) << f;
            bxb |= (uint32_t)(bv[f] & 1) << f;
            if (i0 + f < J.N) vmask |= 1u << f;
        }
    }
    // estimate path: the x bits once more as bytes 0x00 / 0xFF, four flips per
    // word, so a flip's sign mask is one sign-extended byte operand (SDWA)
    constexpr int NXW = (F + 3) / 4;
    uint32_t xbw[NXW];
#pragma unroll
    for (int q = 0; q < NXW; ++q) xbw[q] = 0u;
    if constexpr (gen) {
#pragma unroll
        for (int f = 0; f < F; ++f) xbw[f >> 2] |= ((xb >> f) & 1u) ? (0xFFu << (8 * (f & 3))) : 0u;
    }
    int64_t E = 0, bE = 0, nacc = 0;
    int32_t eoff = 0;
    if (active && !helper) {
        E = J.E[rr];
        bE = J.bE[rr];
        eoff = J.eoff[rr];
        nacc = J.nacc[rr];
    }

    // --- level in force ----------------------------------------------------
    int lvl;
    int64_t s_next;
    if (J.lvl_of_rep) {
        // parallel tempering: one level per replica for the whole launch (a
        // round); with STAGE the workgroup holds one replica and stages its
        // level's brackets
        lvl = active ? J.lvl_of_rep[rr] : 0;
        s_next = INT64_MAX;
    } else {
        lvl = level_of(s0, J.L, J.S);
        s_next = uniform64(next_level_step(lvl, J.L, J.S));
    }
    LevelHdr hd = J.hdr[lvl];
    bool direct = false;   // this level decides in-band flips by its direct table
    bool fast = false;     // ... and this wave does so with one compare per flip
    bool fastb = false;    // wide band: one bracket read per flip, no band tests
    uint32_t ubmax = 0;    // first offset past the level's buckets
    auto stage_brackets = [&]() {
        __syncthreads();
        direct = has_q && hd.q8 >= 0;
        fast = dq && HELP && direct && full;
        // (only in the variants without direct tables: carried beside the
        // one-compare path, its code slows the narrow-band step)
        // (waves holding ghost flips mask them out of the result)
        fastb = !dq && HELP && active && !helper && !perstep && !single && hd.tmax < (1 << 29);
        if (direct) {
            const uint4 *src = reinterpret_cast<const uint4 *>(J.q8 + (size_t)hd.q8 * 65536);
            uint4 *dst = reinterpret_cast<uint4 *>(smem + w_bytes + kMaxBuckets * 4);
            const int bd = blockDim.x;
            // four loads in flight per thread; indices past the end are
            // clamped, so the last piece is just copied more than once
            for (int q0 = threadIdx.x; q0 < 4096; q0 += 4 * bd) {
                const int q1 = min(q0 + bd, 4095), q2 = min(q0 + 2 * bd, 4095),
                          q3 = min(q0 + 3 * bd, 4095);
                const uint4 a = src[q0], b = src[q1], c = src[q2], e = src[q3];
                dst[q0] = a;
                dst[q1] = b;
                dst[q2] = c;
                dst[q3] = e;
            }
        } else {
            const int nb = hd.tmax > hd.tmin ? ((hd.tmax - hd.tmin - 1) >> hd.sh) + 1 : 0;
            ubmax = (uint32_t)nb << hd.sh;
            // the buckets and the reject-all entry after them
            for (int q = threadIdx.x; q <= nb; q += blockDim.x) brk_l[q] = J.brk[hd.off + q];
        }
        __syncthreads();
    };
    if (stage) stage_brackets();

    // 16-bit draw of this lane's flip f from its Philox blocks
    // (forced inline: an out-of-line copy would keep the arrays in scratch)
    auto draw16 = [&](const uint4 (&r)[NB], int f) __attribute__((always_inline)) -> uint32_t {
        const int slice = (F >= 8) ? (f & 7) : ((HELP ? 0 : (i0 & 7)) + f);
        const uint32_t wv = word_of(r[f >> 3], slice >> 1);
        return (slice & 1) ? (wv >> 16) : (wv & 0xFFFFu);
    };
    // direct-table decisions of this lane's flips for the draws in r
    auto lookup_q = [&](const uint4 (&r)[NB], uint32_t (&q)[F]) __attribute__((always_inline)) {
#pragma unroll
        for (int f = 0; f < F; ++f) q[f] = q_l[draw16(r, f)];
    };

    // generator waves: the estimate coefficients of the level of the step
    // they produce (kept in scalar registers; updated when that step opens a
    // new level)
    int ggth = hd.gth;
    float gga = hd.ga, ggb = hd.gb;
    // generator waves: the draws of step st into ring slot st & 1, with the
    // per-draw estimates where its level uses them
    auto produce = [&](int64_t st) {
        const int b = g;   // Philox block of this generator lane
        if (active && b < nblk) {
            const uint4 r = philox((uint32_t)b, (uint32_t)st, rid, kTagMetropolis, k0, k1);
            uint4 *slot = draws + (int)(st & 1) * PB + b * BS;
            slot[0] = r;
            if (gen && ggth) {
                // draw 2q of the block is the low half of word q, 2q + 1 the high half
                int4 e0, e1;
                e0.x = draw_estimate(r.x & 0xFFFFu, gga, ggb);
                e0.y = draw_estimate(r.x >> 16, gga, ggb);
                e0.z = draw_estimate(r.y & 0xFFFFu, gga, ggb);
                e0.w = draw_estimate(r.y >> 16, gga, ggb);
                e1.x = draw_estimate(r.z & 0xFFFFu, gga, ggb);
                e1.y = draw_estimate(r.z >> 16, gga, ggb);
                e1.z = draw_estimate(r.w & 0xFFFFu, gga, ggb);
                e1.w = draw_estimate(r.w >> 16, gga, ggb);
                int4 *dst = reinterpret_cast<int4 *>(slot);
                dst[1] = e0;
                dst[2] = e1;
            }
        }
        // selection draws 64 steps at a time, one step per lane, at the first
        // step of every aligned run of 64 (and at the launch's first step): the
        // ring holds 128, so the run being written never meets the step being
        // read
        if (active && wr == NH - 1 && ((st & 63) == 0 || st == s0)) {
            const int64_t sl = (st & ~(int64_t)63) + lane;
            const uint32_t v = philox(0u, (uint32_t)sl, rid, kTagSelect, k0, k1).x;
            vring[(int)(sl & 127)] = v;
        }
    };
    // compute waves: this lane's draws of step st (written by the generators)
    // (o: element offset of the ring slot, (st & 1) * PB for step st)
    // (lanes past the last variable only hold ghost flips: their block index
    // is clamped, so they read a block in bounds)
    const int dblk = min(i0 >> 3, NH * 64 - 1);
    auto consume_at = [&](int o, uint4 (&dst)[NB]) {
        static_assert(NB == 1, "one Philox block per lane");
        if constexpr (BS > 1) {
            // (estimate variants: the block among its estimates)
            const uint4 *src = draws + o + dblk * BS;
            if (F >= 8) {
                dst[0] = src[0];
            } else {
                const uint2 p = reinterpret_cast<const uint2 *>(src)[(i0 >> 2) & 1];   // half
                dst[0] = make_uint4(p.x, p.y, p.x, p.y);
            }
        } else {
            const uint4 *src = draws + o;
            if (F >= 8) {
                dst[0] = src[dblk];
            } else if (F == 4) {
                const uint2 *s2 = reinterpret_cast<const uint2 *>(src);
                const uint2 p = s2[min(i0 >> 2, 2 * NH * 64 - 1)];   // half of block i0 >> 3
                dst[0] = make_uint4(p.x, p.y, p.x, p.y);
            } else {
                const uint32_t *s1 = reinterpret_cast<const uint32_t *>(src);
                const uint32_t w = s1[min(i0 >> 1, 4 * NH * 64 - 1)];   // word of block i0 >> 3
                dst[0] = make_uint4(w, w, w, w);
            }
        }
    };

    auto consume = [&](int64_t st, uint4 (&dst)[NB]) { consume_at((int)(st & 1) * PB, dst); };

    // compute waves: this lane's per-draw estimates of a step (o: element
    // offset of its ring slot, (st & 1) * PB for step st), stored after each
    // block's draws
    auto read_est_at = [&](int o, int (&dst)[F]) {
        if constexpr (gen && F >= 8) {
            const int4 *src = reinterpret_cast<const int4 *>(draws + o + dblk * BS);
            const int4 a = src[1], b = src[2];
            dst[0] = a.x; dst[1] = a.y; dst[2] = a.z; dst[3] = a.w;
            dst[4] = b.x; dst[5] = b.y; dst[6] = b.z; dst[7] = b.w;
        } else if constexpr (gen) {
            // four flips per lane: half a block, part (i0 >> 2) & 1 of block i0 >> 3
            const int4 *src = reinterpret_cast<const int4 *>(draws + o + dblk * BS);
            const int4 a = src[1 + ((i0 >> 2) & 1)];
            dst[0] = a.x; dst[1] = a.y; dst[2] = a.z; dst[3] = a.w;
        } else {
            (void)o;
        }
    };
    auto read_est = [&](int64_t st, int (&dst)[F]) { read_est_at((int)(st & 1) * PB, dst); };

    uint4 rb[NB];
    int tv[F];   // this step's per-draw estimates (kModeGen)
#pragma unroll
    for (int f = 0; f < F; ++f) tv[f] = 0;
    // with random-number waves the direct-table decisions of a step are read
    // one step ahead, as soon as its draws arrive
    uint32_t qv[F];
#pragma unroll
    for (int f = 0; f < F; ++f) qv[f] = 0u;
    if (HELP) {
        if (helper) produce(s0);
        __syncthreads();
        if (!helper) {
            consume(s0, rb);
            if (direct) lookup_q(rb, qv);
            if (gen) read_est(s0, tv);
        }
    }

    // single trial: the variable proposing at the current step (s mod N)
    int prop = single ? (int)(s0 % J.N) : 0;
    StepT st_next{0.0, -1, -1};
    if (perstep && !helper && s0 < s1) st_next = J.stepT[s0];

    // NW > 1: step s adds the energy change of step s - 1 from dEs (zero when
    // no flip was taken; both slots start at zero)
    if (NW > 1 && !helper && active && wr == 0 && lane == 0) {
        dEs[0] = 0;
        dEs[1] = 0;
    }
    // countdowns (steps left, steps to the next level) tested for equality
    // only: 64-bit equality is a scalar compare, ordering is not
    int64_t to_next = uniform64(s_next - s0);
    int64_t s = s0;
    // generator waves: step s + 1's draws during step s, and the same
    // barriers as the compute waves, level changes included
    if (HELP && helper) {
        for (int64_t left = s1 > s0 ? s1 - s0 : 0; left != 0; --left, ++s, --to_next) {
            if (to_next == 0) {
                lvl = level_of(s, J.L, J.S);
                s_next = next_level_step(lvl, J.L, J.S);
                to_next = uniform64(s_next - s);
                hd = J.hdr[lvl];
                if (stage) stage_brackets();
            }
            if (left != 1) {
                // step s + 1 may open the next level: its estimates use that one
                if (gen && to_next == 1) {
                    const int ln = __builtin_amdgcn_readfirstlane(level_of(s + 1, J.L, J.S));
                    const LevelHdr hn = J.hdr[ln];
                    ggth = __builtin_amdgcn_readfirstlane(hn.gth);
                    gga = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(hn.ga)));
                    ggb = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(hn.gb)));
                }
                produce(s + 1);
            }
            __syncthreads();
        }
    }
    // estimate path of the level in force, in scalar registers (set when a
    // level opens): whether this wave takes it, the window width and the step
    // constant without the offset
    bool gpath = false;
    uint32_t gWt = 0u, gC = 0u;
    auto gen_level = [&]() {
        if constexpr (gen) {
            gpath = J.gth && full && __builtin_amdgcn_readfirstlane(hd.gth) != 0;
            const int glo = __builtin_amdgcn_readfirstlane(hd.glo);
            const int ghi = __builtin_amdgcn_readfirstlane(hd.ghi);
            gWt = (uint32_t)(ghi - glo) + 1u;
            gC = 0u - ((uint32_t)glo + kGenMagic);
        }
    };
    gen_level();
    // LDS slots by step parity, toggled every step: this step's lane records
    // and the next step's draws and estimates (element offsets)
    int rec_o = (int)(s0 & 1) * RS;
    int drw_o = (int)((s0 + 1) & 1) * PB;
    // (the loop ends at step s1e, compared for equality; the random-number
    // waves have already run their steps, and s stands past them)
    const int64_t s1e = (HELP && helper) ? s : (s1 > s0 ? s1 : s0);
    // (a level opens at step s_next: the compute waves compare the step with it)
    for (; s != s1e; ++s, rec_o = RS - rec_o, drw_o = PB - drw_o) {
        if (s == s_next) {
            lvl = level_of(s, J.L, J.S);
            s_next = uniform64(next_level_step(lvl, J.L, J.S));
            hd = J.hdr[lvl];
            gen_level();
            if (stage) {
                stage_brackets();
                if (HELP && direct) lookup_q(rb, qv);
            }
        }
        const int par = (int)(s & 1);
        // per-step schedule: this step's temperature and band (loaded one
        // step ahead)
        double Tstep = 0.0;
        if (perstep) {
            Tstep = st_next.T;
            hd.tmin = st_next.tmin;
            hd.tmax = st_next.tmax;
            if (s + 1 != s1e) st_next = J.stepT[s + 1];
        }
        int d[F];
        uint32_t acc = 0;
        int c = 0, excl = 0, wtot = 0;

        if (gen && gpath) {
            // wide band with per-draw estimates G(u): thr[u] lies in
            // [glo - G, ghi - G], so with z = d - glo + G - 1 (d = (1 - 2x) h -
            // E_off) a flip is accepted when z < 0, rejected when z >= ghi - glo,
            // and only in between is thr[u] read.  Taking (1 - 2x) h as h ^ -x
            // (one's complement, short by one when x = 1) and adding 1 gives
            // zz in {z, z + 1}: zz < 0 still implies z < 0 and zz > ghi - glo
            // still implies z >= ghi - glo, so the same tests hold with a window
            // one wider, at one xor (the sign mask a sign-extended byte operand)
            // and one three-input add per flip.  The host allows this path only
            // for |h| <= kGenFieldMax and levels with tmax < 2^22 and |glo|,
            // |ghi| <= kGenOffMax, so z is in int32; the ring holds G +
            // kGenMagic, so the sum wraps through 2^32 on the way (unsigned
            // arithmetic) and lands on zz.  The sign bits of zz shift straight
            // into the accepted mask.
            const uint32_t negEc = gC - (uint32_t)eoff;
            const uint32_t Wt = gWt;
            if constexpr (!HELP) {
                // no random-number waves: this lane's block of the step, and
                // its estimates, here
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    rb[q] = philox((uint32_t)(i0 >> 3) + q, (uint32_t)s, rid, kTagMetropolis, k0,
                                   k1);
#pragma unroll
                for (int f = 0; f < F; ++f) tv[f] = draw_estimate(draw16(rb, f), hd.ga, hd.gb);
            }
            uint32_t zmin = 0xFFFFFFFFu;
            int zv[F];
#pragma unroll
            for (int f = F - 1; f >= 0; --f) {
                const int mx = (int)(int8_t)(xbw[f >> 2] >> (8 * (f & 3)));   // -x
                const uint32_t hx = (uint32_t)(h[f] ^ mx);
                uint32_t zs;
                asm("v_add3_u32 %0, %1, %2, %3" : "=v"(zs) : "v"(hx), "v"(tv[f]), "v"(negEc));
                const int z = (int)zs;
                zv[f] = z;
                acc = __builtin_amdgcn_alignbit(acc, (uint32_t)z, 31);
                zmin = min(zmin, (uint32_t)z);
            }
            if (ballot(zmin < Wt)) {
                // a flip inside the window (rare): the exact table entry.  This
                // step's draws are still in ring slot s & 1.
                uint4 rt[NB];
                if constexpr (HELP) consume(s, rt);
                else {
#pragma unroll
                    for (int q = 0; q < NB; ++q) rt[q] = rb[q];
                }
                const int32_t *thr = J.thr + (size_t)lvl * 65536;
                int t[F];
#pragma unroll
                for (int f = 0; f < F; ++f)
                    t[f] = thr[((uint32_t)zv[f] < Wt) ? draw16(rt, f) : 0u];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const int mx = -(int)((xb >> f) & 1u);
                    const int dd = ((h[f] ^ mx) - mx) - eoff;
                    acc |= (uint32_t)(((uint32_t)zv[f] < Wt) & (dd <= t[f])) << f;
                }
            }
            c = __popc(acc);
            wave_scan(c, excl, wtot);
            if (NW > 1) rec[rec_o + g] = acc | (xb << 8) | ((uint32_t)(excl + c) << 16);
        } else if (fast) {
            // 1-3a, narrow band with the decisions' table entries already read:
            // with s = (1 - 2x) h the flip is accepted iff s - E_off <= thr[u]
            // = tmin + q[u], i.e. s < q[u] + c with c = tmin + 1 + E_off.  As
            // q <= tmax - tmin this one compare also decides the flips below
            // and above the band.  |s| <= 2^30, E_off <= 2^30 and a direct
            // level's |tmin| <= 256, so nothing here leaves int32.  The wave
            // prefix of the accepted counts is the running sum of the lanes
            // below in the F compare masks.
            const int cc = hd.tmin + 1 + eoff;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                // (h ^ mx) - mx = s, compared as (h ^ mx) < q + c + mx
                const int mx = -(int)((xb >> f) & 1u);
                const bool p = (h[f] ^ mx) < (int)qv[f] + cc + mx;
                const uint64_t pm = ballot(p);
                acc |= (uint32_t)p << f;
                excl = __builtin_amdgcn_mbcnt_hi((uint32_t)(pm >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)pm, excl));
                wtot += (int)__popcll(pm);
            }
            c = __popc(acc);
            if (NW > 1) rec[rec_o + g] = acc | (xb << 8) | ((uint32_t)(excl + c) << 16);
        } else if (fastb) {
            // wide band with the draws at hand: one bracket read per flip and
            // no band tests.  With s = (1 - 2x) h and C = tmin + 1 + E_off,
            // s < C is below the band (accepted).  ub = s - C as an unsigned
            // number indexes the buckets; offsets past them (above the band,
            // and below it after the wrap) read the level's reject-all entry,
            // and costs above tmax inside the last bucket meet its lower cut
            // of 0, so the exact entry decides them.  tmax < 2^29 keeps C in
            // int32.
            const int C = hd.tmin + 1 + eoff;
            int sv[F];
            uint32_t u[F], e[F];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const int mx = -(int)((xb >> f) & 1u);
                sv[f] = (h[f] ^ mx) - mx;
                const uint32_t ub = (uint32_t)sv[f] - (uint32_t)C;
                acc |= (uint32_t)(sv[f] < C) << f;
                u[f] = draw16(rb, f);
                e[f] = brk_l[min(ub, ubmax) >> hd.sh];
            }
            uint32_t fine = 0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const uint32_t lo = e[f] & 0xFFFFu, hi = e[f] >> 16;
                acc |= (uint32_t)(u[f] < lo) << f;
                fine |= (uint32_t)((u[f] >= lo) & (u[f] < hi)) << f;
            }
            if (fine) {
                const int32_t *thr = J.thr + (size_t)lvl * 65536;
                int t[F];
#pragma unroll
                for (int f = 0; f < F; ++f) t[f] = thr[((fine >> f) & 1u) ? u[f] : 0u];
#pragma unroll
                for (int f = 0; f < F; ++f)
                    acc |= (((fine >> f) & 1u) & (uint32_t)(sv[f] - eoff <= t[f])) << f;
            }
            if (!full) acc &= vmask;   // flips past the last variable are never accepted
            c = __popc(acc);
            wave_prefix<CountBits<F>::value>(c, excl, wtot);
            if (NW > 1) rec[rec_o + g] = acc | (xb << 8) | ((uint32_t)(excl + c) << 16);
        } else if (!idle) {
            // 1. cost of every flip and the draw-free decisions (branch-free).
            // Without direct tables the band tmin < d <= tmax is tested as one
            // unsigned compare of ub = d - (tmin + 1) against tmax - tmin, and
            // ub also indexes the brackets (measured faster there; with direct
            // tables the two-compare form is)
            const int t1 = hd.tmin + 1;
            const uint32_t span = (uint32_t)(hd.tmax - hd.tmin);
            uint32_t inb = 0, ub[F];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const int hv = h[f];
                const int dd = (((xb >> f) & 1u) ? -hv : hv) - eoff;
                d[f] = dd;
                const uint32_t v = (vmask >> f) & 1u;
                if constexpr (dq) {
                    acc |= (v & (uint32_t)(dd <= hd.tmin)) << f;
                    inb |= (v & (uint32_t)(dd > hd.tmin) & (uint32_t)(dd <= hd.tmax)) << f;
                } else {
                    ub[f] = (uint32_t)dd - (uint32_t)t1;
                    acc |= (v & (uint32_t)(dd < t1)) << f;
                    inb |= (v & (uint32_t)(ub[f] < span)) << f;
                }
            }
            // single-trial mode: only variable s mod N proposes this step
            if (single) {
                const uint32_t sm = (g == (prop / F)) ? (1u << (prop % F)) : 0u;
                acc &= sm;
                inb &= sm;
            }
            // 2. in-band flips: 16-bit draw and bracket.  Every bracket read is
            // issued (out-of-band flips read entry 0) and waited on once; the
            // threshold table is read only inside a non-exact bracket (rare).
            if (inb && direct) {
                // narrow band: ub = d - tmin - 1 is accepted iff ub < q[u]
                if (!HELP) {
#pragma unroll
                    for (int q = 0; q < NB; ++q)
                        rb[q] = philox((uint32_t)(i0 >> 3) + q, (uint32_t)s, rid, kTagMetropolis,
                                       k0, k1);
                    lookup_q(rb, qv);
                }
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const uint32_t ub = (uint32_t)(d[f] - hd.tmin - 1);
                    acc |= (((inb >> f) & 1u) & (uint32_t)(ub < qv[f])) << f;
                }
            } else if (inb) {
                if (!HELP) {
#pragma unroll
                    for (int q = 0; q < NB; ++q)
                        rb[q] = philox((uint32_t)(i0 >> 3) + q, (uint32_t)s, rid, kTagMetropolis,
                                       k0, k1);
                }
                uint32_t u[F], e[F];
                if (perstep) {
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        const int slice = (F >= 8) ? (f & 7) : ((HELP ? 0 : (i0 & 7)) + f);
                        const uint32_t wv = word_of(rb[f >> 3], slice >> 1);
                        u[f] = (slice & 1) ? (wv >> 16) : (wv & 0xFFFFu);
                    }
                    // per-step schedule: d <= ceil(T G[u]) - 1 <=> d < T G[u]
                    // (G[u] = -ln U_u; one IEEE product, the threshold's own)
                    double gv[F];
#pragma unroll
                    for (int f = 0; f < F; ++f) gv[f] = J.G[((inb >> f) & 1u) ? u[f] : 0u];
#pragma unroll
                    for (int f = 0; f < F; ++f)
                        acc |= (((inb >> f) & 1u) & (uint32_t)((double)d[f] < Tstep * gv[f]))
                               << f;
                    inb = 0;
                }
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const int slice = (F >= 8) ? (f & 7) : ((HELP ? 0 : (i0 & 7)) + f);
                    const uint32_t wv = word_of(rb[f >> 3], slice >> 1);
                    u[f] = (slice & 1) ? (wv >> 16) : (wv & 0xFFFFu);
                    // out-of-band flips read a valid bucket they then ignore
                    const int bi = dq ? (((inb >> f) & 1u) ? ((d[f] - hd.tmin - 1) >> hd.sh) : 0)
                                      : (int)(min(ub[f], span - 1u) >> hd.sh);
                    e[f] = stage ? brk_l[bi] : J.brk[hd.off + bi];
                }
                uint32_t fine = 0;
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const uint32_t ib = (inb >> f) & 1u;
                    const uint32_t lo = e[f] & 0xFFFFu, hi = e[f] >> 16;
                    acc |= (ib & (uint32_t)(u[f] < lo)) << f;
                    fine |= (ib & (uint32_t)(u[f] >= lo) & (uint32_t)(u[f] < hi)) << f;
                }
                if (fine) {
                    const int32_t *thr = J.thr + (size_t)lvl * 65536;
                    int t[F];
#pragma unroll
                    for (int f = 0; f < F; ++f) t[f] = thr[((fine >> f) & 1u) ? u[f] : 0u];
#pragma unroll
                    for (int f = 0; f < F; ++f)
                        acc |= (((fine >> f) & 1u) & (uint32_t)(d[f] <= t[f])) << f;
                }
            }
            // 3a. accepted count, prefix over the wave; publish for the others
            c = __popc(acc);
            wave_prefix<CountBits<F>::value>(c, excl, wtot);
            // record: accepted mask | x bits << 8 | inclusive prefix << 16
            if (NW > 1) rec[rec_o + g] = acc | (xb << 8) | ((uint32_t)(excl + c) << 16);
        }
        if (sync) __syncthreads();
        if (idle) continue;

        // 3b. the chosen flip.  Everything this step needs from LDS is read
        // in one straight-line group (clamped indices, no branches), so the
        // wave waits for LDS once.
        // (on the last step these read draws no step uses: stale, in bounds)
        uint4 rbn[NB];
        if (HELP) consume_at(drw_o, rbn);
        int tvn[F];
        if (gen && HELP) read_est_at(drw_o, tvn);
        const uint32_t vs = HELP ? vring[(int)(s & 127)] : 0u;
        int dEp = 0, tw = 0;
        uint32_t r4[4] = {0u, 0u, 0u, 0u};
        if (NW > 1) {
            dEp = dEs[par ^ 1];
            const int twr = (int)(rec[rec_o + min(lane, NW - 1) * 64 + 63] >> 16);
#pragma unroll
            for (int q = 0; q < 4; ++q) r4[q] = rec[rec_o + q * 64 + lane];
            tw = lane < NW ? twr : 0;
            // keep these reads together: left to itself the compiler sinks
            // the draw and record reads into the branches that use them, so
            // the step would wait for LDS three times in a row
            asm volatile("" ::"v"(r4[0]), "v"(r4[1]), "v"(r4[2]), "v"(r4[3]), "v"(tw), "v"(vs),
                         "v"(dEp));
        } else if (HELP) {
            asm volatile("" ::"v"(vs));
        }
        if (gen && HELP) {
#pragma unroll
            for (int f = 0; f < F; ++f) asm volatile("" ::"v"(tvn[f]));
        }
        int m, k = 0, xk = 0, dk = 0, bit = 0;
        int kw = 0, kl = 0;   // wave and lane holding the chosen flip
        if (NW == 1) {
            m = wtot;
            if (m > 0) {
                const uint32_t v = HELP ? (uint32_t)__builtin_amdgcn_readfirstlane((int)vs)
                                        : philox_x_uniform(0u, (uint32_t)s, rid, kTagSelect, k0, k1);
                const int j = (int)(((uint64_t)v * (uint32_t)m) >> 32);
                const uint64_t bal = ballot(excl + c > j);
                const int ts = (int)__builtin_ctzll(bal);
                const int rloc = j - readlane(excl, ts);
                const uint32_t msk = (uint32_t)readlane((int)acc, ts);
                bit = select_bit<F>(msk, rloc);
                kl = ts;
                k = ts * F + bit;
                xk = (readlane((int)xb, ts) >> bit) & 1;
                // energy change (1 - 2 x_k) h_k of the chosen flip
                int hsel = h[0];
#pragma unroll
                for (int f = 1; f < F; ++f) hsel = (bit == f) ? h[f] : hsel;
                const int hk = readlane(hsel, ts);
                dk = xk ? -hk : hk;
            }
        } else {
            // wave totals sit in lanes 0..NW-1: a scan over 4 lanes suffices
            // for up to 4 waves
            int scan = tw;
            scan += __builtin_amdgcn_update_dpp(0, scan, 0x111, 0xf, 0xf, false);  // row_shr:1
            scan += __builtin_amdgcn_update_dpp(0, scan, 0x112, 0xf, 0xf, false);  // row_shr:2
            if (!nw4 && NW > 4) {
                scan += __builtin_amdgcn_update_dpp(0, scan, 0x114, 0xf, 0xf, false);  // row_shr:4
                scan += __builtin_amdgcn_update_dpp(0, scan, 0x118, 0xf, 0xf, false);  // row_shr:8
            }
            m = readlane(scan, NW - 1);
            if (m > 0) {
                const uint32_t v = HELP ? (uint32_t)__builtin_amdgcn_readfirstlane((int)vs)
                                        : philox_x_uniform(0u, (uint32_t)s, rid, kTagSelect, k0, k1);
                const int j = (int)(((uint64_t)v * (uint32_t)m) >> 32);
                // (lane NW - 1 holds m > j, so the first lane found is a wave
                // index; with four-lane windows the mask is not needed)
                const uint64_t wbal =
                    nw4 ? ballot(scan > j) : ballot(scan > j) & ((1ull << NW) - 1ull);
                const int ws = (int)__builtin_ctzll(wbal);
                const int jw = j - (readlane(scan, ws) - readlane(tw, ws));
                uint32_t r2;
                if (nw4 || NW <= 4) {
                    const uint32_t r01 = (ws & 1) ? r4[1] : r4[0];
                    const uint32_t r23 = (ws & 1) ? r4[3] : r4[2];
                    r2 = (ws & 2) ? r23 : r01;
                } else {
                    r2 = rec[rec_o + ws * 64 + lane];
                }
                // first lane of wave ws whose inclusive prefix passes jw
                const uint64_t bal = ballot((int)(r2 >> 16) > jw);
                const int ts = (int)__builtin_ctzll(bal);
                const uint32_t rs = (uint32_t)readlane((int)r2, ts);
                // the flip: the set bit of the lane's mask with incl - jw set
                // bits at or above it (incl its inclusive prefix; 1 <= incl -
                // jw <= its count), found by lanes 0..F-1 at once
                const uint32_t need = (rs >> 16) - (uint32_t)jw;
                const uint64_t hit = ballot((uint32_t)__popc(rs & ge_mask) == need);
                bit = (int)__builtin_ctz((uint32_t)hit & rs);
                kw = ws;
                kl = ts;
                k = (ws * 64 + ts) * F + bit;
                xk = (rs >> (8 + bit)) & 1;
            }
        }

        // 4. fetch row k of W (the step's only bulk traffic), then, while it
        // is in flight, finish the previous step's energy and best state
        // (one branch on m: the work between the fetch and its use is written
        // out in both arms)
        auto finish_prev = [&]() __attribute__((always_inline)) {
            // the next step's direct-table decisions (its draws arrived with
            // this step's exchange); a level change re-reads them after staging
            if (HELP && direct) lookup_q(rbn, qv);
            if (NW > 1) {
                // the previous step's energy change (written by its owner lane)
                E += (int64_t)__builtin_amdgcn_readfirstlane(dEp);
                const bool better = E < bE;
                bE = better ? E : bE;
                bxb = better ? xb : bxb;
                if (TRACE && active && g == 0 && s != s0) T.E[rr * T.stride + (s - 1 - s0)] = E;
            }
        };
        if (m > 0) {
            RowV raw;
            if (!sparse) {
                // address-space-typed loads: a generic pointer would make this
                // one flat load that waits on both the vector and the LDS
                // counters
                typedef __attribute__((address_space(3))) const RowV LdsRowV;
                typedef __attribute__((address_space(1))) const RowV GlobalRowV;
                if (w_lds) raw = *(LdsRowV *)(Wl + (size_t)k * ld + col0);
                else
                    raw = *(GlobalRowV *)(reinterpret_cast<const WT *>(J.W) + (size_t)k * ld +
                                          col0);
            }
            finish_prev();
            // apply the flip: state, energy, every field
            const int delta = xk ? -1 : 1;
            // the flip's state changes in one lane of one wave: the other
            // waves skip this by a wave-uniform branch
            if (NW == 1 || kw == wr) {
                int hk = 0;
                if (NW > 1) hk = readlane(pick_field<F>(h, bit), kl);
                if (lane == kl) {
                    if (NW > 1) dEs[par] = xk ? -hk : hk;   // (1 - 2 x_k) h_k
                    xb ^= 1u << bit;
                    if constexpr (gen) {
                        const uint32_t mb = 0xFFu << (8 * (bit & 3));
                        xbw[0] ^= bit < 4 ? mb : 0u;
                        if (NXW > 1) xbw[NXW - 1] ^= bit < 4 ? 0u : mb;
                    }
                }
            }
            if (sparse) {
                // only k's neighbours change.  Each wave takes the entries of
                // row k's list that fall in its own columns: one lane per
                // entry scatters the value into the wave's delta buffer, every
                // lane reads its F slots and clears them.  LDS operations of
                // one wave complete in order, so no barrier.
                const int dw = delta * wscale;
                const uint32_t *er = (w_lds ? reinterpret_cast<const uint32_t *>(smem) : J.ell) +
                                     (size_t)k * J.ell_D;
                const int base = wr * 64 * F;
                for (int q0 = 0; q0 < J.ell_D; q0 += 64) {
                    const int j = min(q0 + lane, J.ell_D - 1);
                    const uint32_t e = w_lds ? *(__attribute__((address_space(3))) const uint32_t *)(er + j)
                                               : er[j];
                    const int c = (int)(e & 0xFFFFu) - base;
                    if (q0 + lane < J.ell_D && (unsigned)c < (unsigned)(64 * F))
                        dh[c] = (int)e >> 16;
                }
                int dv[F];
#pragma unroll
                for (int f = 0; f < F; ++f) dv[f] = dh[lane * F + f];
#pragma unroll
                for (int f = 0; f < F; ++f) h[f] += dv[f] * dw;
#pragma unroll
                for (int f = 0; f < F; ++f) dh[lane * F + f] = 0;
            } else if (mul16) {
                update_i16<WT, F>(raw, delta * wscale, h);
            } else if (mul24) {
                // 8/16-bit couplings times a common factor below 2^23: each
                // product is exact as a 24-bit multiply-add, done in place
                const int dw = delta * wscale;
#pragma unroll
                for (int f = 0; f < F; ++f)
                    asm("v_mad_i32_i24 %0, %1, %2, %0" : "+v"(h[f]) : "v"((int)raw[f]), "s"(dw));
            } else if (wscale == 1) {
                // h + (+-raw): xor with the sign, add the sign's two's-complement fix
                const int sx = delta > 0 ? 0 : -1;
#pragma unroll
                for (int f = 0; f < F; ++f) h[f] = h[f] + ((int)raw[f] ^ sx) - sx;
            } else {
#pragma unroll
                for (int f = 0; f < F; ++f) h[f] += delta * ((int)raw[f] * wscale);
            }
            ++nacc;
            if (NW == 1) {
                E += (int64_t)dk;
                const bool better = E < bE;
                bE = better ? E : bE;
                bxb = better ? xb : bxb;
            }
            eoff = 0;
        } else {
            finish_prev();
            if (NW > 1 && wr == 0 && lane == 0) dEs[par] = 0;
            // min(E_off + inc, 2^30) without leaving int32 (E_off, inc in [0, 2^30])
            eoff = min(eoff, eoff_cap) + J.eoff_inc;
            k = -1;
        }
        if (HELP) {
#pragma unroll
            for (int q = 0; q < NB; ++q) rb[q] = rbn[q];
        }
        if (gen && HELP) {
#pragma unroll
            for (int f = 0; f < F; ++f) tv[f] = tvn[f];
        }
        if (single) prop = (prop + 1 == J.N) ? 0 : prop + 1;
        if (TRACE && active && g == 0) {
            T.k[rr * T.stride + (s - s0)] = k;
            T.eoff[rr * T.stride + (s - s0)] = eoff;
            if (NW == 1 || k < 0) T.E[rr * T.stride + (s - s0)] = E;
        }
    }
    if (NW > 1 || HELP) {
        // the last step's energy change
        __syncthreads();
        if (NW > 1 && !helper && s1e != s0) {
            E += (int64_t)dEs[(int)((s1 - 1) & 1)];
            if (E < bE) {
                bE = E;
                bxb = xb;
            }
            if (TRACE && active && g == 0) T.E[rr * T.stride + (s1 - 1 - s0)] = E;
        }
    }
    if (helper) return;

    // --- state back to HBM -------------------------------------------------
    if (lane_has) {
        const size_t base = (size_t)rr * ld + i0;
        typedef typename VecOf<int, F>::type IV;
        typedef typename VecOf<uint8_t, F>::type BV;
        IV hv;
        BV xv, bv;
#pragma unroll
        for (int f = 0; f < F; ++f) {
            hv[f] = h[f];
            xv[f] = (uint8_t)((xb >> f) & 1u);
            bv[f] = (uint8_t)((bxb >> f) & 1u);
        }
        *reinterpret_cast<IV *>(J.h + base) = hv;
        *reinterpret_cast<BV *>(J.x + base) = xv;
        *reinterpret_cast<BV *>(J.bx + base) = bv;
    }
    if (active && g == 0) {
        J.E[rr] = E;
        J.bE[rr] = bE;
        J.eoff[rr] = eoff;
        J.nacc[rr] = nacc;
    }
}

template <typename WT, int F, bool TRACE, bool HELP, bool STAGE, int MODE>
__global__ __launch_bounds__(1024) void k_run(JobDesc J, TraceDesc T) {
    extern __shared__ __align__(16) uint8_t smem[];
    run_block<WT, F, TRACE, HELP, STAGE, MODE>(J, blockIdx.x, smem, T);
}

// Persistent batched form: workgroups pull (job, replica-block) items from a
// device counter until none are left.  Every item of a launch uses the
// launch's workgroup size; jobs of any size and coupling type mix freely.
template <int F, int MODE>
__global__ __launch_bounds__(1024) void k_batch(const JobDesc *__restrict__ jobs,
                                                const BatchItem *__restrict__ items,
                                                const int32_t *n_items_ptr, int32_t *counter) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ int item_id;
    const TraceDesc T{nullptr, nullptr, nullptr, 0};
    const int n_items = *n_items_ptr;
    for (;;) {
        if (threadIdx.x == 0) item_id = atomicAdd(counter, 1);
        __syncthreads();
        const int it = item_id;
        __syncthreads();
        if (it >= n_items) break;
        const BatchItem bi = items[it];
        JobDesc J = jobs[bi.job];
        const int blk = bi.r0 / J.RPW;
        if (J.dtype == 1) run_block<int8_t, F, false, false, true, MODE, true>(J, blk, smem, T);
        else if (J.dtype == 2) run_block<int16_t, F, false, false, true, MODE, true>(J, blk, smem, T);
        else run_block<int32_t, F, false, false, true, MODE, true>(J, blk, smem, T);
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// Initial states.
// --------------------------------------------------------------------------

// Common all-zero start: x = 0, h = b, E = 0 (Algorithm 2 runs all start from
// the same state, which spares computing fields and energies per run).
__global__ void k_state_zero(JobDesc J) {
    const int64_t n = (int64_t)J.R * J.ld;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % J.ld);
        J.h[q] = J.b[i];
        J.x[q] = 0;
        J.bx[q] = 0;
        if (i == 0) {
            const int64_t r = q / J.ld;
            J.E[r] = 0;
            J.bE[r] = 0;
            J.eoff[r] = 0;
            J.nacc[r] = 0;
        }
    }
}

// Random start: bit i of replica id rid_base + r is bit (i & 31) of word
// (i >> 5) & 3 of Philox(i >> 7, 0, rid, init tag).
__global__ void k_rand_bits(uint8_t *X, int32_t R, int32_t N, int32_t ld, uint32_t rid_base,
                            uint64_t seed) {
    const int64_t n = (int64_t)R * ld;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % ld);
        const uint32_t r = (uint32_t)(q / ld);
        uint8_t bit = 0;
        if (i < N) {
            const uint4 w = philox((uint32_t)i >> 7, 0u, rid_base + r, kTagInit, k0, k1);
            bit = (uint8_t)((word_of(w, (i >> 5) & 3) >> (i & 31)) & 1u);
        }
        X[q] = bit;
    }
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Initial fields H = X W^T + b for int8 couplings on the matrix cores:
// v_mfma_i32_32x32x32_i8, exact int8 x int8 -> int32.  One wave per 32 x 32
// output tile (32 replicas x 32 variables); both operands are read with the
// reduction index contiguous (rows of X and rows of the symmetric W).
__global__ __launch_bounds__(256) void k_fields_mfma_i8(const uint8_t *__restrict__ X,
                                                        const int8_t *__restrict__ W,
                                                        const int32_t *__restrict__ b,
                                                        int32_t *__restrict__ H, int32_t R,
                                                        int32_t ld, int32_t wscale) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int tiles_i = ld / 32;
    const int tr = wave / tiles_i, ti = wave - tr * tiles_i;
    const int r0 = tr * 32, c0 = ti * 32;
    if (r0 >= R) return;
    const int row = lane & 31, kh = (lane >> 5) * 16;
    const int ra = min(r0 + row, R - 1);
    const int8_t *pa = reinterpret_cast<const int8_t *>(X) + (size_t)ra * ld + kh;
    const int8_t *pb = W + (size_t)(c0 + row) * ld + kh;
    v16i acc = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int kk = 0; kk < ld; kk += 32) {
        const v4i a = *reinterpret_cast<const v4i *>(pa + kk);
        const v4i bb = *reinterpret_cast<const v4i *>(pb + kk);
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, bb, acc, 0, 0, 0);
    }
    const int col = c0 + (lane & 31);
    const int bcol = b[col];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int r = r0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (r < R) H[(size_t)r * ld + col] = acc[v] * wscale + bcol;
    }
}

// Tiled form of the same product for large R x N: a workgroup computes a
// 128 (replicas) x 128 (variables) block of H with 4 waves of 64 x 64 (2 x 2
// MFMA tiles each); K advances 64 at a time through LDS (both operands are
// K-contiguous: rows of X, rows of the symmetric W), so every operand byte
// read from memory feeds 4 MFMAs.  LDS rows are padded to 80 bytes so the
// 16-byte fragment reads of 32 consecutive rows spread over the banks.
constexpr int kFT = 128, kFK = 64, kFRow = kFK + 16;

__global__ __launch_bounds__(256) void k_fields_mfma_i8_tiled(
    const uint8_t *__restrict__ X, const int8_t *__restrict__ W, const int32_t *__restrict__ b,
    int32_t *__restrict__ H, int32_t R, int32_t ld, int32_t wscale) {
    __shared__ __align__(16) int8_t As[kFT * kFRow];
    __shared__ __align__(16) int8_t Bs[kFT * kFRow];
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    const int r0 = blockIdx.x * kFT, c0 = blockIdx.y * kFT;
    // staging: thread t copies 32 bytes of row t/2 (k half t&1) of each tile
    const int srow = t >> 1, sk = (t & 1) * 32;
    const int ar = min(r0 + srow, R - 1);
    const bool bvalid = c0 + srow < ld;
    const int8_t *ga = reinterpret_cast<const int8_t *>(X) + (size_t)ar * ld + sk;
    const int8_t *gb = W + (size_t)(bvalid ? c0 + srow : 0) * ld + sk;
    v16i acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0;
    const int frow = lane & 31, fk = (lane >> 5) * 16;
    const v4i zero = {0, 0, 0, 0};
    // the next tile's operands are fetched into registers while this one computes
    v4i a0 = *reinterpret_cast<const v4i *>(ga);
    v4i a1 = *reinterpret_cast<const v4i *>(ga + 16);
    v4i b0 = bvalid ? *reinterpret_cast<const v4i *>(gb) : zero;
    v4i b1 = bvalid ? *reinterpret_cast<const v4i *>(gb + 16) : zero;
    for (int k0 = 0; k0 < ld; k0 += kFK) {
        __syncthreads();   // the previous tile is no longer read
        *reinterpret_cast<v4i *>(As + srow * kFRow + sk) = a0;
        *reinterpret_cast<v4i *>(As + srow * kFRow + sk + 16) = a1;
        *reinterpret_cast<v4i *>(Bs + srow * kFRow + sk) = b0;
        *reinterpret_cast<v4i *>(Bs + srow * kFRow + sk + 16) = b1;
        __syncthreads();
        if (k0 + kFK < ld) {
            a0 = *reinterpret_cast<const v4i *>(ga + k0 + kFK);
            a1 = *reinterpret_cast<const v4i *>(ga + k0 + kFK + 16);
            b0 = bvalid ? *reinterpret_cast<const v4i *>(gb + k0 + kFK) : zero;
            b1 = bvalid ? *reinterpret_cast<const v4i *>(gb + k0 + kFK + 16) : zero;
        }
#pragma unroll
        for (int kc = 0; kc < kFK; kc += 32) {
            v4i fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                fa[i] = *reinterpret_cast<const v4i *>(As + (wm * 64 + i * 32 + frow) * kFRow +
                                                       kc + fk);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                fb[j] = *reinterpret_cast<const v4i *>(Bs + (wn * 64 + j * 32 + frow) * kFRow +
                                                       kc + fk);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[i], fb[j], acc[i][j],
                                                                      0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = c0 + wn * 64 + j * 32 + (lane & 31);
        if (col >= ld) continue;
        const int bcol = b[col];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = r0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                if (r < R) H[(size_t)r * ld + col] = acc[i][j][v] * wscale + bcol;
            }
    }
}

// Initial fields for int16 / int32 couplings: one workgroup per replica adds
// row j of W for every set bit x_j (rows are coalesced across the workgroup).
template <typename WT>
__global__ __launch_bounds__(256) void k_fields_rows(const uint8_t *__restrict__ X,
                                                     const WT *__restrict__ W,
                                                     const int32_t *__restrict__ b,
                                                     int32_t *__restrict__ H, int32_t N,
                                                     int32_t ld, int32_t wscale) {
    const int r = blockIdx.x;
    const uint8_t *xr = X + (size_t)r * ld;
    for (int i0 = 0; i0 < ld; i0 += blockDim.x) {
        const int i = i0 + threadIdx.x;
        int acc = 0;
        for (int j = 0; j < N; ++j)
            if (xr[j]) acc += (i < ld ? (int)W[(size_t)j * ld + i] : 0);
        if (i < ld) H[(size_t)r * ld + i] = acc * wscale + b[i];
    }
}

// E = b.x + (1/2) x.(h - b) = (1/2) sum_i x_i (h_i + b_i), exact in int64.
// With finish_state the replica state is completed (x copied to best, offsets
// and counters cleared); otherwise only E_out is written.
__global__ __launch_bounds__(256) void k_energy_from_fields(const uint8_t *__restrict__ X,
                                                            const int32_t *__restrict__ H,
                                                            const int32_t *__restrict__ b,
                                                            int32_t ld, int64_t *E_out,
                                                            int finish, uint8_t *bx,
                                                            int64_t *bE, int32_t *eoff,
                                                            int64_t *nacc) {
    __shared__ long long part[256];
    const int r = blockIdx.x;
    long long acc = 0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        const size_t q = (size_t)r * ld + i;
        if (X[q]) acc += (long long)H[q] + b[i];
        if (finish) bx[q] = X[q];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long long e = part[0] / 2;
        E_out[r] = e;
        if (finish) {
            bE[r] = e;
            eoff[r] = 0;
            nacc[r] = 0;
        }
    }
}

// --------------------------------------------------------------------------
// Parallel tempering: replica exchange on the device (Algorithm 3's exchange
// move; Sec. II.D notes the next DA generation moves it off the host).
// slot2rep[c*M + p] is the replica (0..M-1) at temperature p of chain c.
// One workgroup of 64 lanes per chain: the lanes draw the M-1 exchange
// numbers and look up ln U of each at once, then one lane walks the pairs in
// ascending order (each decision depends on the swaps before it), and the
// lanes write the new slots back.  round[0] is the round index every kernel
// of the round reads; round[1] counts the workgroups that have read it, and
// the last of them advances round[0] (no workgroup waits for another).
// --------------------------------------------------------------------------
constexpr int kPtMaxM = 4096;

__global__ __launch_bounds__(64) void k_pt_exchange(const int64_t *__restrict__ E,
                                                    int32_t *slot2rep, int32_t *lvl_of_rep,
                                                    const double *__restrict__ dbeta,
                                                    const double *__restrict__ lnU, int32_t M,
                                                    int32_t chains, uint64_t seed,
                                                    uint32_t *round, int64_t *n_swaps,
                                                    int64_t *pair_swaps) {
    __shared__ double lnu[kPtMaxM];
    __shared__ int32_t s2r[kPtMaxM];
    __shared__ uint32_t t_sh;
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    if (lane == 0) {
        const uint32_t t = *(volatile uint32_t *)round;
        t_sh = t;
        __threadfence();
        // the last workgroup to have read the round index advances it
        if (atomicAdd(&round[1], 1u) == (uint32_t)chains - 1u) {
            round[1] = 0u;
            __threadfence();
            *(volatile uint32_t *)round = t + 1u;
        }
    }
    __syncthreads();
    const uint32_t t = t_sh;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    int32_t *gs2r = slot2rep + (size_t)c * M;
    for (int p = lane; p < M; p += 64) {
        s2r[p] = gs2r[p];
        if (p + 1 < M) {
            const uint32_t u =
                philox((uint32_t)p, t, (uint32_t)c, kTagExchange, k0, k1).x & 0xFFFFu;
            lnu[p] = lnU[u];
        }
    }
    __syncthreads();
    if (lane == 0) {
        const int64_t *Ec = E + (size_t)c * M;
        int64_t *ps = pair_swaps + (size_t)c * (M > 1 ? M - 1 : 1);
        int64_t sw = 0;
        for (int p = 0; p + 1 < M; ++p) {
            const int a = s2r[p], bq = s2r[p + 1];
            const double diff = (double)(Ec[a] - Ec[bq]);
            const double delta = __dmul_rn(dbeta[p], diff);
            if (lnu[p] < delta) {
                s2r[p] = bq;
                s2r[p + 1] = a;
                ++sw;
                ps[p] += 1;
            }
        }
        n_swaps[c] += sw;
    }
    __syncthreads();
    for (int p = lane; p < M; p += 64) {
        gs2r[p] = s2r[p];
        lvl_of_rep[(size_t)c * M + s2r[p]] = p;
    }
}

__global__ void k_pt_setup(int32_t *slot2rep, int32_t *lvl_of_rep, int64_t *n_swaps,
                           int64_t *pair_swaps, uint32_t *round, int32_t M, int32_t chains) {
    const int npair = chains * (M > 1 ? M - 1 : 1);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < M * chains || q < npair;
         q += gridDim.x * blockDim.x) {
        if (q < M * chains) {
            slot2rep[q] = q % M;
            lvl_of_rep[q] = q % M;
        }
        if (q < chains) n_swaps[q] = 0;
        if (q < npair) pair_swaps[q] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        round[0] = 0u;
        round[1] = 0u;
    }
}

// Copy [R][ld] state rows to dense [R][N] output rows.
__global__ void k_extract(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst, int32_t R,
                          int32_t N, int32_t ld) {
    const int64_t n = (int64_t)R * N;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / N, i = q - r * N;
        dst[q] = src[r * ld + i];
    }
}

__global__ void k_copy_i64(const int64_t *__restrict__ src, int64_t *__restrict__ dst, int32_t n) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x)
        dst[q] = src[q];
}

__global__ void k_fill_i32(int32_t *dst, int32_t value, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = value;
}

// Window of the per-draw estimate of every candidate level: the range of
// thr[u] + G(u) over all 65536 draws (one workgroup per level).  A level keeps
// gth only if the window is narrow and near zero, which also keeps the step
// kernel's sums in int32.
__global__ __launch_bounds__(256) void k_gen_calibrate(LevelHdr *hdr, const int32_t *thr,
                                                       int32_t L) {
    __shared__ int s_lo[256], s_hi[256];
    const int l = blockIdx.x;
    if (l >= L) return;
    const LevelHdr hd = hdr[l];
    if (!hd.gth) return;
    const int32_t *t = thr + (size_t)l * 65536;
    int lo = INT32_MAX, hi = INT32_MIN;
    for (int u = threadIdx.x; u < 65536; u += blockDim.x) {
        const int off =
            t[u] + (int)((uint32_t)draw_estimate((uint32_t)u, hd.ga, hd.gb) - kGenMagic);
        lo = min(lo, off);
        hi = max(hi, off);
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_lo[threadIdx.x] = min(s_lo[threadIdx.x], s_lo[threadIdx.x + w]);
            s_hi[threadIdx.x] = max(s_hi[threadIdx.x], s_hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        lo = s_lo[0];
        hi = s_hi[0];
        const bool ok = lo >= -kGenOffMax && hi <= kGenOffMax && hi - lo <= kGenWindow;
        hdr[l].glo = ok ? lo : 0;
        hdr[l].ghi = ok ? hi : 0;
        hdr[l].gth = ok ? 1 : 0;
    }
}

// --------------------------------------------------------------------------
// Host launch wrappers.
// --------------------------------------------------------------------------
namespace {
inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }
inline int grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 65535) g = 65535;
    return (int)g;
}

template <typename WT, int F, bool TRACE, bool HELP>
int launch_run_t(const JobDesc &J, const TraceDesc &T, int blocks, int threads, size_t lds,
                 void *stream) {
    const dim3 g(blocks), b(threads);
    // (the wide variants take 16-bit couplings' factor as 16-bit too)
    const bool wide = J.NW > 1 && !J.w_lds &&
                      (sizeof(WT) != 2 || (J.wscale < (1 << 15) && J.wscale > -(1 << 15)));
    if (J.lvl_of_rep) {
        // one replica per workgroup: its level's brackets are staged in LDS
        // for the round; several replicas (possibly at different levels) read
        // theirs through L1/L2
        if constexpr (!TRACE) {
            if (J.RPW == 1) {
                if constexpr (F >= 4) {
                    // per-draw estimates, evaluated by the compute lanes
                    if (J.gth && wide) {
                        if (J.NW <= 4)
                            hipLaunchKernelGGL(
                                (k_run<WT, F, false, HELP, true, kModeWide | kModeGen | kModeNW4>),
                                g, b, lds, S(stream), J, T);
                        else
                            hipLaunchKernelGGL(
                                (k_run<WT, F, false, HELP, true, kModeWide | kModeGen>), g, b, lds,
                                S(stream), J, T);
                        return (int)hipGetLastError();
                    }
                }
                if (wide && J.NW <= 4)
                    hipLaunchKernelGGL((k_run<WT, F, false, HELP, true, kModeWide | kModeNW4>), g,
                                       b, lds, S(stream), J, T);
                else if (wide)
                    hipLaunchKernelGGL((k_run<WT, F, false, HELP, true, kModeWide>), g, b, lds,
                                       S(stream), J, T);
                else
                    hipLaunchKernelGGL((k_run<WT, F, false, HELP, true, kModePlain>), g, b, lds,
                                       S(stream), J, T);
                return (int)hipGetLastError();
            }
        }
        if (wide && J.NW <= 4)
            hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, false, kModeWide | kModeNW4>), g, b, lds,
                               S(stream), J, T);
        else if (wide)
            hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, false, kModeWide>), g, b, lds,
                               S(stream), J, T);
        else
            hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, false, kModePlain>), g, b, lds,
                               S(stream), J, T);
        return (int)hipGetLastError();
    }
    const int mode = (J.single ? kModeSingle : 0) | (J.stepT ? kModePerStep : 0);
    if (J.ell) {
        // sparse row lists: the coupling type of dense W plays no part, so
        // these variants exist once (launch_run routes sparse jobs here)
        if constexpr (std::is_same<WT, int16_t>::value) {
            constexpr int SP = kModeSparse;
            switch (mode) {
                case kModePlain:
                    hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, SP>), g, b, lds,
                                       S(stream), J, T);
                    break;
                case kModeSingle:
                    hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, SP | kModeSingle>), g, b,
                                       lds, S(stream), J, T);
                    break;
                case kModePerStep:
                    hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, SP | kModePerStep>), g, b,
                                       lds, S(stream), J, T);
                    break;
                default:
                    hipLaunchKernelGGL(
                        (k_run<WT, F, TRACE, HELP, true, SP | kModeSingle | kModePerStep>), g, b,
                        lds, S(stream), J, T);
                    break;
            }
            return (int)hipGetLastError();
        } else {
            return (int)hipErrorInvalidValue;
        }
    }
    switch (mode) {
        case kModePlain:
            if constexpr (F >= 4) {
                if (J.gth && wide && !J.q8) {
                    if (J.NW <= 4)
                        hipLaunchKernelGGL(
                            (k_run<WT, F, TRACE, HELP, true, kModeWide | kModeGen | kModeNW4>), g,
                            b, lds, S(stream), J, T);
                    else
                        hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModeWide | kModeGen>),
                                           g, b, lds, S(stream), J, T);
                    break;
                }
            }
            if (J.q8 && wide && J.NW <= 4)
                hipLaunchKernelGGL(
                    (k_run<WT, F, TRACE, HELP, true, kModeWide | kModeDirect | kModeNW4>), g, b,
                    lds, S(stream), J, T);
            else if (J.q8 && wide)
                hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModeWide | kModeDirect>), g,
                                   b, lds, S(stream), J, T);
            else if (J.q8)
                hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModeDirect>), g, b, lds,
                                   S(stream), J, T);
            else if (wide && J.NW <= 4)
                hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModeWide | kModeNW4>), g, b,
                                   lds, S(stream), J, T);
            else if (wide)
                hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModeWide>), g, b, lds,
                                   S(stream), J, T);
            else
                hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModePlain>), g, b, lds,
                                   S(stream), J, T);
            break;
        case kModeSingle:
            hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModeSingle>), g, b, lds,
                               S(stream), J, T);
            break;
        case kModePerStep:
            hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModePerStep>), g, b, lds,
                               S(stream), J, T);
            break;
        default:
            hipLaunchKernelGGL((k_run<WT, F, TRACE, HELP, true, kModeSingle | kModePerStep>), g,
                               b, lds, S(stream), J, T);
            break;
    }
    return (int)hipGetLastError();
}

template <typename WT, bool TRACE, bool HELP>
int launch_run_f(const JobDesc &J, int F, const TraceDesc &T, int blocks, int threads, size_t lds,
                 void *stream) {
    switch (F) {
        case 2:
            // two flips per lane: 8- and 16-bit couplings (replicas spread over
            // twice the waves when the chip has room for them)
            if constexpr (sizeof(WT) <= 2)
                return launch_run_t<WT, 2, TRACE, HELP>(J, T, blocks, threads, lds, stream);
            else
                return (int)hipErrorInvalidValue;
        case 4: return launch_run_t<WT, 4, TRACE, HELP>(J, T, blocks, threads, lds, stream);
        case 8: return launch_run_t<WT, 8, TRACE, HELP>(J, T, blocks, threads, lds, stream);
        default: return (int)hipErrorInvalidValue;
    }
}

template <typename WT>
int launch_run_w(const JobDesc &J, int F, bool help, const TraceDesc *trace, int blocks,
                 int threads, size_t lds, void *stream) {
    const TraceDesc none{nullptr, nullptr, nullptr, 0};
    if (trace) {
        return help ? launch_run_f<WT, true, true>(J, F, *trace, blocks, threads, lds, stream)
                    : launch_run_f<WT, true, false>(J, F, *trace, blocks, threads, lds, stream);
    }
    return help ? launch_run_f<WT, false, true>(J, F, none, blocks, threads, lds, stream)
                : launch_run_f<WT, false, false>(J, F, none, blocks, threads, lds, stream);
}
}  // namespace

int launch_run(const JobDesc &J, int F, bool help, const TraceDesc *trace, int blocks,
               int threads, size_t lds_bytes, void *stream) {
    if (job_range_error(J) != nullptr) return (int)hipErrorInvalidValue;
    // the workgroup's LDS must hold at least W when staged and every replica
    // slot in the layout the kernel will use (the estimate ring included)
    {
        const SlotLayout SL = slot_layout(J.NW, help ? J.NH : 0, J.ell ? F : 0,
                                          J.gth != 0 && help);
        const int64_t w_src = J.ell ? (int64_t)J.N * J.ell_D * 4
                                    : (int64_t)J.N * J.ld * (int64_t)J.dtype;
        const int64_t need = (int64_t)SL.bytes * J.RPW + (J.w_lds ? ((w_src + 15) & ~15) : 0);
        if ((int64_t)lds_bytes < need) return (int)hipErrorInvalidValue;
    }
    if (J.ell && !J.lvl_of_rep)
        return launch_run_w<int16_t>(J, F, help, trace, blocks, threads, lds_bytes, stream);
    switch (J.dtype) {
        case 1: return launch_run_w<int8_t>(J, F, help, trace, blocks, threads, lds_bytes, stream);
        case 2: return launch_run_w<int16_t>(J, F, help, trace, blocks, threads, lds_bytes, stream);
        case 4: return launch_run_w<int32_t>(J, F, help, trace, blocks, threads, lds_bytes, stream);
        default: return (int)hipErrorInvalidValue;
    }
}

int launch_batch(const JobDesc *jobs_dev, const BatchItem *items_dev, const int32_t *n_items_dev,
                 int32_t *counter_dev, int blocks, int threads, size_t lds_bytes, void *stream,
                 bool dynamic) {
    if (dynamic)
        hipLaunchKernelGGL((k_batch<8, kModeDynamic>), dim3(blocks), dim3(threads), lds_bytes,
                           S(stream), jobs_dev, items_dev, n_items_dev, counter_dev);
    else
        hipLaunchKernelGGL((k_batch<8, kModePlain | kModeGen>), dim3(blocks), dim3(threads),
                           lds_bytes, S(stream), jobs_dev, items_dev, n_items_dev, counter_dev);
    return (int)hipGetLastError();
}

int launch_state_zero(const JobDesc &J, void *stream) {
    hipLaunchKernelGGL(k_state_zero, dim3(grid_for((int64_t)J.R * J.ld, 256)), dim3(256), 0,
                       S(stream), J);
    return (int)hipGetLastError();
}

int launch_rand_bits(uint8_t *X, int32_t R, int32_t N, int32_t ld, uint32_t rid_base,
                     uint64_t seed, void *stream) {
    hipLaunchKernelGGL(k_rand_bits, dim3(grid_for((int64_t)R * ld, 256)), dim3(256), 0, S(stream),
                       X, R, N, ld, rid_base, seed);
    return (int)hipGetLastError();
}

int launch_fields(const JobDesc &J, const uint8_t *X, int32_t R, int32_t *H, void *stream) {
    if (J.dtype == 1 && (int64_t)R * J.ld >= (int64_t)256 * 128 * 128) {
        // enough 128 x 128 blocks to fill the chip: the LDS-tiled form
        const dim3 grid((R + kFT - 1) / kFT, (J.ld + kFT - 1) / kFT);
        hipLaunchKernelGGL(k_fields_mfma_i8_tiled, grid, dim3(256), 0, S(stream), X,
                           reinterpret_cast<const int8_t *>(J.W), J.b, H, R, J.ld, J.wscale);
    } else if (J.dtype == 1) {
        const int waves = ((R + 31) / 32) * (J.ld / 32);
        hipLaunchKernelGGL(k_fields_mfma_i8, dim3((waves + 3) / 4), dim3(256), 0, S(stream), X,
                           reinterpret_cast<const int8_t *>(J.W), J.b, H, R, J.ld, J.wscale);
    } else if (J.dtype == 2) {
        hipLaunchKernelGGL(k_fields_rows<int16_t>, dim3(R), dim3(256), 0, S(stream), X,
                           reinterpret_cast<const int16_t *>(J.W), J.b, H, J.N, J.ld, J.wscale);
    } else {
        hipLaunchKernelGGL(k_fields_rows<int32_t>, dim3(R), dim3(256), 0, S(stream), X,
                           reinterpret_cast<const int32_t *>(J.W), J.b, H, J.N, J.ld, J.wscale);
    }
    return (int)hipGetLastError();
}

int launch_energy_from_fields(const JobDesc &J, const uint8_t *X, const int32_t *H, int32_t R,
                              int64_t *E_out, bool finish_state, void *stream) {
    hipLaunchKernelGGL(k_energy_from_fields, dim3(R), dim3(256), 0, S(stream), X, H, J.b, J.ld,
                       E_out, finish_state ? 1 : 0, J.bx, J.bE, J.eoff, J.nacc);
    return (int)hipGetLastError();
}

int launch_pt_exchange(int64_t *E, int32_t *slot2rep, int32_t *lvl_of_rep, const double *dbeta,
                       const double *lnU, int32_t M, int32_t chains, uint64_t seed,
                       uint32_t *round_ptr, int64_t *n_swaps, int64_t *pair_swaps,
                       void *stream) {
    if (M < 1 || M > kPtMaxM || chains < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pt_exchange, dim3(chains), dim3(64), 0, S(stream), E, slot2rep,
                       lvl_of_rep, dbeta, lnU, M, chains, seed, round_ptr, n_swaps, pair_swaps);
    return (int)hipGetLastError();
}

int launch_pt_setup(int32_t *slot2rep, int32_t *lvl_of_rep, int64_t *n_swaps,
                    int64_t *pair_swaps, uint32_t *round_ptr, int32_t M, int32_t chains,
                    void *stream) {
    const int64_t n = std::max<int64_t>((int64_t)M * chains, (int64_t)chains * std::max(M - 1, 1));
    hipLaunchKernelGGL(k_pt_setup, dim3(grid_for(n, 256)), dim3(256), 0, S(stream), slot2rep,
                       lvl_of_rep, n_swaps, pair_swaps, round_ptr, M, chains);
    return (int)hipGetLastError();
}

int launch_extract(const JobDesc &J, const uint8_t *src_x, uint8_t *dst_x, int32_t R,
                   void *stream) {
    hipLaunchKernelGGL(k_extract, dim3(grid_for((int64_t)R * J.N, 256)), dim3(256), 0, S(stream),
                       src_x, dst_x, R, J.N, J.ld);
    return (int)hipGetLastError();
}

int launch_copy_i64(const int64_t *src, int64_t *dst, int32_t n, void *stream) {
    hipLaunchKernelGGL(k_copy_i64, dim3(grid_for(n, 256)), dim3(256), 0, S(stream), src, dst, n);
    return (int)hipGetLastError();
}

int launch_fill_i32(int32_t *dst, int32_t value, int64_t n, void *stream) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, S(stream), dst, value, n);
    return (int)hipGetLastError();
}

int launch_gen_calibrate(LevelHdr *hdr, const int32_t *thr, int32_t L, void *stream) {
    if (L < 1 || !hdr || !thr) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gen_calibrate, dim3(L), dim3(256), 0, S(stream), hdr, thr, L);
    return (int)hipGetLastError();
}

}  // namespace dapt
