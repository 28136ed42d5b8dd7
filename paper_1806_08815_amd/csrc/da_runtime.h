// da_runtime.h -- host runtime objects behind the C ABI of include/da.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "da.h"
#include "da_internal.h"

namespace dapt {

// Device-resident Metropolis tables for a list of temperatures (one level per
// temperature), shared by every context on the device through a cache.
struct LevelTables {
    std::vector<double> temps;
    int32_t L = 0;
    int32_t *d_thr = nullptr;      // [L][65536]
    LevelHdr *d_hdr = nullptr;     // [L]
    uint32_t *d_brk = nullptr;     // brackets of all levels
    uint8_t *d_q8 = nullptr;       // direct tables [levels with q8 >= 0][65536], or null
    size_t bytes = 0;
    std::vector<LevelHdr> hdr;     // host copy (tests, footprints), estimate windows included
    bool any_gth = false;          // some level can be decided from per-draw estimates
    ~LevelTables();
};

// Threshold table of one temperature (host): thr[u] = ceil(-T ln U_u) - 1,
// U_u = (u + 1/2) / 65536, clamped to [-1, 2^30]; all -1 for T <= 0.
void build_threshold_table(double T, int32_t *thr);
int32_t threshold_entry(double T, int u);

// Per-step schedules: the step table [S] (temperature and band per step) on
// the device, cached per (device, schedule, S); and -ln U_u [65536] per device.
struct StepTables {
    int64_t S = 0;
    StepT *d_steps = nullptr;
    size_t bytes = 0;
    ~StepTables();
};
std::shared_ptr<StepTables> get_step_tables(const da_schedule &s, int64_t S, std::string &err);
const double *device_neg_log_u(std::string &err);
// Band header and brackets of one level from its threshold table.
void build_brackets(const int32_t *thr, LevelHdr &hd, std::vector<uint32_t> &brk);
// Steps [s0, s1) the autotuner times of an S-step schedule (S >= 1): up to 384
// steps from about a third of the way in, never past the last step (beyond it
// the level index would leave the level tables).
inline void tune_window(int64_t S, int64_t &s0, int64_t &s1) {
    const int64_t w = S < 384 ? S : 384;
    s0 = S / 3 < S - w ? S / 3 : S - w;
    s1 = s0 + w;
}
// Temperature of level l of a schedule.
double schedule_temperature(const da_schedule &s, int l);
// Host image of the tables of a temperature list.
struct HostTables {
    std::vector<double> temps;
    std::vector<int32_t> thr;      // [L][65536]
    std::vector<LevelHdr> hdr;     // [L]
    std::vector<uint32_t> brk;
    std::vector<uint8_t> q8;       // direct tables of the narrow-band levels
};
void build_host_tables(const std::vector<double> &temps, HostTables &ht);
// Tables for a temperature list (cached per device); nullptr on failure with
// `err` set.  `pre`, when given, must hold the host image of these
// temperatures' tables and is uploaded instead of building them again.
std::shared_ptr<LevelTables> get_level_tables(const std::vector<double> &temps, std::string &err,
                                              const HostTables *pre = nullptr);
// Device bytes of the tables of L levels with `buckets` brackets in total.
int64_t level_table_bytes(int32_t L, int64_t buckets);

// Replica state of one context ([cap] replicas of row stride ld).
struct StateBuf {
    int32_t *h = nullptr;
    uint8_t *x = nullptr;
    uint8_t *bx = nullptr;
    int64_t *E = nullptr;
    int64_t *bE = nullptr;
    int32_t *eoff = nullptr;
    int64_t *nacc = nullptr;
    int32_t cap = 0;
    int32_t ld = 0;
    void release();
    bool ensure(int32_t R, int32_t ld_, std::string &err);
    int64_t bytes() const;
    static int64_t bytes_for(int32_t R, int32_t ld);
};

// Launch shape of the step kernel.
struct LaunchShape {
    int F = 8;
    int NW = 1;         // compute waves per replica
    int NH = 0;         // random-number waves per replica (0: lazy draws)
    int RPW = 1;
    int w_lds = 0;
    int direct = 0;     // the level's direct table is staged in LDS (anneal mode)
    int gen = 0;        // random-number waves may hand over per-draw estimates
    int threads = 64;
    int blocks = 1;
    size_t lds = 0;
};

// Runs batches of jobs in one persistent launch of the batched step kernel.
// Descriptor tables have a fixed device capacity so that the launch (counter
// reset + kernel) is captured once as a hipGraph and replayed for every batch;
// only the table contents are re-uploaded, from pinned host staging.
struct BatchRunner {
    static constexpr int kCapJobs = 1024;
    static constexpr int kCapItems = 65536;
    JobDesc *d_jobs = nullptr;
    BatchItem *d_items = nullptr;
    int32_t *d_n = nullptr;
    int32_t *d_counter = nullptr;
    JobDesc *h_jobs = nullptr;       // pinned
    BatchItem *h_items = nullptr;    // pinned
    int32_t *h_n = nullptr;          // pinned
    int blocks = 0;
    size_t lds = 0;
    hipStream_t cap_stream = nullptr;
    // [0]: plain DA step kernel; [1]: the variant reading per-job features
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int prepare(std::string &err);
    // Enqueues the batch on `s` (jobs must already have initialised state).
    int run(const std::vector<JobDesc> &jobs, const std::vector<BatchItem> &items, hipStream_t s,
            std::string &err);
    void release();
    ~BatchRunner() { release(); }
};

// Launch shape of a job inside the batched kernel (16 waves per workgroup).
LaunchShape batch_shape(const da_ctx *ctx);
// The workgroup items of one job, appended to `items`.
void append_batch_items(const JobDesc &J, int job_index, std::vector<BatchItem> &items);

// Storage choice for a Q (shared by da_create and admission): W = Q + Q^T off
// the diagonal, b = diag(Q); returns DA_OK and fills dtype / wscale, or an
// error code with `err` set.
int derive_storage(const int32_t *Q, int32_t N, int32_t dtype_hint, int32_t &dtype,
                   int32_t &wscale, std::string &err);

// Host image of the device copy of W and b: W_ij = (Q_ij + Q_ji) / wscale off
// the diagonal, zero diagonal, rows padded to ld = N rounded up to 64, dtype
// bytes per coupling; b = diag(Q), zero padded.
struct HostMatrix {
    int32_t N = 0, ld = 0, dtype = 0, wscale = 1;
    int64_t hbound = 0;            // max_i |b_i| + sum_j |W_ij|: bounds every |h_i|
    std::vector<uint8_t> W;
    std::vector<int32_t> b;
    int32_t ell_D = 0;             // sparse row lists: D entries per row, 0 = none
    std::vector<uint32_t> ell;     // [N][D] column | (W_ij / wscale) << 16
};
// Adds the sparse row lists to hm; DA_ERANGE (err set) when a value does not
// fit 16 bits or a row has more than 1024 nonzeros.
int prepare_sparse(const int32_t *Q, int32_t N, HostMatrix &hm, std::string &err);
// Fills hm for a storage choice made by derive_storage.
void prepare_matrix(const int32_t *Q, int32_t N, int32_t dtype, int32_t wscale, HostMatrix &hm);
// New context holding hm on the current device (uploaded on stream s, which
// is synchronised before returning).
int create_ctx(const HostMatrix &hm, hipStream_t s, da_ctx **out, std::string &err);

}  // namespace dapt

struct da_ctx {
    int32_t N = 0;
    int32_t ld = 0;
    int32_t dtype = 0;     // bytes per stored coupling
    int32_t wscale = 1;
    int device = 0;
    int cus = 256;               // compute units of the device
    int64_t hbound = 0;          // bound of every |h_i| (max_i |b_i| + sum_j |W_ij|)
    void *d_W = nullptr;
    int32_t *d_b = nullptr;
    uint32_t *d_ell = nullptr;   // sparse row lists [N][ell_D], or null
    int32_t ell_D = 0;
    dapt::StateBuf st;
    hipStream_t own_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;          // last call
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;  // calls since reset
    size_t ev_used = 0;
    double folded_ms = 0.0;      // calls since reset that left the pool
    int64_t folded_calls = 0;
    da_kernel_stats last{};
    bool have_stats = false;
    std::string err;
    // PT scratch
    int32_t *pt_slot2rep = nullptr, *pt_lvl = nullptr;
    int64_t *pt_swaps = nullptr;
    int64_t *pt_pair = nullptr;      // accepted exchanges [chains][M-1]
    uint32_t *pt_round = nullptr;    // [2]: round index, workgroups that read it
    double *pt_dbeta = nullptr, *pt_lnU = nullptr;
    int32_t pt_cap_R = 0, pt_cap_M = 0, pt_cap_chains = 0, pt_cap_pairs = 0;
    std::shared_ptr<dapt::LevelTables> keep_tables;
    std::shared_ptr<dapt::StepTables> keep_steps;
    // what the replica state in `st` holds: replicas st_base .. st_base+st_R-1
    // after st_step steps (st_step < 0: nothing resumable)
    int64_t st_step = -1;
    int64_t st_base = 0;
    int32_t st_R = 0;
};

namespace dapt {

// Shared by da_api.cpp and da_server.cpp.
void set_thread_error(const std::string &msg);
int fail(da_ctx *ctx, int code, const std::string &msg);
int check_hip(da_ctx *ctx, hipError_t e, const char *what);
int validate_schedule(const da_schedule *s, std::string &err);
// direct: the schedule's tables include direct tables (staged when they fit)
LaunchShape choose_shape(const da_ctx *ctx, int32_t R, const da_launch *launch,
                         bool anneal_mode, bool direct = false);
// Fastest measured shape for this instance size, coupling type and replica
// count, into `out`: timed once (when may_time) on the context's replica state,
// which must hold R replicas and is left overwritten, then cached.  Returns
// DA_OK, or the error of the first HIP call that failed (naming the candidate).
int tuned_shape(da_ctx *ctx, const LevelTables &lt, int32_t R, int64_t steps,
                const da_schedule &sched, hipStream_t s, bool may_time, LaunchShape &out);
JobDesc make_job(const da_ctx *ctx, const LevelTables &lt, int32_t R, uint32_t rid_base,
                 uint64_t seed, int64_t steps, const da_schedule &s, const LaunchShape &sh);
int init_state(da_ctx *ctx, const JobDesc &J, int init, hipStream_t stream);
// Event pair for the next timed call (from the context's pool).
int next_events(da_ctx *ctx, hipEvent_t &e0, hipEvent_t &e1);
std::vector<double> schedule_temps(const da_schedule &s);

}  // namespace dapt
