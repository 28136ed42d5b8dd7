// da_api.cpp -- the C ABI of include/da.h: contexts, anneals, parallel
// tempering and energies on one gfx950 device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "da_runtime.h"

using namespace dapt;

namespace dapt {

namespace {
thread_local std::string t_err;
constexpr size_t kEventPool = 1024;

int64_t gcd64(int64_t a, int64_t b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}
}  // namespace

void set_thread_error(const std::string &msg) { t_err = msg; }

int fail(da_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    t_err = msg;
    return code;
}

int check_hip(da_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return DA_OK;
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? DA_ENOMEM : DA_EDEVICE, msg);
}

void StateBuf::release() {
    for (void *p : {(void *)h, (void *)x, (void *)bx, (void *)E, (void *)bE, (void *)eoff,
                    (void *)nacc})
        if (p) (void)hipFree(p);
    h = nullptr; x = bx = nullptr; E = bE = nacc = nullptr; eoff = nullptr;
    cap = 0;
}

int64_t StateBuf::bytes_for(int32_t R, int32_t ld) {
    return (int64_t)R * ld * (4 + 1 + 1) + (int64_t)R * (8 * 3 + 4);
}

int64_t StateBuf::bytes() const { return bytes_for(cap, ld); }

bool StateBuf::ensure(int32_t R, int32_t ld_, std::string &err) {
    if (R <= cap && ld_ == ld) return true;
    release();
    ld = ld_;
    const int32_t n = std::max(R, 1);
    const size_t rows = (size_t)n * ld;
    if (hipMalloc(&h, rows * 4) != hipSuccess || hipMalloc(&x, rows) != hipSuccess ||
        hipMalloc(&bx, rows) != hipSuccess || hipMalloc(&E, (size_t)n * 8) != hipSuccess ||
        hipMalloc(&bE, (size_t)n * 8) != hipSuccess || hipMalloc(&eoff, (size_t)n * 4) != hipSuccess ||
        hipMalloc(&nacc, (size_t)n * 8) != hipSuccess) {
        release();
        err = "out of device memory for replica state";
        return false;
    }
    cap = n;
    return true;
}

int validate_schedule(const da_schedule *s, std::string &err) {
    if (!s) {
        err = "schedule is null";
        return DA_EINVAL;
    }
    if (s->kind != DA_SCHED_GEOMETRIC && s->kind != DA_SCHED_LINEAR_BETA) {
        err = "unknown schedule kind";
        return DA_EINVAL;
    }
    if (s->n_levels < 0 || s->n_levels > kMaxLevels) {
        err = "n_levels must be in [0, 4096] (0: a new temperature every step)";
        return DA_EINVAL;
    }
    if (s->eoff_inc < 0) {
        err = "eoff_inc must be >= 0";
        return DA_EINVAL;
    }
    if (s->init != DA_INIT_ZEROS && s->init != DA_INIT_RANDOM) {
        err = "unknown init";
        return DA_EINVAL;
    }
    if ((s->trial != DA_TRIAL_PARALLEL && s->trial != DA_TRIAL_SINGLE) || s->reserved != 0) {
        err = "trial must be DA_TRIAL_PARALLEL or DA_TRIAL_SINGLE, reserved 0";
        return DA_EINVAL;
    }
    const bool zero = (s->T_hi == 0.0 && s->T_lo == 0.0);
    if (!zero && !(s->T_hi > 0.0 && s->T_lo > 0.0 && std::isfinite(s->T_hi) &&
                   std::isfinite(s->T_lo))) {
        err = "temperatures must be finite and > 0 (or both 0)";
        return DA_EINVAL;
    }
    return DA_OK;
}

// Launch shape: F variables per lane, NW = ceil(N / 64F) waves per replica,
// RPW replicas per workgroup.  W goes to LDS when small (it then serves every
// row fetch at LDS latency).
LaunchShape choose_shape(const da_ctx *ctx, int32_t R, const da_launch *launch,
                         bool anneal_mode, bool direct) {
    LaunchShape sh;
    int stage = anneal_mode ? 1 : 0;
    const int cus = ctx->cus;
    // Few replicas per CU: each replica's step latency is the limit, so spread
    // a replica over more waves (4 variables per lane) and move the random
    // numbers to their own waves.  A full chip is limited by total work: 8
    // variables per lane and lazy draws.
    const bool latency_bound = R <= 2 * cus;
    const int want_help = launch ? launch->rng_waves : 0;
    bool help = want_help > 0 || (want_help == 0 && latency_bound);
    sh.F = (launch && launch->flips_per_lane) ? launch->flips_per_lane : (latency_bound ? 4 : 8);
    if (sh.F != 2 && sh.F != 4 && sh.F != 8) sh.F = 8;
    if (sh.F == 2 && ctx->dtype > 2) sh.F = 4;   // two per lane: 8/16-bit couplings only
    sh.NW = (ctx->N + 64 * sh.F - 1) / (64 * sh.F);
    if (sh.NW > 16) {  // keep a replica within one workgroup (N <= 8192)
        sh.F = 8;
        sh.NW = (ctx->N + 64 * sh.F - 1) / (64 * sh.F);
    }
    const int nblk = (ctx->N + 7) / 8;
    sh.NH = help ? (nblk + 63) / 64 : 0;
    if (sh.NW + sh.NH > 16) sh.NH = 0;
    const int per = sh.NW + sh.NH;
    int rpw = (launch && launch->replicas_per_block) ? launch->replicas_per_block : 1;
    rpw = std::max(1, std::min(rpw, 16 / per));
    rpw = std::min(rpw, std::max(R, 1));
    sh.RPW = rpw;
    // parallel tempering with one replica per workgroup stages the level of
    // that replica for each round (the launcher picks that variant)
    if (!anneal_mode && rpw == 1) stage = 1;
    // what an anneal may stage in LDS: the sparse lists, else dense W
    const int64_t w_bytes = (anneal_mode && ctx->ell_D > 0)
                                ? (int64_t)ctx->N * ctx->ell_D * 4
                                : (int64_t)ctx->N * ctx->ld * ctx->dtype;
    const int want = launch ? launch->w_in_lds : 0;
    const bool sparse = anneal_mode && ctx->ell_D > 0;
    // dense W goes to LDS automatically only when small; row lists whenever they fit
    sh.w_lds = (want >= 0 && w_bytes <= ((want > 0 || sparse) ? device_lds_limit() : 32 * 1024))
                   ? 1
                   : 0;
    sh.threads = 64 * per * sh.RPW;
    sh.blocks = (R + sh.RPW - 1) / sh.RPW;
    // direct tables (narrow bands) are staged too when the schedule has them;
    // W gives way to them, and they give way when even that does not fit
    // (sparse row lists take a kernel variant without them)
    sh.direct = anneal_mode && direct && !sparse ? 1 : 0;
    const size_t limit = (size_t)device_lds_limit();
    sh.lds = run_lds_bytes(sh.NW, sh.RPW, sh.F, sh.w_lds ? (int)w_bytes : 0, stage, sh.NH, sparse,
                           sh.direct);
    if (sh.lds > limit && sh.w_lds) {
        sh.w_lds = 0;
        sh.lds = run_lds_bytes(sh.NW, sh.RPW, sh.F, 0, stage, sh.NH, sparse, sh.direct);
    }
    if (sh.lds > limit && sh.direct) {
        sh.direct = 0;
        sh.lds = run_lds_bytes(sh.NW, sh.RPW, sh.F, 0, stage, sh.NH, sparse);
    }
    // per-draw estimates (handed over by random-number waves, or evaluated by
    // the compute lanes under lazy draws): a multi-wave replica reading W from
    // global memory (the wide variants), 4 or 8 flips per lane, and fields
    // small enough for the estimate path's int32 sums; not with direct tables
    // Left to choose (no tuner), estimates only where fields span many coupling
    // units: a cost then rarely falls inside an estimate's window of a few
    // units, while +-1-like instances meet it every step or two.
    const int want_gen = launch ? launch->draw_estimates : 0;
    const bool wide16 = ctx->dtype != 2 || (ctx->wscale < (1 << 15) && ctx->wscale > -(1 << 15));
    const bool fine_fields = ctx->hbound >= 4096 * (int64_t)std::abs(ctx->wscale);
    if ((want_gen > 0 || (want_gen == 0 && fine_fields)) && anneal_mode && !sparse &&
        !sh.direct && !sh.w_lds && sh.NW > 1 && sh.F >= 4 && wide16 &&
        ctx->hbound <= kGenFieldMax) {
        const size_t lg = run_lds_bytes(sh.NW, sh.RPW, sh.F, 0, stage, sh.NH, false, false, true);
        if (lg <= limit) {
            sh.gen = 1;
            sh.lds = lg;
        }
    }
    return sh;
}

JobDesc make_job(const da_ctx *ctx, const LevelTables &lt, int32_t R, uint32_t rid_base,
                 uint64_t seed, int64_t steps, const da_schedule &s, const LaunchShape &sh) {
    JobDesc J{};
    J.W = ctx->d_W;
    J.b = ctx->d_b;
    J.N = ctx->N;
    J.ld = ctx->ld;
    J.dtype = ctx->dtype;
    J.wscale = ctx->wscale;
    J.h = ctx->st.h;
    J.x = ctx->st.x;
    J.bx = ctx->st.bx;
    J.E = ctx->st.E;
    J.bE = ctx->st.bE;
    J.eoff = ctx->st.eoff;
    J.nacc = ctx->st.nacc;
    J.R = R;
    J.rid_base = rid_base;
    J.seed = seed;
    J.s0 = 0;
    J.s1 = steps;
    J.S = steps;
    J.L = lt.L;
    // increments above 2^30 act as 2^30: the offset saturates there at once
    J.eoff_inc = std::min<int32_t>(s.eoff_inc, kEoffMax);
    J.single = s.trial == DA_TRIAL_SINGLE ? 1 : 0;
    J.ell = ctx->d_ell;
    J.ell_D = ctx->ell_D;
    J.lvl_of_rep = nullptr;
    J.round_ptr = nullptr;
    J.K = 0;
    J.NW = sh.NW;
    J.NH = sh.NH;
    J.RPW = sh.RPW;
    J.w_lds = sh.w_lds;
    J.hdr = lt.d_hdr;
    J.brk = lt.d_brk;
    J.thr = lt.d_thr;
    J.q8 = sh.direct ? lt.d_q8 : nullptr;
    J.gth = (sh.gen && lt.any_gth && s.trial != DA_TRIAL_SINGLE) ? 1 : 0;
    return J;
}

int init_state(da_ctx *ctx, const JobDesc &J, int init, hipStream_t stream) {
    int e;
    if (init == DA_INIT_ZEROS) {
        e = launch_state_zero(J, stream);
    } else {
        e = launch_rand_bits(J.x, J.R, J.N, J.ld, J.rid_base, J.seed, stream);
        if (!e) e = launch_fields(J, J.x, J.R, J.h, stream);
        if (!e) e = launch_energy_from_fields(J, J.x, J.h, J.R, J.E, true, stream);
    }
    return check_hip(ctx, (hipError_t)e, "state initialisation launch");
}

int device_lds_limit() {
    static int limit = -1;
    if (limit < 0) {
        int dev = 0;
        hipDeviceProp_t p;
        limit = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess &&
            p.sharedMemPerBlock > 0)
            limit = (int)p.sharedMemPerBlock;
    }
    return limit;
}

LaunchShape batch_shape(const da_ctx *ctx) {
    LaunchShape sh;
    sh.NH = 0;
    sh.F = 8;
    sh.NW = (ctx->N + 511) / 512;
    sh.RPW = 16 / sh.NW;
    sh.w_lds = 0;
    sh.threads = 1024;
    sh.lds = run_lds_bytes(sh.NW, sh.RPW, sh.F, 0, 1, 0, ctx->ell_D > 0);
    // per-draw estimates evaluated by the compute lanes, as for anneals: fields
    // of many coupling units within the path's int32 bound, dense rows
    sh.gen = (ctx->ell_D == 0 && ctx->hbound <= kGenFieldMax &&
              ctx->hbound >= 4096 * (int64_t)std::abs(ctx->wscale))
                 ? 1
                 : 0;
    return sh;
}

void append_batch_items(const JobDesc &J, int job_index, std::vector<BatchItem> &items) {
    for (int32_t r0 = 0; r0 < J.R; r0 += J.RPW) items.push_back(BatchItem{job_index, r0});
}

int BatchRunner::prepare(std::string &err) {
    if (exec[0] && exec[1]) return DA_OK;
    int dev = 0, cus = 0;
    hipError_t qe = hipGetDevice(&dev);
    if (qe == hipSuccess) qe = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (qe != hipSuccess || cus < 1) {
        err = std::string("batch runner: device query failed: ") + hipGetErrorString(qe);
        return DA_EDEVICE;
    }
    blocks = cus;
    lds = 0;
    // room for any job, sparse row lists' delta buffers included
    for (int nw = 1; nw <= 16; ++nw)
        lds = std::max(lds, run_lds_bytes(nw, 16 / nw, 8, 0, 1, 0, true));
    if (hipMalloc(&d_jobs, sizeof(JobDesc) * kCapJobs) != hipSuccess ||
        hipMalloc(&d_items, sizeof(BatchItem) * kCapItems) != hipSuccess ||
        hipMalloc(&d_n, 4) != hipSuccess || hipMalloc(&d_counter, 4) != hipSuccess ||
        hipHostMalloc(&h_jobs, sizeof(JobDesc) * kCapJobs) != hipSuccess ||
        hipHostMalloc(&h_items, sizeof(BatchItem) * kCapItems) != hipSuccess ||
        hipHostMalloc(&h_n, 4) != hipSuccess) {
        err = "batch descriptor allocation failed";
        release();
        return DA_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking) != hipSuccess) {
        err = "stream creation failed";
        release();
        return DA_EDEVICE;
    }
    // capture: counter reset (a fill kernel, no memset node) + persistent kernel
    const char *stage = "begin capture";
    hipError_t e = hipSuccess;
    for (int v = 0; v < 2 && e == hipSuccess; ++v) {
        stage = "begin capture";
        e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            stage = "counter reset node";
            e = (hipError_t)launch_fill_i32(d_counter, 0, 1, cap_stream);
            if (e == hipSuccess) {
                stage = "kernel node";
                e = (hipError_t)launch_batch(d_jobs, d_items, d_n, d_counter, blocks, 1024, lds,
                                             cap_stream, v == 1);
            }
            const hipError_t e2 = hipStreamEndCapture(cap_stream, &graph[v]);
            if (e == hipSuccess) {
                stage = "end capture";
                e = e2;
            }
        }
        if (e == hipSuccess) {
            stage = "instantiate";
            e = hipGraphInstantiate(&exec[v], graph[v], nullptr, nullptr, 0);
        }
    }
    if (e != hipSuccess) {
        err = std::string("batch graph capture failed at ") + stage + ": " + hipGetErrorString(e);
        release();
        return DA_EDEVICE;
    }
    return DA_OK;
}

int BatchRunner::run(const std::vector<JobDesc> &jobs, const std::vector<BatchItem> &items,
                     hipStream_t s, std::string &err) {
    int rc = prepare(err);
    if (rc) return rc;
    if (jobs.size() > (size_t)kCapJobs) {
        err = "too many jobs in one batch";
        return DA_EINVAL;
    }
    bool dynamic = false;
    for (const JobDesc &J : jobs) dynamic = dynamic || J.single || J.stepT || J.ell;
    // longest items first so the tail of the persistent launch is short
    std::vector<BatchItem> order(items);
    std::stable_sort(order.begin(), order.end(), [&](const BatchItem &p, const BatchItem &q) {
        const JobDesc &a = jobs[(size_t)p.job], &b = jobs[(size_t)q.job];
        return (a.s1 - a.s0) * a.NW > (b.s1 - b.s0) * b.NW;
    });
    std::memcpy(h_jobs, jobs.data(), jobs.size() * sizeof(JobDesc));
    for (size_t off = 0; off < order.size(); off += kCapItems) {
        const size_t n = std::min(order.size() - off, (size_t)kCapItems);
        // the previous chunk must be done with the tables before they change
        if (off) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                err = hipGetErrorString(e);
                return DA_EDEVICE;
            }
        }
        std::memcpy(h_items, order.data() + off, n * sizeof(BatchItem));
        *h_n = (int32_t)n;
        hipError_t e = hipMemcpyAsync(d_jobs, h_jobs, jobs.size() * sizeof(JobDesc),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_items, h_items, n * sizeof(BatchItem), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_n, h_n, 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipGraphLaunch(exec[dynamic ? 1 : 0], s);
        if (e != hipSuccess) {
            err = std::string("batch launch failed: ") + hipGetErrorString(e);
            return DA_EDEVICE;
        }
    }
    return DA_OK;
}

void BatchRunner::release() {
    for (int v = 0; v < 2; ++v) {
        if (exec[v]) (void)hipGraphExecDestroy(exec[v]);
        if (graph[v]) (void)hipGraphDestroy(graph[v]);
        exec[v] = nullptr;
        graph[v] = nullptr;
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void *p : {(void *)d_jobs, (void *)d_items, (void *)d_n, (void *)d_counter})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)h_jobs, (void *)h_items, (void *)h_n})
        if (p) (void)hipHostFree(p);
    cap_stream = nullptr;
    d_jobs = nullptr;
    d_items = nullptr;
    d_n = d_counter = nullptr;
    h_jobs = nullptr;
    h_items = nullptr;
    h_n = nullptr;
}

namespace {
// Calls f(i, j, w_ij) for every pair i < j, w_ij = Q_ij + Q_ji, in 64 x 64
// tiles so that the transposed reads stay in cache.
template <class Fn>
void for_upper_pairs(const int32_t *Q, size_t n, Fn &&f) {
    constexpr size_t B = 64;
    for (size_t I = 0; I < n; I += B)
        for (size_t J = I; J < n; J += B) {
            const size_t ie = std::min(I + B, n), je = std::min(J + B, n);
            for (size_t i = I; i < ie; ++i)
                for (size_t j = std::max(J, i + 1); j < je; ++j)
                    f(i, j, (int64_t)Q[i * n + j] + (int64_t)Q[j * n + i]);
        }
}
}  // namespace

int derive_storage(const int32_t *Q, int32_t N, int32_t dtype_hint, int32_t &dtype,
                   int32_t &wscale, std::string &err) {
    const size_t n = (size_t)N;
    int64_t g = 0, maxw = 0;
    std::vector<int64_t> row(n);
    for (size_t i = 0; i < n; ++i) {
        const int64_t bi = Q[i * n + i];
        row[i] = bi < 0 ? -bi : bi;
    }
    for_upper_pairs(Q, n, [&](size_t i, size_t j, int64_t w) {
        const int64_t aw = w < 0 ? -w : w;
        row[i] += aw;
        row[j] += aw;
        maxw = std::max(maxw, aw);
        if (w && g != 1) g = gcd64(g, w);
    });
    const int64_t maxrow = n ? *std::max_element(row.begin(), row.end()) : 0;
    if (maxrow > (int64_t(1) << 30)) {
        err = "max_i |b_i| + sum_j |W_ij| exceeds 2^30: fields would not fit int32";
        return DA_ERANGE;
    }
    if (g == 0) g = 1;
    maxw /= g;
    int dt = dtype_hint;
    if (dt == DA_DTYPE_AUTO) dt = maxw <= 127 ? 1 : (maxw <= 32767 ? 2 : 4);
    const int64_t lim = dt == 1 ? 127 : (dt == 2 ? 32767 : 2147483647);
    if (maxw > lim) {
        err = "couplings do not fit the requested type";
        return DA_ERANGE;
    }
    dtype = dt;
    wscale = (int32_t)g;
    return DA_OK;
}

namespace {
template <typename T>
void fill_padded(const int32_t *Q, size_t n, size_t ld, int64_t g, uint8_t *dst,
                 std::vector<int64_t> &row) {
    T *W = reinterpret_cast<T *>(dst);
    for_upper_pairs(Q, n, [&](size_t i, size_t j, int64_t w) {
        const T v = (T)(w / g);
        W[i * ld + j] = v;
        W[j * ld + i] = v;
        const int64_t aw = w < 0 ? -w : w;
        row[i] += aw;
        row[j] += aw;
    });
}
}  // namespace

void prepare_matrix(const int32_t *Q, int32_t N, int32_t dtype, int32_t wscale, HostMatrix &hm) {
    hm.N = N;
    hm.ld = (N + 63) / 64 * 64;
    hm.dtype = dtype;
    hm.wscale = wscale;
    const size_t n = (size_t)N, ld = (size_t)hm.ld;
    hm.W.assign(ld * ld * (size_t)dtype, 0);
    std::vector<int64_t> row(n, 0);
    if (dtype == 1) fill_padded<int8_t>(Q, n, ld, wscale, hm.W.data(), row);
    else if (dtype == 2) fill_padded<int16_t>(Q, n, ld, wscale, hm.W.data(), row);
    else fill_padded<int32_t>(Q, n, ld, wscale, hm.W.data(), row);
    hm.b.assign(ld, 0);
    hm.hbound = 0;
    for (size_t i = 0; i < n; ++i) {
        hm.b[i] = Q[i * n + i];
        hm.hbound = std::max(hm.hbound, row[i] + (hm.b[i] < 0 ? -(int64_t)hm.b[i] : hm.b[i]));
    }
}

int prepare_sparse(const int32_t *Q, int32_t N, HostMatrix &hm, std::string &err) {
    const size_t n = (size_t)N;
    const int64_t g = hm.wscale;
    std::vector<std::vector<uint32_t>> rows(n);
    for (size_t i = 0; i < n; ++i)
        for (size_t j = 0; j < n; ++j) {
            if (i == j) continue;
            const int64_t w = ((int64_t)Q[i * n + j] + (int64_t)Q[j * n + i]) / g;
            if (!w) continue;
            if (w < -32768 || w > 32767) {
                err = "a coupling does not fit the 16-bit sparse entry";
                return DA_ERANGE;
            }
            rows[i].push_back((uint32_t)j | ((uint32_t)(uint16_t)(int16_t)w << 16));
        }
    size_t D = 4;
    for (auto &r : rows) D = std::max(D, (r.size() + 3) / 4 * 4);
    if (D > 1024) {
        err = "a row has more than 1024 nonzeros: use dense storage";
        return DA_ERANGE;
    }
    hm.ell_D = (int32_t)D;
    hm.ell.assign(n * D, 0xFFFFu);   // padding: column 0xFFFF, value 0
    for (size_t i = 0; i < n; ++i)
        std::copy(rows[i].begin(), rows[i].end(), hm.ell.begin() + (ptrdiff_t)(i * D));
    return DA_OK;
}

int create_ctx(const HostMatrix &hm, hipStream_t s, da_ctx **out, std::string &err) {
    da_ctx *ctx = new (std::nothrow) da_ctx();
    if (!ctx) {
        err = "host allocation failed";
        return DA_ENOMEM;
    }
    ctx->N = hm.N;
    ctx->ld = hm.ld;
    ctx->dtype = hm.dtype;
    ctx->wscale = hm.wscale;
    ctx->hbound = hm.hbound;
    const char *what = nullptr;
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) what = "device query";
    if (!what && (e = hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount,
                                            ctx->device)) != hipSuccess)
        what = "compute-unit count";
    if (!what && (e = hipMalloc(&ctx->d_W, hm.W.size())) != hipSuccess) what = "W allocation";
    if (!what && (e = hipMalloc(&ctx->d_b, hm.b.size() * 4)) != hipSuccess) what = "b allocation";
    if (!what && (e = hipMemcpyAsync(ctx->d_W, hm.W.data(), hm.W.size(), hipMemcpyHostToDevice,
                                     s)) != hipSuccess)
        what = "W upload";
    if (!what && (e = hipMemcpyAsync(ctx->d_b, hm.b.data(), hm.b.size() * 4,
                                     hipMemcpyHostToDevice, s)) != hipSuccess)
        what = "b upload";
    if (!what && hm.ell_D > 0) {
        ctx->ell_D = hm.ell_D;
        if ((e = hipMalloc(&ctx->d_ell, hm.ell.size() * 4)) != hipSuccess) what = "sparse allocation";
        else if ((e = hipMemcpyAsync(ctx->d_ell, hm.ell.data(), hm.ell.size() * 4,
                                     hipMemcpyHostToDevice, s)) != hipSuccess)
            what = "sparse upload";
    }
    // the host image may be freed when this returns
    if (!what && (e = hipStreamSynchronize(s)) != hipSuccess) what = "upload";
    if (!what && (e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking)) !=
                     hipSuccess)
        what = "stream";
    if (what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        da_destroy(ctx);
        return (e == hipErrorOutOfMemory) ? DA_ENOMEM : DA_EDEVICE;
    }
    *out = ctx;
    return DA_OK;
}

// ---------------------------------------------------------------------------
// Autotuner.  Launch shapes never change results, only speed, so the first
// anneal of each (device, N, coupling type, replica-count bucket) times every
// candidate shape on a window of its own schedule, run on scratch state, and
// keeps the fastest for later calls.  DAPT_AUTOTUNE=0 disables it.
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
    int dev, N, dtype, rbucket;
    bool operator<(const TuneKey &o) const {
        if (dev != o.dev) return dev < o.dev;
        if (N != o.N) return N < o.N;
        if (dtype != o.dtype) return dtype < o.dtype;
        return rbucket < o.rbucket;
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, da_launch> g_tune;

bool tune_enabled() {
    const char *e = std::getenv("DAPT_AUTOTUNE");
    return !(e && e[0] == '0');
}
}  // namespace

// Direct tables pay for their staging (64 KiB per level and workgroup) only
// when levels last a few hundred steps.
static bool want_direct(const LevelTables &lt, const da_schedule &sched, int64_t steps) {
    return lt.d_q8 != nullptr && sched.n_levels > 0 && steps >= 256 * (int64_t)sched.n_levels;
}

int tuned_shape(da_ctx *ctx, const LevelTables &lt, int32_t R, int64_t steps,
                const da_schedule &sched, hipStream_t s, bool may_time, LaunchShape &out) {
    const bool direct = want_direct(lt, sched, steps);
    int dev = 0;
    int rc = check_hip(ctx, hipGetDevice(&dev), "autotuner: device query");
    if (rc) return rc;
    int rb = 1;
    while (rb < R) rb <<= 1;
    const TuneKey key{dev, ctx->N, ctx->dtype, rb};
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            out = choose_shape(ctx, R, &it->second, true, direct);
            return DA_OK;
        }
    }
    const int64_t window = std::min<int64_t>(steps, 384);
    out = choose_shape(ctx, R, nullptr, true, direct);
    if (window < 64 || !may_time) return DA_OK;
    // The candidates run on the context's own replica state (it must hold R
    // replicas already); the caller initialises it for the real run afterwards.
    if (ctx->st.cap < R || ctx->st.ld != ctx->ld)
        return fail(ctx, DA_EINVAL, "autotuner: replica state not allocated");
    hipEvent_t a = nullptr, b = nullptr;
    rc = check_hip(ctx, hipEventCreate(&a), "autotuner: event create");
    if (!rc) rc = check_hip(ctx, hipEventCreate(&b), "autotuner: event create");
    da_launch best{0, 0, 0, 0, 0};
    float best_ms = 1e30f;
    // W staged in LDS is a candidate whenever it fits there
    const bool w_fits = ctx->ell_D == 0 &&
                        (int64_t)ctx->N * ctx->ld * ctx->dtype <= (int64_t)device_lds_limit();
    for (int F : {2, 4, 8}) {
        if (F == 2 && ctx->dtype > 2) continue;
        for (int rpw : {1, 2, 4}) {
            for (int rng : {1, -1})
            for (int wl : {-1, 1})
            for (int ge : {1, -1}) {
                if (rc) break;
                if (wl > 0 && !w_fits) continue;
                const da_launch cand{F, rpw, wl, rng, ge};
                const LaunchShape sh = choose_shape(ctx, R, &cand, true, direct);
                if (sh.RPW != rpw || sh.F != F || sh.w_lds != (wl > 0 ? 1 : 0) ||
                    sh.threads > 1024 || sh.lds > (size_t)device_lds_limit())
                    continue;
                // the estimate candidate only where the shape can take it
                if (ge > 0 && (!sh.gen || !lt.any_gth)) continue;
                JobDesc J = make_job(ctx, lt, R, 0u, 1u, steps, sched, sh);
                tune_window(steps, J.s0, J.s1);
                if (const char *why = job_range_error(J)) {
                    rc = fail(ctx, DA_EINVAL, std::string("autotuner: ") + why);
                    break;
                }
                // any failure here is a device fault or a launch the device
                // refused: report it with the candidate instead of moving on
                char what[160];
                std::snprintf(what, sizeof what,
                              "autotuner candidate (flips/lane %d, replicas/workgroup %d, "
                              "rng waves %d, W in LDS %d, draw estimates %d)", F, rpw, rng, wl,
                              ge);
                rc = check_hip(ctx, (hipError_t)launch_state_zero(J, s), what);
                if (!rc) rc = check_hip(ctx, hipEventRecord(a, s), what);
                if (!rc)
                    rc = check_hip(ctx,
                                   (hipError_t)launch_run(J, sh.F, sh.NH > 0, nullptr, sh.blocks,
                                                          sh.threads, sh.lds, s),
                                   what);
                if (!rc) rc = check_hip(ctx, hipEventRecord(b, s), what);
                if (!rc) rc = check_hip(ctx, hipEventSynchronize(b), what);
                float ms = 0.f;
                if (!rc) rc = check_hip(ctx, hipEventElapsedTime(&ms, a, b), what);
                if (!rc && ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                }
            }
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (rc) return rc;
    if (best.flips_per_lane == 0) return DA_OK;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[key] = best;
    }
    out = choose_shape(ctx, R, &best, true, direct);
    return DA_OK;
}

int next_events(da_ctx *ctx, hipEvent_t &e0, hipEvent_t &e1) {
    if (ctx->ev_used == kEventPool) {
        // fold the window into running totals so the pool stays bounded
        int rc = check_hip(ctx, hipEventSynchronize(ctx->ev1), "event synchronise");
        for (size_t q = 0; q < ctx->ev_used && !rc; ++q) {
            float ms = 0.f;
            rc = check_hip(ctx, hipEventElapsedTime(&ms, ctx->ev_pool[q].first, ctx->ev_pool[q].second),
                           "event elapsed time");
            ctx->folded_ms += ms;
        }
        if (rc) return rc;
        ctx->folded_calls += (int64_t)ctx->ev_used;
        ctx->ev_used = 0;
    }
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        int rc = check_hip(ctx, hipEventCreate(&a), "event create");
        if (!rc) rc = check_hip(ctx, hipEventCreate(&b), "event create");
        if (rc) return rc;
        ctx->ev_pool.emplace_back(a, b);
    }
    e0 = ctx->ev_pool[ctx->ev_used].first;
    e1 = ctx->ev_pool[ctx->ev_used].second;
    ++ctx->ev_used;
    ctx->ev0 = e0;
    ctx->ev1 = e1;
    return DA_OK;
}

}  // namespace dapt

namespace {

constexpr int64_t kMaxSteps = (int64_t(1) << 31) - 1;

bool device_is_gfx950(std::string &err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        err = std::string("no HIP device: ") + hipGetErrorString(e);
        return false;
    }
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) {
        err = std::string("hipGetDeviceProperties failed: ") + hipGetErrorString(e);
        return false;
    }
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) {
        err = std::string("device is ") + p.gcnArchName + ", this library is built for gfx950";
        return false;
    }
    return true;
}

hipStream_t ctx_stream(da_ctx *ctx, void *stream) {
    return stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
}

// Copy-out of one anneal's outputs from the context state into device buffers.
int extract_outputs(da_ctx *ctx, const JobDesc &J, int32_t R, const da_result *o, hipStream_t s) {
    int e = 0;
    if (o->best_x && !e) e = launch_extract(J, J.bx, o->best_x, R, s);
    if (o->final_x && !e) e = launch_extract(J, J.x, o->final_x, R, s);
    if (o->best_E && !e) e = launch_copy_i64(J.bE, o->best_E, R, s);
    if (o->final_E && !e) e = launch_copy_i64(J.E, o->final_E, R, s);
    if (o->n_accept && !e) e = launch_copy_i64(J.nacc, o->n_accept, R, s);
    return check_hip(ctx, (hipError_t)e, "output extraction launch");
}

int copy_outputs_to_host(da_ctx *ctx, const JobDesc &J, int32_t R, const da_result *o,
                         hipStream_t s) {
    hipError_t e = hipSuccess;
    const size_t N = (size_t)J.N, ld = (size_t)J.ld;
    if (o->best_x && e == hipSuccess)
        e = hipMemcpy2DAsync(o->best_x, N, J.bx, ld, N, (size_t)R, hipMemcpyDeviceToHost, s);
    if (o->final_x && e == hipSuccess)
        e = hipMemcpy2DAsync(o->final_x, N, J.x, ld, N, (size_t)R, hipMemcpyDeviceToHost, s);
    if (o->best_E && e == hipSuccess)
        e = hipMemcpyAsync(o->best_E, J.bE, (size_t)R * 8, hipMemcpyDeviceToHost, s);
    if (o->final_E && e == hipSuccess)
        e = hipMemcpyAsync(o->final_E, J.E, (size_t)R * 8, hipMemcpyDeviceToHost, s);
    if (o->n_accept && e == hipSuccess)
        e = hipMemcpyAsync(o->n_accept, J.nacc, (size_t)R * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return check_hip(ctx, e, "copy of outputs to host");
}

void record_stats(da_ctx *ctx, const LaunchShape &sh, int64_t launches, int gth = 0) {
    (void)launches;
    ctx->last = da_kernel_stats{};
    ctx->last.blocks = sh.blocks;
    ctx->last.threads = sh.threads;
    ctx->last.flips_per_lane = sh.F;
    ctx->last.replicas_per_block = sh.RPW;
    ctx->last.w_in_lds = sh.w_lds;
    ctx->last.rng_waves = sh.NH;
    ctx->last.dtype = ctx->dtype;
    ctx->last.draw_estimates = gth;
    ctx->have_stats = true;
}

// Enqueue a full anneal: state init, step kernel between timing events.
// Tables a schedule needs: per-level decision tables, or, for a per-step
// schedule (n_levels = 0), one dummy level (T = 0, empty band) plus the step
// table and -ln U_u.
struct JobTables {
    std::shared_ptr<LevelTables> levels;
    std::shared_ptr<StepTables> steps;
    const double *G = nullptr;
};

int job_tables(const da_schedule &sch, int64_t steps, JobTables &jt, std::string &err) {
    if (sch.n_levels == 0) {
        if (steps > kMaxPerStepSteps) {
            err = "per-step schedules take at most 2^24 steps";
            return DA_EINVAL;
        }
        jt.levels = get_level_tables(std::vector<double>{0.0}, err);
        if (!jt.levels) return DA_ENOMEM;
        if (steps > 0) {
            jt.steps = get_step_tables(sch, steps, err);
            jt.G = device_neg_log_u(err);
            if (!jt.steps || !jt.G) return DA_ENOMEM;
        }
        return DA_OK;
    }
    jt.levels = get_level_tables(schedule_temps(sch), err);
    return jt.levels ? DA_OK : DA_ENOMEM;
}

void attach_step_tables(JobDesc &J, const JobTables &jt) {
    J.stepT = jt.steps ? jt.steps->d_steps : nullptr;
    J.G = jt.G;
}

// Steps [step_begin, step_end) of a `steps`-step anneal; step_begin > 0
// continues from the state the context holds.
int enqueue_anneal(da_ctx *ctx, const da_schedule *schedule, int64_t replica_base,
                   int32_t replicas, int64_t steps, uint64_t seed, const da_launch *launch,
                   const da_trace *trace_dev, hipStream_t s, JobDesc &J,
                   int64_t step_begin = 0, int64_t step_end = -1) {
    std::string err;
    if (!ctx) return fail(nullptr, DA_EINVAL, "ctx is null");
    int rc = validate_schedule(schedule, err);
    if (rc) return fail(ctx, rc, err);
    if (replicas < 1) return fail(ctx, DA_EINVAL, "replicas must be >= 1");
    if (steps < 0 || steps > kMaxSteps) return fail(ctx, DA_EINVAL, "steps must be in [0, 2^31)");
    if (step_end < 0) step_end = steps;
    if (step_begin < 0 || step_begin > step_end || step_end > steps)
        return fail(ctx, DA_EINVAL, "need 0 <= step_begin <= step_end <= total steps");
    if (replica_base < 0 || replica_base + replicas > (int64_t(1) << 31))
        return fail(ctx, DA_EINVAL, "replica ids must lie in [0, 2^31)");
    if (step_begin > 0 && (ctx->st_step != step_begin || ctx->st_base != replica_base ||
                           ctx->st_R < replicas))
        return fail(ctx, DA_EINVAL, "the context holds no state of these replicas at step_begin");
    JobTables jt;
    rc = job_tables(*schedule, steps, jt, err);
    if (rc) return fail(ctx, rc, err);
    ctx->keep_tables = jt.levels;
    ctx->keep_steps = jt.steps;
    if (!ctx->st.ensure(replicas, ctx->ld, err)) return fail(ctx, DA_ENOMEM, err);
    const LevelTables &lt0 = *jt.levels;
    // from here on the state changes: it is resumable again only on success
    ctx->st_step = -1;
    LaunchShape sh;
    // the tuner times its candidates on the replica state, so only when the
    // run starts from the initial state (which is written after it); a resumed
    // piece takes the cached choice or the default
    if (launch == nullptr && trace_dev == nullptr && tune_enabled() && !jt.steps) {
        rc = tuned_shape(ctx, lt0, replicas, steps, *schedule, s, step_begin == 0, sh);
        if (rc) return rc;
    } else {
        sh = choose_shape(ctx, replicas, launch, true,
                          !jt.steps && want_direct(lt0, *schedule, steps));
    }
    J = make_job(ctx, lt0, replicas, (uint32_t)replica_base, seed, steps, *schedule, sh);
    attach_step_tables(J, jt);
    J.s0 = step_begin;
    J.s1 = step_end;
    if (const char *why = job_range_error(J)) return fail(ctx, DA_EINVAL, why);
    if (step_begin == 0) {
        rc = init_state(ctx, J, schedule->init, s);
        if (rc) return rc;
    }
    hipEvent_t e0, e1;
    rc = next_events(ctx, e0, e1);
    if (rc) return rc;
    rc = check_hip(ctx, hipEventRecord(e0, s), "event record");
    if (rc) return rc;
    if (step_end > step_begin) {
        TraceDesc T{nullptr, nullptr, nullptr, steps};
        if (trace_dev) {
            T.k = trace_dev->k;
            T.E = trace_dev->E;
            T.eoff = trace_dev->eoff;
        }
        const int e = launch_run(J, sh.F, sh.NH > 0, trace_dev ? &T : nullptr, sh.blocks,
                                 sh.threads, sh.lds, s);
        rc = check_hip(ctx, (hipError_t)e, "step kernel launch");
        if (rc) return rc;
    }
    rc = check_hip(ctx, hipEventRecord(e1, s), "event record");
    if (rc) return rc;
    record_stats(ctx, sh, 1, J.gth);
    ctx->st_step = step_end;
    ctx->st_base = replica_base;
    ctx->st_R = replicas;
    return DA_OK;
}

}  // namespace

extern "C" {

int da_create(const int32_t *Q, int32_t N, int32_t dtype_hint, da_ctx **out) {
    if (!out) return fail(nullptr, DA_EINVAL, "out is null");
    *out = nullptr;
    if (!Q) return fail(nullptr, DA_EINVAL, "Q is null");
    if (N < 1 || N > DA_MAX_N) return fail(nullptr, DA_EINVAL, "N must be in [1, 8192]");
    const bool sparse = (dtype_hint & DA_STORE_SPARSE) != 0;
    dtype_hint &= ~DA_STORE_SPARSE;
    if (dtype_hint != DA_DTYPE_AUTO && dtype_hint != DA_DTYPE_I8 && dtype_hint != DA_DTYPE_I16 &&
        dtype_hint != DA_DTYPE_I32)
        return fail(nullptr, DA_EINVAL, "unknown dtype hint");
    std::string err;
    if (!device_is_gfx950(err)) return fail(nullptr, DA_EDEVICE, err);

    int32_t dtype = 0, wscale = 1;
    int rc = derive_storage(Q, N, dtype_hint, dtype, wscale, err);
    if (rc) return fail(nullptr, rc, err);
    HostMatrix hm;
    prepare_matrix(Q, N, dtype, wscale, hm);
    if (sparse) {
        rc = prepare_sparse(Q, N, hm, err);
        if (rc) return fail(nullptr, rc, err);
    }
    rc = create_ctx(hm, nullptr, out, err);
    if (rc) return fail(nullptr, rc, err);
    return DA_OK;
}

void da_destroy(da_ctx *ctx) {
    if (!ctx) return;
    if (ctx->own_stream) (void)hipStreamSynchronize(ctx->own_stream);
    (void)hipDeviceSynchronize();
    ctx->st.release();
    if (ctx->d_W) (void)hipFree(ctx->d_W);
    if (ctx->d_b) (void)hipFree(ctx->d_b);
    if (ctx->d_ell) (void)hipFree(ctx->d_ell);
    for (void *p : {(void *)ctx->pt_slot2rep, (void *)ctx->pt_lvl, (void *)ctx->pt_swaps,
                    (void *)ctx->pt_pair, (void *)ctx->pt_round, (void *)ctx->pt_dbeta,
                    (void *)ctx->pt_lnU})
        if (p) (void)hipFree(p);
    for (auto &pr : ctx->ev_pool) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    delete ctx;
}

int da_get_info(const da_ctx *ctx, da_info *info) {
    if (!ctx || !info) return fail(nullptr, DA_EINVAL, "null argument");
    info->N = ctx->N;
    info->ld = ctx->ld;
    info->dtype = ctx->dtype;
    info->wscale = ctx->wscale;
    info->device_bytes = (int64_t)ctx->ld * ctx->ld * ctx->dtype + (int64_t)ctx->ld * 4 +
                         ctx->st.bytes() + (int64_t)ctx->N * ctx->ell_D * 4;
    info->sparse_degree = ctx->ell_D;
    info->reserved = 0;
    return DA_OK;
}

int da_anneal_async(da_ctx *ctx, const da_schedule *schedule, int64_t replica_base,
                    int32_t replicas, int64_t steps, uint64_t seed, const da_launch *launch,
                    const da_result *out_dev, void *stream) {
    if (!ctx) return fail(nullptr, DA_EINVAL, "ctx is null");
    hipStream_t s = ctx_stream(ctx, stream);
    JobDesc J;
    int rc = enqueue_anneal(ctx, schedule, replica_base, replicas, steps, seed, launch, nullptr, s, J);
    if (rc) return rc;
    if (out_dev) rc = extract_outputs(ctx, J, replicas, out_dev, s);
    return rc;
}

int da_anneal_ex(da_ctx *ctx, const da_schedule *schedule, int64_t replica_base,
                 int32_t replicas, int64_t steps, uint64_t seed, const da_launch *launch,
                 da_result *out, const da_trace *trace) {
    if (!ctx) return fail(nullptr, DA_EINVAL, "ctx is null");
    hipStream_t s = ctx->own_stream;
    da_trace dev_trace{nullptr, nullptr, nullptr};
    const size_t cells = (size_t)std::max<int64_t>(replicas, 0) * (size_t)std::max<int64_t>(steps, 0);
    int rc = DA_OK;
    if (trace && cells) {
        if (trace->k) rc = check_hip(ctx, hipMalloc(&dev_trace.k, cells * 4), "trace allocation");
        if (!rc && trace->E) rc = check_hip(ctx, hipMalloc(&dev_trace.E, cells * 8), "trace allocation");
        if (!rc && trace->eoff) rc = check_hip(ctx, hipMalloc(&dev_trace.eoff, cells * 8), "trace allocation");
        // the traced kernel writes every column it is given; give it all three
        if (!rc && !dev_trace.k) rc = check_hip(ctx, hipMalloc(&dev_trace.k, cells * 4), "trace allocation");
        if (!rc && !dev_trace.E) rc = check_hip(ctx, hipMalloc(&dev_trace.E, cells * 8), "trace allocation");
        if (!rc && !dev_trace.eoff) rc = check_hip(ctx, hipMalloc(&dev_trace.eoff, cells * 8), "trace allocation");
    }
    JobDesc J;
    if (!rc)
        rc = enqueue_anneal(ctx, schedule, replica_base, replicas, steps, seed, launch,
                            (trace && cells) ? &dev_trace : nullptr, s, J);
    if (!rc && out) rc = copy_outputs_to_host(ctx, J, replicas, out, s);
    if (!rc && trace && cells) {
        hipError_t e = hipSuccess;
        if (trace->k) e = hipMemcpy(trace->k, dev_trace.k, cells * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && trace->E) e = hipMemcpy(trace->E, dev_trace.E, cells * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess && trace->eoff) e = hipMemcpy(trace->eoff, dev_trace.eoff, cells * 8, hipMemcpyDeviceToHost);
        rc = check_hip(ctx, e, "trace copy");
    }
    if (!rc && !out) rc = check_hip(ctx, hipStreamSynchronize(s), "stream synchronise");
    if (dev_trace.k) (void)hipFree(dev_trace.k);
    if (dev_trace.E) (void)hipFree(dev_trace.E);
    if (dev_trace.eoff) (void)hipFree(dev_trace.eoff);
    return rc;
}

int da_anneal(da_ctx *ctx, const da_schedule *schedule, int32_t replicas, int64_t steps,
              uint64_t seed, da_result *out) {
    return da_anneal_ex(ctx, schedule, 0, replicas, steps, seed, nullptr, out, nullptr);
}

int da_anneal_steps(da_ctx *ctx, const da_schedule *schedule, int64_t replica_base,
                    int32_t replicas, int64_t total_steps, int64_t step_begin,
                    int64_t step_end, uint64_t seed, da_result *out) {
    if (!ctx) return fail(nullptr, DA_EINVAL, "ctx is null");
    hipStream_t s = ctx->own_stream;
    JobDesc J;
    int rc = enqueue_anneal(ctx, schedule, replica_base, replicas, total_steps, seed, nullptr,
                            nullptr, s, J, step_begin, step_end);
    if (rc) return rc;
    if (out) return copy_outputs_to_host(ctx, J, replicas, out, s);
    return check_hip(ctx, hipStreamSynchronize(s), "stream synchronise");
}

int64_t da_state_bytes(int32_t N, int32_t replicas) {
    if (N < 1 || N > DA_MAX_N || replicas < 1) return -1;
    const int64_t n = N, r = replicas;
    return (int64_t)sizeof(da_state_header) + r * (2 * n + 4 * n) + r * (8 * 3 + 4);
}

int da_state_save(da_ctx *ctx, int32_t replicas, void *buf, size_t bytes) {
    if (!ctx || !buf) return fail(ctx, DA_EINVAL, "null argument");
    if (ctx->st_step < 0 || replicas < 1 || replicas > ctx->st_R)
        return fail(ctx, DA_EINVAL, "the context holds no anneal state for that many replicas");
    const int64_t need = da_state_bytes(ctx->N, replicas);
    if ((int64_t)bytes < need) return fail(ctx, DA_EINVAL, "buffer shorter than da_state_bytes");
    const size_t N = (size_t)ctx->N, ld = (size_t)ctx->ld, R = (size_t)replicas;
    auto *hdr = static_cast<da_state_header *>(buf);
    hdr->magic = 0x54534144u;
    hdr->version = 1;
    hdr->N = ctx->N;
    hdr->replicas = replicas;
    hdr->step = ctx->st_step;
    hdr->replica_base = (uint64_t)ctx->st_base;
    uint8_t *p = static_cast<uint8_t *>(buf) + sizeof(da_state_header);
    hipStream_t s = ctx->own_stream;
    uint8_t *x = p, *bx = p + R * N;
    int32_t *h = reinterpret_cast<int32_t *>(p + 2 * R * N);
    uint8_t *tail = p + 6 * R * N;
    hipError_t e = hipMemcpy2DAsync(x, N, ctx->st.x, ld, N, R, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(bx, N, ctx->st.bx, ld, N, R, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(h, N * 4, ctx->st.h, ld * 4, N * 4, R, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tail, ctx->st.E, R * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(tail + R * 8, ctx->st.bE, R * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(tail + R * 16, ctx->st.nacc, R * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(tail + R * 24, ctx->st.eoff, R * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return check_hip(ctx, e, "state copy to host");
}

int da_state_load(da_ctx *ctx, const void *buf, size_t bytes) {
    if (!ctx || !buf) return fail(ctx, DA_EINVAL, "null argument");
    if (bytes < sizeof(da_state_header)) return fail(ctx, DA_EINVAL, "buffer too short");
    const auto *hdr = static_cast<const da_state_header *>(buf);
    if (hdr->magic != 0x54534144u || hdr->version != 1)
        return fail(ctx, DA_EINVAL, "not a version-1 state snapshot");
    if (hdr->N != ctx->N) return fail(ctx, DA_EINVAL, "snapshot is of a different N");
    if (hdr->replicas < 1 || hdr->step < 0 || hdr->step > kMaxSteps ||
        hdr->replica_base + (uint64_t)hdr->replicas > (uint64_t(1) << 31))
        return fail(ctx, DA_EINVAL, "corrupt snapshot header");
    const int64_t need = da_state_bytes(hdr->N, hdr->replicas);
    if ((int64_t)bytes < need) return fail(ctx, DA_EINVAL, "buffer shorter than the snapshot");
    {
        // the step kernel keeps E_offset in [0, 2^30]; a snapshot outside is corrupt
        const size_t R = (size_t)hdr->replicas, N = (size_t)hdr->N;
        const uint8_t *eo = static_cast<const uint8_t *>(buf) + sizeof(da_state_header) +
                            6 * R * N + 24 * R;
        for (size_t r = 0; r < R; ++r) {
            int32_t v;
            std::memcpy(&v, eo + 4 * r, 4);
            if (v < 0 || v > kEoffMax) return fail(ctx, DA_EINVAL, "snapshot offset out of range");
        }
    }
    std::string err;
    ctx->st_step = -1;
    if (!ctx->st.ensure(hdr->replicas, ctx->ld, err)) return fail(ctx, DA_ENOMEM, err);
    const size_t N = (size_t)ctx->N, ld = (size_t)ctx->ld, R = (size_t)hdr->replicas;
    const uint8_t *p = static_cast<const uint8_t *>(buf) + sizeof(da_state_header);
    const uint8_t *x = p, *bx = p + R * N, *h = p + 2 * R * N, *tail = p + 6 * R * N;
    hipStream_t s = ctx->own_stream;
    // padding columns of the state rows are zero, as the initialisers leave them
    hipError_t e = hipMemsetAsync(ctx->st.x, 0, R * ld, s);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->st.bx, 0, R * ld, s);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->st.h, 0, R * ld * 4, s);
    if (e == hipSuccess) e = hipMemcpy2DAsync(ctx->st.x, ld, x, N, N, R, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(ctx->st.bx, ld, bx, N, N, R, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(ctx->st.h, ld * 4, h, N * 4, N * 4, R, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->st.E, tail, R * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->st.bE, tail + R * 8, R * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->st.nacc, tail + R * 16, R * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->st.eoff, tail + R * 24, R * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int rc = check_hip(ctx, e, "state upload");
    if (rc) return rc;
    ctx->st_step = hdr->step;
    ctx->st_base = (int64_t)hdr->replica_base;
    ctx->st_R = hdr->replicas;
    return DA_OK;
}

int da_anneal_batch(const da_batch_item *items, int32_t count, void *stream) {
    if (!items || count < 1) return fail(nullptr, DA_EINVAL, "empty batch");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : nullptr;
    for (int32_t a = 0; a < count; ++a)
        for (int32_t c = a + 1; c < count; ++c)
            if (items[a].ctx == items[c].ctx)
                return fail(nullptr, DA_EINVAL, "batch items must use distinct contexts");
    std::vector<JobDesc> jobs((size_t)count);
    std::vector<BatchItem> work;
    std::vector<std::shared_ptr<LevelTables>> keep;
    std::vector<std::shared_ptr<StepTables>> keep_steps;
    // no context claims a resumable state until the whole batch has run
    for (int32_t a = 0; a < count; ++a)
        if (items[a].ctx) items[a].ctx->st_step = -1;
    for (int32_t a = 0; a < count; ++a) {
        const da_batch_item &it = items[a];
        da_ctx *ctx = it.ctx;
        if (!ctx) return fail(nullptr, DA_EINVAL, "batch item without context");
        if (!s) s = ctx->own_stream;
        std::string err;
        int rc = validate_schedule(&it.schedule, err);
        if (rc) return fail(ctx, rc, err);
        if (it.replicas < 1 || it.steps < 0 || it.steps > kMaxSteps || it.replica_base < 0 ||
            it.replica_base + it.replicas > (int64_t(1) << 31))
            return fail(ctx, DA_EINVAL, "bad replicas / steps / replica_base in batch item");
        JobTables jt;
        rc = job_tables(it.schedule, it.steps, jt, err);
        if (rc) return fail(ctx, rc, err);
        auto lt = jt.levels;
        if (jt.steps) keep_steps.push_back(jt.steps);
        if (!lt) return fail(ctx, DA_ENOMEM, err);
        keep.push_back(lt);
        ctx->keep_tables = lt;
        if (!ctx->st.ensure(it.replicas, ctx->ld, err)) return fail(ctx, DA_ENOMEM, err);
        const LaunchShape sh = batch_shape(ctx);
        jobs[(size_t)a] = make_job(ctx, *lt, it.replicas, (uint32_t)it.replica_base, it.seed,
                                   it.steps, it.schedule, sh);
        attach_step_tables(jobs[(size_t)a], jt);
        if (const char *why = job_range_error(jobs[(size_t)a])) return fail(ctx, DA_EINVAL, why);
        rc = init_state(ctx, jobs[(size_t)a], it.schedule.init, s);
        if (rc) return rc;
        if (it.steps > 0) append_batch_items(jobs[(size_t)a], a, work);
        record_stats(ctx, sh, 1);
    }
    da_ctx *c0 = items[0].ctx;
    // process-lifetime runner (never destroyed: no device frees at exit)
    static std::mutex runner_mu;
    static BatchRunner *runner_p = new BatchRunner();
    BatchRunner &runner = *runner_p;
    std::lock_guard<std::mutex> lock(runner_mu);
    std::string err;
    hipEvent_t be0 = nullptr, be1 = nullptr;
    int rc = next_events(c0, be0, be1);
    if (!rc) rc = check_hip(c0, hipEventRecord(be0, s), "event record");
    if (!rc && !work.empty()) {
        rc = runner.run(jobs, work, s, err);
        if (rc) fail(c0, rc, err);
        c0->last.blocks = runner.blocks;
        c0->last.threads = 1024;
    }
    if (!rc) rc = check_hip(c0, hipEventRecord(be1, s), "event record");
    for (int32_t a = 0; a < count && !rc; ++a)
        rc = extract_outputs(items[a].ctx, jobs[(size_t)a], items[a].replicas, &items[a].out_dev, s);
    // descriptor tables are reused by the next batch: finish this one first
    if (!rc) rc = check_hip(c0, hipStreamSynchronize(s), "stream synchronise");
    if (rc) return rc;
    for (int32_t a = 0; a < count; ++a) {
        da_ctx *ctx = items[a].ctx;
        ctx->st_step = items[a].steps;
        ctx->st_base = items[a].replica_base;
        ctx->st_R = items[a].replicas;
    }
    return DA_OK;
}

}  // extern "C"

namespace {

int check_pt_args(da_ctx *ctx, const double *temps, int32_t M, int32_t chains, int64_t rounds,
                  int32_t steps_per_round, int32_t eoff_inc) {
    if (!temps || M < 1 || M > kMaxLevels || chains < 1 || rounds < 0 || steps_per_round < 0 ||
        eoff_inc < 0)
        return fail(ctx, DA_EINVAL, "bad PT arguments");
    if ((int64_t)M * chains > (int64_t(1) << 30)) return fail(ctx, DA_EINVAL, "too many replicas");
    if (rounds * (int64_t)steps_per_round > kMaxSteps || rounds > kMaxSteps)
        return fail(ctx, DA_EINVAL, "rounds * steps_per_round must be < 2^31");
    for (int p = 0; p < M; ++p) {
        if (!(temps[p] > 0.0) || !std::isfinite(temps[p]))
            return fail(ctx, DA_EINVAL, "temperatures must be finite and > 0");
        if (p + 1 < M && !(temps[p] < temps[p + 1]))
            return fail(ctx, DA_EINVAL, "temperatures must be strictly increasing");
    }
    return DA_OK;
}

// One PT run on the device (arguments already checked): random starts, then
// `rounds` rounds of steps_per_round DA steps and an exchange sweep.
int pt_run(da_ctx *ctx, const double *temps, int32_t M, int32_t chains, int64_t rounds,
           int32_t steps_per_round, int32_t eoff_inc, uint64_t seed, da_pt_result *out) {
    const int32_t R = M * chains;
    const int32_t npair = chains * std::max(M - 1, 1);
    std::string err;
    std::vector<double> tv(temps, temps + M);
    auto lt = get_level_tables(tv, err);
    if (!lt) return fail(ctx, DA_ENOMEM, err);
    ctx->keep_tables = lt;
    ctx->st_step = -1;   // PT state is not a resumable anneal
    if (!ctx->st.ensure(R, ctx->ld, err)) return fail(ctx, DA_ENOMEM, err);
    hipStream_t s = ctx->own_stream;
    int rc = DA_OK;
    if (R > ctx->pt_cap_R || M > ctx->pt_cap_M || chains > ctx->pt_cap_chains ||
        npair > ctx->pt_cap_pairs) {
        for (void *p : {(void *)ctx->pt_slot2rep, (void *)ctx->pt_lvl, (void *)ctx->pt_swaps,
                        (void *)ctx->pt_pair, (void *)ctx->pt_round, (void *)ctx->pt_dbeta,
                        (void *)ctx->pt_lnU})
            if (p) (void)hipFree(p);
        ctx->pt_slot2rep = ctx->pt_lvl = nullptr;
        ctx->pt_swaps = ctx->pt_pair = nullptr;
        ctx->pt_round = nullptr;
        ctx->pt_dbeta = ctx->pt_lnU = nullptr;
        ctx->pt_cap_R = ctx->pt_cap_M = ctx->pt_cap_chains = ctx->pt_cap_pairs = 0;
        rc = check_hip(ctx, hipMalloc(&ctx->pt_slot2rep, (size_t)R * 4), "PT allocation");
        if (!rc) rc = check_hip(ctx, hipMalloc(&ctx->pt_lvl, (size_t)R * 4), "PT allocation");
        if (!rc) rc = check_hip(ctx, hipMalloc(&ctx->pt_swaps, (size_t)chains * 8), "PT allocation");
        if (!rc) rc = check_hip(ctx, hipMalloc(&ctx->pt_pair, (size_t)npair * 8), "PT allocation");
        if (!rc) rc = check_hip(ctx, hipMalloc(&ctx->pt_round, 8), "PT allocation");
        if (!rc) rc = check_hip(ctx, hipMalloc(&ctx->pt_dbeta, (size_t)M * 8), "PT allocation");
        if (!rc) rc = check_hip(ctx, hipMalloc(&ctx->pt_lnU, 65536 * 8), "PT allocation");
        if (rc) return rc;
        ctx->pt_cap_R = R;
        ctx->pt_cap_M = M;
        ctx->pt_cap_chains = chains;
        ctx->pt_cap_pairs = npair;
    }
    // exchange tables: 1/T_p - 1/T_{p+1} and ln U_u, U_u = (u + 1/2)/65536
    std::vector<double> dbeta((size_t)M, 0.0), lnU(65536);
    for (int p = 0; p + 1 < M; ++p) dbeta[(size_t)p] = 1.0 / temps[p] - 1.0 / temps[p + 1];
    for (int u = 0; u < 65536; ++u) lnU[(size_t)u] = std::log(((double)u + 0.5) / 65536.0);
    rc = check_hip(ctx, hipMemcpyAsync(ctx->pt_dbeta, dbeta.data(), (size_t)M * 8, hipMemcpyHostToDevice, s), "PT upload");
    if (!rc) rc = check_hip(ctx, hipMemcpyAsync(ctx->pt_lnU, lnU.data(), 65536 * 8, hipMemcpyHostToDevice, s), "PT upload");
    if (rc) return rc;

    da_schedule sched{temps[0], temps[0], DA_SCHED_GEOMETRIC, 1, eoff_inc, DA_INIT_RANDOM,
                      DA_TRIAL_PARALLEL, 0};
    LaunchShape sh = choose_shape(ctx, R, nullptr, false);
    JobDesc J = make_job(ctx, *lt, R, 0u, seed, 0, sched, sh);
    // per-draw estimates (one replica per workgroup, several compute waves,
    // fields of many coupling units, as for anneals; the levels' windows are
    // measured when the tables are made): handed over by the random-number
    // waves, whose ring then needs its estimate part in LDS, or evaluated by
    // the compute lanes themselves
    const bool wide16 = ctx->dtype != 2 || (ctx->wscale < (1 << 15) && ctx->wscale > -(1 << 15));
    J.gth = (lt->any_gth && sh.RPW == 1 && sh.NW > 1 && sh.F >= 4 && !sh.w_lds && wide16 &&
             ctx->ell_D == 0 && ctx->hbound <= kGenFieldMax &&
             ctx->hbound >= 4096 * (int64_t)std::abs(ctx->wscale))
                ? 1
                : 0;
    if (J.gth && sh.NH > 0) {
        const size_t lg = run_lds_bytes(sh.NW, sh.RPW, sh.F, 0, 1, sh.NH, false, false, true);
        if (lg <= (size_t)device_lds_limit()) sh.lds = lg;
        else J.gth = 0;
    }
    J.L = M;
    J.lvl_of_rep = ctx->pt_lvl;
    J.round_ptr = ctx->pt_round;
    J.K = steps_per_round;
    if (const char *why = job_range_error(J)) return fail(ctx, DA_EINVAL, why);
    rc = init_state(ctx, J, DA_INIT_RANDOM, s);
    if (!rc)
        rc = check_hip(ctx, (hipError_t)launch_pt_setup(ctx->pt_slot2rep, ctx->pt_lvl,
                                                        ctx->pt_swaps, ctx->pt_pair,
                                                        ctx->pt_round, M, chains, s),
                       "PT setup");
    hipEvent_t pe0 = nullptr, pe1 = nullptr;
    if (!rc) rc = next_events(ctx, pe0, pe1);
    if (!rc) rc = check_hip(ctx, hipEventRecord(pe0, s), "event record");
    if (rc) return rc;

    auto one_round = [&]() -> int {
        int e = 0;
        if (steps_per_round > 0)
            e = launch_run(J, sh.F, sh.NH > 0, nullptr, sh.blocks, sh.threads, sh.lds, s);
        if (!e)
            e = launch_pt_exchange(J.E, ctx->pt_slot2rep, ctx->pt_lvl, ctx->pt_dbeta, ctx->pt_lnU,
                                   M, chains, seed, ctx->pt_round, ctx->pt_swaps, ctx->pt_pair, s);
        return e;
    };
    // Rounds are captured into a hipGraph (kernels only, no memsets) and
    // replayed; each kernel reads the round index from the device counter.
    const int64_t G = std::min<int64_t>(rounds, 32);
    int64_t done = 0;
    if (G >= 2 && rounds >= 2 * G) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        rc = check_hip(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture");
        for (int64_t q = 0; q < G && !rc; ++q) rc = check_hip(ctx, (hipError_t)one_round(), "PT round launch");
        hipError_t ee = hipStreamEndCapture(s, &graph);
        if (!rc) rc = check_hip(ctx, ee, "graph capture end");
        if (!rc) rc = check_hip(ctx, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
        for (; !rc && done + G <= rounds; done += G)
            rc = check_hip(ctx, hipGraphLaunch(exec, s), "graph launch");
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (rc) return rc;
    }
    for (; done < rounds && !rc; ++done) rc = check_hip(ctx, (hipError_t)one_round(), "PT round launch");
    if (!rc) rc = check_hip(ctx, hipEventRecord(pe1, s), "event record");
    if (rc) return rc;
    record_stats(ctx, sh, 1, J.gth);

    if (out) {
        da_result o{out->best_x, out->best_E, out->final_x, out->final_E, out->n_accept};
        rc = copy_outputs_to_host(ctx, J, R, &o, s);
        hipError_t e = hipSuccess;
        if (!rc && out->slot) e = hipMemcpy(out->slot, ctx->pt_lvl, (size_t)R * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && !rc && out->n_swaps)
            e = hipMemcpy(out->n_swaps, ctx->pt_swaps, (size_t)chains * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess && !rc && out->pair_swaps && M > 1)
            e = hipMemcpy(out->pair_swaps, ctx->pt_pair, (size_t)chains * (M - 1) * 8,
                          hipMemcpyDeviceToHost);
        if (!rc) rc = check_hip(ctx, e, "PT output copy");
    } else {
        rc = check_hip(ctx, hipStreamSynchronize(s), "stream synchronise");
    }
    return rc;
}

}  // namespace

extern "C" {

int da_pt(da_ctx *ctx, const double *temps, int32_t M, int32_t chains, int64_t rounds,
          int32_t steps_per_round, int32_t eoff_inc, uint64_t seed, da_pt_result *out) {
    if (!ctx) return fail(nullptr, DA_EINVAL, "ctx is null");
    const int rc = check_pt_args(ctx, temps, M, chains, rounds, steps_per_round, eoff_inc);
    if (rc) return rc;
    return pt_run(ctx, temps, M, chains, rounds, steps_per_round, eoff_inc, seed, out);
}

int da_pt_ladder_update(int32_t M, const double *temps, const int64_t *accepted,
                        int64_t proposals, double *out) {
    if (!temps || !out || (M > 1 && !accepted) || M < 1 || proposals < 0)
        return fail(nullptr, DA_EINVAL, "bad ladder-update arguments");
    for (int p = 0; p < M; ++p) out[p] = temps[p];
    if (M < 3 || proposals < 1) return DA_OK;
    // in inverse temperature: the span beta_0 - beta_{M-1} stays, and each
    // pair's interval becomes proportional to (its interval) * (its
    // acceptance, floored at half a swap), so more-accepting pairs widen
    const double beta_cold = 1.0 / temps[0];
    const double beta_hot = 1.0 / temps[M - 1];
    const double floor_acc = 0.5 / (double)proposals;
    std::vector<double> w((size_t)M - 1);
    double total = 0.0;
    for (int p = 0; p + 1 < M; ++p) {
        double a = (double)accepted[p] / (double)proposals;
        if (a < floor_acc) a = floor_acc;
        w[(size_t)p] = (1.0 / temps[p] - 1.0 / temps[p + 1]) * a;
        total += w[(size_t)p];
    }
    double beta = beta_cold;
    for (int p = 0; p + 2 < M; ++p) {
        beta = beta - (beta_cold - beta_hot) * (w[(size_t)p] / total);
        out[p + 1] = 1.0 / beta;
    }
    return DA_OK;
}

int da_pt_adapt(da_ctx *ctx, double *temps, int32_t M, int32_t chains, int32_t iterations,
                int64_t rounds, int32_t steps_per_round, int32_t eoff_inc, uint64_t seed,
                double *acceptance) {
    if (!ctx) return fail(nullptr, DA_EINVAL, "ctx is null");
    if (M < 2 || iterations < 0 || rounds < 1)
        return fail(ctx, DA_EINVAL, "ladder adaptation needs M >= 2, rounds >= 1");
    int rc = check_pt_args(ctx, temps, M, chains, rounds, steps_per_round, eoff_inc);
    if (rc) return rc;
    std::vector<int64_t> ps((size_t)chains * (M - 1)), acc((size_t)M - 1);
    std::vector<double> next((size_t)M);
    const int64_t proposals = (int64_t)chains * rounds;
    for (int32_t it = 0; it < iterations; ++it) {
        da_pt_result o{};
        o.pair_swaps = ps.data();
        rc = pt_run(ctx, temps, M, chains, rounds, steps_per_round, eoff_inc,
                    seed + (uint64_t)it, &o);
        if (rc) return rc;
        for (int p = 0; p + 1 < M; ++p) {
            int64_t a = 0;
            for (int32_t c = 0; c < chains; ++c) a += ps[(size_t)c * (M - 1) + p];
            acc[(size_t)p] = a;
            if (acceptance)
                acceptance[(size_t)it * (M - 1) + p] = (double)a / (double)proposals;
        }
        rc = da_pt_ladder_update(M, temps, acc.data(), proposals, next.data());
        if (rc) return rc;
        for (int p = 0; p < M; ++p) temps[p] = next[(size_t)p];
    }
    return DA_OK;
}

int da_energy(da_ctx *ctx, const uint8_t *x, int32_t count, int64_t *E) {
    if (!ctx || !x || !E || count < 1) return fail(ctx, DA_EINVAL, "bad energy arguments");
    const size_t ld = (size_t)ctx->ld, N = (size_t)ctx->N;
    std::vector<uint8_t> xp((size_t)count * ld, 0);
    for (size_t r = 0; r < (size_t)count; ++r)
        for (size_t i = 0; i < N; ++i) xp[r * ld + i] = x[r * N + i] ? 1 : 0;
    uint8_t *dX = nullptr;
    int32_t *dH = nullptr;
    int64_t *dE = nullptr;
    hipStream_t s = ctx->own_stream;
    int rc = check_hip(ctx, hipMalloc(&dX, xp.size()), "energy allocation");
    if (!rc) rc = check_hip(ctx, hipMalloc(&dH, (size_t)count * ld * 4), "energy allocation");
    if (!rc) rc = check_hip(ctx, hipMalloc(&dE, (size_t)count * 8), "energy allocation");
    if (!rc) rc = check_hip(ctx, hipMemcpyAsync(dX, xp.data(), xp.size(), hipMemcpyHostToDevice, s), "energy upload");
    JobDesc J{};
    J.W = ctx->d_W;
    J.b = ctx->d_b;
    J.N = ctx->N;
    J.ld = ctx->ld;
    J.dtype = ctx->dtype;
    J.wscale = ctx->wscale;
    if (!rc) rc = check_hip(ctx, (hipError_t)launch_fields(J, dX, count, dH, s), "field launch");
    if (!rc) rc = check_hip(ctx, (hipError_t)launch_energy_from_fields(J, dX, dH, count, dE, false, s), "energy launch");
    if (!rc) rc = check_hip(ctx, hipMemcpyAsync(E, dE, (size_t)count * 8, hipMemcpyDeviceToHost, s), "energy copy");
    if (!rc) rc = check_hip(ctx, hipStreamSynchronize(s), "stream synchronise");
    if (dX) (void)hipFree(dX);
    if (dH) (void)hipFree(dH);
    if (dE) (void)hipFree(dE);
    return rc;
}

int da_last_kernel_stats(da_ctx *ctx, da_kernel_stats *stats) {
    if (!ctx || !stats) return fail(ctx, DA_EINVAL, "null argument");
    if (!ctx->have_stats || ctx->ev_used == 0) return fail(ctx, DA_EINVAL, "no launch recorded yet");
    int rc = check_hip(ctx, hipEventSynchronize(ctx->ev1), "event synchronise");
    if (rc) return rc;
    double total = 0.0;
    float ms = 0.f;
    for (size_t q = 0; q < ctx->ev_used; ++q) {
        rc = check_hip(ctx, hipEventElapsedTime(&ms, ctx->ev_pool[q].first, ctx->ev_pool[q].second),
                       "event elapsed time");
        if (rc) return rc;
        total += ms;
    }
    ctx->last.kernel_ms = ms;
    ctx->last.total_ms = total + ctx->folded_ms;
    ctx->last.launches = (int64_t)ctx->ev_used + ctx->folded_calls;
    *stats = ctx->last;
    return DA_OK;
}

int da_reset_kernel_stats(da_ctx *ctx) {
    if (!ctx) return fail(nullptr, DA_EINVAL, "ctx is null");
    if (ctx->ev1) {
        const int rc = check_hip(ctx, hipEventSynchronize(ctx->ev1), "event synchronise");
        if (rc) return rc;
    }
    ctx->ev_used = 0;
    ctx->folded_ms = 0.0;
    ctx->folded_calls = 0;
    return DA_OK;
}

const char *da_last_error(const da_ctx *ctx) {
    if (ctx) return ctx->err.c_str();
    return t_err.c_str();
}

#ifndef DAPT_BUILD_ID
#define DAPT_BUILD_ID "unknown"
#endif
const char *da_build_id(void) { return DAPT_BUILD_ID; }

const char *da_strerror(int status) {
    switch (status) {
        case DA_OK: return "ok";
        case DA_EINVAL: return "invalid argument";
        case DA_ERANGE: return "coefficients out of range";
        case DA_ENOMEM: return "out of memory";
        case DA_EDEVICE: return "device error";
        case DA_ENOTREADY: return "not ready";
        case DA_ENOTFOUND: return "unknown ticket";
        default: return "unknown status";
    }
}

int da_threshold_table(double T, int32_t *thr) {
    if (!thr) return fail(nullptr, DA_EINVAL, "thr is null");
    build_threshold_table(T, thr);
    return DA_OK;
}

double da_level_temperature(const da_schedule *schedule, int32_t level) {
    if (!schedule) return NAN;
    return schedule_temperature(*schedule, level);
}

}  // extern "C"
