// da_tables.cpp -- temperature levels and the Metropolis decision tables.
//
// The Metropolis acceptance exp(-dE/T) (Sec. III of arXiv:1806.08815) is
// decided in integers.  A 16-bit draw u stands for U_u = (u + 1/2)/65536, and a
// flip of offset-shifted cost d is accepted iff U_u < exp(-d/T), which for an
// integer d is d <= thr[u] with thr[u] = ceil(-T ln U_u) - 1.  Every decision
// the device takes is this comparison against these host-built tables, so it
// is bit-identical wherever it is made; the device's own fp32 estimate of
// thr[u] (LevelHdr) only brackets it, with a window measured over all draws.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>

#include "da_runtime.h"

namespace dapt {

namespace {
constexpr int64_t kThrMax = int64_t(1) << 30;
}

namespace {
// ln U_u for every draw, computed once: a level's table is then one product
// per entry, the same product -T * ln(U_u) either way.
const double *log_u_table() {
    static const std::vector<double> t = [] {
        std::vector<double> v(65536);
        for (int u = 0; u < 65536; ++u) v[(size_t)u] = std::log(((double)u + 0.5) / 65536.0);
        return v;
    }();
    return t.data();
}
}  // namespace

int32_t threshold_entry(double T, int u) {
    if (!(T > 0.0)) return -1;
    const double y = -T * log_u_table()[u];
    const double c = std::ceil(y) - 1.0;
    int64_t t = (c >= (double)kThrMax) ? kThrMax : (int64_t)c;
    if (t < -1) t = -1;
    return (int32_t)t;
}

void build_threshold_table(double T, int32_t *thr) {
    for (int u = 0; u < 65536; ++u) thr[u] = threshold_entry(T, u);
}

// Number of draws accepting cost d: thr is non-increasing in u, so the
// accepting draws form the prefix [0, ucut(d)).
static int ucut(const int32_t *thr, int64_t d) {
    int lo = 0, hi = 65536;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)thr[mid] >= d) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

void build_brackets(const int32_t *thr, LevelHdr &hd, std::vector<uint32_t> &brk) {
    hd.tmin = thr[65535];
    hd.tmax = thr[0];
    hd.sh = 0;
    hd.q8 = -1;
    hd.gth = 0;
    hd.ga = hd.gb = 0.0f;
    hd.glo = hd.ghi = 0;
    hd.pad[0] = hd.pad[1] = 0;
    hd.off = (int32_t)brk.size();
    // every level ends with a reject-all entry (lo = hi = 0), which costs
    // past the last bucket may read
    if (hd.tmax <= hd.tmin) {   // no draw ever changes a decision
        brk.push_back(0);
        return;
    }
    const int64_t range = (int64_t)hd.tmax - hd.tmin;
    int sh = 0;
    while (((range + (int64_t(1) << sh) - 1) >> sh) > kMaxBuckets - 1) ++sh;
    const int64_t nb = (range + (int64_t(1) << sh) - 1) >> sh;
    for (int64_t D = 0; D < nb; ++D) {
        // the lower cut at the bucket's true end: past tmax it is 0, so
        // costs above the band that fall into the last bucket are decided
        // by the exact table entry
        const int64_t ds = (int64_t)hd.tmin + 1 + (D << sh);
        const int64_t de = ds + (int64_t(1) << sh) - 1;
        const uint32_t lo = (uint32_t)ucut(thr, de);
        const uint32_t hi = (uint32_t)ucut(thr, ds);
        brk.push_back(lo | (hi << 16));
    }
    brk.push_back(0);
    hd.sh = sh;
}

double schedule_temperature(const da_schedule &s, int l) {
    if (s.n_levels <= 1) return s.T_hi;
    const double frac = (double)l / (double)(s.n_levels - 1);
    if (s.kind == DA_SCHED_LINEAR_BETA)
        return 1.0 / (1.0 / s.T_hi + (1.0 / s.T_lo - 1.0 / s.T_hi) * frac);
    return s.T_hi * std::pow(s.T_lo / s.T_hi, frac);
}

std::vector<double> schedule_temps(const da_schedule &s) {
    std::vector<double> t((size_t)s.n_levels);
    for (int l = 0; l < s.n_levels; ++l) t[(size_t)l] = schedule_temperature(s, l);
    return t;
}

int64_t level_table_bytes(int32_t L, int64_t buckets) {
    // direct tables: at most one per level, only for short schedules
    const int64_t q8 = L <= kMaxDirectLevels ? (int64_t)L * 65536 : 0;
    return (int64_t)L * 65536 * 4 + (int64_t)L * (int64_t)sizeof(LevelHdr) + buckets * 4 + q8;
}

LevelTables::~LevelTables() {
    if (d_thr) (void)hipFree(d_thr);
    if (d_hdr) (void)hipFree(d_hdr);
    if (d_brk) (void)hipFree(d_brk);
    if (d_q8) (void)hipFree(d_q8);
}

namespace {
struct CacheKey {
    int device;
    std::string bits;
    bool operator<(const CacheKey &o) const {
        return device != o.device ? device < o.device : bits < o.bits;
    }
};
std::mutex g_cache_mu;
std::map<CacheKey, std::weak_ptr<LevelTables>> g_cache;
}  // namespace

void build_host_tables(const std::vector<double> &temps, HostTables &ht) {
    const size_t L = temps.size();
    ht.temps = temps;
    ht.thr.resize(L * 65536);
    ht.hdr.resize(L);
    ht.brk.clear();
    ht.q8.clear();
    int32_t nq = 0;
    for (size_t l = 0; l < L; ++l) {
        const int32_t *thr = ht.thr.data() + l * 65536;
        build_threshold_table(temps[l], ht.thr.data() + l * 65536);
        build_brackets(thr, ht.hdr[l], ht.brk);
        LevelHdr &hd = ht.hdr[l];
        if (L <= (size_t)kMaxDirectLevels && hd.tmax > hd.tmin &&
            hd.tmax - hd.tmin <= kDirectSpan && hd.tmin >= -kDirectTmin &&
            hd.tmin <= kDirectTmin) {
            hd.q8 = nq++;
            for (int u = 0; u < 65536; ++u) ht.q8.push_back((uint8_t)(thr[u] - hd.tmin));
        }
        // candidates for the per-draw estimate: -G(u) ~ T ln(65536 / (u + 1/2));
        // the device measures the window (launch_gen_calibrate)
        const double T = temps[l];
        if (T > 0.0 && std::isfinite(T) && hd.tmax < kGenTmax) {
            hd.gth = 1;
            hd.ga = (float)(T * std::log(2.0));
            hd.gb = (float)(1.5 * 8388608.0 - 16.0 * T * std::log(2.0));
        }
    }
    if (ht.brk.empty()) ht.brk.push_back(0);
}

std::shared_ptr<LevelTables> get_level_tables(const std::vector<double> &temps, std::string &err,
                                              const HostTables *pre) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return nullptr;
    }
    CacheKey key{dev, std::string(reinterpret_cast<const char *>(temps.data()),
                                  temps.size() * sizeof(double))};
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        if (auto sp = it->second.lock()) return sp;
    }
    HostTables own;
    if (!pre || pre->temps != temps) {
        build_host_tables(temps, own);
        pre = &own;
    }
    auto lt = std::make_shared<LevelTables>();
    lt->temps = temps;
    lt->L = (int32_t)temps.size();
    lt->hdr = pre->hdr;
    const size_t thr_b = pre->thr.size() * 4, hdr_b = pre->hdr.size() * sizeof(LevelHdr),
                 brk_b = pre->brk.size() * 4;
    const size_t q8_b = pre->q8.size();
    if (hipMalloc(&lt->d_thr, thr_b) != hipSuccess || hipMalloc(&lt->d_hdr, hdr_b) != hipSuccess ||
        hipMalloc(&lt->d_brk, brk_b) != hipSuccess ||
        (q8_b && hipMalloc(&lt->d_q8, q8_b) != hipSuccess)) {
        err = "out of device memory for level tables";
        return nullptr;
    }
    if (hipMemcpy(lt->d_thr, pre->thr.data(), thr_b, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(lt->d_hdr, pre->hdr.data(), hdr_b, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(lt->d_brk, pre->brk.data(), brk_b, hipMemcpyHostToDevice) != hipSuccess ||
        (q8_b && hipMemcpy(lt->d_q8, pre->q8.data(), q8_b, hipMemcpyHostToDevice) != hipSuccess)) {
        err = "upload of level tables failed";
        return nullptr;
    }
    // windows of the per-draw estimates, measured on this device; the host
    // copy of the headers takes them over
    if (launch_gen_calibrate(lt->d_hdr, lt->d_thr, lt->L, nullptr) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess ||
        hipMemcpy(lt->hdr.data(), lt->d_hdr, hdr_b, hipMemcpyDeviceToHost) != hipSuccess) {
        err = "estimate window pass over the level tables failed";
        return nullptr;
    }
    for (const LevelHdr &h : lt->hdr) lt->any_gth = lt->any_gth || h.gth != 0;
    lt->bytes = thr_b + hdr_b + brk_b + q8_b;
    g_cache[key] = lt;
    return lt;
}

StepTables::~StepTables() {
    if (d_steps) (void)hipFree(d_steps);
}

namespace {
std::mutex g_step_mu;
std::map<std::string, std::weak_ptr<StepTables>> g_step_cache;
std::mutex g_G_mu;
std::map<int, double *> g_G;   // per device, held until the process ends
}  // namespace

std::shared_ptr<StepTables> get_step_tables(const da_schedule &s, int64_t S, std::string &err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return nullptr;
    }
    if (S < 1 || S > kMaxPerStepSteps) {
        err = "per-step schedules take 1 .. 2^24 steps";
        return nullptr;
    }
    std::string key(reinterpret_cast<const char *>(&dev), sizeof dev);
    key.append(reinterpret_cast<const char *>(&s.T_hi), sizeof s.T_hi);
    key.append(reinterpret_cast<const char *>(&s.T_lo), sizeof s.T_lo);
    key.append(reinterpret_cast<const char *>(&s.kind), sizeof s.kind);
    key.append(reinterpret_cast<const char *>(&S), sizeof S);
    std::lock_guard<std::mutex> lock(g_step_mu);
    auto it = g_step_cache.find(key);
    if (it != g_step_cache.end()) {
        if (auto sp = it->second.lock()) return sp;
    }
    // step s runs at level s of an S-level schedule
    da_schedule lv = s;
    lv.n_levels = (int32_t)std::min<int64_t>(S, INT32_MAX);
    std::vector<StepT> host((size_t)S);
    for (int64_t q = 0; q < S; ++q) {
        const double T = schedule_temperature(lv, (int)q);
        host[(size_t)q] = StepT{T, threshold_entry(T, 65535), threshold_entry(T, 0)};
    }
    auto st = std::make_shared<StepTables>();
    st->S = S;
    st->bytes = host.size() * sizeof(StepT);
    if (hipMalloc(&st->d_steps, st->bytes) != hipSuccess ||
        hipMemcpy(st->d_steps, host.data(), st->bytes, hipMemcpyHostToDevice) != hipSuccess) {
        err = "per-step table allocation or upload failed";
        return nullptr;
    }
    g_step_cache[key] = st;
    return st;
}

const double *device_neg_log_u(std::string &err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_G_mu);
    auto it = g_G.find(dev);
    if (it != g_G.end()) return it->second;
    std::vector<double> G(65536);
    const double *lnU = log_u_table();
    for (int u = 0; u < 65536; ++u) G[(size_t)u] = -lnU[u];
    double *d = nullptr;
    if (hipMalloc(&d, G.size() * 8) != hipSuccess ||
        hipMemcpy(d, G.data(), G.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        err = "-ln U table allocation or upload failed";
        return nullptr;
    }
    g_G[dev] = d;
    return d;
}

}  // namespace dapt
