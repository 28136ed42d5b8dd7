// Host checks of the library's level tables against the way the step kernel
// uses them: every level's bucket count fits the LDS staging area and its
// reject-all entry sits where staging and the one-read form look for it; the
// three in-kernel decision forms (band tests + bracket, one bracket read per
// flip, direct table) agree with the definition d <= thr[u] of the Metropolis
// test as a threshold on the 16-bit draw; and the autotuner's timing window
// stays inside its schedule.  Exit status 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "da_internal.h"
#include "da_runtime.h"

using namespace dapt;

static long g_bad = 0;
#define CHECK(c, ...)                    \
    do {                                 \
        if (!(c)) {                      \
            if (g_bad < 20) {            \
                std::printf(__VA_ARGS__); \
                std::printf("\n");       \
            }                            \
            ++g_bad;                     \
        }                                \
    } while (0)

// band tests, then the bracket of an in-band cost, then the exact entry
static bool band_form(const int32_t *thr, const LevelHdr &hd, const uint32_t *brk, int64_t d,
                      uint32_t u) {
    const int64_t t1 = (int64_t)hd.tmin + 1, span = (int64_t)hd.tmax - hd.tmin;
    if (d < t1) return true;
    const int64_t ub = d - t1;
    if (ub >= span) return false;
    const uint32_t e = brk[hd.off + (ub >> hd.sh)];
    const uint32_t lo = e & 0xFFFFu, hi = e >> 16;
    if (u < lo) return true;
    if (u >= hi) return false;
    return d <= thr[u];
}

// one bracket read, no band tests: the offset wraps as a 32-bit unsigned
// number and is clamped to the first offset past the buckets
static bool one_read_form(const int32_t *thr, const LevelHdr &hd, const uint32_t *brk, int64_t d,
                          uint32_t u) {
    const int64_t t1 = (int64_t)hd.tmin + 1;
    const int nb = hd.tmax > hd.tmin ? ((hd.tmax - hd.tmin - 1) >> hd.sh) + 1 : 0;
    const uint32_t ubmax = (uint32_t)nb << hd.sh;
    const uint32_t ub = (uint32_t)(uint64_t)(d - t1);
    const uint32_t idx = (ub < ubmax ? ub : ubmax) >> hd.sh;
    bool acc = d < t1;
    const uint32_t e = brk[hd.off + idx];
    const uint32_t lo = e & 0xFFFFu, hi = e >> 16;
    acc = acc || u < lo;
    if (u >= lo && u < hi) acc = acc || d <= thr[u];
    return acc;
}

// The per-draw estimate path (kModeGen) with an estimate of the device's form
// evaluated on the host (the host's log2f stands in for v_log_f32; the window
// is measured over all draws either way): the ring value is the fp32 sum's
// bits, G = bits - kGenMagic; with z = s + bits - (E_off + glo + 1 + kGenMagic)
// in wrapping 32-bit arithmetic, z < 0 accepts, ghi - glo <= z rejects, and in
// between the exact entry decides.  Also checks that the sum lands in
// [2^23, 2^24) (so the bits are the rounded value) and that the true z fits
// int32 for |s| <= kGenFieldMax, E_off in [0, 2^30] and tmax < 2^22.
static int32_t host_estimate_bits(uint32_t u, float ga, float gb) {
    const float x = (float)u + 0.5f;
    const float v = std::fma(std::log2(x), ga, gb);
    CHECK(v >= 8388608.0f && v < 16777216.0f, "estimate sum %g outside [2^23, 2^24)", (double)v);
    int32_t b;
    std::memcpy(&b, &v, 4);
    return b;
}

static bool estimate_form(const int32_t *thr, int glo, int ghi, int32_t bits, int64_t s,
                          int32_t eoff, uint32_t u, bool &wrapped) {
    const uint32_t Ec = (uint32_t)eoff + (uint32_t)glo + 1u + kGenMagic;
    const int32_t z = (int32_t)((uint32_t)(int32_t)s + (uint32_t)bits - Ec);
    const int64_t G = (int64_t)bits - (int64_t)kGenMagic;
    const int64_t zt = s + G - ((int64_t)eoff + glo + 1);
    wrapped = zt < INT32_MIN || zt > INT32_MAX || (int64_t)z != zt;
    if (z < 0) return true;
    if ((uint32_t)z >= (uint32_t)(ghi - glo)) return false;
    return s - eoff <= thr[u];
}

// never called here: the host check builds tables without uploading them
namespace dapt {
int launch_gen_calibrate(LevelHdr *, const int32_t *, int32_t, void *) { return 1; }
}  // namespace dapt

int main() {
    std::vector<std::vector<double>> lists;
    for (double Thi : {0.3, 3.0, 20.0, 60.0, 196608.0, 1e6, 3e8, 5e9})
        for (int L : {1, 6, 64})
            for (double ratio : {1.0, 0.05}) {
                std::vector<double> t;
                for (int l = 0; l < L; ++l)
                    t.push_back(L == 1 ? Thi : Thi * std::pow(ratio, (double)l / (L - 1)));
                lists.push_back(t);
            }
    lists.push_back({0.0});
    std::mt19937_64 rng(12345);
    long levels = 0, decisions = 0;
    for (const auto &t : lists) {
        HostTables ht;
        build_host_tables(t, ht);
        int nq = 0;
        for (size_t l = 0; l < t.size(); ++l) {
            const LevelHdr &hd = ht.hdr[l];
            const int32_t *thr = ht.thr.data() + l * 65536;
            const uint32_t *brk = ht.brk.data();
            ++levels;
            CHECK(hd.tmin == thr[65535] && hd.tmax == thr[0], "T=%g: band limits", t[l]);
            const int nb = hd.tmax > hd.tmin ? ((hd.tmax - hd.tmin - 1) >> hd.sh) + 1 : 0;
            CHECK(nb + 1 <= kMaxBuckets, "T=%g: %d buckets", t[l], nb);
            CHECK((size_t)hd.off + nb < ht.brk.size() && brk[hd.off + nb] == 0,
                  "T=%g: reject-all entry missing", t[l]);
            const bool narrow = hd.tmax > hd.tmin && hd.tmax - hd.tmin <= kDirectSpan &&
                                hd.tmin >= -kDirectTmin && hd.tmin <= kDirectTmin &&
                                t.size() <= (size_t)kMaxDirectLevels;
            CHECK(narrow == (hd.q8 >= 0), "T=%g: direct table %d", t[l], hd.q8);
            const uint8_t *q = hd.q8 >= 0 ? ht.q8.data() + (size_t)hd.q8 * 65536 : nullptr;
            if (hd.q8 >= 0) CHECK(hd.q8 == nq++, "T=%g: direct table order", t[l]);
            // costs across and beyond the band, and the extremes of the int32 range
            std::vector<int64_t> ds = {INT32_MIN, -(int64_t(1) << 30), -1, 0, 1, int64_t(1) << 30};
            for (int64_t k = -300; k <= 300; ++k) {
                ds.push_back((int64_t)hd.tmin + k);
                ds.push_back((int64_t)hd.tmax + k);
            }
            std::uniform_int_distribution<int64_t> band((int64_t)hd.tmin - 5, (int64_t)hd.tmax + 5);
            for (int k = 0; k < 600; ++k) ds.push_back(band(rng));
            for (int64_t d : ds)
                for (int k = 0; k < 6; ++k) {
                    const uint32_t u = k == 0 ? 0u : (k == 1 ? 65535u : (uint32_t)(rng() & 0xFFFFu));
                    const bool want = d <= thr[u];
                    ++decisions;
                    CHECK(band_form(thr, hd, brk, d, u) == want, "T=%g d=%lld u=%u: band form",
                          t[l], (long long)d, u);
                    if (hd.tmax < (1 << 29))
                        CHECK(one_read_form(thr, hd, brk, d, u) == want,
                              "T=%g d=%lld u=%u: one-read form", t[l], (long long)d, u);
                    if (q && d >= -(int64_t(1) << 30) - (int64_t(1) << 30) + 512)
                        CHECK(((d - ((int64_t)hd.tmin + 1)) < (int64_t)q[u]) == want,
                              "T=%g d=%lld u=%u: direct table", t[l], (long long)d, u);
                }
            // the estimate path: candidates are exactly the levels with T > 0
            // and tmax < 2^29; window measured over every draw
            CHECK(hd.gth == ((t[l] > 0.0 && hd.tmax < kGenTmax) ? 1 : 0), "T=%g: estimate flag",
                  t[l]);
            if (!hd.gth) continue;
            int glo = INT32_MAX, ghi = INT32_MIN;
            std::vector<int32_t> G(65536);
            for (uint32_t u = 0; u < 65536; ++u) {
                G[u] = host_estimate_bits(u, hd.ga, hd.gb);
                const int32_t off = thr[u] + (int32_t)((uint32_t)G[u] - kGenMagic);
                glo = std::min(glo, off);
                ghi = std::max(ghi, off);
            }
            // the device keeps a level only when its window is narrow (fp32
            // rounding widens it with T: a few units up to T ~ 1e6)
            const bool ok = glo >= -kGenOffMax && ghi <= kGenOffMax && ghi - glo <= kGenWindow;
            if (t[l] <= 1e6)
                CHECK(ok && ghi - glo <= 4, "T=%g: estimate window [%d, %d]", t[l], glo, ghi);
            if (!ok) continue;
            for (int32_t eoff : {0, 1, 1 << 20, 1 << 29, (1 << 30) - 1, 1 << 30})
                for (int64_t d : ds) {
                    const int64_t s = d + eoff;
                    if (s > kGenFieldMax || s < -kGenFieldMax) continue;
                    for (int k = 0; k < 3; ++k) {
                        const uint32_t u =
                            k == 0 ? 0u : (k == 1 ? 65535u : (uint32_t)(rng() & 0xFFFFu));
                        bool wrapped = false;
                        ++decisions;
                        CHECK(estimate_form(thr, glo, ghi, G[u], s, eoff, u, wrapped) ==
                                  (d <= thr[u]),
                              "T=%g d=%lld eoff=%d u=%u: estimate form", t[l], (long long)d,
                              eoff, u);
                        CHECK(!wrapped, "T=%g s=%lld eoff=%d: estimate sum wraps", t[l],
                              (long long)s, eoff);
                    }
                }
            // the extreme sums: |s| at the bound, largest offset, both ends of G
            for (int64_t s : {-kGenFieldMax, kGenFieldMax})
                for (uint32_t u : {0u, 65535u}) {
                    bool wrapped = false;
                    (void)estimate_form(thr, glo, ghi, G[u], s, 1 << 30, u, wrapped);
                    CHECK(!wrapped, "T=%g: extreme estimate sum wraps", t[l]);
                    (void)estimate_form(thr, glo, ghi, G[u], s, 0, u, wrapped);
                    CHECK(!wrapped, "T=%g: extreme estimate sum wraps", t[l]);
                }
        }
    }
    for (int64_t S = 1; S <= 5000; ++S) {
        int64_t s0 = 0, s1 = 0;
        tune_window(S, s0, s1);
        CHECK(s0 >= 0 && s1 <= S && s1 - s0 == (S < 384 ? S : 384), "tune window S=%lld",
              (long long)S);
    }
    // the host guard of every step-kernel launch: a step range inside the
    // schedule passes (the autotuner's window included), anything reaching
    // step S or beyond -- where the level index would leave the tables -- and
    // offset increments that could overflow the saturating update do not
    {
        LevelHdr hdr0{};
        JobDesc J{};
        J.N = 1000;
        J.ld = 1024;
        J.R = 8;
        J.NW = 2;
        J.NH = 2;
        J.RPW = 1;
        J.L = 128;
        J.hdr = &hdr0;
        J.eoff_inc = 1;
        for (int64_t S : {1, 2, 63, 64, 383, 384, 575, 576, 100000}) {
            J.S = S;
            J.s0 = 0;
            J.s1 = S;
            CHECK(job_range_error(J) == nullptr, "guard rejects the whole schedule S=%lld",
                  (long long)S);
            tune_window(S, J.s0, J.s1);
            CHECK(job_range_error(J) == nullptr, "guard rejects the tuner window S=%lld",
                  (long long)S);
            J.s0 = S / 3;              // the old window: starts at S/3 whatever S
            J.s1 = J.s0 + 384;
            CHECK((job_range_error(J) == nullptr) == (J.s1 <= S),
                  "guard and a window past the end disagree, S=%lld", (long long)S);
            J.s0 = 0;
            J.s1 = S + 1;
            CHECK(job_range_error(J) != nullptr, "guard lets s1 = S + 1 through");
            J.s0 = -1;
            J.s1 = S;
            CHECK(job_range_error(J) != nullptr, "guard lets s0 < 0 through");
            J.s0 = S;
            J.s1 = S - 1;
            CHECK(job_range_error(J) != nullptr, "guard lets s0 > s1 through");
        }
        J.S = 1000;
        J.s0 = 0;
        J.s1 = 1000;
        for (int32_t inc : {0, 1, 65536, kEoffMax}) {
            J.eoff_inc = inc;
            CHECK(job_range_error(J) == nullptr, "guard rejects increment %d", inc);
        }
        J.eoff_inc = kEoffMax + 1;
        CHECK(job_range_error(J) != nullptr, "guard lets an increment above 2^30 through");
        J.eoff_inc = -1;
        CHECK(job_range_error(J) != nullptr, "guard lets a negative increment through");
        J.eoff_inc = 1;
        J.NW = 15;                    // 15 + 2 waves do not fit one workgroup
        CHECK(job_range_error(J) != nullptr, "guard lets 17 waves through");
        J.NW = 2;
        J.L = 0;
        CHECK(job_range_error(J) != nullptr, "guard lets a job without levels through");
        // the saturating offset update equals min(E_off + inc, 2^30) over [0, 2^30]
        for (int64_t e : {int64_t(0), int64_t(1), int64_t(kEoffMax) - 1, int64_t(kEoffMax)})
            for (int64_t inc : {int64_t(0), int64_t(1), int64_t(1) << 29, int64_t(kEoffMax)}) {
                const int32_t cap = kEoffMax - (int32_t)inc;
                const int64_t got = (int64_t)std::min<int32_t>((int32_t)e, cap) + inc;
                const int64_t want = std::min<int64_t>(e + inc, kEoffMax);
                CHECK(got == want, "offset update e=%lld inc=%lld", (long long)e,
                      (long long)inc);
            }
    }
    std::printf("levels %ld decisions %ld failures %ld\n", levels, decisions, g_bad);
    return g_bad != 0;
}
