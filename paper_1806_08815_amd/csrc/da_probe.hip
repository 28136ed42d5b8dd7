// da_probe.hip -- memory roofline of the DA row stream.
//
// Each step of the annealer fetches one row of the coupling matrix, chosen by
// the previous step's selection, so a replica has exactly one dependent row
// fetch in flight.  This probe reproduces that access pattern without the
// rest of the step: `chains` independent chains (one workgroup of `waves`
// waves each, like a replica) walk a random permutation of the rows of an
// n_rows x row_elems matrix; every wave loads its share of the current row
// with the same vector loads as the step kernel, and the next row index is
// read out of the loaded data, so fetches are serialised per chain.  The time
// per step is the dependent-fetch latency at that working-set size (L2, MALL
// or HBM); rows * chains / time is the achievable row-stream bandwidth for a
// given number of chains in flight.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "da.h"
#include "da_internal.h"

namespace {

template <typename WT>
__global__ __launch_bounds__(1024) void k_row_chase(const WT *__restrict__ M, int32_t ld,
                                                    int32_t n_rows, int64_t steps, int32_t *sink) {
    constexpr int F = 8;
    typedef WT V __attribute__((ext_vector_type(F)));
    __shared__ int next;
    const int lane = threadIdx.x & 63;
    const int g = threadIdx.x;
    int k = (int)((blockIdx.x * 2654435761u) % (uint32_t)n_rows);
    int acc = 0;
    const int col = (g * F < ld) ? g * F : 0;
    for (int64_t s = 0; s < steps; ++s) {
        const V v = *reinterpret_cast<const V *>(M + (size_t)k * ld + col);
        int part = 0;
#pragma unroll
        for (int f = 0; f < F; ++f) part += (int)v[f];
        acc += part;
        // row index of the next step, from the first element of this row
        if (blockDim.x > 64) {
            if (g == 0) next = (int)v[0];
            __syncthreads();
            k = next;
            __syncthreads();
        } else {
            k = __builtin_amdgcn_readfirstlane((int)v[0]);
        }
        k = (k & 0x7fffffff) % n_rows;
    }
    if (lane == 0) sink[blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)] = acc;
}

template <typename WT>
int run_probe(int32_t n_rows, int32_t row_elems, int32_t chains, int32_t waves, int64_t steps,
              double *ns_per_step, double *gbytes_per_s) {
    const int32_t ld = (row_elems + 511) / 512 * 512;
    if (waves * 64 * 8 < row_elems) return DA_EINVAL;
    // random permutation cycle: element 0 of row r names the next row
    std::vector<WT> host((size_t)n_rows * ld, (WT)1);
    std::vector<int32_t> perm((size_t)n_rows);
    for (int32_t r = 0; r < n_rows; ++r) perm[(size_t)r] = r;
    uint64_t x = 0x9E3779B97F4A7C15ull;
    for (int32_t r = n_rows - 1; r > 0; --r) {
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        const int32_t j = (int32_t)(x % (uint64_t)(r + 1));
        std::swap(perm[(size_t)r], perm[(size_t)j]);
    }
    for (int32_t q = 0; q < n_rows; ++q)
        host[(size_t)perm[(size_t)q] * ld] = (WT)perm[(size_t)((q + 1) % n_rows)];
    WT *dM = nullptr;
    int32_t *sink = nullptr;
    if (hipMalloc(&dM, host.size() * sizeof(WT)) != hipSuccess) return DA_ENOMEM;
    if (hipMalloc(&sink, (size_t)chains * waves * 4) != hipSuccess) {
        (void)hipFree(dM);
        return DA_ENOMEM;
    }
    int rc = DA_OK;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = DA_EDEVICE;
    if (!rc &&
        hipMemcpy(dM, host.data(), host.size() * sizeof(WT), hipMemcpyHostToDevice) != hipSuccess)
        rc = DA_EDEVICE;
    float ms = 0.f;
    if (!rc) {
        // warm caches with a short run, then time
        hipLaunchKernelGGL(k_row_chase<WT>, dim3(chains), dim3(64 * waves), 0, 0, dM, ld, n_rows,
                           (int64_t)(steps / 10 + 1), sink);
        if (hipGetLastError() != hipSuccess || hipEventRecord(a, 0) != hipSuccess) rc = DA_EDEVICE;
    }
    if (!rc) {
        hipLaunchKernelGGL(k_row_chase<WT>, dim3(chains), dim3(64 * waves), 0, 0, dM, ld, n_rows,
                           steps, sink);
        if (hipGetLastError() != hipSuccess || hipEventRecord(b, 0) != hipSuccess ||
            hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
            rc = DA_EDEVICE;
    }
    if (!rc) {
        const double t = ms * 1e-3;
        *ns_per_step = t / (double)steps * 1e9;
        *gbytes_per_s = (double)row_elems * sizeof(WT) * chains * (double)steps / t / 1e9;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(dM);
    (void)hipFree(sink);
    return rc;
}

}  // namespace

// Initial fields of R random states of a random +-1 N-variable instance on the
// matrix cores (the int8 path of the random start): average time of `iters`
// launches of the field kernel alone, and int8 ops/s (2 ld^2 R per launch).
extern "C" int da_probe_fields_mfma(int32_t N, int32_t R, int32_t iters, double *ms_per_call,
                                    double *tera_ops) {
    if (N < 32 || N > DA_MAX_N || R < 1 || iters < 1 || !ms_per_call || !tera_ops)
        return DA_EINVAL;
    const int32_t ld = (N + 63) / 64 * 64;
    std::vector<int8_t> w((size_t)ld * ld, 0);
    std::vector<uint8_t> x((size_t)R * ld, 0);
    uint64_t st = 0x243F6A8885A308D3ull;
    auto next = [&]() {
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        return st;
    };
    for (int32_t i = 0; i < N; ++i)
        for (int32_t j = i + 1; j < N; ++j) {
            const int8_t v = (next() & 1) ? 1 : -1;
            w[(size_t)i * ld + j] = v;
            w[(size_t)j * ld + i] = v;
        }
    for (int32_t r = 0; r < R; ++r)
        for (int32_t i = 0; i < N; ++i) x[(size_t)r * ld + i] = (uint8_t)(next() & 1);
    int8_t *dW = nullptr;
    uint8_t *dX = nullptr;
    int32_t *db = nullptr, *dH = nullptr;
    int rc = DA_OK;
    if (hipMalloc(&dW, w.size()) != hipSuccess || hipMalloc(&dX, x.size()) != hipSuccess ||
        hipMalloc(&db, (size_t)ld * 4) != hipSuccess ||
        hipMalloc(&dH, (size_t)R * ld * 4) != hipSuccess)
        rc = DA_ENOMEM;
    if (!rc && (hipMemcpy(dW, w.data(), w.size(), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(dX, x.data(), x.size(), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemset(db, 0, (size_t)ld * 4) != hipSuccess))
        rc = DA_EDEVICE;
    hipEvent_t a = nullptr, b = nullptr;
    if (!rc) {
        dapt::JobDesc J{};
        J.W = dW;
        J.b = db;
        J.N = N;
        J.ld = ld;
        J.dtype = 1;
        J.wscale = 1;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = DA_EDEVICE;
        if (!rc && dapt::launch_fields(J, dX, R, dH, nullptr) != 0) rc = DA_EDEVICE;
        if (!rc && hipEventRecord(a, 0) != hipSuccess) rc = DA_EDEVICE;
        for (int32_t q = 0; q < iters && !rc; ++q)
            if (dapt::launch_fields(J, dX, R, dH, nullptr) != 0) rc = DA_EDEVICE;
        float ms = 0.f;
        if (!rc && (hipEventRecord(b, 0) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                    hipEventElapsedTime(&ms, a, b) != hipSuccess))
            rc = DA_EDEVICE;
        if (!rc) {
            *ms_per_call = ms / iters;
            *tera_ops = 2.0 * ld * (double)ld * R / (*ms_per_call * 1e-3) / 1e12;
        }
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    (void)hipFree(dW);
    (void)hipFree(dX);
    (void)hipFree(db);
    (void)hipFree(dH);
    return rc;
}

extern "C" int da_probe_row_stream(int32_t n_rows, int32_t row_elems, int32_t dtype_bytes,
                                   int32_t chains, int32_t waves_per_chain, int64_t steps,
                                   double *ns_per_step, double *gbytes_per_s) {
    if (n_rows < 2 || row_elems < 8 || chains < 1 || waves_per_chain < 1 ||
        waves_per_chain > 16 || steps < 1 || !ns_per_step || !gbytes_per_s)
        return DA_EINVAL;
    if (dtype_bytes == 2 && n_rows > 32767) return DA_EINVAL;
    switch (dtype_bytes) {
        case 2: return run_probe<int16_t>(n_rows, row_elems, chains, waves_per_chain, steps,
                                          ns_per_step, gbytes_per_s);
        case 4: return run_probe<int32_t>(n_rows, row_elems, chains, waves_per_chain, steps,
                                          ns_per_step, gbytes_per_s);
        default: return DA_EINVAL;
    }
}
