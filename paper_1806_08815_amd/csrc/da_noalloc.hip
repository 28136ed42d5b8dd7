// da_noalloc.hip -- an allocation-free form of da_energy, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// da_energy stages the states in padded rows and computes the local fields
// H = X W^T + b (int8 matrix cores or the row kernel) before the energies
// E = (1/2) sum_i x_i (h_i + b_i); both intermediates live in device scratch.
// Here that scratch is one file-scope device array per GPU, of a fixed
// maximum size.  Its address on each device is taken once, with that device
// current, and only that address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "da_runtime.h"

namespace dapt {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB on every device
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device (taken once per device).
int scratch_on_device(int dev, uint8_t **out, std::string &err) {
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device index out of range";
        return DA_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("scratch symbol address: ") + hipGetErrorString(e);
            return DA_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return DA_OK;
}

// [count][N] states (nonzero = 1) into [count][ld] rows, zero padded.
__global__ void k_pad_states(const uint8_t *__restrict__ x, uint8_t *__restrict__ X,
                             int32_t count, int32_t N, int32_t ld) {
    const int64_t n = (int64_t)count * ld;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / ld;
        const int i = (int)(q - r * ld);
        X[q] = i < N ? (uint8_t)(x[r * N + i] != 0) : (uint8_t)0;
    }
}

}  // namespace
}  // namespace dapt

using namespace dapt;

namespace {
// Largest count whose padded states and fields fit the scratch at this N:
// ceil(count ld / 256) 256 + 4 count ld <= kScratchBytes.
int64_t max_states(int32_t N) {
    const int64_t ld = ((int64_t)N + 63) / 64 * 64;
    int64_t lo = 0, hi = (int64_t)kScratchBytes;
    while (lo < hi) {
        const int64_t c = (lo + hi + 1) / 2;
        const int64_t need = ((c * ld + 255) / 256) * 256 + c * ld * 4;
        if (need <= (int64_t)kScratchBytes) lo = c;
        else hi = c - 1;
    }
    return lo;
}
}  // namespace

extern "C" int da_energy_noalloc(da_ctx *ctx, const uint8_t *x_dev, int32_t count,
                                 int64_t *E_dev, void *stream) {
    if (!ctx || !x_dev || !E_dev || count < 1)
        return fail(ctx, DA_EINVAL, "bad energy arguments");
    const int64_t cap = max_states(ctx->N);
    if (count > cap)
        return fail(ctx, DA_EINVAL,
                    "count exceeds what the 32 MiB scratch holds at this N (" +
                        std::to_string(cap) + " states)");
    int dev = 0;
    int rc = check_hip(ctx, hipGetDevice(&dev), "device query");
    if (rc) return rc;
    if (dev != ctx->device)
        return fail(ctx, DA_EINVAL, "the context lives on another device than the current one");
    uint8_t *base = nullptr;
    std::string err;
    rc = scratch_on_device(dev, &base, err);
    if (rc) return fail(ctx, rc, err);
    // both intermediates are written in full before they are read: nothing in
    // the scratch has to start at zero
    const size_t ld = (size_t)ctx->ld;
    uint8_t *X = base;
    int32_t *H = reinterpret_cast<int32_t *>(base + ((size_t)count * ld + 255) / 256 * 256);
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : nullptr;
    JobDesc J{};
    J.W = ctx->d_W;
    J.b = ctx->d_b;
    J.N = ctx->N;
    J.ld = ctx->ld;
    J.dtype = ctx->dtype;
    J.wscale = ctx->wscale;
    const int64_t n = (int64_t)count * ctx->ld;
    int64_t grid = (n + 255) / 256;
    if (grid > 65535) grid = 65535;
    hipLaunchKernelGGL(k_pad_states, dim3((unsigned)grid), dim3(256), 0, s, x_dev, X, count,
                       ctx->N, ctx->ld);
    rc = check_hip(ctx, hipGetLastError(), "state padding launch");
    if (!rc) rc = check_hip(ctx, (hipError_t)launch_fields(J, X, count, H, s), "field launch");
    if (!rc)
        rc = check_hip(ctx, (hipError_t)launch_energy_from_fields(J, X, H, count, E_dev, false, s),
                       "energy launch");
    return rc;
}
