// rhosvd_t2c_noalloc: the Tucker-to-canonical transform (Remark 2.6) in one
// call that allocates nothing, for callers that cannot allocate device memory.
// Its workspace is a fixed static device array (one per GPU, held until the
// process ends); every result, including the status, is written to device
// memory, so the call never waits for the GPU.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr size_t T2C_SCRATCH_BYTES = (size_t)8 << 20;   // 8 MiB per device

// In host code this name is only a stand-in for the device array: its device
// address comes from hipGetSymbolAddress (per device, below).
__device__ __align__(256) char scratch[T2C_SCRATCH_BYTES];

constexpr int MAXDEV = 64;
std::mutex g_mu;
char* g_scratch[MAXDEV] = {};

// The device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array at its own address).
hipError_t scratch_address(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = (char*)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// the scratch layout for an r1 x r2 x r3 core; base == nullptr only measures
struct Layout {
    double *W, *sig, *tails;
    int *p, *flags;
    int64_t *off, *R_lim;
    size_t bytes;
};

Layout layout_for(char* base, int r1, int r2, int r3) {
    const size_t L = (size_t)std::max(r1, r2), c = (size_t)std::min(r1, r2);
    Layout o{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += a256(bytes);
        return p;
    };
    o.W = (double*)take((size_t)r3 * L * c * 8);
    o.sig = (double*)take((size_t)r3 * c * 8);
    o.tails = (double*)take((size_t)r3 * 8);
    o.p = (int*)take((size_t)r3 * 4);
    o.off = (int64_t*)take(((size_t)r3 + 1) * 8);
    o.flags = (int*)take(16);
    o.R_lim = (int64_t*)take(8);
    o.bytes = off;
    return o;
}

}  // namespace

extern "C" rhosvd_status rhosvd_t2c_noalloc(void* hip_stream, int32_t r1, int32_t r2, int32_t r3, const double* beta,
                                            double eps, int64_t cap, double* weights, double* F1, double* F2,
                                            int32_t* slice, int64_t* R, double* bound, int32_t* status) {
    if (!beta || !R || !status || cap < 0) return RHOSVD_ERR_ARG;
    if (cap > 0 && (!weights || !F1 || !F2 || !slice)) return RHOSVD_ERR_ARG;
    if (r1 < 1 || r2 < 1 || r3 < 1) return RHOSVD_ERR_ARG;
    if (!(eps > 0.0) || !isfinite(eps)) return RHOSVD_ERR_ARG;
    if (std::min(r1, r2) > T2C_MAXC || t2c_lds_bytes(r1, r2) > T2C_MAX_LDS) return RHOSVD_ERR_UNSUPPORTED;
    if (layout_for(nullptr, r1, r2, r3).bytes > T2C_SCRATCH_BYTES) return RHOSVD_ERR_UNSUPPORTED;
    char* base = nullptr;
    if (scratch_address(&base) != hipSuccess) return RHOSVD_ERR_DEVICE;
    const Layout w = layout_for(base, r1, r2, r3);
    hipStream_t st = (hipStream_t)hip_stream;
    const int c = std::min(r1, r2);
    const double thr = eps / ((double)r3 * sqrt((double)c));
    // every call on this device shares the array: the flags start from zero, all
    // other words are written before they are read
    if (launch_t2c_clear_flags(w.flags, st) != hipSuccess) return RHOSVD_ERR_DEVICE;
    if (launch_t2c_jacobi(beta, r1, r2, r3, thr, 60, w.W, w.sig, w.p, w.tails, w.flags, st) != hipSuccess)
        return RHOSVD_ERR_DEVICE;
    if (launch_t2c_offsets(w.p, w.tails, r3, cap, w.flags, w.off, w.R_lim, R, bound, status, st) != hipSuccess)
        return RHOSVD_ERR_DEVICE;
    // a grid for the capacity; terms at or beyond the device-side R exit at once
    const int64_t grid = std::min<int64_t>(cap, (int64_t)r3 * c);
    if (grid > 0 && launch_t2c_terms(beta, r1, r2, r3, w.W, w.sig, w.off, grid, weights, F1, r1, F2, r2, slice, st,
                                     w.R_lim) != hipSuccess)
        return RHOSVD_ERR_DEVICE;
    return RHOSVD_OK;
}
