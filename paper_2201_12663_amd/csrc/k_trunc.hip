// a4: truncation (sort, tails, ranks).
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int TB = 1024;   // threads of the truncation block
constexpr int MAXM = 2048;

// deterministic block sum of per-thread values (fixed tree order)
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
        red[32] = s;
    }
    __syncthreads();
    s = red[32];
    __syncthreads();
    return s;
}

// one block per mode
__global__ __launch_bounds__(TB) void k_truncate(TruncArgs a) {
    __shared__ double key[MAXM];
    __shared__ int idx[MAXM];
    __shared__ double scan[MAXM + 1];
    __shared__ double red[40];
    __shared__ int rmin;
    const int mode = blockIdx.x, t = threadIdx.x;

    // |xi'|^2 and |A|^2 (same fixed order in every block)
    double v = 0.0;
    for (int64_t i = t; i < a.R_pad; i += TB) v += a.xip[i] * a.xip[i];
    const double xi2 = block_sum(v, red);
    v = 0.0;
    for (int64_t i = t; i < a.anorm_ntiles; i += TB) v += a.anorm_part[i];
    const double a2 = block_sum(v, red);
    const double xi_norm = sqrt(xi2), a_norm = sqrt(fmax(a2, 0.0));
    const double tau = (xi_norm > 0.0) ? a.eps * a_norm / (3.0 * xi_norm) : 0.0;

    // eigenvalues, padded to a power of two with -inf
    int N2 = 1;
    while (N2 < a.m) N2 <<= 1;
    const double* lam = a.lam[mode];
    for (int i = t; i < N2; i += TB) {
        key[i] = (i < a.m) ? lam[i] : -INFINITY;
        idx[i] = i;
    }
    __syncthreads();
    // bitonic sort: descending key, ascending index on ties
    for (int size = 2; size <= N2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < N2; i += TB) {
                int j = i ^ stride;
                if (j > i) {
                    bool desc = ((i & size) == 0);
                    double ki = key[i], kj = key[j];
                    int ii = idx[i], ij = idx[j];
                    // "i before j" in the final descending order?
                    bool i_first = (ki > kj) || (ki == kj && ii < ij);
                    if (desc ? !i_first : i_first) {
                        key[i] = kj; key[j] = ki;
                        idx[i] = ij; idx[j] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    // suffix sums of max(lambda, 0): scan[r] = sum_{k >= r} lambda_k, scan[m] = 0
    for (int i = t; i <= a.m; i += TB) scan[i] = (i < a.m) ? fmax(key[i], 0.0) : 0.0;
    __syncthreads();
    for (int off = 1; off < a.m; off <<= 1) {
        double add[2];
        int cnt = 0;
        for (int i = t; i < a.m; i += TB) add[cnt++] = (i + off < a.m) ? scan[i + off] : 0.0;
        __syncthreads();
        cnt = 0;
        for (int i = t; i < a.m; i += TB) scan[i] += add[cnt++];
        __syncthreads();
    }
    if (t == 0) rmin = a.m;
    __syncthreads();
    // r = min{ r >= 1 : t_r <= tau }, t_r = sqrt(scan[r])
    for (int r = 1 + t; r <= a.m; r += TB)
        if (sqrt(scan[r]) <= tau) atomicMin(&rmin, r);
    __syncthreads();
    const int r = (xi_norm > 0.0) ? rmin : 0;
    for (int i = t; i < a.m; i += TB) {
        a.sigma[mode][i] = sqrt(fmax(key[i], 0.0));
        a.order[mode][i] = idx[i];
    }
    for (int i = t; i <= a.m; i += TB) a.tails[mode][i] = sqrt(scan[i]);
    if (t == 0) {
        a.ranks[mode] = r;
        if (mode == 0) { a.scal[0] = xi_norm; a.scal[1] = a_norm; a.scal[2] = tau; }
    }
}

}  // namespace

hipError_t launch_truncate(const TruncArgs& a, hipStream_t st) {
    if (a.m < 1 || a.m > MAXM) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_truncate, dim3(3), dim3(TB), 0, st, a);
    return hipGetLastError();
}
