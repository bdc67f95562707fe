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

// one block per mode: sorted spectrum, tails, rank; mode 0 also writes the norms
// floor2: a squared tail that every t_r carries in addition to the discarded
// eigenvalues (the residual of a range finder; 0 on the Gram path).  When no
// r <= m certifies t_r <= tau the rank is set to m + 1.  signed_tails: the tails sum
// the eigenvalues with their signs (then clamp at zero) instead of their positive
// parts: for a Gram whose small eigenvalues are rounding noise of either sign, the
// noise then largely cancels in the tails instead of adding up.
__device__ __forceinline__ void truncate_mode(int mode, const double* __restrict__ lam, int m, const double* __restrict__ xip,
                              int64_t R_pad, const double* __restrict__ anorm_part, int64_t anorm_ntiles, double eps,
                              double* __restrict__ sigma, int* __restrict__ order, double* __restrict__ tails,
                              int* __restrict__ ranks, double* __restrict__ scal, double floor2 = 0.0,
                              bool presorted = false, double tau_fixed = 0.0, bool signed_tails = false) {
    __shared__ double key[MAXM];
    __shared__ int idx[MAXM];
    __shared__ double scan[MAXM + 1];
    __shared__ double red[40];
    __shared__ int rmin;
    const int t = threadIdx.x;

    // |xi'|^2 and |A|^2 (same fixed order in every block)
    double v = 0.0;
    for (int64_t i = t; i < R_pad; i += TB) v += xip[i] * xip[i];
    const double xi2 = block_sum(v, red);
    v = 0.0;
    for (int64_t i = t; i < anorm_ntiles; i += TB) v += anorm_part[i];
    const double a2 = block_sum(v, red);
    const double xi_norm = sqrt(xi2), a_norm = sqrt(fmax(a2, 0.0));
    const double tau = tau_fixed > 0.0 ? tau_fixed : (xi_norm > 0.0) ? eps * a_norm / (3.0 * xi_norm) : 0.0;

    // eigenvalues, padded to a power of two with -inf
    int N2 = 1;
    while (N2 < m) N2 <<= 1;
    for (int i = t; i < N2; i += TB) {
        key[i] = (i < m) ? lam[i] : -INFINITY;
        idx[i] = i;
    }
    __syncthreads();
    // bitonic sort: descending key, ascending index on ties (skipped when the values
    // come in the order of the vectors they belong to: the tails then follow that order)
    for (int size = 2; size <= (presorted ? 1 : N2); size <<= 1) {
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
    for (int i = t; i <= m; i += TB) scan[i] = (i < m) ? (signed_tails ? key[i] : fmax(key[i], 0.0)) : 0.0;
    __syncthreads();
    for (int off = 1; off < m; off <<= 1) {
        double add[2];
        int cnt = 0;
        for (int i = t; i < m; i += TB) add[cnt++] = (i + off < m) ? scan[i + off] : 0.0;
        __syncthreads();
        cnt = 0;
        for (int i = t; i < m; i += TB) scan[i] += add[cnt++];
        __syncthreads();
    }
    if (floor2 != 0.0 || signed_tails) {
        for (int i = t; i <= m; i += TB) scan[i] = fmax(scan[i] + floor2, 0.0);
        __syncthreads();
    }
    if (t == 0) rmin = m + 1;
    __syncthreads();
    // r = min{ r >= 1 : t_r <= tau }, t_r = sqrt(scan[r])
    for (int r = 1 + t; r <= m; r += TB)
        if (sqrt(scan[r]) <= tau) atomicMin(&rmin, r);
    __syncthreads();
    const int r = (xi_norm > 0.0) ? rmin : 0;
    for (int i = t; i < m; i += TB) {
        sigma[i] = sqrt(fmax(key[i], 0.0));
        order[i] = idx[i];
    }
    for (int i = t; i <= m; i += TB) tails[i] = sqrt(scan[i]);
    if (t == 0) {
        ranks[mode] = r;
        scal[3 + mode] = sqrt(scan[r < m ? r : m]);
        scal[6 + mode] = fmax(key[0], 0.0);                        // lambda_1
        scal[9 + mode] = r >= 1 && r <= m ? fmax(key[r - 1], 0.0) : 0.0;   // lambda_r
        if (mode == 0) { scal[0] = xi_norm; scal[1] = a_norm; scal[2] = tau; }
    }
}

__global__ __launch_bounds__(TB) void k_truncate(TruncArgs a) {
    const int mode = blockIdx.x;
    const int m = a.m_mode[mode] > 0 ? a.m_mode[mode] : a.m;
    truncate_mode(mode, a.lam[mode], m, a.xip, a.R_pad, a.anorm_part, a.anorm_ntiles, a.eps, a.sigma[mode],
                  a.order[mode], a.tails[mode], a.ranks, a.scal, a.floor2 ? a.floor2[mode] : 0.0, a.presorted != 0,
                  a.tau_fixed, a.signed_tails != 0);
}

// part[b] = sum of x[i]^2 over i = b, b + nparts, ... (one block per part, fixed order)
__global__ __launch_bounds__(256) void k_sumsq_partials(const double* __restrict__ x, int64_t count,
                                                        double* __restrict__ part, int nparts) {
    __shared__ double red[40];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x + (int64_t)nparts * threadIdx.x; i < count; i += (int64_t)nparts * 256)
        v += x[i] * x[i];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// batched: grid (3, problems); problems with non-finite input are skipped
__global__ __launch_bounds__(TB) void k_truncate_b(const BProb* __restrict__ P) {
    const int mode = blockIdx.x;
    const BProb& q = P[blockIdx.y];
    if (q.flags[0] != 0) {
        if (threadIdx.x == 0) q.ranks[mode] = 0;
        return;
    }
    truncate_mode(mode, q.lam[mode], q.m, q.xip, q.R_pad, q.anorm_part, q.anorm_ntiles, q.eps, q.sigma[mode],
                  q.order[mode], q.tails[mode], q.ranks, q.scal);
}

// status word per problem (one thread each)
__global__ void k_status_b(const BProb* __restrict__ P, int np) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const BProb& q = P[p];
    int st = 0;
    if (q.flags[0] != 0) st = -2;                  // non-finite input
    else if (*q.abort_w != 0) st = -4;             // eigensolver wait ran out
    else {
        const int64_t r1 = q.ranks[0], r2 = q.ranks[1], r3 = q.ranks[2];
        const bool zcap = (q.Zo[0] || q.Zo[1] || q.Zo[2] || q.Vo[0] || q.Vo[1] || q.Vo[2]) &&
                          (r1 > q.cap_rank || r2 > q.cap_rank || r3 > q.cap_rank);
        const bool rcap = r1 > q.rcap || r2 > q.rcap || r3 > q.rcap;
        const bool bcap = q.beta && r1 * r2 * r3 > q.cap_beta;
        if (zcap || rcap || bcap) st = -8;          // capacity
    }
    q.ranks[3] = st;
}

}  // namespace

hipError_t launch_truncate(const TruncArgs& a, hipStream_t st) {
    if (a.m < 1 || a.m > MAXM) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_truncate, dim3(3), dim3(TB), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_truncate_b(const BProb* P, int np, hipStream_t st) {
    if (np < 1) return hipSuccess;
    hipLaunchKernelGGL(k_truncate_b, dim3(3, (unsigned)np), dim3(TB), 0, st, P);
    hipLaunchKernelGGL(k_status_b, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, P, np);
    return hipGetLastError();
}

namespace {
// Spectrum and tails of a deflated reduction: the first k singular values from
// the first pass (sig1), then those of the deflated side matrix (sig2, tails2
// over its own index).  tails[i] for i >= k is tails2[i - k]; below k the first
// pass values are added: tails[i]^2 = sum_{i <= j < k} sig1[j]^2 + tails2[0]^2.
__global__ void k_combine_spectrum(int k, int m, const double* __restrict__ sig1, const double* __restrict__ sig2,
                                   const double* __restrict__ tails2, double* __restrict__ sigma,
                                   double* __restrict__ tails) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) sigma[i] = i < k ? sig1[i] : sig2[i - k];
    for (int i = k + threadIdx.x; i <= m; i += blockDim.x) tails[i] = tails2[i - k];
    if (threadIdx.x == 0) {
        double s = tails2[0] * tails2[0];
        for (int i = k - 1; i >= 0; --i) {
            s += sig1[i] * sig1[i];
            tails[i] = sqrt(s);
        }
    }
}
}  // namespace

hipError_t launch_combine_spectrum(int k, int m, const double* sig1, const double* sig2, const double* tails2,
                                   double* sigma, double* tails, hipStream_t st) {
    hipLaunchKernelGGL(k_combine_spectrum, dim3(1), dim3(256), 0, st, k, m, sig1, sig2, tails2, sigma, tails);
    return hipGetLastError();
}

hipError_t launch_sumsq_partials(const double* x, int64_t count, double* part, int nparts, hipStream_t st) {
    if (nparts < 1 || nparts > 1024 || count < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sumsq_partials, dim3((unsigned)nparts), dim3(256), 0, st, x, count, part, nparts);
    return hipGetLastError();
}
