// Tucker-to-canonical transform of a 3rd-order core (Section 2.3, Remark 2.6):
// every third-mode slice B_m = beta[:, :, m] (r1 x r2) is decomposed by its SVD
// and truncated at a threshold; the kept rank-one terms of all slices form a
// canonical tensor (eq. beta_R).
//
// One workgroup per slice runs a one-sided (Hestenes) Jacobi SVD in LDS, so the
// singular values carry no squaring of the condition number: the L x c matrix X
// (c = min(r1, r2) columns of length L = max(r1, r2); X = B_m when r2 <= r1, else
// B_m^T) is rotated column pair by column pair until its columns are mutually
// orthogonal, X J = W; then sigma_k = |w_k| and w_k / sigma_k are the singular
// vectors on X's row side.  The pairs of a round of the round-robin (tournament)
// ordering are disjoint, so the four waves rotate different pairs at once; rounds
// are separated by barriers.  The other factor of each kept term is formed from
// the slice itself (k_t2c_terms): v_k = B_m^T u_k / sigma_k, or u_k = B_m v_k /
// sigma_k, which keeps its absolute error at rounding level.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int T2C_THREADS = 256;
constexpr double U64 = 1.1102230246251565e-16;   // 2^-53

// partner of player q in round rd of the round-robin over cc (even) players:
// player cc-1 stays, the others rotate
__device__ __forceinline__ void tournament_pair(int rd, int q, int cc, int& i, int& j) {
    const int nm = cc - 1;
    if (q == 0) {
        i = nm;
        j = rd;
    } else {
        i = (rd + q) % nm;
        j = (rd + nm - q) % nm;
    }
    if (i > j) { const int t = i; i = j; j = t; }
}

__global__ __launch_bounds__(T2C_THREADS) void k_t2c_jacobi(const double* __restrict__ beta, int r1, int r2, int r3,
                                                          double thr, int max_sweeps, double* __restrict__ Wout,
                                                          double* __restrict__ sig_out, int* __restrict__ p_out,
                                                          double* __restrict__ tail_out, int* __restrict__ flags) {
    extern __shared__ double X[];                   // L x c, column j at X + j * L
    __shared__ double s_red[8];
    __shared__ int s_rot[4];
    __shared__ double s_sig[T2C_MAXC];
    __shared__ double s_sorted[T2C_MAXC];
    __shared__ int s_rank[T2C_MAXC];
    const int m = blockIdx.x;
    const bool trans = r1 < r2;                     // X = B^T
    const int L = trans ? r2 : r1, c = trans ? r1 : r2;
    const double* B = beta + (int64_t)m * r1 * r2;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // load the slice and its squared Frobenius norm (fixed order: thread sums, then waves)
    double fro = 0.0;
    for (int e = tid; e < L * c; e += T2C_THREADS) {
        const int i = e % L, j = e / L;
        const double v = trans ? B[j + (int64_t)r1 * i] : B[i + (int64_t)r1 * j];
        X[e] = v;
        fro += v * v;
    }
    fro = wave_sum(fro);
    if (lane == 0) s_red[w] = fro;
    __syncthreads();
    fro = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    // pairs count as orthogonal when |x.y| <= L u |x||y|, or below the absolute
    // floor (2 L u |B|_F)^2 where both columns are at rounding level of the slice
    const double tol = (double)L * U64;
    const double floor2 = (2.0 * L * U64) * (2.0 * L * U64) * fro;
    const int cc = (c + 1) & ~1;
    int sweep = 0;
    bool converged = (c < 2);
    for (; sweep < max_sweeps && !converged; ++sweep) {
        int rotated = 0;
        for (int rd = 0; rd < cc - 1; ++rd) {
            for (int q = w; q < cc / 2; q += 4) {
                int i, j;
                tournament_pair(rd, q, cc, i, j);
                if (j >= c) continue;                // the idle player when c is odd
                double* x = X + (int64_t)i * L;
                double* y = X + (int64_t)j * L;
                double a = 0.0, b = 0.0, g = 0.0;
                for (int k = lane; k < L; k += 64) {
                    const double xv = x[k], yv = y[k];
                    a += xv * xv;
                    b += yv * yv;
                    g += xv * yv;
                }
                a = wave_sum(a);
                b = wave_sum(b);
                g = wave_sum(g);
                if (fabs(g) <= tol * sqrt(a) * sqrt(b) || fabs(g) <= floor2) continue;
                rotated = 1;
                const double zeta = (b - a) / (2.0 * g);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int k = lane; k < L; k += 64) {
                    const double xv = x[k], yv = y[k];
                    x[k] = cs * xv - sn * yv;
                    y[k] = sn * xv + cs * yv;
                }
            }
            __syncthreads();
        }
        if (lane == 0) s_rot[w] = rotated;
        __syncthreads();
        converged = !(s_rot[0] | s_rot[1] | s_rot[2] | s_rot[3]);
        __syncthreads();
    }
    if (!converged && tid == 0) atomicOr(flags, 1);
    // singular values: column norms; descending order by counting (ties: lower index first)
    for (int j = w; j < c; j += 4) {
        double a = 0.0;
        for (int k = lane; k < L; k += 64) a += X[(int64_t)j * L + k] * X[(int64_t)j * L + k];
        a = wave_sum(a);
        if (lane == 0) s_sig[j] = sqrt(a);
    }
    __syncthreads();
    for (int j = tid; j < c; j += T2C_THREADS) {
        const double sj = s_sig[j];
        int rk = 0;
        for (int i = 0; i < c; ++i) rk += (s_sig[i] > sj) || (s_sig[i] == sj && i < j);
        s_rank[j] = rk;
    }
    __syncthreads();
    double* Wm = Wout + (int64_t)m * L * c;
    double* sg = sig_out + (int64_t)m * c;
    for (int e = tid; e < L * c; e += T2C_THREADS) {
        const int k = e % L, j = e / L;
        const double s = s_sig[j];
        Wm[k + (int64_t)L * s_rank[j]] = s > 0.0 ? X[e] / s : 0.0;
    }
    for (int j = tid; j < c; j += T2C_THREADS) {
        sg[s_rank[j]] = s_sig[j];
        s_sorted[s_rank[j]] = s_sig[j];
    }
    __syncthreads();
    // kept terms: sigma > thr; the tail of the dropped ones, summed smallest first
    if (tid == 0) {
        int p = 0;
        while (p < c && s_sorted[p] > thr) ++p;
        double t2 = 0.0;
        for (int k = c - 1; k >= p; --k) t2 += s_sorted[k] * s_sorted[k];
        p_out[m] = p;
        tail_out[m] = sqrt(t2);
    }
}

// One workgroup per kept term t (slice m = slice_of[t], position k < p_m): the
// weight sigma_k, the Jacobi-side unit vector, and the other factor formed from
// the slice.  F1 (r1 x R, ld ld1) holds u_k, F2 (r2 x R, ld ld2) holds v_k.
__global__ __launch_bounds__(T2C_THREADS) void k_t2c_terms(const double* __restrict__ beta, int r1, int r2,
                                                         const double* __restrict__ Wj, const double* __restrict__ sig,
                                                         const int64_t* __restrict__ off, int r3,
                                                         double* __restrict__ weights, double* __restrict__ F1,
                                                         int64_t ld1, double* __restrict__ F2, int64_t ld2,
                                                         int* __restrict__ slice_of, const int64_t* __restrict__ R_lim) {
    const int64_t t = blockIdx.x;
    if (R_lim && t >= *R_lim) return;               // grid sized for a capacity, R known on the device
    int lo = 0, hi = r3;                             // slice m: off[m] <= t < off[m + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid;
    }
    const int m = lo;
    const int k = (int)(t - off[m]);
    const bool trans = r1 < r2;
    const int L = trans ? r2 : r1, c = trans ? r1 : r2;
    const double s = sig[(int64_t)m * c + k];
    const double* q = Wj + (int64_t)m * L * c + (int64_t)L * k;    // unit vector on X's row side
    const double* B = beta + (int64_t)m * r1 * r2;
    double* fq = trans ? F2 + t * ld2 : F1 + t * ld1;                // same side as q
    double* fo = trans ? F1 + t * ld1 : F2 + t * ld2;                // the other side
    for (int i = threadIdx.x; i < L; i += T2C_THREADS) fq[i] = q[i];
    // other[j] = sum_i X[i, j'] ... : with X = B (no trans) v_j = sum_i B[i, j] u_i / s;
    // with X = B^T, u_i = sum_j B[i, j] v_j / s
    const int No = trans ? r1 : r2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = w; o < No; o += 4) {
        double a = 0.0;
        if (!trans)
            for (int i = lane; i < r1; i += 64) a += B[i + (int64_t)r1 * o] * q[i];
        else
            for (int j = lane; j < r2; j += 64) a += B[o + (int64_t)r1 * j] * q[j];
        a = wave_sum(a);
        if (lane == 0) fo[o] = a / s;
    }
    if (threadIdx.x == 0) {
        weights[t] = s;
        slice_of[t] = m;
    }
}

// Counts to offsets on the device (one thread, slices in order): off[m + 1] =
// off[m] + p[m], R = off[r3], bound = sum of the tails, status NOCONV when a
// slice did not converge, CAPACITY when R > cap; *R_lim = R when the terms may be
// written, else 0.
__global__ void k_t2c_offsets(const int* __restrict__ p, const double* __restrict__ tails, int r3, int64_t cap,
                              const int* __restrict__ flags, int64_t* __restrict__ off, int64_t* __restrict__ R_lim,
                              int64_t* __restrict__ R_out, double* __restrict__ bound_out, int* __restrict__ status) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t acc = 0;
    double b = 0.0;
    off[0] = 0;
    for (int m = 0; m < r3; ++m) {
        acc += p[m];
        b += tails[m];
        off[m + 1] = acc;
    }
    int st = 0;
    if (flags[0] & 1) st = RHOSVD_ERR_NOCONV;
    else if (acc > cap) st = RHOSVD_ERR_CAPACITY;
    *R_lim = st == 0 ? acc : 0;
    *R_out = acc;
    if (bound_out) *bound_out = b;
    *status = st;
}

__global__ void k_t2c_clear_flags(int* __restrict__ flags) {
    if (threadIdx.x < 4) flags[threadIdx.x] = 0;
}

// C[:, t] = Z3[:, slice_of[t]] for every term (n rows, ld ldc / ldz)
__global__ void k_t2c_gather_cols(int n, int64_t R, const double* __restrict__ Z, int64_t ldz,
                                  const int* __restrict__ slice_of, double* __restrict__ C, int64_t ldc) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * R;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, t = e / n;
        C[i + t * ldc] = Z[i + (int64_t)slice_of[t] * ldz];
    }
}

}  // namespace

size_t t2c_lds_bytes(int r1, int r2) { return (size_t)r1 * r2 * sizeof(double); }

hipError_t launch_t2c_jacobi(const double* beta, int r1, int r2, int r3, double thr, int max_sweeps, double* Wout,
                             double* sig_out, int* p_out, double* tail_out, int* flags, hipStream_t st) {
    if (r1 < 1 || r2 < 1 || r3 < 1 || std::min(r1, r2) > T2C_MAXC) return hipErrorInvalidValue;
    const size_t lds = t2c_lds_bytes(r1, r2);
    if (lds > T2C_MAX_LDS) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_t2c_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)T2C_MAX_LDS);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_t2c_jacobi, dim3((unsigned)r3), dim3(T2C_THREADS), lds, st, beta, r1, r2, r3, thr,
                       max_sweeps, Wout, sig_out, p_out, tail_out, flags);
    return hipGetLastError();
}

hipError_t launch_t2c_terms(const double* beta, int r1, int r2, int r3, const double* Wj, const double* sig,
                            const int64_t* off, int64_t R, double* weights, double* F1, int64_t ld1, double* F2,
                            int64_t ld2, int* slice_of, hipStream_t st, const int64_t* R_lim) {
    if (R < 1) return hipSuccess;
    hipLaunchKernelGGL(k_t2c_terms, dim3((unsigned)R), dim3(T2C_THREADS), 0, st, beta, r1, r2, Wj, sig, off, r3,
                       weights, F1, ld1, F2, ld2, slice_of, R_lim);
    return hipGetLastError();
}

hipError_t launch_t2c_offsets(const int* p, const double* tails, int r3, int64_t cap, const int* flags, int64_t* off,
                              int64_t* R_lim, int64_t* R_out, double* bound_out, int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_t2c_offsets, dim3(1), dim3(64), 0, st, p, tails, r3, cap, flags, off, R_lim, R_out, bound_out,
                       status);
    return hipGetLastError();
}

hipError_t launch_t2c_clear_flags(int* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_t2c_clear_flags, dim3(1), dim3(64), 0, st, flags);
    return hipGetLastError();
}

hipError_t launch_t2c_gather_cols(int n, int64_t R, const double* Z, int64_t ldz, const int* slice_of, double* C,
                                  int64_t ldc, hipStream_t st) {
    if (R < 1 || n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_t2c_gather_cols, dim3(1024), dim3(256), 0, st, n, R, Z, ldz, slice_of, C, ldc);
    return hipGetLastError();
}
