// Normalization (a1), Gram (a2), exact |A| identity and projection (a6) kernels.
#include "common.hpp"
#include "kernels.hpp"

// ===========================================================================
// a1: one wave per canonical term nu handles its three columns.
// Scaled Euclidean norm (max-abs, then sum of squares of the scaled entries),
// xi'_nu = xi_nu * s1 * s2 * s3; a term with xi = 0 or a zero column is dropped
// (xi' = 0, normalized columns zero).  Padded rows/terms are written as zero.
// ===========================================================================
__device__ __forceinline__ void colnorm_term(int64_t n, int64_t R, int64_t n_pad, int64_t R_pad, const double* __restrict__ U0,
                             const double* __restrict__ U1, const double* __restrict__ U2,
                             const double* __restrict__ xi, double* __restrict__ T0, double* __restrict__ T1,
                             double* __restrict__ T2, double* __restrict__ xip, int* __restrict__ flags, int64_t nu) {
    const int lane = threadIdx.x & 63;
    if (nu >= R_pad) return;
    const double* U[3] = {U0, U1, U2};
    double* T[3] = {T0, T1, T2};
    if (nu >= R) {
        for (int l = 0; l < 3; ++l)
            for (int64_t i = lane; i < n_pad; i += 64) T[l][i + nu * n_pad] = 0.0;
        if (lane == 0) xip[nu] = 0.0;
        return;
    }
    double s[3];
    int bad = 0;
    for (int l = 0; l < 3; ++l) {
        const double* col = U[l] + nu * n;
        double mx = 0.0;
        for (int64_t i = lane; i < n; i += 64) {
            double v = col[i];
            if (!isfinite(v)) bad = 1;
            mx = fmax(mx, fabs(v));
        }
        mx = wave_max(mx);
        double acc = 0.0;
        if (mx > 0.0 && isfinite(mx)) {
            // 1/mx overflows for a subnormal mx (and loses bits for a huge one):
            // outside [2^-1000, 2^1000] divide instead (mx is uniform across the wave)
            if (mx >= 0x1p-1000 && mx <= 0x1p1000) {
                const double inv = 1.0 / mx;
                for (int64_t i = lane; i < n; i += 64) {
                    const double v = col[i] * inv;
                    acc += v * v;
                }
            } else {
                for (int64_t i = lane; i < n; i += 64) {
                    const double v = col[i] / mx;
                    acc += v * v;
                }
            }
        }
        acc = wave_sum(acc);
        s[l] = (mx > 0.0) ? mx * sqrt(acc) : 0.0;
    }
    bad = wave_or(bad);
    double x = xi[nu];
    if (!isfinite(x)) bad = 1;
    const bool keep = !bad && x != 0.0 && s[0] > 0.0 && s[1] > 0.0 && s[2] > 0.0;
    for (int l = 0; l < 3; ++l) {
        const double* col = U[l] + nu * n;
        double* out = T[l] + nu * n_pad;
        for (int64_t i = lane; i < n_pad; i += 64)
            out[i] = (keep && i < n) ? col[i] / s[l] : 0.0;
    }
    if (lane == 0) {
        xip[nu] = keep ? x * s[0] * s[1] * s[2] : 0.0;
        if (bad) atomicOr(&flags[0], 1);
        if (!keep) atomicAdd(&flags[1], 1);
    }
}

__global__ __launch_bounds__(256) void k_colnorm(int64_t n, int64_t R, int64_t n_pad, int64_t R_pad,
                                                 const double* __restrict__ U0,
                                                 const double* __restrict__ U1,
                                                 const double* __restrict__ U2,
                                                 const double* __restrict__ xi,
                                                 double* __restrict__ T0, double* __restrict__ T1,
                                                 double* __restrict__ T2, double* __restrict__ xip,
                                                 int* __restrict__ flags) {
    colnorm_term(n, R, n_pad, R_pad, U0, U1, U2, xi, T0, T1, T2, xip, flags,
                 (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
}

hipError_t launch_colnorm(int64_t n, int64_t R, int64_t n_pad, int64_t R_pad,
                          const double* const U[3], const double* xi,
                          double* const Ut[3], double* xip, int* flags, hipStream_t st) {
    dim3 grid((unsigned)ceil_div(R_pad, 4));
    hipLaunchKernelGGL(k_colnorm, grid, dim3(256), 0, st, n, R, n_pad, R_pad, U[0], U[1], U[2],
                       xi, Ut[0], Ut[1], Ut[2], xip, flags);
    return hipGetLastError();
}

// ===========================================================================
// FP64 MFMA tile engine: a 64x64 output tile per 256-thread block, 4 waves in
// a 2x2 arrangement (32x32 each = 2x2 MFMA 16x16 sub-tiles), K in chunks of 16
// staged through LDS.  Operands are padded, so no bounds checks are needed.
//   A "M-contiguous": A(i,k) = A[i + k*lda];  "K-contiguous": A(i,k) = A[k + i*lda]
//   B "N-contiguous": B(k,j) = B[j + k*ldb];  "K-contiguous": B(k,j) = B[k + j*ldb]
// ===========================================================================
constexpr int T64 = 64;
constexpr int KC = 16;
constexpr int LDS_STRIDE = T64 + 4;   // doubles per k-row in LDS

// thread t's four entries of a 64 x 16 chunk: (i, k) = (t % 64, t / 64 + 4q) for an
// M-contiguous operand, (t / 4, 4 (t % 4) + q) for a K-contiguous one
template <bool AK>
__device__ __forceinline__ void gload64(const double* __restrict__ A, int64_t lda, int64_t m0, int64_t k0,
                                        double (&r)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!AK) r[q] = A[(m0 + (t & 63)) + (k0 + (t >> 6) + 4 * q) * lda];
        else r[q] = A[(k0 + ((t & 3) << 2) + q) + (m0 + (t >> 2)) * lda];
    }
}

template <bool AK>
__device__ __forceinline__ void sstore64(const double (&r)[4], double* __restrict__ s) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!AK) s[((t >> 6) + 4 * q) * LDS_STRIDE + (t & 63)] = r[q];
        else s[(((t & 3) << 2) + q) * LDS_STRIDE + (t >> 2)] = r[q];
    }
}

// acc[a][b] += A[m0 + wave rows][k0 .. k1) * B[k0 .. k1)[n0 + wave cols].  sA and sB
// hold two chunk buffers each (2 * KC * LDS_STRIDE doubles): the next chunk's global
// loads are in flight during the current chunk's MFMAs, one barrier per chunk.
template <bool AK, bool BK>
__device__ __forceinline__ void tile64_f64(const double* __restrict__ A, int64_t lda,
                                           const double* __restrict__ B, int64_t ldb,
                                           int64_t m0, int64_t n0, int64_t k0, int64_t k1,
                                           double* sA, double* sB, d4_t acc[2][2]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    if (k0 >= k1) return;
    double ra[4], rb[4];
    gload64<AK>(A, lda, m0, k0, ra);
    gload64<BK>(B, ldb, n0, k0, rb);
    sstore64<AK>(ra, sA);
    sstore64<BK>(rb, sB);
    __syncthreads();
    int buf = 0;
    for (int64_t kb = k0; kb < k1; kb += KC) {
        const bool more = kb + KC < k1;
        if (more) {
            gload64<AK>(A, lda, m0, kb + KC, ra);
            gload64<BK>(B, ldb, n0, kb + KC, rb);
        }
        const double* cA = sA + buf * KC * LDS_STRIDE;
        const double* cB = sB + buf * KC * LDS_STRIDE;
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            const int k = kk * 4 + (lane >> 4);
            double a0 = cA[k * LDS_STRIDE + wr + (lane & 15)];
            double a1 = cA[k * LDS_STRIDE + wr + 16 + (lane & 15)];
            double b0 = cB[k * LDS_STRIDE + wc + (lane & 15)];
            double b1 = cB[k * LDS_STRIDE + wc + 16 + (lane & 15)];
            acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
            acc[0][1] = mfma_f64(a0, b1, acc[0][1]);
            acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
            acc[1][1] = mfma_f64(a1, b1, acc[1][1]);
        }
        if (more) {
            sstore64<AK>(ra, sA + (buf ^ 1) * KC * LDS_STRIDE);
            sstore64<BK>(rb, sB + (buf ^ 1) * KC * LDS_STRIDE);
        }
        __syncthreads();
        buf ^= 1;
    }
}

__device__ __forceinline__ void zero_acc(d4_t acc[2][2]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
}

// ===========================================================================
// a2: Gram G = U~ U~^T on the n side (n <= R).  Lower-triangle tiles only;
// split-K partials are summed in a fixed order by k_gram_reduce, which also
// mirrors the tile into the upper triangle.
// grid: (tile pairs, splits, mode)
// ===========================================================================
__device__ __forceinline__ void gram_tile(int64_t n_pad, int64_t R_pad, const double* __restrict__ T, double* __restrict__ G,
                          double* __restrict__ part, int splits, int64_t t, int split, int mode) {
    __shared__ double sA[2 * KC * LDS_STRIDE];
    __shared__ double sB[2 * KC * LDS_STRIDE];
    // lower-triangle tile (ti >= tj) from the linear index
    int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int64_t tj = t - ti * (ti + 1) / 2;
    const int64_t chunk = round_up(ceil_div(R_pad, splits), KC);
    const int64_t k0 = split * chunk, k1 = (k0 + chunk < R_pad) ? k0 + chunk : R_pad;
    d4_t acc[2][2];
    zero_acc(acc);
    if (k0 < k1)
        tile64_f64<false, false>(T, n_pad, T, n_pad, ti * T64, tj * T64, k0, k1, sA, sB, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    if (splits == 1) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int64_t r = ti * T64 + wr + a * 16 + c_row64(lane, i);
                    int64_t c = tj * T64 + wc + b * 16 + c_col(lane);
                    if (r < c) continue;   // diagonal tiles: the r >= c lane writes both
                    double v = acc[a][b][i];
                    G[r + c * n_pad] = v;
                    G[c + r * n_pad] = v;
                }
    } else {
        double* P = part + ((int64_t)split * 3 + mode) * n_pad * n_pad;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int64_t r = ti * T64 + wr + a * 16 + c_row64(lane, i);
                    int64_t c = tj * T64 + wc + b * 16 + c_col(lane);
                    P[r + c * n_pad] = acc[a][b][i];
                }
    }
}

__global__ __launch_bounds__(256) void k_gram(int64_t n_pad, int64_t R_pad, const double* __restrict__ T0,
                                              const double* __restrict__ T1, const double* __restrict__ T2,
                                              double* __restrict__ G0, double* __restrict__ G1,
                                              double* __restrict__ G2, double* __restrict__ part, int splits) {
    const int mode = blockIdx.z;
    const double* T = mode == 0 ? T0 : (mode == 1 ? T1 : T2);
    double* G = mode == 0 ? G0 : (mode == 1 ? G1 : G2);
    gram_tile(n_pad, R_pad, T, G, part, splits, blockIdx.x, blockIdx.y, mode);
}

__global__ void k_gram_reduce(int64_t n_pad, const double* __restrict__ part, int splits,
                              double* __restrict__ G0, double* __restrict__ G1, double* __restrict__ G2) {
    const int mode = blockIdx.y;
    double* G = mode == 0 ? G0 : (mode == 1 ? G1 : G2);
    const int64_t NN = n_pad * n_pad;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < NN; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e % n_pad, c = e / n_pad;
        if (r < c) continue;   // lower triangle (partials exist for every lower tile)
        double s = 0.0;
        for (int sp = 0; sp < splits; ++sp) s += part[((int64_t)sp * 3 + mode) * NN + e];
        G[r + c * n_pad] = s;
        G[c + r * n_pad] = s;
    }
}

hipError_t launch_gram_nt(int64_t n_pad, int64_t R_pad, double* const Ut[3], double* const G[3],
                          double* part, int splits, hipStream_t st) {
    const int64_t nt = n_pad / T64;
    dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)splits, 3);
    hipLaunchKernelGGL(k_gram, grid, dim3(256), 0, st, n_pad, R_pad, Ut[0], Ut[1], Ut[2], G[0], G[1],
                       G[2], part, splits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    hipLaunchKernelGGL(k_gram_reduce, dim3(1024, 3), dim3(256), 0, st, n_pad, part, splits, G[0], G[1], G[2]);
    return hipGetLastError();
}

hipError_t launch_gram_reduce(int64_t n_pad, const double* part, int splits, double* const G[3], hipStream_t st) {
    hipLaunchKernelGGL(k_gram_reduce, dim3(1024, 3), dim3(256), 0, st, n_pad, part, splits, G[0], G[1], G[2]);
    return hipGetLastError();
}

// ===========================================================================
// |A|^2 = sum_{nu,mu} xi'_nu xi'_mu prod_l <u~_nu^(l), u~_mu^(l)>  (the inner
// product of two canonical sums).  One block per lower-triangle tile (nu-tile
// >= mu-tile) of the R x R Gram matrices; the three mode Grams of the tile are
// formed with FP64 MFMA, multiplied entrywise, weighted, and reduced to one
// partial sum per tile (off-diagonal tiles count twice).
// ===========================================================================
template <bool STORE_G>
__device__ __forceinline__ void anorm_tile(int64_t n_pad, int64_t R_pad, const double* __restrict__ T0,
                           const double* __restrict__ T1, const double* __restrict__ T2,
                           const double* __restrict__ xip, double* __restrict__ part, double* __restrict__ G0,
                           double* __restrict__ G1, double* __restrict__ G2, int64_t t) {
    __shared__ double sA[2 * KC * LDS_STRIDE];
    __shared__ double sB[2 * KC * LDS_STRIDE];
    __shared__ double red[4];
    int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int64_t tj = t - ti * (ti + 1) / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    d4_t prod[2][2];
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        const double* Tl = l == 0 ? T0 : (l == 1 ? T1 : T2);
        d4_t acc[2][2];
        zero_acc(acc);
        tile64_f64<true, true>(Tl, n_pad, Tl, n_pad, ti * T64, tj * T64, 0, n_pad, sA, sB, acc);
        double* Gl = l == 0 ? G0 : (l == 1 ? G1 : G2);
        if (STORE_G && Gl) {   // R < n: this tile of U~^T U~ is the mode's Gram on the R side
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        int64_t r = ti * T64 + wr + a * 16 + c_row64(lane, i);
                        int64_t c = tj * T64 + wc + b * 16 + c_col(lane);
                        if (r < c) continue;
                        Gl[r + c * R_pad] = acc[a][b][i];
                        Gl[c + r * R_pad] = acc[a][b][i];
                    }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) prod[a][b] = (l == 0) ? acc[a][b] : prod[a][b] * acc[a][b];
    }
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int64_t nu = ti * T64 + wr + a * 16 + c_row64(lane, i);
                int64_t mu = tj * T64 + wc + b * 16 + c_col(lane);
                s += xip[nu] * xip[mu] * prod[a][b][i];
            }
    s = wave_sum(s);
    if (lane == 0) red[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = (red[0] + red[1]) + (red[2] + red[3]);
        part[t] = (ti == tj) ? tot : 2.0 * tot;
    }
}

template <bool STORE_G>
__global__ __launch_bounds__(256) void k_anorm(int64_t n_pad, int64_t R_pad, const double* __restrict__ T0,
                                               const double* __restrict__ T1, const double* __restrict__ T2,
                                               const double* __restrict__ xip, double* __restrict__ part,
                                               double* __restrict__ G0, double* __restrict__ G1,
                                               double* __restrict__ G2) {
    anorm_tile<STORE_G>(n_pad, R_pad, T0, T1, T2, xip, part, G0, G1, G2, blockIdx.x);
}

hipError_t launch_anorm_partials(int64_t n_pad, int64_t R_pad, double* const Ut[3],
                                 const double* xip, double* part, int64_t* ntiles, double* const Gr[3],
                                 hipStream_t st) {
    const int64_t nt = R_pad / T64;
    *ntiles = nt * (nt + 1) / 2;
    if (Gr)
        hipLaunchKernelGGL(k_anorm<true>, dim3((unsigned)*ntiles), dim3(256), 0, st, n_pad, R_pad, Ut[0], Ut[1],
                           Ut[2], xip, part, Gr[0], Gr[1], Gr[2]);
    else
        hipLaunchKernelGGL(k_anorm<false>, dim3((unsigned)*ntiles), dim3(256), 0, st, n_pad, R_pad, Ut[0], Ut[1],
                           Ut[2], xip, part, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

// ===========================================================================
// a6: V = Z^T U~  (r_pad x R_pad, col-major ld r_pad), K = n_pad.
// Z: n_pad x r_pad (ld n_pad) -> A(j,i) = Z[i + j*n_pad] (K-contiguous);
// U~: n_pad x R_pad -> B(i,nu) = U~[i + nu*n_pad] (K-contiguous).
// ===========================================================================
__device__ __forceinline__ void project_tile(int64_t n_pad, int64_t R_pad, int64_t r_pad, const double* __restrict__ Z,
                             const double* __restrict__ T, double* __restrict__ out64, float* __restrict__ out32,
                             int64_t tm, int64_t tn) {
    __shared__ double sA[2 * KC * LDS_STRIDE];
    __shared__ double sB[2 * KC * LDS_STRIDE];
    d4_t acc[2][2];
    zero_acc(acc);
    tile64_f64<true, true>(Z, n_pad, T, n_pad, tm * T64, tn * T64, 0, n_pad, sA, sB, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int64_t j = tm * T64 + wr + a * 16 + c_row64(lane, i);
                int64_t nu = tn * T64 + wc + b * 16 + c_col(lane);
                if (out64) out64[j + nu * r_pad] = acc[a][b][i];
                else out32[j + nu * r_pad] = (float)acc[a][b][i];
            }
}

__global__ __launch_bounds__(256) void k_project(int64_t n_pad, int64_t R_pad, int64_t r_pad,
                                                 const double* __restrict__ Z, const double* __restrict__ T,
                                                 double* __restrict__ out64, float* __restrict__ out32) {
    project_tile(n_pad, R_pad, r_pad, Z, T, out64, out32, blockIdx.y, blockIdx.x);
}

hipError_t launch_project(int64_t n_pad, int64_t R_pad, int64_t r_pad, const double* Z,
                          const double* Ut, double* out_f64, float* out_f32, hipStream_t st) {
    dim3 grid((unsigned)(R_pad / T64), (unsigned)(r_pad / T64));
    hipLaunchKernelGGL(k_project, grid, dim3(256), 0, st, n_pad, R_pad, r_pad, Z, Ut, out_f64, out_f32);
    return hipGetLastError();
}

// ===========================================================================
// Generic FP64 MFMA GEMM on padded operands: C (M x N, col-major, ldc) =
// alpha * A * B with A M- or K-contiguous and B N- or K-contiguous (see
// tile64_f64).  M, N multiples of 64, K multiple of 16.  grid (N/64, M/64).
// ===========================================================================
template <bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm64(int64_t K, const double* __restrict__ A, int64_t lda,
                                                const double* __restrict__ B, int64_t ldb, double* __restrict__ C,
                                                int64_t ldc, double alpha) {
    __shared__ double sA[2 * KC * LDS_STRIDE];
    __shared__ double sB[2 * KC * LDS_STRIDE];
    const int64_t tm = blockIdx.y, tn = blockIdx.x;
    d4_t acc[2][2];
    zero_acc(acc);
    tile64_f64<AK, BK>(A, lda, B, ldb, tm * T64, tn * T64, 0, K, sA, sB, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int64_t r = tm * T64 + wr + a * 16 + c_row64(lane, i);
                int64_t c = tn * T64 + wc + b * 16 + c_col(lane);
                C[r + c * ldc] = alpha * acc[a][b][i];
            }
}

hipError_t launch_gemm64(bool a_kcontig, bool b_kcontig, int64_t M, int64_t N, int64_t K, const double* A,
                         int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, double alpha,
                         hipStream_t st) {
    if (M % T64 || N % T64 || K % KC) return hipErrorInvalidValue;
    dim3 grid((unsigned)(N / T64), (unsigned)(M / T64));
    if (a_kcontig && b_kcontig)
        hipLaunchKernelGGL((k_gemm64<true, true>), grid, dim3(256), 0, st, K, A, lda, B, ldb, C, ldc, alpha);
    else if (a_kcontig)
        hipLaunchKernelGGL((k_gemm64<true, false>), grid, dim3(256), 0, st, K, A, lda, B, ldb, C, ldc, alpha);
    else if (b_kcontig)
        hipLaunchKernelGGL((k_gemm64<false, true>), grid, dim3(256), 0, st, K, A, lda, B, ldb, C, ldc, alpha);
    else
        hipLaunchKernelGGL((k_gemm64<false, false>), grid, dim3(256), 0, st, K, A, lda, B, ldb, C, ldc, alpha);
    return hipGetLastError();
}

// Wr[:, k] = W[:, order[k]] / sigma_k for k < r; zero columns r..r_pad-1 (ld = m_pad)
__global__ void k_gather_scaled(int m_pad, int r, int r_pad, const double* __restrict__ W,
                                const int* __restrict__ order, const double* __restrict__ sigma,
                                double* __restrict__ Wr, const int* __restrict__ r_dev) {
    if (r_dev) r = min(r, *r_dev);
    const int64_t tot = (int64_t)m_pad * r_pad;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m_pad), k = (int)(e / m_pad);
        double v = 0.0;
        if (k < r && sigma[k] > 0.0) v = W[i + (int64_t)(order ? order[k] : k) * m_pad] / sigma[k];
        Wr[e] = v;
    }
}

// M (mp x mp, leading dimension ld): keep the leading r x r block, identity elsewhere
__global__ void k_pad_identity(int r, int mp, int ld, double* __restrict__ M, const int* __restrict__ r_dev) {
    if (r_dev) r = min(r, *r_dev);
    const int64_t tot = (int64_t)mp * mp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % mp), j = (int)(e / mp);
        if (i >= r || j >= r) M[i + (int64_t)j * ld] = (i == j) ? 1.0 : 0.0;
    }
}

// out[:, j] = P[:, j] * mu_j^(-1/2) (mp x mp, leading dimension ld)
__global__ void k_scale_cols_invsqrt(int mp, int ld, const double* __restrict__ mu, const double* __restrict__ P,
                                     double* __restrict__ out) {
    const int64_t tot = (int64_t)mp * mp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % mp), j = (int)(e / mp);
        const int64_t o = i + (int64_t)j * ld;
        out[o] = (mu[j] > 0.0) ? P[o] / sqrt(mu[j]) : 0.0;
    }
}

// sign rule on the columns of Z (n_pad x r, in place): largest-magnitude entry positive
__global__ __launch_bounds__(256) void k_sign_cols(int n, int n_pad, int r, double* __restrict__ Z) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= r) return;
    double* z = Z + (int64_t)k * n_pad;
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < n; i += 64) {
        double a = fabs(z[i]);
        if (a > best) { best = a; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sgn = (z[bi] < 0.0) ? -1.0 : 1.0;
    for (int i = lane; i < n_pad; i += 64) z[i] = (i < n) ? sgn * z[i] : 0.0;
}

hipError_t launch_gather_scaled(int m_pad, int r, int r_pad, const double* W, const int* order,
                                const double* sigma, double* Wr, hipStream_t st, const int* r_dev) {
    hipLaunchKernelGGL(k_gather_scaled, dim3(512), dim3(256), 0, st, m_pad, r, r_pad, W, order, sigma, Wr, r_dev);
    return hipGetLastError();
}
hipError_t launch_pad_identity(int r, int mp, int ld, double* M, hipStream_t st, const int* r_dev) {
    hipLaunchKernelGGL(k_pad_identity, dim3(256), dim3(256), 0, st, r, mp, ld, M, r_dev);
    return hipGetLastError();
}
hipError_t launch_scale_cols_invsqrt(int mp, int ld, const double* mu, const double* P, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_cols_invsqrt, dim3(256), dim3(256), 0, st, mp, ld, mu, P, out);
    return hipGetLastError();
}
hipError_t launch_sign_cols(int n, int n_pad, int r, double* Z, hipStream_t st) {
    if (r < 1) return hipSuccess;
    hipLaunchKernelGGL(k_sign_cols, dim3((unsigned)ceil_div(r, 4)), dim3(256), 0, st, n, n_pad, r, Z);
    return hipGetLastError();
}

// ===========================================================================
// Batched variants: one launch covers every problem of a batch.  The grid is
// flattened; pre[p] .. pre[p+1]-1 are problem p's blocks (pre[0] = 0).
// ===========================================================================
__device__ __forceinline__ int find_problem(const int64_t* __restrict__ pre, int np, int64_t b) {
    int lo = 0, hi = np;   // largest p with pre[p] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_colnorm_b(const BProb* __restrict__ P, const int64_t* __restrict__ pre, int np) {
    const int p = find_problem(pre, np, blockIdx.x);
    const BProb& q = P[p];
    const int64_t nu = (blockIdx.x - pre[p]) * 4 + (threadIdx.x >> 6);
    colnorm_term(q.n, q.R, q.n_pad, q.R_pad, q.U[0], q.U[1], q.U[2], q.xi, q.Ut[0], q.Ut[1], q.Ut[2], q.xip, q.flags,
                 nu);
}

// RSIDE: the instance for problems with R < n (which also store the R-side
// Grams); each instance skips the other kind of problem
template <bool RSIDE>
__global__ __launch_bounds__(256) void k_anorm_b(const BProb* __restrict__ P, const int64_t* __restrict__ pre, int np) {
    const int p = find_problem(pre, np, blockIdx.x);
    const BProb& q = P[p];
    if ((q.rside != 0) != RSIDE) return;
    anorm_tile<RSIDE>(q.n_pad, q.R_pad, q.Ut[0], q.Ut[1], q.Ut[2], q.xip, q.anorm_part, q.G[0], q.G[1], q.G[2],
                      blockIdx.x - pre[p]);
}

__global__ __launch_bounds__(256) void k_gram_b(const BProb* __restrict__ P, const int64_t* __restrict__ pre, int np) {
    const int p = find_problem(pre, np, blockIdx.x);
    const BProb& q = P[p];
    const int64_t nt = q.n_pad / T64, per = nt * (nt + 1) / 2;
    const int64_t local = blockIdx.x - pre[p];
    const int mode = (int)(local / per);
    gram_tile(q.n_pad, q.R_pad, q.Ut[mode], q.G[mode], nullptr, 1, local % per, 0, mode);
}

// V_l = Z_l^T U~_l for the row tiles below round_up(min(r_l, rcap), 128)
__global__ __launch_bounds__(256) void k_project_b(const BProb* __restrict__ P, const int64_t* __restrict__ pre, int np,
                                                   int f32) {
    const int p = find_problem(pre, np, blockIdx.x);
    const BProb& q = P[p];
    const int64_t TMc = q.rcap_pad / T64, TN = q.R_pad / T64;
    const int64_t local = blockIdx.x - pre[p];
    const int mode = (int)(local / (TMc * TN));
    const int64_t rem = local % (TMc * TN);
    const int64_t tm = rem / TN, tn = rem % TN;
    const int r = min(q.ranks[mode], q.rcap);
    if (q.ranks[3] != 0 || r < 1 || tm * T64 >= round_up(r, 128)) return;
    project_tile(q.n_pad, q.R_pad, q.rcap_pad, q.Z[mode], q.Ut[mode], f32 ? nullptr : (double*)q.V[mode],
                 f32 ? (float*)q.V[mode] : nullptr, tm, tn);
}

// sign rule on columns k < min(r, rcap) of Z_l, zero columns up to rcap_pad
__global__ __launch_bounds__(256) void k_sign_b(const BProb* __restrict__ P, const int64_t* __restrict__ pre, int np) {
    const int p = find_problem(pre, np, blockIdx.x);
    const BProb& q = P[p];
    const int64_t per = q.rcap_pad / 4;
    const int64_t local = blockIdx.x - pre[p];
    const int mode = (int)(local / per);
    const int k = (int)((local % per) * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int r = min(q.ranks[mode], q.rcap);
    double* z = q.Z[mode] + (int64_t)k * q.n_pad;
    if (k >= r) {
        for (int i = lane; i < q.n_pad; i += 64) z[i] = 0.0;
        return;
    }
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < q.n; i += 64) {
        double a = fabs(z[i]);
        if (a > best) { best = a; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sgn = (z[bi] < 0.0) ? -1.0 : 1.0;
    for (int i = lane; i < q.n_pad; i += 64) z[i] = (i < q.n) ? sgn * z[i] : 0.0;
}

hipError_t launch_batched_dense(int which, const BProb* P, const int64_t* pre, int np, int64_t nblocks, int f32,
                                hipStream_t st) {
    if (nblocks < 1) return hipSuccess;
    const dim3 grid((unsigned)nblocks), blk(256);
    switch (which) {
        case BK_COLNORM: hipLaunchKernelGGL(k_colnorm_b, grid, blk, 0, st, P, pre, np); break;
        case BK_ANORM:
            hipLaunchKernelGGL(k_anorm_b<false>, grid, blk, 0, st, P, pre, np);
            if (hipGetLastError() != hipSuccess) break;
            hipLaunchKernelGGL(k_anorm_b<true>, grid, blk, 0, st, P, pre, np);
            break;
        case BK_GRAM: hipLaunchKernelGGL(k_gram_b, grid, blk, 0, st, P, pre, np); break;
        case BK_PROJECT: hipLaunchKernelGGL(k_project_b, grid, blk, 0, st, P, pre, np, f32); break;
        case BK_SIGN: hipLaunchKernelGGL(k_sign_b, grid, blk, 0, st, P, pre, np); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ===========================================================================
// Residual of a range finder: partial sums over 64 x 64 tiles of
// |U~ - Q B|_F^2 with Q (n_pad x p_pad, ld n_pad) and B = Q^T U~ (p_pad x R_pad).
// grid: (R_pad / 64, n_pad / 64); part[ti + tj * tiles_i]
// ===========================================================================
__global__ __launch_bounds__(256) void k_resid_partials(int64_t n_pad, int64_t R_pad, int64_t p_pad,
                                                        const double* __restrict__ Q, const double* __restrict__ B,
                                                        const double* __restrict__ T, double* __restrict__ part) {
    __shared__ double sA[2 * KC * LDS_STRIDE];
    __shared__ double sB[2 * KC * LDS_STRIDE];
    __shared__ double red[4];
    const int64_t tn = blockIdx.x, tm = blockIdx.y;
    d4_t acc[2][2];
    zero_acc(acc);
    tile64_f64<false, true>(Q, n_pad, B, p_pad, tm * T64, tn * T64, 0, p_pad, sA, sB, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t r = tm * T64 + wr + a * 16 + c_row64(lane, i);
                const int64_t c = tn * T64 + wc + b * 16 + c_col(lane);
                const double d = T[r + c * n_pad] - acc[a][b][i];
                s += d * d;
            }
    s = wave_sum(s);
    if (lane == 0) red[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[tm + tn * (n_pad / T64)] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out = T - Q B (n_pad x N_pad, ld n_pad): Q n_pad x p_pad (ld n_pad), B p_pad x
// N_pad (ld p_pad).  Each block reads and writes only its own 64 x 64 tile of T
// and out, so out may be T.
__global__ __launch_bounds__(256) void k_residual(int64_t n_pad, int64_t p_pad, const double* __restrict__ Q,
                                                  const double* __restrict__ B, const double* T, double* out) {
    __shared__ double sA[2 * KC * LDS_STRIDE];
    __shared__ double sB[2 * KC * LDS_STRIDE];
    const int64_t tn = blockIdx.x, tm = blockIdx.y;
    d4_t acc[2][2];
    zero_acc(acc);
    tile64_f64<false, true>(Q, n_pad, B, p_pad, tm * T64, tn * T64, 0, p_pad, sA, sB, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t r = tm * T64 + wr + a * 16 + c_row64(lane, i);
                const int64_t c = tn * T64 + wc + b * 16 + c_col(lane);
                out[r + c * n_pad] = T[r + c * n_pad] - acc[a][b][i];
            }
}

hipError_t launch_residual(int64_t n_pad, int64_t N_pad, int64_t p_pad, const double* Q, const double* B,
                           const double* T, double* out, hipStream_t st) {
    if (n_pad % T64 || N_pad % T64 || p_pad % KC) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_residual, dim3((unsigned)(N_pad / T64), (unsigned)(n_pad / T64)), dim3(256), 0, st, n_pad,
                       p_pad, Q, B, T, out);
    return hipGetLastError();
}

hipError_t launch_resid_partials(int64_t n_pad, int64_t R_pad, int64_t p_pad, const double* Q, const double* B,
                                 const double* Ut, double* part, hipStream_t st) {
    if (n_pad % T64 || R_pad % T64 || p_pad % KC) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_resid_partials, dim3((unsigned)(R_pad / T64), (unsigned)(n_pad / T64)), dim3(256), 0, st,
                       n_pad, R_pad, p_pad, Q, B, Ut, part);
    return hipGetLastError();
}

// ===========================================================================
// The certificate inside the proof of Theorem 2.3:
//   c_l = sum_nu |xi'_nu| |U~[:, nu] - Z V[:, nu]|   (V = Z^T U~ in FP64),
// every residual column formed directly.  k_colresid2: per 64 x 64 tile the sum of
// squares of each column's 64 residual entries -> part[tm * R_pad + col];
// k_cert_cols: per column the fixed-order sum over the row tiles, its root times
// |xi'|, one partial per 256 columns -> out[blockIdx.x].
// ===========================================================================
__global__ __launch_bounds__(256) void k_colresid2(int64_t n_pad, int64_t R_pad, int64_t p_pad,
                                                   const double* __restrict__ Q, const double* __restrict__ B,
                                                   const double* __restrict__ T, double* __restrict__ part) {
    __shared__ double sA[2 * KC * LDS_STRIDE];
    __shared__ double sB[2 * KC * LDS_STRIDE];
    __shared__ double cs[2][T64];
    const int64_t tn = blockIdx.x, tm = blockIdx.y;
    d4_t acc[2][2];
    zero_acc(acc);
    tile64_f64<false, true>(Q, n_pad, B, p_pad, tm * T64, tn * T64, 0, p_pad, sA, sB, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    double sq[2] = {0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t r = tm * T64 + wr + a * 16 + c_row64(lane, i);
                const int64_t c = tn * T64 + wc + b * 16 + c_col(lane);
                const double d = T[r + c * n_pad] - acc[a][b][i];
                sq[b] += d * d;
            }
    // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same column
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        sq[b] += __shfl_xor(sq[b], 16);
        sq[b] += __shfl_xor(sq[b], 32);
    }
    if (lane < 16) {
        cs[w >> 1][wc + lane] = sq[0];
        cs[w >> 1][wc + 16 + lane] = sq[1];
    }
    __syncthreads();
    if (threadIdx.x < T64) part[tm * R_pad + tn * T64 + threadIdx.x] = cs[0][threadIdx.x] + cs[1][threadIdx.x];
}

__global__ __launch_bounds__(256) void k_cert_cols(const double* __restrict__ part, int64_t ntm, int64_t R_pad,
                                                   const double* __restrict__ xip, double* __restrict__ out) {
    __shared__ double red[4];
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (c < R_pad) {
        double s = 0.0;
        for (int64_t rt = 0; rt < ntm; ++rt) s += part[rt * R_pad + c];
        v = fabs(xip[c]) * sqrt(s);
    }
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

int64_t cert_blocks(int64_t R_pad) { return (R_pad + 255) / 256; }

hipError_t launch_cert_mode(int64_t n_pad, int64_t R_pad, int64_t p_pad, const double* Z, const double* V64,
                            const double* Ut, const double* xip, double* part, double* out, hipStream_t st) {
    if (n_pad % T64 || R_pad % T64 || p_pad % KC) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_colresid2, dim3((unsigned)(R_pad / T64), (unsigned)(n_pad / T64)), dim3(256), 0, st, n_pad,
                       R_pad, p_pad, Z, V64, Ut, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cert_cols, dim3((unsigned)cert_blocks(R_pad)), dim3(256), 0, st, part, n_pad / T64, R_pad,
                       xip, out);
    return hipGetLastError();
}
