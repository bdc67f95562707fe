// a2 in reduced precision: the Gram matrix G = U~ U~^T (n <= R side) from FP32
// MFMA or from BF16x3 MFMA (a = a_hi + a_lo in bf16, a*b ~ hi*hi + hi*lo + lo*hi),
// both accumulating in FP32.  Its eigenvalues then carry rounding noise of about
// u_32 |G| (FP32) or 2^-17 |G| (BF16x3) instead of u_64 |G|; the reduction that
// uses it recovers FP64 accuracy by a Rayleigh-Ritz step on the leading
// eigenvectors (FP64 projection, residual and small eigenproblem).
//
// Same tiling as the FP64 Gram: lower-triangle 64 x 64 output tiles, 4 waves of
// 32 x 32 (2 x 2 MFMA 16 x 16 fragments), the same split-K partials (summed in
// FP64 by the FP64 Gram's reduction kernel).  K runs in chunks of 32 terms; the
// FP32 accumulators are added into FP64 ones every GLP_FLUSH terms, which bounds
// the growth of the FP32 rounding over long contractions.
#include <hip/hip_runtime.h>
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int GT = 64;          // output tile
constexpr int GK = 32;          // K chunk
constexpr int F32_STRIDE = 80;  // floats per k row of an FP32 chunk: the four k rows a
                                // wave reads together fall 16 banks apart
constexpr int GLP_FLUSH = 4096;

// one chunk of both operands in LDS
union LpChunk {
    struct {
        float a[GK][F32_STRIDE];
        float b[GK][F32_STRIDE];
    } f32;
    struct {
        // row r (64 bytes: 32 bf16 k values) of a plane; its 8-k group q at slot
        // lds_slot(r, q)
        char ah[GT * 64], al[GT * 64], bh[GT * 64], bl[GT * 64];
    } b16;
};

// hi = bf16(x), lo = bf16(x - hi), eight values at once
__device__ __forceinline__ void split8(const float (&x)[8], bf8_t& hi, bf8_t& lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 h = (__bf16)x[e];
        hi[e] = h;
        lo[e] = (__bf16)(x[e] - (float)h);
    }
}

template <int PREC>
__global__ __launch_bounds__(256) void k_gram_lp(int64_t n_pad, int64_t R_pad, const double* __restrict__ T0,
                                                 const double* __restrict__ T1, const double* __restrict__ T2,
                                                 double* __restrict__ G0, double* __restrict__ G1,
                                                 double* __restrict__ G2, double* __restrict__ part, int splits) {
    __shared__ LpChunk S;
    const int mode = blockIdx.z;
    const double* __restrict__ T = mode == 0 ? T0 : (mode == 1 ? T1 : T2);
    double* __restrict__ G = mode == 0 ? G0 : (mode == 1 ? G1 : G2);
    // lower-triangle tile (ti >= tj) from the linear index
    const int64_t tl = blockIdx.x;
    int64_t ti = (int64_t)((sqrt(8.0 * (double)tl + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tl) ++ti;
    while (ti * (ti + 1) / 2 > tl) --ti;
    const int64_t tj = tl - ti * (ti + 1) / 2;
    const int64_t chunk = round_up(ceil_div(R_pad, splits), GK);
    const int64_t k0 = (int64_t)blockIdx.y * chunk, k1 = (k0 + chunk < R_pad) ? k0 + chunk : R_pad;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    // loading map: row lr of the tile, k values 8 lq .. 8 lq + 7 of the chunk (each
    // load instruction of a wave reads 64 consecutive rows of one column of U~)
    const int lr = t & 63, lq = t >> 6;
    const double* pa = T + (ti * GT + lr) + (k0 + 8 * lq) * n_pad;
    const double* pb = T + (tj * GT + lr) + (k0 + 8 * lq) * n_pad;

    f4_t acc[2][2];
    double acc64[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; ++i) acc64[a][b][i] = 0.0;
        }
    auto flush = [&]() {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
#pragma unroll
                for (int i = 0; i < 4; ++i) acc64[a][b][i] += (double)acc[a][b][i];
                acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};
            }
    };

    int since = 0;
    for (int64_t kc = k0; kc < k1; kc += GK) {
        float xa[8], xb[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            xa[e] = (float)pa[(kc - k0 + e) * n_pad];
            xb[e] = (float)pb[(kc - k0 + e) * n_pad];
        }
        __syncthreads();   // every wave is done with the previous chunk
        if constexpr (PREC == 1) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                S.f32.a[8 * lq + e][lr] = xa[e];
                S.f32.b[8 * lq + e][lr] = xb[e];
            }
        } else {
            bf8_t h, l;
            const int off = lr * 64 + 16 * lds_slot(lr, lq);
            split8(xa, h, l);
            *reinterpret_cast<bf8_t*>(S.b16.ah + off) = h;
            *reinterpret_cast<bf8_t*>(S.b16.al + off) = l;
            split8(xb, h, l);
            *reinterpret_cast<bf8_t*>(S.b16.bh + off) = h;
            *reinterpret_cast<bf8_t*>(S.b16.bl + off) = l;
        }
        __syncthreads();
        if constexpr (PREC == 1) {
#pragma unroll
            for (int s = 0; s < GK / 4; ++s) {
                const int k = 4 * s + (lane >> 4);
                float av[2], bv[2];
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    av[f] = S.f32.a[k][wr + 16 * f + (lane & 15)];
                    bv[f] = S.f32.b[k][wc + 16 * f + (lane & 15)];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f32(av[a], bv[b], acc[a][b]);
            }
        } else {
            bf8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const int ra = wr + 16 * f + (lane & 15), rb = wc + 16 * f + (lane & 15);
                const int oa = ra * 64 + 16 * lds_slot(ra, lane >> 4);
                const int ob = rb * 64 + 16 * lds_slot(rb, lane >> 4);
                ah[f] = *reinterpret_cast<const bf8_t*>(S.b16.ah + oa);
                al[f] = *reinterpret_cast<const bf8_t*>(S.b16.al + oa);
                bh[f] = *reinterpret_cast<const bf8_t*>(S.b16.bh + ob);
                bl[f] = *reinterpret_cast<const bf8_t*>(S.b16.bl + ob);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b] = mfma_bf16(ah[a], bh[b], acc[a][b]);
                    acc[a][b] = mfma_bf16(ah[a], bl[b], acc[a][b]);
                    acc[a][b] = mfma_bf16(al[a], bh[b], acc[a][b]);
                }
        }
        since += GK;
        if (since == GLP_FLUSH) {
            flush();
            since = 0;
        }
    }
    flush();
    // register i of lane l: row 4 (l / 16) + i, column l % 16 of its fragment
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t r = ti * GT + wr + a * 16 + c_row32(lane, i);
                const int64_t c = tj * GT + wc + b * 16 + c_col(lane);
                const double v = acc64[a][b][i];
                if (splits == 1) {
                    if (r < c) continue;   // diagonal tiles: the r >= c lane writes both
                    G[r + c * n_pad] = v;
                    G[c + r * n_pad] = v;
                } else {
                    part[((int64_t)blockIdx.y * 3 + mode) * n_pad * n_pad + r + c * n_pad] = v;
                }
            }
}

}  // namespace

hipError_t launch_gram_lp(int prec, int64_t n_pad, int64_t R_pad, double* const Ut[3], double* const G[3],
                          double* part, int splits, hipStream_t st) {
    if (prec != 1 && prec != 2) return hipErrorInvalidValue;
    if (n_pad % GT != 0 || R_pad % GK != 0 || (splits > 1 && !part)) return hipErrorInvalidValue;
    const int64_t nt = n_pad / GT;
    dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)splits, 3);
    if (prec == 1)
        hipLaunchKernelGGL(k_gram_lp<1>, grid, dim3(256), 0, st, n_pad, R_pad, Ut[0], Ut[1], Ut[2], G[0], G[1], G[2],
                           part, splits);
    else
        hipLaunchKernelGGL(k_gram_lp<2>, grid, dim3(256), 0, st, n_pad, R_pad, Ut[0], Ut[1], Ut[2], G[0], G[1], G[2],
                           part, splits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    return launch_gram_reduce(n_pad, part, splits, G, st);
}
