// a7: the Khatri-Rao core contraction (Proposition 2.2)
//     beta[j1, j2, j3] = sum_nu xi'_nu V1[j1,nu] V2[j2,nu] V3[j3,nu]
// as one MFMA GEMM  beta_(1) = (V1 diag(xi')) * (V3 (.) V2)^T  with M = r1,
// N = r2*r3, K = R.  The Khatri-Rao operand is never stored: each K-chunk of
// V2 and V3 (16 rows each) is staged in LDS and the B fragments are formed in
// registers as V2[j2,nu]*V3[j3,nu].
//
// Workgroup tile: TM rows of j1 x 256 columns = 16 (j2) x 16 (j3); 4 waves, wave
// w owns columns j3 in [4w, 4w+4).  FP64/FP32: K chunks double-buffered in LDS
// with the next chunk's global loads in flight during the current chunk's MFMAs;
// BF16x3: a ring of three chunks filled by direct global-to-LDS loads.
// Tiles are assigned XCD-contiguously: block b runs on XCD b % 8, and each XCD
// gets one contiguous range of tiles, ordered so neighbouring tiles share V1 rows
// and, in groups of 8 x 8 (j2, j3) tiles, their V2 and V3 slices.
//
// Variants: FP64 (v_mfma_f64_16x16x4, TM=64), FP32 (v_mfma_f32_16x16x4, TM=64)
// and BF16x3 (v_mfma_f32_16x16x32_bf16, TM=128): a = a_hi + a_lo, b = b_hi + b_lo
// in bf16, a*b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi, FP32 accumulation restarted
// every KFLUSH values of nu (partial sums added in beta's precision).  The BF16x3
// core reads V1 diag(xi') already split (launch_split_a: hi and lo planes, nu
// contiguous), so its vector ALUs only form and split the Khatri-Rao operand.
#include <hip/hip_runtime.h>
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int NXCD = 8;
constexpr int TN2 = 16, TN3 = 16;

__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t per) {
    return (bid % NXCD) * per + bid / NXCD;
}

// tile index -> (row block, j2 tile, j3 tile).  Within one row block the j2 x j3
// tiles run in groups of GN2 j2 tiles with j3 slowest inside a group, so that the
// workgroups one XCD holds at a time (consecutive tiles) cover a near-square block
// of (j2, j3) tiles and share their V2 and V3 slices in that XCD's L2.
constexpr int GN2 = 8;
__device__ __forceinline__ void tile_coords(int64_t tile, int N2T, int N3T, int& mt, int& n2t, int& n3t) {
    const int NT = N2T * N3T;
    mt = (int)(tile / NT);
    const int t = (int)(tile % NT);
    const int g = t / (GN2 * N3T), first = g * GN2;
    const int gs = min(N2T - first, GN2);
    const int u = t - g * GN2 * N3T;
    n2t = first + u % gs;
    n3t = u / gs;
}

// beta entries are written as O: double, or float (the mixed cores' option)
template <typename O, typename T>
__device__ __forceinline__ void store_beta(O* __restrict__ beta, int r1, int r2, int r3, int j1, int j2, int j3, T v) {
    if (j1 < r1 && j2 < r2 && j3 < r3) beta[(int64_t)j1 + (int64_t)r1 * ((int64_t)j2 + (int64_t)r2 * j3)] = (O)v;
}

// The FP32-accumulating cores hand their accumulators to beta every KFLUSH
// values of nu: the first hand-over stores, later ones add in FP64 (FP32 for a
// float beta) and the accumulators restart from zero.  A workgroup owns its
// tile, and every lane reads back only what it wrote itself, so no
// synchronization is needed.  Rounding of a sequential FP32 sum grows with the
// running total; restarting every KFLUSH terms bounds that growth (R = 90000:
// about 10x smaller error).  The hand-over variants run only when R_pad > KFLUSH;
// shorter contractions keep the single final store.
constexpr int64_t KFLUSH = 8192;

// NF x 4 accumulator fragments of a 16 x 16 FP32 MFMA (rows 4 (lane / 16) + i,
// column lane % 16) into beta: store (first) or add, then reset to zero.  One
// base pointer per j3 column and constant offsets 16 f + i keep the addressing
// out of the registers.
template <int NF, typename O>
__device__ __forceinline__ void hand_over(O* __restrict__ beta, int r1, int r2, int r3, int m0, int b2, int b3,
                                          int lane, int w, f4_t (&acc)[NF][4], bool first) {
    const int rb = m0 + 4 * (lane >> 4);
    const int rows = r1 - rb;                       // rows rb + o exist for o < rows
    const int j2 = b2 + c_col(lane);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int j3 = b3 + 4 * w + g;
        if (j2 < r2 && j3 < r3) {
            O* p = beta + rb + (int64_t)r1 * ((int64_t)j2 + (int64_t)r2 * j3);
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (16 * f + i < rows) {
                        O& x = p[16 * f + i];
                        x = first ? (O)acc[f][g][i] : (O)((double)x + (double)acc[f][g][i]);
                    }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f][g] = f4_t{0.f, 0.f, 0.f, 0.f};
    }
}

// ---------------------------------------------------------------------------
// FP64 / FP32 variant, TM = 64, KC = 16
// ---------------------------------------------------------------------------
template <typename T>
struct MF;
template <>
struct MF<double> {
    typedef d4_t acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) { return mfma_f64(a, b, c); }
    static __device__ __forceinline__ int row(int lane, int i) { return c_row64(lane, i); }
};
template <>
struct MF<float> {
    typedef f4_t acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) { return mfma_f32(a, b, c); }
    static __device__ __forceinline__ int row(int lane, int i) { return c_row32(lane, i); }
};

template <typename T, typename O, bool FLUSH, int NF>
__device__ __forceinline__ void core_tile_std(int r1, int r2, int r3, int ld1, int ld2, int ld3, int64_t Kp,
                              const T* __restrict__ V1, const T* __restrict__ V2, const T* __restrict__ V3,
                              const double* __restrict__ xip, O* __restrict__ beta, int N2T, int N3T,
                              int64_t tile, int mbase = 0) {
    constexpr int TM = 16 * NF, KC = 16;
    constexpr int PA = TM * KC / 256, AS = 256 / TM;   // A entries per thread, their k stride
    typedef typename MF<T>::acc_t acc_t;
    // rows of sA padded by 64 bytes: the two k rows a half-wave reads fall 16 banks apart
    __shared__ T sA[2][KC][TM + 64 / sizeof(T)];
    __shared__ T s2[2][KC][TN2];
    __shared__ T s3[2][KC][TN3];
    int mt, n2t, n3t;
    tile_coords(tile, N2T, N3T, mt, n2t, n3t);
    const int m0 = mbase + mt * TM, b2 = n2t * TN2, b3 = n3t * TN3;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;

    // staging maps: A TM x 16 (PA per thread), V2/V3 16 x 16 (1 each)
    const int ai = t % TM, ak = t / TM;
    const int vi = t & 15, vk = t >> 4;
    T ra[PA], rv2, rv3;
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < PA; ++q) {
            const int64_t k = k0 + ak + AS * q;
            ra[q] = V1[(int64_t)(m0 + ai) + k * ld1] * (T)xip[k];
        }
        rv2 = V2[(int64_t)(b2 + vi) + (k0 + vk) * ld2];
        rv3 = V3[(int64_t)(b3 + vi) + (k0 + vk) * ld3];
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PA; ++q) sA[buf][ak + AS * q][ai] = ra[q];
        s2[buf][vk][vi] = rv2;
        s3[buf][vk][vi] = rv3;
    };

    acc_t acc[NF][4];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[f][g] = acc_t{0, 0, 0, 0};

    constexpr bool f32 = sizeof(T) == 4 && FLUSH;
    constexpr int64_t FL = KFLUSH / KC;   // chunks between hand-overs (FP32 only)
    bool first = true;

    const int64_t nchunk = Kp / KC;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int64_t c = 0; c < nchunk; ++c) {
        const int buf = (int)(c & 1);
        if (c + 1 < nchunk) gload((c + 1) * KC);
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            const int k = 4 * kk + (lane >> 4);
            T a[NF], b[4];
#pragma unroll
            for (int f = 0; f < NF; ++f) a[f] = sA[buf][k][16 * f + (lane & 15)];
            const T v2 = s2[buf][k][lane & 15];
#pragma unroll
            for (int g = 0; g < 4; ++g) b[g] = v2 * s3[buf][k][4 * w + g];
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int g = 0; g < 4; ++g) acc[f][g] = MF<T>::mma(a[f], b[g], acc[f][g]);
        }
        if constexpr (f32) {
            if ((c + 1) % FL == 0 && c + 1 < nchunk) {
                hand_over<NF, O>(beta, r1, r2, r3, m0, b2, b3, lane, w, acc, first);
                first = false;
            }
        }
        if (c + 1 < nchunk) lstore(buf ^ 1);
        __syncthreads();
    }
    if constexpr (f32) {
        hand_over<NF, O>(beta, r1, r2, r3, m0, b2, b3, lane, w, acc, first);
        return;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                store_beta<O>(beta, r1, r2, r3, m0 + 16 * f + MF<T>::row(lane, i), b2 + c_col(lane), b3 + 4 * w + g,
                           acc[f][g][i]);
}

// Two waves per SIMD at least: the FP32 instances with the hand-over of long
// contractions then fit without spills (436 -> 256 registers at 128 rows,
// 212 -> 126 at 64), and the 128-row tile without it drops from 268 to 192.
template <typename T, typename O, bool FLUSH, int NF>
__global__ __launch_bounds__(256, 2) void k_core_std(int r1, int r2, int r3, int ld1, int ld2, int ld3,
                                                  int64_t Kp, const T* __restrict__ V1,
                                                  const T* __restrict__ V2, const T* __restrict__ V3,
                                                  const double* __restrict__ xip, O* __restrict__ beta,
                                                  int MT, int N2T, int N3T, int64_t per, int mbase) {
    const int64_t tile = xcd_tile(blockIdx.x, per);
    if (tile >= (int64_t)MT * N2T * N3T) return;
    core_tile_std<T, O, FLUSH, NF>(r1, r2, r3, ld1, ld2, ld3, Kp, V1, V2, V3, xip, beta, N2T, N3T, tile, mbase);
}

// ---------------------------------------------------------------------------
// BF16x3 variant, TM = 64 or 128, KC = 32.  V_l are FP32.
// ---------------------------------------------------------------------------
constexpr int BKC = 32;   // K chunk

typedef float f2_t __attribute__((ext_vector_type(2)));
typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
union bf8_pairs {
    bf8_t v;
    b2_t p[4];
};

// two values at once: hi = bf16(x), lo = bf16(x - hi) (packed conversions)
__device__ __forceinline__ void split2(f2_t x, b2_t& hi, b2_t& lo) {
    hi = __builtin_convertvector(x, b2_t);
    lo = __builtin_convertvector(x - __builtin_convertvector(hi, f2_t), b2_t);
}


// The BF16x3 tile with its operands streamed straight from global memory into
// LDS (global_load_lds: lane L of a wave writes its 16 bytes at the
// instruction's LDS base + 16 L, so no registers hold them on the way) through
// a ring of three K-chunk stages: chunk c+2 is in flight while chunk c is
// multiplied.  Layouts (bytes within a stage), chosen so that the reads of a
// K-chunk meet no bank conflicts:
//   A plane (hi, lo): row r at 64 r, its 8-k group q (16 B) at slot lds_slot(r, q);
//   V2, V3: k row at 64 s(k), s(k) = 4 (k & 7) + (k >> 3), so that the four k
//   rows a wave reads together (k, k+8, k+16, k+24) form one 256-byte block.
template <int NF>
struct DmaStage {
    static constexpr int TM = 16 * NF;
    static constexpr int A_BYTES = TM * 64;              // one plane of one chunk
    static constexpr int V_BYTES = BKC * TN2 * 4;        // V2 or V3 of one chunk (2 KB)
    static constexpr int BYTES = 2 * A_BYTES + 2 * V_BYTES;
    static constexpr int LOADS = TM / 32 + 1;            // global_load_lds per wave per chunk
};

typedef __attribute__((address_space(3))) void* lds_void_ptr;

template <typename O, bool FLUSH, int NF>
__device__ __forceinline__ void core_tile_bf16x3_dma(int r1, int r2, int r3, int ld2, int ld3, int64_t Kp,
                                                     const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al,
                                                     const float* __restrict__ V2, const float* __restrict__ V3,
                                                     O* __restrict__ beta, int N2T, int N3T, int64_t tile,
                                                     int mbase = 0) {
    typedef DmaStage<NF> S;
    constexpr int TM = S::TM, NS = 3;
    __shared__ __attribute__((aligned(1024))) char ring[NS * S::BYTES];
    int mt, n2t, n3t;
    tile_coords(tile, N2T, N3T, mt, n2t, n3t);
    const int m0 = mbase + mt * TM, b2 = n2t * TN2, b3 = n3t * TN3;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t nchunk = Kp / BKC;

    // issue this wave's loads of chunk c into stage c % NS
    auto issue = [&](int64_t c) {
        char* st = ring + (int)(c % NS) * S::BYTES;
        const int64_t k0 = c * BKC;
        // A: 16-row blocks (1 KB each) of both planes; wave w takes blocks w, w + 4, ...
#pragma unroll
        for (int i = 0; i < TM / 32; ++i) {
            const int blk = w + 4 * i;                    // 0 .. 2 TM / 16 - 1 over both planes
            const int plane = blk / (TM / 16), rb = (blk % (TM / 16)) * 16;
            const int r = rb + (lane >> 2);
            const int q = lds_slot(r, lane & 3);
            const __bf16* src = (plane ? Al : Ah) + (int64_t)(m0 + r) * Kp + k0 + 8 * q;
            __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_ptr)(st + plane * S::A_BYTES + rb * 64), 16,
                                             0, 0);
        }
        // V2 (waves 0, 1) and V3 (waves 2, 3): 16 k rows per instruction
        {
            const int half = w & 1;
            const int s = 16 * half + (lane >> 2);
            const int k = 8 * (s & 3) + (s >> 2);
            const float* src = (w < 2) ? V2 + (int64_t)(b2 + 4 * (lane & 3)) + (k0 + k) * ld2
                                       : V3 + (int64_t)(b3 + 4 * (lane & 3)) + (k0 + k) * ld3;
            char* dst = st + 2 * S::A_BYTES + (w < 2 ? 0 : S::V_BYTES) + half * 1024;
            __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_ptr)dst, 16, 0, 0);
        }
    };

    f4_t acc[NF][4];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[f][g] = f4_t{0.f, 0.f, 0.f, 0.f};
    constexpr int64_t FL = KFLUSH / BKC;
    bool first = true;

    issue(0);
    if (nchunk > 1) issue(1);
    const int kq = lane >> 4, kg = 8 * kq;
    for (int64_t c = 0; c < nchunk; ++c) {
        // chunk c has landed (this wave's loads; chunk c+1's may still fly), every
        // wave's own LDS reads are done, then all waves meet: chunk c is visible
        // to all and the stage of chunk c-1 is free
        if (c + 1 < nchunk) {
            static_assert(S::LOADS == 2 || S::LOADS == 3 || S::LOADS == 5, "vmcnt of one chunk");
            if constexpr (S::LOADS == 5) asm volatile("s_waitcnt vmcnt(5) lgkmcnt(0)\n\ts_barrier" ::: "memory");
            else if constexpr (S::LOADS == 3) asm volatile("s_waitcnt vmcnt(3) lgkmcnt(0)\n\ts_barrier" ::: "memory");
            else asm volatile("s_waitcnt vmcnt(2) lgkmcnt(0)\n\ts_barrier" ::: "memory");
        } else {
            asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
        }
        if (c + 2 < nchunk) issue(c + 2);
        const char* st = ring + (int)(c % NS) * S::BYTES;
        const float* s2 = (const float*)(st + 2 * S::A_BYTES);
        const float* s3 = (const float*)(st + 2 * S::A_BYTES + S::V_BYTES);
        // B fragments: 8 k values of column (j2 = lane%16, j3 = 4w+g), split hi/lo
        bf8_pairs bh[4], bl[4];
        float v2[8];
        f4_t v3[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int srow = 4 * e + kq;                  // s(kg + e)
            v2[e] = s2[srow * 16 + (lane & 15)];
            v3[e] = *reinterpret_cast<const f4_t*>(&s3[srow * 16 + 4 * w]);
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                split2(f2_t{v2[2 * e] * v3[2 * e][g], v2[2 * e + 1] * v3[2 * e + 1][g]}, bh[g].p[e], bl[g].p[e]);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int row = 16 * f + (lane & 15);
            const int off = row * 64 + 16 * lds_slot(row, kq);
            const bf8_t ah = *reinterpret_cast<const bf8_t*>(st + off);
            const bf8_t al = *reinterpret_cast<const bf8_t*>(st + S::A_BYTES + off);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                acc[f][g] = mfma_bf16(ah, bh[g].v, acc[f][g]);
                acc[f][g] = mfma_bf16(ah, bl[g].v, acc[f][g]);
                acc[f][g] = mfma_bf16(al, bh[g].v, acc[f][g]);
            }
        }
        if constexpr (FLUSH) {
            if ((c + 1) % FL == 0 && c + 1 < nchunk) {
                hand_over<NF, O>(beta, r1, r2, r3, m0, b2, b3, lane, w, acc, first);
                first = false;
            }
        }
    }
    // the ring is reused by the next tile of a persistent workgroup: every wave is
    // done reading it
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if constexpr (FLUSH) {
        hand_over<NF, O>(beta, r1, r2, r3, m0, b2, b3, lane, w, acc, first);
        return;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                store_beta<O>(beta, r1, r2, r3, m0 + 16 * f + c_row32(lane, i), b2 + c_col(lane), b3 + 4 * w + g,
                           acc[f][g][i]);
}

// Two waves per SIMD: the 128-row tile fits 234 registers (its accumulators are
// 128 of them; the operands travel to LDS without registers), the 64-row tile
// 158.  The 128-row tile forms each Khatri-Rao fragment once for twice the
// MFMAs.  Measured at the 1024 x 4096 workload and not kept: a 256-row tile at
// one wave per SIMD, accumulators in AGPRs, the next chunk's fragments formed
// during the current chunk's MFMAs (9.9 ms against 6.6: one wave per SIMD leaves
// the matrix cores idle on every dependency); a 256-row tile of 8 waves, each
// with 2 j3 columns and all 16 row fragments, half the Khatri-Rao work per MFMA
// for twice the A-fragment reads, one workgroup per CU (7.1 ms).
template <typename O, bool FLUSH, int NF>
__global__ __launch_bounds__(256, 2) void k_core_bf16x3(int r1, int r2, int r3, int ld2, int ld3, int64_t Kp,
                                                     const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al,
                                                     const float* __restrict__ V2, const float* __restrict__ V3,
                                                     O* __restrict__ beta, int MT, int N2T, int N3T, int64_t per,
                                                     int mbase) {
    const int64_t tile = xcd_tile(blockIdx.x, per);
    if (tile >= (int64_t)MT * N2T * N3T) return;
    core_tile_bf16x3_dma<O, FLUSH, NF>(r1, r2, r3, ld2, ld3, Kp, Ah, Al, V2, V3, beta, N2T, N3T, tile, mbase);
}


// ---------------------------------------------------------------------------
// The BF16x3 core's A operand: x = V1[j1, nu] * xi'_nu (FP32, as the FP32 core
// forms it), split into hi = bf16(x) and lo = bf16(x - hi), stored as two planes
// with nu contiguous: plane[j1 * Kp + nu].  One 64 x 64 tile per workgroup,
// transposed through LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split_tile(const float* __restrict__ V1, int64_t ld, const double* __restrict__ xip,
                                           int64_t Kp, __bf16* __restrict__ Ah, __bf16* __restrict__ Al, int64_t tm,
                                           int64_t tn) {
    __shared__ float s[64][65];
    const int t = threadIdx.x;
    const int64_t r0 = tm * 64, k0 = tn * 64;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int kk = (t >> 6) + 4 * q, rr = t & 63;
        s[kk][rr] = V1[(r0 + rr) + (k0 + kk) * ld] * (float)xip[k0 + kk];
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int idx = t + 256 * g;
        const int rr = idx >> 3, kq = (idx & 7) * 8;
        bf8_pairs h8, l8;
#pragma unroll
        for (int e = 0; e < 4; ++e) split2(f2_t{s[kq + 2 * e][rr], s[kq + 2 * e + 1][rr]}, h8.p[e], l8.p[e]);
        const int64_t off = (r0 + rr) * Kp + k0 + kq;
        *reinterpret_cast<bf8_t*>(Ah + off) = h8.v;
        *reinterpret_cast<bf8_t*>(Al + off) = l8.v;
    }
}

__global__ __launch_bounds__(256) void k_split_a(const float* __restrict__ V1, int64_t ld,
                                                 const double* __restrict__ xip, int64_t Kp,
                                                 __bf16* __restrict__ Ah, __bf16* __restrict__ Al) {
    split_tile(V1, ld, xip, Kp, Ah, Al, blockIdx.y, blockIdx.x);
}

// batched: problem p's blocks cover rcap_pad / 64 x R_pad / 64 tiles of mode 1;
// tiles beyond the rank (rounded to the 128-row core tile) are skipped
__global__ __launch_bounds__(256) void k_split_b(const BProb* __restrict__ P, const int64_t* __restrict__ pre, int np) {
    int lo = 0, hi = np;   // largest p with pre[p] <= blockIdx.x
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid;
    }
    const BProb& q = P[lo];
    const int64_t TN = q.R_pad / 64;
    const int64_t local = (int64_t)blockIdx.x - pre[lo];
    const int64_t tm = local / TN, tn = local % TN;
    const int r = min(q.ranks[0], q.rcap);
    if (q.ranks[3] != 0 || r < 1 || tm * 64 >= round_up(r, 128)) return;
    const __bf16* base = (const __bf16*)q.Asplit;
    split_tile((const float*)q.V[0], q.rcap_pad, q.xip, q.R_pad, (__bf16*)base,
               (__bf16*)base + (int64_t)q.rcap_pad * q.R_pad, tm, tn);
}

// ---------------------------------------------------------------------------
// Batched cores: the plan kernel counts each eligible problem's tiles (status 0,
// beta requested, all ranks >= 1) and writes the prefix sums; the persistent
// kernel's workgroups then take tiles from a shared counter until none is left.
// work[0]: counter, work[1]: total tiles, work[2 .. np+2]: prefix.
// ---------------------------------------------------------------------------
__global__ void k_core_plan_b(const BProb* __restrict__ P, int np, int tm, int64_t* __restrict__ work) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    for (int p = 0; p < np; ++p) {
        const BProb& q = P[p];
        work[2 + p] = acc;
        const int r1 = q.ranks[0], r2 = q.ranks[1], r3 = q.ranks[2];
        if (q.ranks[3] == 0 && q.beta && r1 > 0 && r2 > 0 && r3 > 0)
            acc += ceil_div(r1, tm) * ceil_div(r2, TN2) * ceil_div(r3, TN3);
    }
    work[2 + np] = acc;
    work[1] = acc;
    work[0] = 0;
}

// the BF16x3 instances at two waves per SIMD, as k_core_bf16x3
template <int PREC, typename O, bool FLUSH, int NF>
__global__ __launch_bounds__(256, PREC == 2 ? 2 : 1) void k_core_persist_b(const BProb* __restrict__ P, int np,
                                                        int64_t* __restrict__ work) {
    __shared__ int64_t s_tile;
    const int64_t total = work[1];
    const int64_t* pre = work + 2;
    for (;;) {
        if (threadIdx.x == 0)
            s_tile = (int64_t)atomicAdd((unsigned long long*)&work[0], 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile >= total) break;
        int lo = 0, hi = np;   // largest p with pre[p] <= tile
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= tile) lo = mid;
            else hi = mid;
        }
        const BProb& q = P[lo];
        const int r1 = q.ranks[0], r2 = q.ranks[1], r3 = q.ranks[2];
        const int N2T = (int)ceil_div(r2, TN2), N3T = (int)ceil_div(r3, TN3);
        const int64_t local = tile - pre[lo];
        if (PREC == 0)
            core_tile_std<double, O, false, 4>(r1, r2, r3, q.rcap_pad, q.rcap_pad, q.rcap_pad, q.R_pad, (const double*)q.V[0],
                                  (const double*)q.V[1], (const double*)q.V[2], q.xip, (O*)q.beta, N2T, N3T, local);
        else if (PREC == 1)
            core_tile_std<float, O, FLUSH, NF>(r1, r2, r3, q.rcap_pad, q.rcap_pad, q.rcap_pad, q.R_pad, (const float*)q.V[0],
                                 (const float*)q.V[1], (const float*)q.V[2], q.xip, (O*)q.beta, N2T, N3T, local);
        else
            core_tile_bf16x3_dma<O, FLUSH, NF>(r1, r2, r3, q.rcap_pad, q.rcap_pad, q.R_pad, (const __bf16*)q.Asplit,
                             (const __bf16*)q.Asplit + (int64_t)q.rcap_pad * q.R_pad, (const float*)q.V[1],
                             (const float*)q.V[2], (O*)q.beta, N2T, N3T, local);
    }
}

}  // namespace

template <typename O, bool FLUSH, int NF>
static void launch_core_t(const CoreArgs& a, dim3 grid, int MT, int N2T, int N3T, int64_t per, int mbase,
                          hipStream_t st) {
    O* beta = (O*)a.beta;
    if constexpr (NF == 2) {   // 32-row tiles: the last row block of the FP32 and BF16x3 cores only
        if (a.prec == 1) {
            hipLaunchKernelGGL((k_core_std<float, O, FLUSH, 2>), grid, dim3(256), 0, st, a.r[0], a.r[1], a.r[2],
                               a.r_pad[0], a.r_pad[1], a.r_pad[2], a.R_pad, (const float*)a.V[0],
                               (const float*)a.V[1], (const float*)a.V[2], a.xip, beta, MT, N2T, N3T, per, mbase);
        } else {
            const __bf16* Ah = (const __bf16*)a.Asplit;
            hipLaunchKernelGGL((k_core_bf16x3<O, FLUSH, 2>), grid, dim3(256), 0, st, a.r[0], a.r[1], a.r[2],
                               a.r_pad[1], a.r_pad[2], a.R_pad, Ah, Ah + (int64_t)a.r_pad[0] * a.R_pad,
                               (const float*)a.V[1], (const float*)a.V[2], beta, MT, N2T, N3T, per, mbase);
        }
    } else if (a.prec == 0) {
        hipLaunchKernelGGL((k_core_std<double, O, false, 4>), grid, dim3(256), 0, st, a.r[0], a.r[1], a.r[2],
                           a.r_pad[0], a.r_pad[1], a.r_pad[2], a.R_pad, (const double*)a.V[0],
                           (const double*)a.V[1], (const double*)a.V[2], a.xip, beta, MT, N2T, N3T, per, mbase);
    } else if (a.prec == 1) {
        hipLaunchKernelGGL((k_core_std<float, O, FLUSH, NF>), grid, dim3(256), 0, st, a.r[0], a.r[1], a.r[2],
                           a.r_pad[0], a.r_pad[1], a.r_pad[2], a.R_pad, (const float*)a.V[0],
                           (const float*)a.V[1], (const float*)a.V[2], a.xip, beta, MT, N2T, N3T, per, mbase);
    } else {
        const __bf16* Ah = (const __bf16*)a.Asplit;
        hipLaunchKernelGGL((k_core_bf16x3<O, FLUSH, NF>), grid, dim3(256), 0, st, a.r[0], a.r[1], a.r[2],
                           a.r_pad[1], a.r_pad[2], a.R_pad, Ah, Ah + (int64_t)a.r_pad[0] * a.R_pad,
                           (const float*)a.V[1], (const float*)a.V[2], beta, MT, N2T, N3T, per, mbase);
    }
}

template <typename O, bool FLUSH>
static void launch_core_nf(const CoreArgs& a, int nf, int MT, int N2T, int N3T, int mbase, hipStream_t st) {
    const int64_t per = ceil_div((int64_t)MT * N2T * N3T, NXCD);
    const dim3 grid((unsigned)(per * NXCD));
    if (nf == 8) launch_core_t<O, FLUSH, 8>(a, grid, MT, N2T, N3T, per, mbase, st);
    else if (nf == 4) launch_core_t<O, FLUSH, 4>(a, grid, MT, N2T, N3T, per, mbase, st);
    else launch_core_t<O, FLUSH, 2>(a, grid, MT, N2T, N3T, per, mbase, st);
}

int core_tile_default(int prec) { return (prec & 3) == 2 ? 128 : 64; }

bool core_tile_valid(int prec, int tile) {
    return (prec & 3) == 0 ? tile == 64 : (tile == 64 || tile == 128);
}

hipError_t launch_core(const CoreArgs& a, hipStream_t st) {
    if (a.r[0] < 1 || a.r[1] < 1 || a.r[2] < 1) return hipSuccess;
    const int TMv = a.tile ? a.tile : core_tile_default(a.prec);
    if (!core_tile_valid(a.prec, TMv)) return hipErrorInvalidValue;
    const int KCv = (a.prec == 2) ? BKC : 16;
    if (a.R_pad % KCv != 0) return hipErrorInvalidValue;
    if (a.prec == 2 && !a.Asplit) return hipErrorInvalidValue;
    const int MT = (int)ceil_div(a.r[0], TMv), N2T = (int)ceil_div(a.r[1], TN2), N3T = (int)ceil_div(a.r[2], TN3);
    // the kernels read whole tiles: padded rows must exist (and be zero)
    if (a.r_pad[0] < MT * TMv || a.r_pad[1] < N2T * TN2 || a.r_pad[2] < N3T * TN3) return hipErrorInvalidValue;
    const bool flush = a.R_pad > KFLUSH;   // the hand-over variants only where they act
    // a last row block that is mostly padding runs in a second launch with smaller
    // tiles: at most 32 rows as 32-row tiles (FP32, BF16x3), else at most 64 rows of
    // a 128-row tile as 64-row tiles (656 rows at 128: 5 x 128 + 1 x 32 row tiles,
    // 672 rows of MFMA work instead of 768).  Only where the launches run many
    // rounds of workgroups: the second launch's last round is a tail of its own, and
    // with few tiles per row block it costs more than the padding rows (274 x 271 x
    // 270 at R = 90000, 289 tiles per row block: FP32 core 38.2 -> 40.7 ms split).
    // Rounds of two workgroups per CU; a smaller tile's round counted as half.
    const int rem = a.r[0] - (MT - 1) * TMv;
    int nf_last = 0;
    if (MT > 1) {
        if (a.prec != 0 && rem <= 32) nf_last = 2;
        else if (TMv == 128 && rem <= 64) nf_last = 4;
    }
    if (nf_last) {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
            ncu = 256;
        const int64_t slots = 2 * (int64_t)ncu, n23 = (int64_t)N2T * N3T;
        const int64_t whole = ceil_div((int64_t)MT * n23, slots);
        const int64_t split2 = 2 * ceil_div((int64_t)(MT - 1) * n23, slots) + ceil_div(n23, slots);
        if (split2 >= 2 * whole) nf_last = 0;   // split rounds (x2) not fewer than whole rounds (x2)
    }
    const bool split_last = nf_last != 0;
    // every launch reads rows mbase .. mbase + 16 nf mt - 1 of the A operand
    if (split_last && (MT - 1) * TMv + 16 * nf_last > a.r_pad[0]) return hipErrorInvalidValue;
    auto go = [&](int nf, int mt, int mbase) {
        if (a.beta_f32) {
            if (flush) launch_core_nf<float, true>(a, nf, mt, N2T, N3T, mbase, st);
            else launch_core_nf<float, false>(a, nf, mt, N2T, N3T, mbase, st);
        } else {
            if (flush) launch_core_nf<double, true>(a, nf, mt, N2T, N3T, mbase, st);
            else launch_core_nf<double, false>(a, nf, mt, N2T, N3T, mbase, st);
        }
    };
    if (split_last) {
        go(TMv / 16, MT - 1, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        go(nf_last, 1, (MT - 1) * TMv);
    } else {
        go(TMv / 16, MT, 0);
    }
    return hipGetLastError();
}

template <typename O, bool FLUSH, int NF>
static void launch_persist_t(const BProb* P, int np, int prec, int64_t* work, int grid, hipStream_t st) {
    const dim3 g((unsigned)grid), b(256);
    if (prec == 0) hipLaunchKernelGGL((k_core_persist_b<0, O, false, 4>), g, b, 0, st, P, np, work);
    else if (prec == 1) hipLaunchKernelGGL((k_core_persist_b<1, O, FLUSH, NF>), g, b, 0, st, P, np, work);
    else hipLaunchKernelGGL((k_core_persist_b<2, O, FLUSH, NF>), g, b, 0, st, P, np, work);
}

template <typename O, bool FLUSH>
static void launch_persist_nf(const BProb* P, int np, int prec, int nf, int64_t* work, int grid, hipStream_t st) {
    if (nf == 8) launch_persist_t<O, FLUSH, 8>(P, np, prec, work, grid, st);
    else launch_persist_t<O, FLUSH, 4>(P, np, prec, work, grid, st);
}

// prec: 0 FP64, 1 FP32, 2 BF16x3; +16 float beta; +32 some problem has R_pad > KFLUSH
hipError_t launch_core_b(const BProb* P, int np, int prec, int tile, int64_t* work, int grid, hipStream_t st) {
    if (np < 1) return hipSuccess;
    const int TMv = tile ? tile : core_tile_default(prec);
    if (!core_tile_valid(prec, TMv)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_core_plan_b, dim3(1), dim3(64), 0, st, P, np, TMv, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool f32 = (prec & 16) != 0, flush = (prec & 32) != 0;
    const int nf = TMv / 16;
    if (f32) {
        if (flush) launch_persist_nf<float, true>(P, np, prec & 3, nf, work, grid, st);
        else launch_persist_nf<float, false>(P, np, prec & 3, nf, work, grid, st);
    } else {
        if (flush) launch_persist_nf<double, true>(P, np, prec & 3, nf, work, grid, st);
        else launch_persist_nf<double, false>(P, np, prec & 3, nf, work, grid, st);
    }
    return hipGetLastError();
}

int64_t core_flush_span() { return KFLUSH; }

hipError_t launch_split_a(int64_t rows_pad, int64_t R_pad, int64_t ld, const float* V1, const double* xip,
                          void* planes, hipStream_t st) {
    if (rows_pad % 64 || R_pad % 64 || ld < rows_pad) return hipErrorInvalidValue;
    __bf16* Ah = (__bf16*)planes;
    hipLaunchKernelGGL(k_split_a, dim3((unsigned)(R_pad / 64), (unsigned)(rows_pad / 64)), dim3(256), 0, st, V1, ld,
                       xip, R_pad, Ah, Ah + rows_pad * R_pad);
    return hipGetLastError();
}

hipError_t launch_split_b(const BProb* P, const int64_t* pre, int np, int64_t nblocks, hipStream_t st) {
    if (nblocks < 1) return hipSuccess;
    hipLaunchKernelGGL(k_split_b, dim3((unsigned)nblocks), dim3(256), 0, st, P, pre, np);
    return hipGetLastError();
}

template <typename O, bool FLUSH, int NF>
static const void* persist_fn(int prec) {
    switch (prec) {
        case 0: return (const void*)k_core_persist_b<0, O, false, 4>;
        case 1: return (const void*)k_core_persist_b<1, O, FLUSH, NF>;
        default: return (const void*)k_core_persist_b<2, O, FLUSH, NF>;
    }
}

template <int NF>
static const void* persist_fn_nf(int prec) {
    const bool f32 = (prec & 16) != 0, flush = (prec & 32) != 0;
    return f32 ? (flush ? persist_fn<float, true, NF>(prec & 3) : persist_fn<float, false, NF>(prec & 3))
               : (flush ? persist_fn<double, true, NF>(prec & 3) : persist_fn<double, false, NF>(prec & 3));
}

int core_b_max_grid(int prec, int tile) {
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    const int TMv = tile ? tile : core_tile_default(prec);
    const void* f = TMv == 128 ? persist_fn_nf<8>(prec) : persist_fn_nf<4>(prec);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, 256, 0) != hipSuccess || occ < 1) occ = 1;
    return ncu * occ;
}
