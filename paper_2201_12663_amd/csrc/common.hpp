// Shared device helpers for the gfx950 kernels of the Reduced HOSVD library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

#define WAVE 64

// ---------------------------------------------------------------------------
// MFMA fragment layouts (CDNA3/CDNA4, 16x16 output tiles, one wave):
//   A operand (16 x K):  lane l holds rows  (l % 16), k-group (l / 16)
//   B operand (K x 16):  lane l holds cols  (l % 16), k-group (l / 16)
//   C/D (16 x 16), register i = 0..3 of lane l holds column l % 16 and row
//       f64 16x16x4:              4*i + l/16   (rows interleaved across lane groups)
//       f32 16x16x4, bf16 16x16x32: 4*(l/16) + i (4 consecutive rows per lane)
// f64/f32 16x16x4: k-group g = single k index g (4 k per instruction)
// bf16 16x16x32:   k-group g = k indices 8g .. 8g+7 (8 bf16 per lane)
// (checked on gfx950 with one-hot operands)
// ---------------------------------------------------------------------------
__device__ __forceinline__ d4_t mfma_f64(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_f32(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_bf16(bf8_t a, bf8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int c_row64(int lane, int i) { return 4 * i + (lane >> 4); }

// LDS placement of bf16 MFMA operands held as 64-byte rows (32 k values in four
// 16-byte groups): group q of row r sits in slot q ^ f(r), f(r) = ((r >> 1) ^ (r >> 2)) & 3.
// The 16 rows of a fragment read with one group index then fall on distinct banks
// both with 32 banks (8 lanes per cycle for a 16-byte read: rows 2 apart share
// banks unless f separates them) and with 64 banks (16 lanes per cycle).
__device__ __forceinline__ int lds_slot(int r, int q) { return q ^ (((r >> 1) ^ (r >> 2)) & 3); }
__device__ __forceinline__ int c_row32(int lane, int i) { return 4 * (lane >> 4) + i; }
__device__ __forceinline__ int c_col(int lane) { return lane & 15; }

// ---------------------------------------------------------------------------
// wave reductions (64 lanes)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, WAVE);
    return v;
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
__host__ __device__ static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ static inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
