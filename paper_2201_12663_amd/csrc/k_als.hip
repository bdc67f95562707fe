// Kernels of the canonical-to-Tucker ALS refinement (Section 2.1, after
// Definition 2.1; eq. eqn:can_A_Tuck_als).  For mode l with the other modes a, b,
// the contracted unfolding M_l = U~_l diag(xi') (V_b (.) V_a)^T has the Gram matrix
//     M_l M_l^T = U~_l P U~_l^T,   P = diag(xi') (V_a^T V_a o V_b^T V_b) diag(xi'),
// formed with FP64 MFMA GEMMs (V^T V, U~ P, (U~ P) U~^T) and the Hadamard scaling
// below; its leading eigenvectors are the new Z_l.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace {

// Ha <- diag(xi') (Ha o Hb) diag(xi') (R_pad x R_pad, column-major)
__global__ void k_als_hadamard(int64_t Rp, double* __restrict__ Ha, const double* __restrict__ Hb,
                               const double* __restrict__ xip) {
    const int64_t tot = Rp * Rp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % Rp, j = e / Rp;
        Ha[e] = xip[i] * xip[j] * (Ha[e] * Hb[e]);
    }
}

// order[k] = index of the k-th largest of lam[0 .. m) (ties: lower index first)
__global__ __launch_bounds__(1024) void k_order_desc(const double* __restrict__ lam, int m, int* __restrict__ order) {
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const double v = lam[j];
        int rk = 0;
        for (int i = 0; i < m; ++i) {
            const double u = lam[i];
            rk += (u > v) || (u == v && i < j);
        }
        order[rk] = j;
    }
}

}  // namespace

hipError_t launch_als_hadamard(int64_t R_pad, double* Ha, const double* Hb, const double* xip, hipStream_t st) {
    hipLaunchKernelGGL(k_als_hadamard, dim3(2048), dim3(256), 0, st, R_pad, Ha, Hb, xip);
    return hipGetLastError();
}

hipError_t launch_order_desc(const double* lam, int m, int* order, hipStream_t st) {
    if (m < 1 || m > 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_order_desc, dim3(1), dim3(1024), 0, st, lam, m, order);
    return hipGetLastError();
}
