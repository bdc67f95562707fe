// Kernels of the learned rank proposal and its randomized range finder.
//
//   features   : the 32 singular values of a Gaussian sketch Y = U~ Omega[:, :32]
//                (from the eigenvalues of Y^T Y) -> log10(sigma_k / sigma_1) / 16,
//                clamped at -1, 32 zeros, ln(n)/10, ln(R)/10, ln(eps)/10
//   pad_omega  : the caller's R x w test matrix into a zero-padded R_pad x cols block
//   lowdin     : Q = Y P Lambda^(-1/2) column scaling (directions with an eigenvalue
//                below rel * max dropped)
//   floor_sum  : fixed-order sum of the residual partial sums per mode
#include "common.hpp"
#include "kernels.hpp"

namespace {

// one block per mode; lam: the 32 eigenvalues of the sketch Gram (any order)
__global__ void k_features(const double* __restrict__ lam0, const double* __restrict__ lam1,
                           const double* __restrict__ lam2, int n, int64_t R, double eps, float* __restrict__ feat) {
    __shared__ double s[32];
    const int l = blockIdx.x, t = threadIdx.x;
    const double* lam = l == 0 ? lam0 : (l == 1 ? lam1 : lam2);
    if (t < 32) s[t] = sqrt(fmax(lam[t], 0.0));
    __syncthreads();
    if (t == 0) {   // 32 values: insertion sort, descending
        for (int i = 1; i < 32; ++i) {
            const double x = s[i];
            int k = i;
            while (k > 0 && s[k - 1] < x) { s[k] = s[k - 1]; --k; }
            s[k] = x;
        }
    }
    __syncthreads();
    float* f = feat + (int64_t)l * NET_IN;
    if (t < 32) {
        const double s1 = s[0];
        double v = -1.0;
        if (s1 > 0.0 && s[t] > 0.0) v = fmax(log10(s[t] / s1) / 16.0, -1.0);
        f[t] = (float)v;
    } else if (t < 64) {
        f[t] = 0.0f;
    } else if (t == 64) {
        f[64] = (float)(log((double)n) / 10.0);
        f[65] = (float)(log((double)R) / 10.0);
        f[66] = (float)(log(eps) / 10.0);
    }
}

__global__ void k_pad_omega(int64_t R, int64_t R_pad, int w, int cols, const double* __restrict__ omega,
                            double* __restrict__ out) {
    const int64_t tot = R_pad * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % R_pad;
        const int j = (int)(e / R_pad);
        out[e] = (i < R && j < w) ? omega[i + (int64_t)j * R] : 0.0;
    }
}

// out[:, j] = P[:, j] / sqrt(mu_j) when mu_j > rel * max(mu), else 0 (mp x mp, ld)
__global__ void k_lowdin(int mp, int ld, const double* __restrict__ mu, const double* __restrict__ P,
                         double* __restrict__ out, double rel) {
    __shared__ double mx;
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int j = 0; j < mp; ++j) v = fmax(v, mu[j]);
        mx = v;
    }
    __syncthreads();
    const double thr = rel * mx;
    const int64_t tot = (int64_t)mp * mp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % mp), j = (int)(e / mp);
        const int64_t o = i + (int64_t)j * ld;
        out[o] = (mu[j] > thr && mu[j] > 0.0) ? P[o] / sqrt(mu[j]) : 0.0;
    }
}

__global__ void k_floor_sum(const double* __restrict__ part, int64_t ntiles, double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < ntiles; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// out[k] = sigma[k]^2, k < r (sorted singular values back to eigenvalues)
__global__ void k_square_prefix(int r, const double* __restrict__ sigma, double* __restrict__ out) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < r; k += gridDim.x * blockDim.x) out[k] = sigma[k] * sigma[k];
}

// out[k] = sum_nu V[k, nu]^2, one thread per row (coalesced across k)
__global__ void k_row_norms2(int p, int ld, int64_t R_pad, const double* __restrict__ V, double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p) return;
    double acc = 0.0;
    for (int64_t nu = 0; nu < R_pad; ++nu) {
        const double v = V[k + nu * ld];
        acc = fma(v, v, acc);
    }
    out[k] = acc;
}

// dst = src with rows >= keep set to zero (ld x R_pad, column-major); dst may be src
template <typename O>
__global__ void k_v_finalize(int keep, int ld, int64_t R_pad, const double* __restrict__ src, O* __restrict__ dst) {
    const int64_t tot = (int64_t)ld * R_pad;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % ld);
        dst[e] = (O)(j < keep ? src[e] : 0.0);
    }
}

}  // namespace

hipError_t launch_square_prefix(int r, const double* sigma, double* out, hipStream_t st) {
    if (r < 1) return hipSuccess;
    hipLaunchKernelGGL(k_square_prefix, dim3((unsigned)((r + 255) / 256)), dim3(256), 0, st, r, sigma, out);
    return hipGetLastError();
}

hipError_t launch_row_norms2(int p, int ld, int64_t R_pad, const double* V, double* out, hipStream_t st) {
    if (p < 1) return hipSuccess;
    hipLaunchKernelGGL(k_row_norms2, dim3((unsigned)((p + 63) / 64)), dim3(64), 0, st, p, ld, R_pad, V, out);
    return hipGetLastError();
}

hipError_t launch_v_finalize(int keep, int ld, int64_t R_pad, const double* src, double* dst64, float* dst32,
                             hipStream_t st) {
    if (dst64)
        hipLaunchKernelGGL(k_v_finalize<double>, dim3(2048), dim3(256), 0, st, keep, ld, R_pad, src, dst64);
    else
        hipLaunchKernelGGL(k_v_finalize<float>, dim3(2048), dim3(256), 0, st, keep, ld, R_pad, src, dst32);
    return hipGetLastError();
}

hipError_t launch_features(const double* const lam[3], int n, int64_t R, double eps, float* feat, hipStream_t st) {
    hipLaunchKernelGGL(k_features, dim3(3), dim3(128), 0, st, lam[0], lam[1], lam[2], n, R, eps, feat);
    return hipGetLastError();
}

hipError_t launch_pad_omega(int64_t R, int64_t R_pad, int w, int cols, const double* omega, double* out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_pad_omega, dim3(512), dim3(256), 0, st, R, R_pad, w, cols, omega, out);
    return hipGetLastError();
}

hipError_t launch_lowdin(int mp, int ld, const double* mu, const double* P, double* out, double rel, hipStream_t st) {
    // one block: the threshold needs max(mu) before any column is scaled
    hipLaunchKernelGGL(k_lowdin, dim3(1), dim3(1024), 0, st, mp, ld, mu, P, out, rel);
    return hipGetLastError();
}

hipError_t launch_floor_sum(const double* part, int64_t ntiles, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_floor_sum, dim3(1), dim3(256), 0, st, part, ntiles, out);
    return hipGetLastError();
}
