// a3: FP64 symmetric eigensolver — two-sided block Jacobi on the Gram matrix.
//
// The m_pad x m_pad matrix is cut into nb = m_pad/16 blocks of 16 indices.  One
// step pairs the blocks (round-robin, every pair once per sweep); pair k forms a
// "super-block" S_k of 32 indices.  Per step:
//   phase 1: each 32x32 diagonal sub-problem G[S_k,S_k] is diagonalized
//            completely by a parallel cyclic Jacobi inside one workgroup
//            (each thread owns a 2x2 block; rows/columns move between
//            threads in round-robin order so the active pairs are always
//            the thread-local 2x2 diagonal blocks) -> orthogonal Q_k;
//   phase 2: G <- J^T G J and W <- W J with J = diag(Q_k) (permuted), tile by
//            tile as 32x32x32 FP64 MFMA products: G[S_j,S_k] <- Q_j^T G[S_j,S_k] Q_k
//            (j <= k, mirrored), W[rows,S_k] <- W[rows,S_k] Q_k.
// Rotations are applied only where |G_pq| > tol * |G|_F; a sweep in which no
// sub-problem rotates ends the iteration.  On exit diag(G) holds the
// eigenvalues and the columns of W the eigenvectors.  Every workgroup is
// resident (cooperative launch); phases are separated by grid barriers and
// every workgroup takes the same number of barriers, so the grid always drains.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int SB = 2 * JB;    // 32 indices per super-block
constexpr int LDT = SB + 1;   // LDS leading dimension of 32x32 tiles
constexpr int MAX_INNER = 12; // inner sweeps per sub-problem
constexpr int MAXBLK = 1024;

struct JacobiDev {
    double* G[3];
    double* W[3];
    int nmat;
    int m_pad;
    int max_sweeps;
    double tol;
    double* Q;          // nmat * P * SB*SB (col-major 32x32 each)
    int* qflag;         // nmat * P (1 = Q is not the identity)
    double* partials;   // MAXBLK * 3
    unsigned* bar;      // barrier count, generation
    int* rot;           // per sweep: any rotation applied
    int* sweeps_out;
};

__device__ __forceinline__ int ring(int s, int i, int nb) {
    return i == 0 ? 0 : 1 + ((i - 1 + s) % (nb - 1));
}
// global index of local position p (0..31) of super-block (I, J)
__device__ __forceinline__ int sidx(int I, int J, int p) {
    return p < JB ? I * JB + p : J * JB + (p - JB);
}
// circle-method move of a position (pairs are positions (2i, 2i+1))
__device__ __forceinline__ int next_pos(int p) {
    if (p == 0) return 0;
    if (p == 1) return 2;
    if ((p & 1) == 0) return p < SB - 2 ? p + 2 : SB - 1;
    return p - 2;
}

// ---------------------------------------------------------------------------
// phase 1: diagonalize S = G[S_k, S_k] (32x32), write Q_k
// ---------------------------------------------------------------------------
__device__ void solve_pair(const JacobiDev& d, int mat, int k, int I, int J, double thr, int sweep,
                           double* sm) {
    double* bufS = sm;                 // 32 x LDT
    double* bufQ = sm + SB * LDT;      // 32 x LDT
    double* cs = sm + 2 * SB * LDT;    // 16 cosines
    double* sn = cs + 16;              // 16 sines
    const int m = d.m_pad;
    const double* G = d.G[mat];
    const int t = threadIdx.x, bi = t >> 4, bj = t & 15;
    const int r0 = 2 * bi, c0 = 2 * bj;
    const int gr0 = sidx(I, J, r0), gr1 = sidx(I, J, r0 + 1);
    const int gc0 = sidx(I, J, c0), gc1 = sidx(I, J, c0 + 1);
    double s00 = G[gr0 + (int64_t)gc0 * m], s01 = G[gr0 + (int64_t)gc1 * m];
    double s10 = G[gr1 + (int64_t)gc0 * m], s11 = G[gr1 + (int64_t)gc1 * m];
    double q00 = (bi == bj) ? 1.0 : 0.0, q01 = 0.0, q10 = 0.0, q11 = q00;
    int any = 0;
    for (int isw = 0; isw < MAX_INNER; ++isw) {
        int rot = 0;
        for (int round = 0; round < SB - 1; ++round) {
            int here = 0;
            if (bi == bj) {
                double c = 1.0, s = 0.0;
                if (fabs(s01) > thr) {
                    double zeta = (s11 - s00) / (2.0 * s01);
                    double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = c * tt;
                    here = 1;
                    rot = 1;
                }
                cs[bi] = c;
                sn[bi] = s;
            }
            __syncthreads();
            const double cI = cs[bi], sI = sn[bi], cJ = cs[bj], sJ = sn[bj];
            // S <- R_I^T S R_J,  R = [[c, s], [-s, c]]
            double x00 = s00 * cJ - s01 * sJ, x01 = s00 * sJ + s01 * cJ;
            double x10 = s10 * cJ - s11 * sJ, x11 = s10 * sJ + s11 * cJ;
            double y00 = cI * x00 - sI * x10, y01 = cI * x01 - sI * x11;
            double y10 = sI * x00 + cI * x10, y11 = sI * x01 + cI * x11;
            if (here) { y01 = 0.0; y10 = 0.0; }   // the annihilated pair is exactly zero
            // Q <- Q R_J
            double z00 = q00 * cJ - q01 * sJ, z01 = q00 * sJ + q01 * cJ;
            double z10 = q10 * cJ - q11 * sJ, z11 = q10 * sJ + q11 * cJ;
            const int pr0 = next_pos(r0), pr1 = next_pos(r0 + 1);
            const int pc0 = next_pos(c0), pc1 = next_pos(c0 + 1);
            bufS[pc0 * LDT + pr0] = y00;
            bufS[pc1 * LDT + pr0] = y01;
            bufS[pc0 * LDT + pr1] = y10;
            bufS[pc1 * LDT + pr1] = y11;
            bufQ[pc0 * LDT + r0] = z00;
            bufQ[pc1 * LDT + r0] = z01;
            bufQ[pc0 * LDT + r0 + 1] = z10;
            bufQ[pc1 * LDT + r0 + 1] = z11;
            __syncthreads();
            s00 = bufS[c0 * LDT + r0];
            s01 = bufS[(c0 + 1) * LDT + r0];
            s10 = bufS[c0 * LDT + r0 + 1];
            s11 = bufS[(c0 + 1) * LDT + r0 + 1];
            q00 = bufQ[c0 * LDT + r0];
            q01 = bufQ[(c0 + 1) * LDT + r0];
            q10 = bufQ[c0 * LDT + r0 + 1];
            q11 = bufQ[(c0 + 1) * LDT + r0 + 1];
        }
        rot = __syncthreads_or(rot);
        if (!rot) break;
        any = 1;
    }
    // after whole inner sweeps the positions are back in their original order
    const int P = m / SB;
    double* Qk = d.Q + ((int64_t)mat * P + k) * SB * SB;
    Qk[c0 * SB + r0] = q00;
    Qk[(c0 + 1) * SB + r0] = q01;
    Qk[c0 * SB + r0 + 1] = q10;
    Qk[(c0 + 1) * SB + r0 + 1] = q11;
    if (t == 0) {
        d.qflag[mat * P + k] = any;
        if (any) atomicOr(&d.rot[sweep], 1);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// phase 2 helpers: 32x32x32 FP64 MFMA product, operands in LDS (col-major, LDT)
//   C = op(A) * B, op(A) = A or A^T; wave w computes rows 16*(w>>1), cols 16*(w&1)
// ---------------------------------------------------------------------------
template <bool TRANS_A>
__device__ __forceinline__ d4_t mm32(const double* A, const double* B) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int R0 = 16 * (w >> 1), C0 = 16 * (w & 1);
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < SB / 4; ++kk) {
        const int k = 4 * kk + (lane >> 4);
        const int r = R0 + (lane & 15), c = C0 + (lane & 15);
        double a = TRANS_A ? A[r * LDT + k] : A[k * LDT + r];
        double b = B[c * LDT + k];
        acc = mfma_f64(a, b, acc);
    }
    return acc;
}

__device__ __forceinline__ void load_q(const double* Qg, double* s) {
    for (int e = threadIdx.x; e < SB * SB; e += blockDim.x) s[(e / SB) * LDT + (e % SB)] = Qg[e];
}

__device__ void update_g(const JacobiDev& d, int mat, int j, int k, int Ij, int Jj, int Ik, int Jk,
                         double* sm) {
    const int m = d.m_pad, P = m / SB;
    if (!d.qflag[mat * P + j] && !d.qflag[mat * P + k]) return;
    double* sG = sm;
    double* sQj = sm + SB * LDT;
    double* sQk = sm + 2 * SB * LDT;
    double* sT = sm + 3 * SB * LDT;
    double* G = d.G[mat];
    for (int e = threadIdx.x; e < SB * SB; e += blockDim.x) {
        int r = e % SB, c = e / SB;
        sG[c * LDT + r] = G[sidx(Ij, Jj, r) + (int64_t)sidx(Ik, Jk, c) * m];
    }
    load_q(d.Q + ((int64_t)mat * P + j) * SB * SB, sQj);
    load_q(d.Q + ((int64_t)mat * P + k) * SB * SB, sQk);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int R0 = 16 * (w >> 1), C0 = 16 * (w & 1);
    d4_t t = mm32<false>(sG, sQk);
#pragma unroll
    for (int i = 0; i < 4; ++i) sT[(C0 + c_col(lane)) * LDT + R0 + c_row64(lane, i)] = t[i];
    __syncthreads();
    d4_t y = mm32<true>(sQj, sT);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = R0 + c_row64(lane, i), c = C0 + c_col(lane);
        const int gr = sidx(Ij, Jj, r), gc = sidx(Ik, Jk, c);
        if (j == k) {
            if (r < c) continue;   // diagonal super-block: keep it exactly symmetric
            G[gr + (int64_t)gc * m] = y[i];
            G[gc + (int64_t)gr * m] = y[i];
        } else {
            G[gr + (int64_t)gc * m] = y[i];
            G[gc + (int64_t)gr * m] = y[i];
        }
    }
    __syncthreads();
}

__device__ void update_w(const JacobiDev& d, int mat, int i0, int k, int Ik, int Jk, double* sm) {
    const int m = d.m_pad, P = m / SB;
    if (!d.qflag[mat * P + k]) return;
    double* sW = sm;
    double* sQk = sm + 2 * SB * LDT;
    double* W = d.W[mat];
    for (int e = threadIdx.x; e < SB * SB; e += blockDim.x) {
        int r = e % SB, c = e / SB;
        sW[c * LDT + r] = W[(i0 * SB + r) + (int64_t)sidx(Ik, Jk, c) * m];
    }
    load_q(d.Q + ((int64_t)mat * P + k) * SB * SB, sQk);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int R0 = 16 * (w >> 1), C0 = 16 * (w & 1);
    d4_t y = mm32<false>(sW, sQk);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = R0 + c_row64(lane, i), c = C0 + c_col(lane);
        W[(i0 * SB + r) + (int64_t)sidx(Ik, Jk, c) * m] = y[i];
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_jacobi(JacobiDev d) {
    __shared__ double sm[4 * SB * LDT + 64];
    __shared__ double red[4];
    const unsigned nblk = gridDim.x;
    const int m = d.m_pad, P = m / SB, nb = 2 * P;
    const int64_t mm = (int64_t)m * m;

    // phase 0: W = I and |G|_F
    for (int mat = 0; mat < d.nmat; ++mat) {
        double acc = 0.0;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mm;
             e += (int64_t)nblk * blockDim.x) {
            double g = d.G[mat][e];
            acc += g * g;
            d.W[mat][e] = ((e % m) == (e / m)) ? 1.0 : 0.0;
        }
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) d.partials[blockIdx.x * 3 + mat] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
    grid_barrier(d.bar, d.bar + 1, nblk);
    double thr[3] = {0.0, 0.0, 0.0};
    for (int mat = 0; mat < d.nmat; ++mat) {
        double s = 0.0;
        for (unsigned b = 0; b < nblk; ++b) s += d.partials[b * 3 + mat];
        thr[mat] = d.tol * sqrt(s);
    }

    const int NG = P * (P + 1) / 2, NW = P * P;   // (m/32 row blocks) x P pairs
    int sweep = 0, converged = 0;
    for (; sweep < d.max_sweeps; ++sweep) {
        for (int step = 0; step < nb - 1; ++step) {
            for (int it = blockIdx.x; it < d.nmat * P; it += nblk) {
                const int mat = it / P, k = it % P;
                solve_pair(d, mat, k, ring(step, k, nb), ring(step, nb - 1 - k, nb), thr[mat], sweep, sm);
            }
            grid_barrier(d.bar, d.bar + 1, nblk);
            for (int it = blockIdx.x; it < d.nmat * (NG + NW); it += nblk) {
                const int mat = it / (NG + NW), r = it % (NG + NW);
                if (r < NG) {
                    int kk = (int)((sqrt(8.0 * r + 1.0) - 1.0) * 0.5);
                    while ((kk + 1) * (kk + 2) / 2 <= r) ++kk;
                    while (kk * (kk + 1) / 2 > r) --kk;
                    const int jj = r - kk * (kk + 1) / 2;   // jj <= kk
                    update_g(d, mat, jj, kk, ring(step, jj, nb), ring(step, nb - 1 - jj, nb),
                             ring(step, kk, nb), ring(step, nb - 1 - kk, nb), sm);
                } else {
                    const int q = r - NG, i0 = q / P, kk = q % P;
                    update_w(d, mat, i0, kk, ring(step, kk, nb), ring(step, nb - 1 - kk, nb), sm);
                }
            }
            grid_barrier(d.bar, d.bar + 1, nblk);
        }
        const int any = __hip_atomic_load(&d.rot[sweep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (!any) { converged = 1; ++sweep; break; }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *d.sweeps_out = converged ? sweep : -1;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t jacobi_work_bytes(int nmat, int m_pad, int max_sweeps) {
    const int P = m_pad / SB;
    return align256((size_t)nmat * P * SB * SB * 8) + align256((size_t)nmat * P * 4) +
           align256((size_t)MAXBLK * 3 * 8) + align256(16) + align256((size_t)(max_sweeps + 1) * 4);
}

hipError_t launch_jacobi(const JacobiProblem& p, void* work, size_t work_bytes, int* sweeps_dev,
                         hipStream_t st) {
    if (p.m_pad % SB != 0 || p.nmat < 1 || p.nmat > 3) return hipErrorInvalidValue;
    if (work_bytes < jacobi_work_bytes(p.nmat, p.m_pad, p.max_sweeps)) return hipErrorInvalidValue;
    const int P = p.m_pad / SB;
    JacobiDev d{};
    for (int i = 0; i < 3; ++i) { d.G[i] = p.G[i]; d.W[i] = p.W[i]; }
    d.nmat = p.nmat;
    d.m_pad = p.m_pad;
    d.max_sweeps = p.max_sweeps;
    d.tol = p.tol;
    char* w = (char*)work;
    d.Q = (double*)w;            w += align256((size_t)p.nmat * P * SB * SB * 8);
    d.qflag = (int*)w;           w += align256((size_t)p.nmat * P * 4);
    d.partials = (double*)w;     w += align256((size_t)MAXBLK * 3 * 8);
    d.bar = (unsigned*)w;        w += align256(16);
    d.rot = (int*)w;
    d.sweeps_out = sweeps_dev;
    hipError_t e = hipMemsetAsync(d.bar, 0, 16, st);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(d.rot, 0, (size_t)(p.max_sweeps + 1) * 4, st);
    if (e != hipSuccess) return e;
    int dev = 0, ncu = 0, occ = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_jacobi, 256, 0)) != hipSuccess) return e;
    if (occ < 1) return hipErrorInvalidConfiguration;
    const int NG = P * (P + 1) / 2, NW = P * P;
    int want = p.nmat * (NG + NW);
    int nblk = ncu;                 // one resident workgroup per CU at most
    if (want < nblk) nblk = want;
    if (nblk > MAXBLK) nblk = MAXBLK;
    if (nblk < 1) nblk = 1;
    void* args[] = {&d};
    return hipLaunchCooperativeKernel((const void*)k_jacobi, dim3(nblk), dim3(256), args, 0, st);
}
