// a3: FP64 symmetric eigensolver for the Gram matrices.
//
//   1. Householder tridiagonalization G = H T H^T (H = H_0 ... H_{m-3}),
//      one cooperative kernel: the columns of each matrix live in the
//      registers of a group of workgroups (at most 16 columns per workgroup);
//      per column, the owner forms the reflector, every workgroup computes its
//      part of p = tau G v, then applies the rank-2 update G -= v w^T + w v^T
//      to its own columns.  Per column, v is broadcast and p all-gathered
//      through flag-tagged words; nothing else travels through memory.
//   2. Divide and conquer on T (Cuppen): T is split recursively into blocks of
//      at most 32 (the coupling b = e_mid is removed as T = diag(T1, T2) +
//      b u u^T); leaves are diagonalized by a parallel Jacobi in one
//      workgroup; each merge solves the rank-one update D + rho z z^T:
//      deflation of tiny z_i and of close poles (Givens), the secular equation
//      1 + rho sum z_i^2/(d_i - lambda) = 0 by bisection on lambda - d_origin
//      (origin = the nearer pole, so every d_i - lambda is formed accurately),
//      z recomputed from the roots (Gu & Eisenstat) so the eigenvectors are
//      orthogonal, and the children's eigenvectors multiplied by the merge's
//      eigenvector matrix (FP64 MFMA).  One launch per phase per tree level.
//   3. Back-transformation of the selected eigenvectors by the reflectors.
#include <math.h>

#include <string.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr double U64 = 1.1102230246251565e-16;
constexpr int LEAF = 32;
constexpr int MAXN = 2048;
constexpr int TCOL = 16;   // columns per workgroup in the tridiagonalization (in registers)

__device__ double block_sum256(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// 1. tridiagonalization
// ---------------------------------------------------------------------------
// Matrices of one tridiagonalization launch: matrix q owns blocks
// [blk0, blk0 + bpm), each holding cpb consecutive columns in LDS.
struct TriMat {
    double* G;          // m x m (ld): in the symmetric matrix, out the reflectors below the diagonal
    double* d;          // m
    double* e;          // m - 1
    double* tau;        // m
    uint64_t* x;        // exchange area, tri_xwords(m) words, zero before the launch
    int m, ld, cpb, bpm, blk0;
};
constexpr int TRI_MAXMAT = 24;
struct TriArgs {
    TriMat mat[TRI_MAXMAT];
    int nmat;
    int* abort_w;       // set to 1 when an exchange wait ran out
};

__host__ __device__ constexpr size_t tri_xwords(int m) { return (size_t)8 * ((m + 63) & ~63) + 8; }

// Cross-workgroup exchange of the tridiagonalization.  A double travels as two
// 64-bit words {32 data bits, 32 flag bits}, each written by one agent-scope
// atomic store; a reader polls the words until both carry the flag of the
// current column step, so the data needs no separate barrier or cache
// maintenance.  Buffers alternate by the parity of the step: a slot is
// rewritten two steps later, after every reader has provably consumed it.
// Every wait is bounded: past the spin limit the reader raises the launch's
// abort word, all other waits end at once and the host reports an error.
constexpr int SPIN_LIMIT = 1 << 22;

__device__ __forceinline__ void ll_put(uint64_t* w, double v, uint32_t flag) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    __hip_atomic_store(w, (bits & 0xffffffffull) | ((uint64_t)flag << 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, (bits >> 32) | ((uint64_t)flag << 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ll_ld(const uint64_t* w) {
    return __hip_atomic_load(const_cast<uint64_t*>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ll_val(uint64_t lo, uint64_t hi) {
    return __longlong_as_double((long long)((lo & 0xffffffffull) | (hi << 32)));
}

// Receive N values: value q from the word pair at w[q] (skipped when w[q] is null).
// All pending pairs are loaded together, so one round trip serves every value
// that is already there.
template <int N>
__device__ __forceinline__ void ll_get(const uint64_t* const (&w)[N], double (&out)[N], uint32_t flag,
                                       int* abort_w) {
    bool ready[N];
#pragma unroll
    for (int q = 0; q < N; ++q) ready[q] = (w[q] == nullptr);
    for (int spin = 0;; ++spin) {
        uint64_t lo[N], hi[N];
#pragma unroll
        for (int q = 0; q < N; ++q)
            if (!ready[q]) {
                lo[q] = ll_ld(w[q]);
                hi[q] = ll_ld(w[q] + 1);
            }
        bool all = true;
#pragma unroll
        for (int q = 0; q < N; ++q)
            if (!ready[q]) {
                if ((uint32_t)(lo[q] >> 32) == flag && (uint32_t)(hi[q] >> 32) == flag) {
                    out[q] = ll_val(lo[q], hi[q]);
                    ready[q] = true;
                } else {
                    all = false;
                }
            }
        if (all) return;
        if ((spin & 63) == 63) {
            if (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || spin > SPIN_LIMIT) {
                __hip_atomic_store(abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int q = 0; q < N; ++q)
                    if (!ready[q]) out[q] = 0.0;
                return;
            }
        }
    }
}

// word offsets inside a matrix's exchange area (a word pair per value; v and p
// by row, per step parity)
__device__ __forceinline__ uint64_t* xv(const TriMat& M, int par) { return M.x + (size_t)par * 2 * ((M.m + 63) & ~63); }
__device__ __forceinline__ uint64_t* xp(const TriMat& M, int par) {
    return M.x + (size_t)(2 + par) * 2 * ((M.m + 63) & ~63);
}
__device__ __forceinline__ uint64_t* xtau(const TriMat& M, int par) {
    return M.x + (size_t)8 * ((M.m + 63) & ~63) + 2 * par;
}

// Block sum over NT threads (4 or 8 waves), added in a fixed order, so that every
// workgroup that sums the same values gets the same result.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    constexpr int NW = NT / 64;
    static_assert(NW == 4 || NW == 8, "4 or 8 waves");
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = (red[0] + red[1]) + (red[2] + red[3]);
    if constexpr (NW == 8) s += (red[4] + red[5]) + (red[6] + red[7]);
    __syncthreads();
    return s;
}

// Sums of 16 values across the wave at once: four halving butterfly steps
// (each lane keeps half of its values and adds its partner's copy of that
// half) and two last pairwise adds.  Lane l ends with the wave total of value
// l >> 2.  18 shuffles instead of 16 separate 6-step reductions.
__device__ __forceinline__ double wave_sum16(const double (&a)[16], int lane) {
    double b8[8], b4[4], b2[2];
    {
        const bool h = lane & 32;
#pragma unroll
        for (int j = 0; j < 8; ++j) b8[j] = (h ? a[j + 8] : a[j]) + __shfl_xor(h ? a[j] : a[j + 8], 32, WAVE);
    }
    {
        const bool h = lane & 16;
#pragma unroll
        for (int j = 0; j < 4; ++j) b4[j] = (h ? b8[j + 4] : b8[j]) + __shfl_xor(h ? b8[j] : b8[j + 4], 16, WAVE);
    }
    {
        const bool h = lane & 8;
#pragma unroll
        for (int j = 0; j < 2; ++j) b2[j] = (h ? b4[j + 2] : b4[j]) + __shfl_xor(h ? b4[j] : b4[j + 2], 8, WAVE);
    }
    const bool h = lane & 4;
    double b1 = (h ? b2[1] : b2[0]) + __shfl_xor(h ? b2[0] : b2[1], 4, WAVE);
    b1 += __shfl_xor(b1, 2, WAVE);
    return b1 + __shfl_xor(b1, 1, WAVE);
}

// Reflector j from column j (this thread's rows t + NT q in x, already updated
// by every step before j): v (rows j+1..m-1, v[j+1] = 1) and tau are sent for
// step j; G[:, j] below the diagonal, tau_j, e_j = beta and d_j are stored for
// the later kernels.  bc: one shared word for the broadcast of x[j+1].
template <int RPT, int NT>
__device__ __forceinline__ void send_reflector(const double (&x)[RPT], int j, const TriMat& M, double* red,
                                               double* bc) {
    const int t = threadIdx.x, m = M.m;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = t + NT * q;
        if (i > j + 1 && i < m) s += x[q] * x[q];
        if (i == j + 1) bc[0] = x[q];
        if (i == j) M.d[j] = x[q];
    }
    s = block_sum<NT>(s, red);   // its barriers publish bc[0]
    const double alpha = bc[0];
    double tau, beta, scal;
    if (s == 0.0) {
        tau = 0.0; beta = alpha; scal = 0.0;
    } else {
        const double nrm = sqrt(alpha * alpha + s);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
    }
    const uint32_t flag = (uint32_t)j + 1;
    uint64_t* vx = xv(M, j & 1);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = t + NT * q;
        if (i > j && i < m) {
            const double v = (i == j + 1) ? 1.0 : x[q] * scal;
            ll_put(vx + 2 * i, v, flag);
            M.G[i + (int64_t)j * M.ld] = v;
        }
    }
    if (t == 0) {
        ll_put(xtau(M, j & 1), tau, flag);
        M.tau[j] = tau;
        M.e[j] = beta;
    }
}

// One-sided Householder tridiagonalization H^T G H = T, column-distributed:
// step k broadcasts v_k, every block forms p_j = tau (G v)_j for its columns,
// the p_j and the per-block sums of p_j v_j are all-gathered, and each block
// applies G <- G - v w^T - w v^T with w = p - (tau/2)(p.v) v to its columns.
// The owner of column k+1 then forms reflector k+1 from it and sends it.
// Each block keeps its (at most TCOL) columns in registers: thread t holds rows
// t + NT q, q < RPT, of every column and vector, so neither the dot products
// nor the updates touch memory; rows >= m are zero, v_k and w_k are zero on
// rows <= k, and a column that is not live takes a zero update, so the loops
// run over every register column without bounds or branches.
template <int RPT, int NT>
__global__ __launch_bounds__(NT) void k_tridiag(TriArgs a) {
    constexpr int NW = NT / 64;
    __shared__ double red[NW];
    __shared__ double red2[TCOL * NW];
    __shared__ double vjs[TCOL], wjs[TCOL], pjs[TCOL];
    __shared__ double bc[1];
    static_assert(TCOL == 16, "one butterfly reduction covers the columns");
    int q0 = 0;
    while (q0 + 1 < a.nmat && (int)blockIdx.x >= a.mat[q0 + 1].blk0) ++q0;
    const TriMat& M = a.mat[q0];
    const int gb = blockIdx.x - M.blk0;
    if (gb >= M.bpm) return;
    const int m = M.m, ld = M.ld, cpb = M.cpb;
    const int c0 = gb * cpb;
    const int nc = max(0, min(cpb, m - c0));
    const int t = threadIdx.x, lane = t & 63;
    double C[TCOL][RPT];
#pragma unroll
    for (int c = 0; c < TCOL; ++c)
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = t + NT * q;
            C[c][q] = (c < nc && i < m) ? M.G[i + (int64_t)(c0 + c) * ld] : 0.0;
        }
    if (m > 2 && c0 == 0 && nc > 0) send_reflector<RPT, NT>(C[0], 0, M, red, bc);
    for (int k = 0; k + 2 < m; ++k) {
        // every own column is final (none > k): leave
        if (c0 + nc <= k + 1) break;
        const int par = k & 1;
        const uint32_t flag = (uint32_t)k + 1;
        // receive v_k (this thread's rows > k) and tau_k in one poll
        double vr[RPT];
        double tau;
        {
            const uint64_t* w[RPT + 1];
            double val[RPT + 1];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = t + NT * q;
                w[q] = (i > k && i < m) ? xv(M, par) + 2 * i : nullptr;
                val[q] = 0.0;
            }
            w[RPT] = xtau(M, par);
            ll_get<RPT + 1>(w, val, flag, a.abort_w);
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = t + NT * q;
                vr[q] = val[q];
                if (i >= c0 && i < c0 + nc) vjs[i - c0] = vr[q];
            }
            tau = val[RPT];
        }
        const int cs = max(0, k + 1 - c0);   // first local column with j > k
        const int cn = k + 1 - c0;           // local index of column k+1
        // p_j = tau sum_i G[i,j] v_i for own columns j > k (exchanged even when
        // tau = 0: the all-gather of p orders the reuse of the step buffers)
        double acc[TCOL];
#pragma unroll
        for (int c = 0; c < TCOL; ++c) {
            acc[c] = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) acc[c] += C[c][q] * vr[q];
        }
        const double sw = wave_sum16(acc, lane);   // lane l: column l >> 2
        if ((lane & 3) == 0) red2[(lane >> 2) * NW + (t >> 6)] = sw;
        __syncthreads();   // red2, vjs
        if (t < nc && t >= cs) {
            double sp = (red2[t * NW] + red2[t * NW + 1]) + (red2[t * NW + 2] + red2[t * NW + 3]);
            if constexpr (NW == 8)
                sp += (red2[t * NW + 4] + red2[t * NW + 5]) + (red2[t * NW + 6] + red2[t * NW + 7]);
            const double pj = tau * sp;
            ll_put(xp(M, par) + 2 * (c0 + t), pj, flag);
            pjs[t] = pj;
        }
        // receive p (this thread's rows > k)
        double pr[RPT], partial = 0.0;
        {
            const uint64_t* w[RPT];
            double val[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = t + NT * q;
                w[q] = (i > k && i < m) ? xp(M, par) + 2 * i : nullptr;
                val[q] = 0.0;
            }
            ll_get<RPT>(w, val, flag, a.abort_w);
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                pr[q] = val[q];
                partial += pr[q] * vr[q];
            }
        }
        // p.v over all rows, by the same threads in the same order in every
        // workgroup of the matrix, so the sum does not depend on how the
        // columns are split among workgroups (and needs no exchange of its own)
        const double cw = 0.5 * tau * block_sum<NT>(partial, red);
        if (t >= cs && t < nc) wjs[t] = pjs[t] - cw * vjs[t];
        __syncthreads();
        double wr[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) wr[q] = pr[q] - cw * vr[q];
        // the owner's column k+1 first, then its reflector goes out; then the rest
        if (cn >= 0 && cn < nc) {
            const double wc = wjs[cn], vc = vjs[cn];
            double x[RPT] = {};
#pragma unroll
            for (int c = 0; c < TCOL; ++c)
                if (c == cn) {
#pragma unroll
                    for (int q = 0; q < RPT; ++q) {
                        C[c][q] -= vr[q] * wc + wr[q] * vc;
                        x[q] = C[c][q];
                    }
                }
            if (k + 3 < m) send_reflector<RPT, NT>(x, k + 1, M, red, bc);
        }
#pragma unroll
        for (int c = 0; c < TCOL; ++c) {
            const bool live = c > cn && c >= cs && c < nc;
            const double wc = live ? wjs[c] : 0.0, vc = live ? vjs[c] : 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) C[c][q] -= vr[q] * wc + wr[q] * vc;
        }
        __syncthreads();   // vjs, wjs, pjs are rewritten next step
    }
    // the last 2 x 2 block (and T itself when m <= 2), from the registers
#pragma unroll
    for (int c = 0; c < TCOL; ++c) {
        const int j = c0 + c;
        if (c < nc && j >= m - 2) {
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = t + NT * q;
                if (i == j) M.d[j] = C[c][q];
                if (j == m - 2 && i == j + 1) M.e[j] = C[c][q];
            }
        }
    }
}

// rows per thread and threads per workgroup: 256 threads up to m = 1024, 512
// beyond, and the smallest RPT with NT RPT >= m (1..4)
static int tri_nt(int m) { return m <= 1024 ? 256 : 512; }
static int tri_rpt(int m) { return std::max(1, (m + tri_nt(m) - 1) / tri_nt(m)); }

static const void* tri_kernel(int rpt, int nt) {
    if (nt == 256) {
        switch (rpt) {
            case 1: return (const void*)k_tridiag<1, 256>;
            case 2: return (const void*)k_tridiag<2, 256>;
            case 3: return (const void*)k_tridiag<3, 256>;
            default: return (const void*)k_tridiag<4, 256>;
        }
    }
    return rpt <= 3 ? (const void*)k_tridiag<3, 512> : (const void*)k_tridiag<4, 512>;
}

__global__ void k_zero_words(uint64_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// 2. divide and conquer
// ---------------------------------------------------------------------------
struct Node {
    int mat, lo, mid, hi;     // leaf: mid == hi
    long long soff;           // byte offset of the node's scratch (merge nodes)
};

struct DCArgs {
    const Node* nodes;        // nodes of this pass
    int nnodes;
    const EigMat* mats;       // matrix table
    char* scratch;            // per-node scratch (node_scratch_bytes(n) each)
};

// node scratch: header, then 8 arrays of n doubles (D, z, dd, zk, tau, zh, rc x 2)
// and 5 arrays of n ints (perm, keep, org, rp x 2)
struct NodeScratch {
    double rho;
    double sgn;
    int k;
    int nrot;
    int pad[2];
};
__host__ __device__ constexpr size_t node_scratch_bytes(int n) {
    return (sizeof(NodeScratch) + (size_t)8 * n * sizeof(double) + (size_t)5 * n * sizeof(int) + 255) & ~(size_t)255;
}
__device__ __forceinline__ NodeScratch* ns_head(const DCArgs& a, int node) {
    return (NodeScratch*)(a.scratch + a.nodes[node].soff);
}
__device__ __forceinline__ int ns_n(const DCArgs& a, int node) { return a.nodes[node].hi - a.nodes[node].lo; }
__device__ __forceinline__ double* ns_D(const DCArgs& a, int node) { return (double*)(ns_head(a, node) + 1); }
__device__ __forceinline__ double* ns_z(const DCArgs& a, int node) { return ns_D(a, node) + ns_n(a, node); }
__device__ __forceinline__ double* ns_dd(const DCArgs& a, int node) { return ns_D(a, node) + 2 * ns_n(a, node); }
__device__ __forceinline__ double* ns_zk(const DCArgs& a, int node) { return ns_D(a, node) + 3 * ns_n(a, node); }
__device__ __forceinline__ double* ns_tau(const DCArgs& a, int node) { return ns_D(a, node) + 4 * ns_n(a, node); }
__device__ __forceinline__ double* ns_zh(const DCArgs& a, int node) { return ns_D(a, node) + 5 * ns_n(a, node); }
__device__ __forceinline__ double* ns_rc(const DCArgs& a, int node) { return ns_D(a, node) + 6 * ns_n(a, node); }   // 2n
__device__ __forceinline__ int* ns_perm(const DCArgs& a, int node) { return (int*)(ns_D(a, node) + 8 * ns_n(a, node)); }
__device__ __forceinline__ int* ns_keep(const DCArgs& a, int node) { return ns_perm(a, node) + ns_n(a, node); }
__device__ __forceinline__ int* ns_org(const DCArgs& a, int node) { return ns_perm(a, node) + 2 * ns_n(a, node); }
__device__ __forceinline__ int* ns_rp(const DCArgs& a, int node) { return ns_perm(a, node) + 3 * ns_n(a, node); }    // 2n

// leaves: dense Jacobi on the (<= 32) tridiagonal block, one workgroup each
__device__ __forceinline__ int next_pos32(int p) {
    if (p == 0) return 0;
    if (p == 1) return 2;
    if ((p & 1) == 0) return p < 30 ? p + 2 : 31;
    return p - 2;
}

__global__ __launch_bounds__(256) void k_dc_leaves(DCArgs a) {
    __shared__ double bufS[32 * 33];
    __shared__ double bufQ[32 * 33];
    __shared__ double cs[16], sn[16];
    __shared__ double red[4];
    const Node nd = a.nodes[blockIdx.x];
    const int n = nd.hi - nd.lo;
    const EigMat& mt = a.mats[nd.mat];
    const double* d = mt.d + nd.lo;
    const double* e = mt.e + nd.lo;
    const int t = threadIdx.x, bi = t >> 4, bj = t & 15;
    const int r0 = 2 * bi, c0 = 2 * bj;
    auto T = [&](int r, int c) -> double {
        if (r >= n || c >= n) return 0.0;
        if (r == c) return d[r];
        if (r == c + 1) return e[c];
        if (c == r + 1) return e[r];
        return 0.0;
    };
    double s00 = T(r0, c0), s01 = T(r0, c0 + 1), s10 = T(r0 + 1, c0), s11 = T(r0 + 1, c0 + 1);
    double q00 = (bi == bj) ? 1.0 : 0.0, q01 = 0.0, q10 = 0.0, q11 = q00;
    double f2 = s00 * s00 + s01 * s01 + s10 * s10 + s11 * s11;
    f2 = block_sum256(f2, red);
    const double thr = 0.5 * U64 * sqrt(f2);
    for (int isw = 0; isw < 40; ++isw) {
        int rot = 0;
        for (int round = 0; round < 31; ++round) {
            int here = 0;
            if (bi == bj) {
                double c = 1.0, s = 0.0;
                if (fabs(s01) > thr) {
                    const double zeta = (s11 - s00) / (2.0 * s01);
                    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
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
            const double x00 = s00 * cJ - s01 * sJ, x01 = s00 * sJ + s01 * cJ;
            const double x10 = s10 * cJ - s11 * sJ, x11 = s10 * sJ + s11 * cJ;
            double y00 = cI * x00 - sI * x10, y01 = cI * x01 - sI * x11;
            double y10 = sI * x00 + cI * x10, y11 = sI * x01 + cI * x11;
            if (here) { y01 = 0.0; y10 = 0.0; }
            const double z00 = q00 * cJ - q01 * sJ, z01 = q00 * sJ + q01 * cJ;
            const double z10 = q10 * cJ - q11 * sJ, z11 = q10 * sJ + q11 * cJ;
            const int pr0 = next_pos32(r0), pr1 = next_pos32(r0 + 1);
            const int pc0 = next_pos32(c0), pc1 = next_pos32(c0 + 1);
            bufS[pc0 * 33 + pr0] = y00;
            bufS[pc1 * 33 + pr0] = y01;
            bufS[pc0 * 33 + pr1] = y10;
            bufS[pc1 * 33 + pr1] = y11;
            bufQ[pc0 * 33 + r0] = z00;
            bufQ[pc1 * 33 + r0] = z01;
            bufQ[pc0 * 33 + r0 + 1] = z10;
            bufQ[pc1 * 33 + r0 + 1] = z11;
            __syncthreads();
            s00 = bufS[c0 * 33 + r0];
            s01 = bufS[(c0 + 1) * 33 + r0];
            s10 = bufS[c0 * 33 + r0 + 1];
            s11 = bufS[(c0 + 1) * 33 + r0 + 1];
            q00 = bufQ[c0 * 33 + r0];
            q01 = bufQ[(c0 + 1) * 33 + r0];
            q10 = bufQ[c0 * 33 + r0 + 1];
            q11 = bufQ[(c0 + 1) * 33 + r0 + 1];
        }
        if (!__syncthreads_or(rot)) break;
    }
    // eigenvalues on the diagonal (positions are back in order after whole sweeps)
    double* lam = mt.lam + nd.lo;
    double* Q = mt.Q;
    const int ld = mt.ld;
    if (bi == bj) {
        if (r0 < n) lam[r0] = s00;
        if (r0 + 1 < n) lam[r0 + 1] = s11;
    }
    const double qv[4] = {q00, q01, q10, q11};
    for (int u = 0; u < 4; ++u) {
        const int r = r0 + (u >> 1), c = c0 + (u & 1);
        if (r < n && c < n) Q[(nd.lo + r) + (int64_t)(nd.lo + c) * ld] = qv[u];
    }
}

// phase A (one workgroup per node): z, sort, deflation.  The deflation scan is
// sequential where a close-pole rotation occurs (a rotation changes the next
// comparison).  All threads first test every consecutive pair of undeflated
// entries with the unrotated values: when no pair calls for a rotation the
// scan's result is the compacted list of undeflated entries, formed in
// parallel; otherwise one thread runs the scan.  Both work on LDS copies of D
// and z, written out afterwards by all threads.
__global__ __launch_bounds__(256) void k_dc_prep(DCArgs a) {
    __shared__ double key[MAXN];
    __shared__ int idx[MAXN];
    __shared__ double zs[MAXN];
    __shared__ int keep_s[MAXN];
    __shared__ double red[4];
    __shared__ int s_k, s_rot;
    __shared__ int cnt_s[256];
    const int node = blockIdx.x;
    const Node nd = a.nodes[node];
    const int n1 = nd.mid - nd.lo, n = nd.hi - nd.lo;
    const int t = threadIdx.x;
    const EigMat& mt = a.mats[nd.mat];
    const double* lam = mt.lam + nd.lo;
    const double* Q = mt.Q;
    const int ld = mt.ld;
    double rho = 2.0 * mt.e[nd.mid - 1];
    const double sgn = rho < 0.0 ? -1.0 : 1.0;
    rho = fabs(rho);
    const double rs2 = 0.7071067811865476;
    int N2 = 1;
    while (N2 < n) N2 <<= 1;
    double* z = ns_z(a, node);
    for (int i = t; i < N2; i += 256) {
        key[i] = (i < n) ? sgn * lam[i] : INFINITY;
        idx[i] = i;
    }
    __syncthreads();
    for (int size = 2; size <= N2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < N2; i += 256) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool asc = ((i & size) == 0);
                    const double ki = key[i], kj = key[j];
                    const int ii = idx[i], ij = idx[j];
                    const bool i_first = (ki < kj) || (ki == kj && ii < ij);
                    if (asc ? !i_first : i_first) {
                        key[i] = kj; key[j] = ki;
                        idx[i] = ij; idx[j] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    double* D = ns_D(a, node);
    int* perm = ns_perm(a, node);
    double mx = 0.0;
    for (int s = t; s < n; s += 256) {
        const int i = idx[s];
        perm[s] = i;
        // column lo+i: last row of child 1 (row mid-1) or first row of child 2 (row mid)
        const int row = (i < n1) ? nd.mid - 1 : nd.mid;
        zs[s] = rs2 * Q[row + (int64_t)(nd.lo + i) * ld];
        mx = fmax(mx, fabs(key[s]));
    }
    mx = wave_max(mx);
    if ((t & 63) == 0) red[t >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double tol = 8.0 * U64 * fmax(mx, rho);
    // undeflated entries of this thread's range, compacted in order
    const int per = (n + 255) / 256, b0 = min(n, t * per), b1 = min(n, b0 + per);
    int c = 0;
    for (int i = b0; i < b1; ++i) c += fabs(rho * zs[i]) > tol;
    cnt_s[t] = c;
    if (t == 0) s_rot = 0;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int q = 0; q < 256; ++q) {
            const int v = cnt_s[q];
            cnt_s[q] = acc;
            acc += v;
        }
        s_k = acc;
    }
    __syncthreads();
    {
        int o = cnt_s[t];
        for (int i = b0; i < b1; ++i)
            if (fabs(rho * zs[i]) > tol) keep_s[o++] = i;
    }
    __syncthreads();
    for (int q = t + 1; q < s_k; q += 256) {
        const int pv = keep_s[q - 1], i = keep_s[q];
        const double tt = hypot(zs[pv], zs[i]);
        const double cc = zs[i] / tt, ss = -zs[pv] / tt;
        if (fabs((key[i] - key[pv]) * cc * ss) <= tol) s_rot = 1;
    }
    __syncthreads();
    if (t == 0 && !s_rot) {
        NodeScratch* h = ns_head(a, node);
        h->rho = rho;
        h->sgn = sgn;
        h->k = s_k;
        h->nrot = 0;
    }
    if (t == 0 && s_rot) {
        // the scan over the undeflated entries (keep_s, in order: an entry that is
        // not yet visited still has its original z, so the parallel deflation test
        // holds for it); prev's values travel in registers, and the next eight
        // entries are read from LDS ahead of the dependent arithmetic.  keep_s is
        // rewritten in place: position k < q when entry q is read.
        double* rc = ns_rc(a, node);
        int* rp = ns_rp(a, node);
        double* Dl = key;
        const int K0 = s_k;
        int k = 0, nrot = 0;
        int prev = K0 > 0 ? keep_s[0] : -1;
        double zp = prev >= 0 ? zs[prev] : 0.0, dp = prev >= 0 ? Dl[prev] : 0.0;
        for (int q0 = 1; q0 < K0; q0 += 8) {
            const int cnt = min(8, K0 - q0);
            int ii[8];
            double zz[8], dv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) ii[u] = u < cnt ? keep_s[q0 + u] : 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                zz[u] = zs[ii[u]];
                dv[u] = Dl[ii[u]];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (u >= cnt) break;
                const int i = ii[u];
                const double zi = zz[u], di = dv[u];
                const double tt = hypot(zp, zi);
                const double c = zi / tt, s = -zp / tt;
                if (fabs((di - dp) * c * s) <= tol) {
                    // close poles: rotate so that z[prev] = 0 and deflate prev
                    const double dnew = dp * s * s + di * c * c;
                    Dl[prev] = dp * c * c + di * s * s;
                    Dl[i] = dnew;
                    zs[i] = tt;
                    zs[prev] = 0.0;
                    rp[2 * nrot] = prev;
                    rp[2 * nrot + 1] = i;
                    rc[2 * nrot] = c;
                    rc[2 * nrot + 1] = s;
                    ++nrot;
                    prev = i;
                    zp = tt;
                    dp = dnew;
                } else {
                    keep_s[k++] = prev;
                    prev = i;
                    zp = zi;
                    dp = di;
                }
            }
        }
        if (prev >= 0) keep_s[k++] = prev;
        s_k = k;
        NodeScratch* h = ns_head(a, node);
        h->rho = rho;
        h->sgn = sgn;
        h->k = k;
        h->nrot = nrot;
    }
    __syncthreads();
    const int k = s_k;
    double* dd = ns_dd(a, node);
    double* zk = ns_zk(a, node);
    for (int s = t; s < n; s += 256) {
        D[s] = key[s];
        z[s] = zs[s];
    }
    int* keep = ns_keep(a, node);
    for (int q = t; q < k; q += 256) {
        keep[q] = keep_s[q];
        dd[q] = key[keep_s[q]];
        zk[q] = zs[keep_s[q]];
    }
}

// phase B: secular roots; one wave per root, nodes x roots flattened in y.  The
// workgroup's four waves share one LDS copy of the poles and of z^2.
__global__ __launch_bounds__(256) void k_dc_roots(DCArgs a) {
    __shared__ double s_dd[MAXN];
    __shared__ double s_z2[MAXN];
    const int node = blockIdx.y;
    const NodeScratch* h = ns_head(a, node);
    const int k = h->k;
    if ((int)blockIdx.x * 4 >= k) return;   // uniform across the workgroup
    const double* dd = ns_dd(a, node);
    const double* zk = ns_zk(a, node);
    for (int i = threadIdx.x; i < k; i += 256) {
        s_dd[i] = dd[i];
        s_z2[i] = zk[i] * zk[i];
    }
    __syncthreads();
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= k) return;
    const double rho = h->rho;
    double zz2 = 0.0;
    for (int i = lane; i < k; i += 64) zz2 += s_z2[i];
    zz2 = wave_sum(zz2);
    const double lo_pole = s_dd[j];
    const double hi_pole = (j + 1 < k) ? s_dd[j + 1] : s_dd[j] + rho * zz2;
    int o = j;
    if (j + 1 < k) {
        const double mid = 0.5 * (hi_pole - lo_pole);
        double f = 0.0;
        for (int i = lane; i < k; i += 64) f += s_z2[i] / ((s_dd[i] - lo_pole) - mid);
        f = 1.0 + rho * wave_sum(f);
        o = (f > 0.0) ? j : j + 1;
    }
    // f(t) = 1 + rho sum z_i^2 / ((d_i - d_o) - t) increases between the poles.
    // Bisection until the bracket is 2^-20 of its first width, then Newton steps
    // kept inside the bracket (which every evaluation narrows; a step leaving it is
    // replaced by the midpoint) until a step falls below two ulps of t or no double
    // is left inside the bracket.
    const double dorg = s_dd[o];
    double lo = lo_pole - dorg, hi = hi_pole - dorg;
    const double w0 = hi - lo;
    for (int it = 0; it < 200; ++it) {
        const double tm = 0.5 * (lo + hi);
        if (tm == lo || tm == hi || hi - lo <= w0 * 0x1p-20) break;
        double f = 0.0;
        for (int i = lane; i < k; i += 64) f += s_z2[i] / ((s_dd[i] - dorg) - tm);
        f = 1.0 + rho * wave_sum(f);
        if (f > 0.0) hi = tm;
        else lo = tm;
    }
    double tm = 0.5 * (lo + hi);
    for (int it = 0; it < 64; ++it) {
        if (tm == lo || tm == hi) break;
        double f = 0.0, fp = 0.0;
        for (int i = lane; i < k; i += 64) {
            const double inv = 1.0 / ((s_dd[i] - dorg) - tm);
            const double q = s_z2[i] * inv;
            f += q;
            fp += q * inv;
        }
        f = 1.0 + rho * wave_sum(f);
        fp = rho * wave_sum(fp);
        if (f == 0.0) break;
        if (f > 0.0) hi = tm;
        else lo = tm;
        double nt = tm - f / fp;
        if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
        const bool small = fabs(nt - tm) <= 2.0 * U64 * fabs(nt);
        tm = nt;
        if (small) break;
    }
    if (lane == 0) {
        ns_tau(a, node)[j] = tm;
        ns_org(a, node)[j] = o;
    }
}

// phase C1: z-hat (Gu & Eisenstat), one thread per i
__global__ __launch_bounds__(256) void k_dc_zhat(DCArgs a) {
    const int node = blockIdx.y;
    const NodeScratch* h = ns_head(a, node);
    const int k = h->k;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= k) return;
    const double* dd = ns_dd(a, node);
    const double* zk = ns_zk(a, node);
    const double* tau = ns_tau(a, node);
    const int* org = ns_org(a, node);
    const double rho = h->rho;
    // delta(i,j) = d_i - lambda_j = (d_i - d_org(j)) - tau_j ;  lambda_j - d_i = -delta
    auto lmd = [&](int jj) { return -((dd[i] - dd[org[jj]]) - tau[jj]); };
    double prod = lmd(k - 1) / rho;
    for (int jj = 0; jj < k - 1; ++jj) {
        const double den = (jj < i) ? dd[jj] - dd[i] : dd[jj + 1] - dd[i];
        prod *= lmd(jj) / den;
    }
    ns_zh(a, node)[i] = copysign(sqrt(fmax(prod, 0.0)), zk[i]);
}

// phase C2: merge matrix M (n x n at the node's block of a.M), one wave per column.
// Columns are in sorted coordinates; rows are mapped back through perm; the
// Givens rotations of the close-pole deflation are applied to the rows.
__global__ __launch_bounds__(256) void k_dc_vectors(DCArgs a) {
    const int node = blockIdx.y;
    const Node nd = a.nodes[node];
    const NodeScratch* h = ns_head(a, node);
    const int n = nd.hi - nd.lo, k = h->k, nrot = h->nrot;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (col >= n) return;
    __shared__ double xs[4][MAXN];
    double* x = xs[threadIdx.x >> 6];
    const int* keep = ns_keep(a, node);
    const double* dd = ns_dd(a, node);
    const double* tau = ns_tau(a, node);
    const int* org = ns_org(a, node);
    const double* zh = ns_zh(a, node);
    const double* D = ns_D(a, node);
    for (int i = lane; i < n; i += 64) x[i] = 0.0;
    // is this sorted column a kept one?  keep[] is increasing: binary search
    int lo = 0, hi = k;
    while (lo < hi) {
        const int md = (lo + hi) >> 1;
        if (keep[md] < col) lo = md + 1;
        else hi = md;
    }
    const bool kept = (lo < k && keep[lo] == col);
    double lamc;
    if (kept) {
        const int jc = lo;
        double nrm = 0.0;
        for (int q = lane; q < k; q += 64) {
            const double delta = (dd[q] - dd[org[jc]]) - tau[jc];
            const double u = zh[q] / delta;
            nrm += u * u;
        }
        nrm = sqrt(wave_sum(nrm));
        for (int q = lane; q < k; q += 64) {
            const double delta = (dd[q] - dd[org[jc]]) - tau[jc];
            x[keep[q]] = zh[q] / delta / nrm;
        }
        lamc = dd[org[jc]] + tau[jc];
    } else {
        if (lane == 0) x[col] = 1.0;
        lamc = D[col];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // rows <- R_1 R_2 ... R_t x : apply the rotations in reverse order
    if (lane == 0) {
        const double* rc = ns_rc(a, node);
        const int* rp = ns_rp(a, node);
        for (int q = nrot - 1; q >= 0; --q) {
            const int p = rp[2 * q], i = rp[2 * q + 1];
            const double c = rc[2 * q], s = rc[2 * q + 1];
            const double xp = x[p], xi = x[i];
            x[p] = c * xp - s * xi;
            x[i] = s * xp + c * xi;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int* perm = ns_perm(a, node);
    const EigMat& mt = a.mats[nd.mat];
    double* M = mt.M;
    const int ld = mt.ld;
    for (int s = lane; s < n; s += 64) M[(nd.lo + perm[s]) + (int64_t)(nd.lo + col) * ld] = x[s];
    if (lane == 0) mt.lam[nd.lo + col] = h->sgn * lamc;
}

// phase D: Qn[rows of child c, lo:hi] = Q[child block] * M[child rows, lo:hi]
// (block-diagonal product), masked FP64 MFMA tiles of 64 x 64; one tile per block.
struct GemmTask {
    int mat, r0, nr, c0, nc, k0, nk;   // rows [r0, r0+nr), cols [c0, c0+nc), k range [k0, k0+nk)
};

__global__ __launch_bounds__(256) void k_dc_gemm(DCArgs a, const GemmTask* tasks) {
    __shared__ double sA[16][68];
    __shared__ double sB[16][68];
    const GemmTask tk = tasks[blockIdx.y];
    const int tiles_n = (tk.nc + 63) / 64;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= tk.nr) return;
    const EigMat& mt = a.mats[tk.mat];
    const int ld = mt.ld;
    const double* Q = mt.Q;
    const double* M = mt.M;
    double* Qn = mt.Qn;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    d4_t acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int rbase = tk.r0 + tm * 64, cbase = tk.c0 + tn * 64;
    for (int kb = 0; kb < tk.nk; kb += 16) {
        for (int q = 0; q < 4; ++q) {
            const int kk = (t >> 6) + 4 * q, i = t & 63;
            const int gr = rbase + i, gk = tk.k0 + kb + kk;
            sA[kk][i] = (rbase + i < tk.r0 + tk.nr && kb + kk < tk.nk) ? Q[gr + (int64_t)gk * ld] : 0.0;
            const int gc = cbase + i;
            sB[kk][i] = (cbase + i < tk.c0 + tk.nc && kb + kk < tk.nk) ? M[gk + (int64_t)gc * ld] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = kk * 4 + (lane >> 4);
            const double a0 = sA[k][wr + (lane & 15)], a1 = sA[k][wr + 16 + (lane & 15)];
            const double b0 = sB[k][wc + (lane & 15)], b1 = sB[k][wc + 16 + (lane & 15)];
            acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
            acc[0][1] = mfma_f64(a0, b1, acc[0][1]);
            acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
            acc[1][1] = mfma_f64(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int i = 0; i < 4; ++i) {
                const int r = rbase + wr + 16 * x + c_row64(lane, i);
                const int c = cbase + wc + 16 * y + c_col(lane);
                if (r < tk.r0 + tk.nr && c < tk.c0 + tk.nc) Qn[r + (int64_t)c * ld] = acc[x][y][i];
            }
}

// copy a node's block of Qn back into Q (so every node's result is in Q)
__global__ void k_dc_copyback(DCArgs a) {
    const Node nd = a.nodes[blockIdx.y];
    const EigMat& mt = a.mats[nd.mat];
    const int n = nd.hi - nd.lo, ld = mt.ld;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
        const int r = e % n, c = e / n;
        const int64_t o = (nd.lo + r) + (int64_t)(nd.lo + c) * ld;
        mt.Q[o] = mt.Qn[o];
    }
}

// ---------------------------------------------------------------------------
// 3. back-transformation: out[:, k] = H_0 H_1 ... H_{m-3} Q[:, order[k]], k < r,
// in compact-WY form: blocks of NB = 32 reflectors, B_b = I - V_b T_b V_b^T with
// T_b upper triangular (T[i,i] = tau_i, T[0:i,i] = -tau_i T[0:i,0:i] V[:,0:i]^T v_i),
// applied last block first.  Rows m..nrows-1 of out are zero.
// ---------------------------------------------------------------------------
constexpr int NB = 32;

// v_j of block b at row i (zero above its leading 1)
__device__ __forceinline__ double vb(const double* Hv, int ld, int m, int k0, int j, int kc, int i) {
    return (j < kc && i > k0 + j && i < m) ? Hv[i + (int64_t)(k0 + j) * ld] : 0.0;
}

// T_b from Y = V_b^T V_b, computed with FP64 MFMA (one 16 x 16 tile of Y per wave).
// grid: (blocks of the largest job, jobs)
__global__ __launch_bounds__(256) void k_larft(BtJobs J) {
    __shared__ double Y[NB][NB + 1];
    __shared__ double T[NB][NB + 1];
    const BtJob& jb = J.job[blockIdx.y];
    const int m = jb.m, ld = jb.ld;
    const double* __restrict__ Hv = jb.Hv;
    const int b = blockIdx.x, k0 = NB * b;
    if (m < 3 || k0 >= m - 2) return;
    const int kc = min(NB, (m - 2) - k0);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int ti = w & 1, tj = w >> 1;
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int row0 = k0 + 1; row0 < m; row0 += 32) {
        double av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int row = row0 + 4 * u + (lane >> 4);
            av[u] = vb(Hv, ld, m, k0, 16 * ti + (lane & 15), kc, row);
            bv[u] = vb(Hv, ld, m, k0, 16 * tj + (lane & 15), kc, row);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = mfma_f64(av[u], bv[u], acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Y[16 * ti + c_row64(lane, q)][16 * tj + c_col(lane)] = acc[q];
    for (int e = t; e < NB * (NB + 1); e += 256) (&T[0][0])[e] = 0.0;
    __syncthreads();
    if (t < 64) {
        for (int i = 0; i < kc; ++i) {
            const double tv = jb.tau[k0 + i];
            double v = 0.0;
            if (t < i) {
                for (int q = t; q < i; ++q) v += T[t][q] * Y[q][i];
                v = -tv * v;
            }
            __builtin_amdgcn_wave_barrier();
            if (t < i) T[t][i] = v;
            if (t == 0) T[i][i] = tv;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();
    for (int e = t; e < NB * NB; e += 256) jb.Tw[(int64_t)b * NB * NB + e] = T[e % NB][e / NB];
}

// X <- H X for a slab of CW columns of X (one workgroup), blocks applied last first:
//   Wm = V_b^T X (MFMA, 2 tiles x 2 halves of the rows), W2 = T_b Wm, X -= V_b W2 (MFMA).
// XL: the slab lives in LDS as X[i * CW + c]; otherwise it is updated in place in out.
// CW = 16, or 8 where 16 columns of m rows do not fit in LDS (the MFMA lanes of
// columns 8 .. 15 then carry zeros and their results are not stored).
// grid: (slabs of the largest job, jobs); slabs at or beyond the job's rank exit.
// BT_WAVES waves per workgroup (two per SIMD: the steps are latency-bound).
constexpr int BT_WAVES = 8, BT_THREADS = 64 * BT_WAVES, BT_H = BT_WAVES / 2;
template <bool XL, int CW>
__global__ __launch_bounds__(BT_THREADS) void k_apply_wy(BtJobs J) {
    extern __shared__ double Xs[];              // mr x 16 when XL
    __shared__ double P[BT_H][NB][17];
    __shared__ double W2[NB][17];
    __shared__ double Ts[NB][NB + 1];           // T_b of the current block, Ts[q][j] = T[j, q]
    const BtJob& jb = J.job[blockIdx.y];
    const int m = jb.m, ld = jb.ld, ldo = jb.ldo, nrows = jb.nrows;
    const int r = jb.r_dev ? min(*jb.r_dev, jb.r) : jb.r;
    const double* __restrict__ Hv = jb.Hv;
    const int mr = (m + 63) & ~63;
    const int c0 = blockIdx.x * CW;
    if (c0 >= r) return;
    const int nc = min(CW, r - c0);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double* Xo = jb.out + (int64_t)c0 * ldo;
    auto X = [&](int i, int c) -> double& { return XL ? Xs[i * CW + c] : Xo[i + (int64_t)c * ldo]; };
    // load the slab (columns beyond nc and rows beyond m are zero)
    const int rows_ld = XL ? mr : m;
    for (int e = t; e < rows_ld * CW; e += BT_THREADS) {
        const int c = e % CW, i = e / CW;
        double v = 0.0;
        if (c < nc && i < m) v = jb.Q[i + (int64_t)(jb.order ? jb.order[c0 + c] : c0 + c) * ld];
        if (XL || c < nc) X(i, c) = v;
    }
    for (int e = t; e < NB * 17; e += BT_THREADS) (&W2[0][0])[e] = 0.0;   // columns >= CW stay zero
    __syncthreads();
    const int nblk = m >= 3 ? (m - 2 + NB - 1) / NB : 0;
    for (int b = nblk - 1; b >= 0; --b) {
        const int k0 = NB * b, kc = min(NB, (m - 2) - k0);
        // T_b into LDS (used after the barrier that ends pass 1)
        {
            const double* T = jb.Tw + (int64_t)b * NB * NB;
            for (int e = t; e < NB * NB; e += BT_THREADS) Ts[e / NB][e % NB] = T[e];
        }
        // pass 1: wave w -> tile jt = w & 1 of Wm and the groups of 4 rows h, h + BT_H,
        // h + 2 BT_H, .. (h = w / 2); the reflector values of the next 8 groups are
        // loaded before this step's MFMAs, which alternate between two accumulators
        {
            constexpr int RS = 4 * BT_H, RSTEP = 8 * RS;   // row stride between MFMAs, per step
            const int jt = w & 1, h = w >> 1;
            d4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
            double an[8];
            const int rfirst = k0 + 1 + 4 * h;
#pragma unroll
            for (int u = 0; u < 8; ++u) an[u] = vb(Hv, ld, m, k0, 16 * jt + (lane & 15), kc, rfirst + RS * u + (lane >> 4));
            for (int row0 = rfirst; row0 < m; row0 += RSTEP) {
                double av[8], bv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) av[u] = an[u];
                if (row0 + RSTEP < m) {
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        an[u] = vb(Hv, ld, m, k0, 16 * jt + (lane & 15), kc, row0 + RSTEP + RS * u + (lane >> 4));
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int row = row0 + RS * u + (lane >> 4);
                    bv[u] = (row < m && (lane & 15) < (XL ? CW : nc)) ? X(row, lane & 15) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    acc0 = mfma_f64(av[u], bv[u], acc0);
                    acc1 = mfma_f64(av[u + 1], bv[u + 1], acc1);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) P[h][16 * jt + c_row64(lane, q)][c_col(lane)] = acc0[q] + acc1[q];
        }
        __syncthreads();
        // Wm = the sum of the wave groups' partial products (into P[0]), then
        // W2 = T_b Wm (T_b upper triangular), both from LDS
        for (int e = t; e < NB * CW; e += BT_THREADS) {
            const int q = e % NB, c = e / NB;
            double pq = P[0][q][c];
#pragma unroll
            for (int hh = 1; hh < BT_H; ++hh) pq += P[hh][q][c];
            P[0][q][c] = pq;
        }
        __syncthreads();
        for (int e = t; e < NB * CW; e += BT_THREADS) {
            const int j = e % NB, c = e / NB;
            double s = 0.0;
            for (int q = j; q < kc; ++q) s += Ts[q][j] * P[0][q][c];
            W2[j][c] = s;
        }
        __syncthreads();
        // pass 2: X[i, :] -= V_b[i, :] W2 for rows k0+1 .. m-1, 16-row tiles over the waves;
        // the reflector values of the next tile are loaded before this tile's MFMAs
        {
            const int i0 = k0 + 1;
            const int ntile = (m - i0 + 15) / 16;
            double an[NB / 4];
            if (w < ntile) {
#pragma unroll
                for (int st = 0; st < NB / 4; ++st)
                    an[st] = vb(Hv, ld, m, k0, 4 * st + (lane >> 4), kc, i0 + 16 * w + (lane & 15));
            }
            for (int tl = w; tl < ntile; tl += BT_WAVES) {
                const int rb = i0 + 16 * tl;
                double av[NB / 4];
#pragma unroll
                for (int st = 0; st < NB / 4; ++st) av[st] = an[st];
                if (tl + BT_WAVES < ntile) {
#pragma unroll
                    for (int st = 0; st < NB / 4; ++st)
                        an[st] = vb(Hv, ld, m, k0, 4 * st + (lane >> 4), kc, rb + 16 * BT_WAVES + (lane & 15));
                }
                d4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < NB / 4; st += 2) {
                    acc0 = mfma_f64(av[st], W2[4 * st + (lane >> 4)][lane & 15], acc0);
                    acc1 = mfma_f64(av[st + 1], W2[4 * (st + 1) + (lane >> 4)][lane & 15], acc1);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = rb + c_row64(lane, q);
                    if (row < m && c_col(lane) < (XL ? CW : nc)) X(row, c_col(lane)) -= acc0[q] + acc1[q];
                }
            }
        }
        __syncthreads();
    }
    if (XL) {
        for (int e = t; e < nrows * CW; e += BT_THREADS) {
            const int i = e % nrows, c = e / nrows;
            if (c < nc) Xo[i + (int64_t)c * ldo] = (i < m) ? Xs[i * CW + c] : 0.0;
        }
    } else {
        for (int e = t; e < nrows * CW; e += BT_THREADS) {
            const int i = e % nrows, c = e / nrows;
            if (c < nc && i >= m) Xo[i + (int64_t)c * ldo] = 0.0;
        }
    }
}

void build_tree(int mat, int lo, int hi, std::vector<std::vector<Node>>& by_height, int& height) {
    if (hi - lo <= LEAF) {
        if ((int)by_height.size() < 1) by_height.resize(1);
        by_height[0].push_back(Node{mat, lo, hi, hi, 0});
        height = 0;
        return;
    }
    const int mid = lo + (hi - lo) / 2;
    int h1 = 0, h2 = 0;
    build_tree(mat, lo, mid, by_height, h1);
    build_tree(mat, mid, hi, by_height, h2);
    height = 1 + std::max(h1, h2);
    if ((int)by_height.size() <= height) by_height.resize(height + 1);
    by_height[height].push_back(Node{mat, lo, mid, hi, 0});
}

// the coupling of every split at mid is removed from the diagonal: d[mid-1] -= b,
// d[mid] -= b with b = e[mid-1].  Splits touch disjoint entries (children have at
// least LEAF/2 rows), so one thread per split.
__global__ void k_dc_modify(const EigMat* __restrict__ mats, const int2* __restrict__ mids, int nmids) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nmids) return;
    const EigMat& mt = mats[mids[q].x];
    const int mid = mids[q].y;
    const double b = mt.e[mid - 1];
    mt.d[mid - 1] -= b;
    mt.d[mid] -= b;
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// A plan holds everything about the eigensolver's launches that depends only on
// the matrix sizes and addresses: the packing of the tridiagonalization into
// cooperative launches, the divide-and-conquer trees, and the device tables
// (matrix table, split list, node and GEMM task lists per tree level).
struct EigPlan {
    std::vector<EigMat> mats;
    // tridiagonalization
    struct TriLaunch {
        std::vector<int> mats;   // indices into mats
        int cpb;                 // columns per workgroup (at most TCOL)
        int rpt, nt;             // rows per thread, threads per workgroup (set by the largest m of the launch)
        int nblocks;
        TriArgs args;
    };
    std::vector<TriLaunch> tri;
    std::vector<size_t> xoff;    // word offset of each matrix's exchange area
    size_t xwords = 0;
    // divide and conquer
    std::vector<std::vector<Node>> levels;
    std::vector<std::vector<GemmTask>> tasks;
    std::vector<int2> mids;
    // device layout (byte offsets into the bound work area)
    size_t off_mats = 0, off_mids = 0, off_x = 0, off_scratch = 0, total = 0;
    std::vector<size_t> off_nodes, off_tasks;
    size_t scratch_bytes = 0;
    std::vector<char> blob;      // host copy of the tables (mats, mids, nodes, tasks)
    size_t blob_bytes = 0;
    char* work = nullptr;
};

EigPlan* eig_plan_create(const EigMat* mats, int nmat, size_t* work_bytes) {
    if (nmat < 1) return nullptr;
    for (int i = 0; i < nmat; ++i)
        if (mats[i].m < 1 || mats[i].m > MAXN || mats[i].ld < mats[i].m) return nullptr;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return nullptr;
    EigPlan* P = new EigPlan();
    P->mats.assign(mats, mats + nmat);
    // ---- tridiagonalization: largest matrices first, packed while every block of
    // a launch can be resident at once (occupancy of the kernel's registers)
    std::vector<int> ord(nmat);
    for (int i = 0; i < nmat; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return mats[x].m > mats[y].m; });
    P->xoff.resize(nmat);
    for (int i = 0; i < nmat; ++i) {
        P->xoff[i] = P->xwords;
        P->xwords += tri_xwords(mats[i].m);
    }
    for (size_t q = 0; q < ord.size();) {
        EigPlan::TriLaunch L;
        const int m0 = mats[ord[q]].m;
        L.rpt = tri_rpt(m0);
        L.nt = tri_nt(m0);
        const int cpb0 = TCOL;
        L.cpb = cpb0;
        const void* kf = tri_kernel(L.rpt, L.nt);
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kf, L.nt, 0) != hipSuccess || occ < 1) {
            delete P;
            return nullptr;
        }
        const int cap = occ * ncu;
        int blocks = 0;
        while (q < ord.size() && (int)L.mats.size() < TRI_MAXMAT) {
            const int mi = mats[ord[q]].m;
            // every matrix of the launch uses the launch's columns per block
            const int bpm = (mi + cpb0 - 1) / cpb0;
            if (bpm > 256 || bpm > cap) { delete P; return nullptr; }
            if (blocks + bpm > cap) break;
            L.mats.push_back(ord[q]);
            blocks += bpm;
            ++q;
        }
        // fewer columns per workgroup while every workgroup of the launch still
        // has a CU of its own: each column step then updates fewer columns per
        // CU (three m = 1024 matrices: 16 -> 13 columns, 192 -> 237 workgroups);
        // two workgroups sharing a CU would serialize their steps
        for (int c = cpb0 - 1; c >= 1; --c) {
            int nb = 0, most = 0;
            for (int i : L.mats) {
                const int b = (mats[i].m + c - 1) / c;
                nb += b;
                most = std::max(most, b);
            }
            if (nb > ncu || most > 256) break;
            L.cpb = c;
            blocks = nb;
        }
        L.nblocks = blocks;
        P->tri.push_back(L);
    }
    // ---- divide and conquer trees, levels across all matrices
    for (int i = 0; i < nmat; ++i) {
        int h = 0;
        build_tree(i, 0, mats[i].m, P->levels, h);
    }
    for (size_t h = 1; h < P->levels.size(); ++h)
        for (auto& nd : P->levels[h]) P->mids.push_back(int2{nd.mat, nd.mid});
    size_t scratch = 0;
    P->tasks.resize(P->levels.size());
    for (size_t h = 1; h < P->levels.size(); ++h) {
        size_t off = 0;
        for (auto& nd : P->levels[h]) {
            nd.soff = (long long)off;
            off += node_scratch_bytes(nd.hi - nd.lo);
            const int n1 = nd.mid - nd.lo, n2 = nd.hi - nd.mid, n = nd.hi - nd.lo;
            P->tasks[h].push_back(GemmTask{nd.mat, nd.lo, n1, nd.lo, n, nd.lo, n1});
            P->tasks[h].push_back(GemmTask{nd.mat, nd.mid, n2, nd.lo, n, nd.mid, n2});
        }
        scratch = std::max(scratch, off);
    }
    P->scratch_bytes = scratch;
    // ---- device layout: tables blob, exchange words, node scratch
    size_t o = 0;
    P->off_mats = o;  o += a256(nmat * sizeof(EigMat));
    P->off_mids = o;  o += a256(std::max<size_t>(1, P->mids.size()) * sizeof(int2));
    P->off_nodes.resize(P->levels.size());
    P->off_tasks.resize(P->levels.size());
    for (size_t h = 0; h < P->levels.size(); ++h) {
        P->off_nodes[h] = o;  o += a256(P->levels[h].size() * sizeof(Node));
        P->off_tasks[h] = o;  o += a256(std::max<size_t>(1, P->tasks[h].size()) * sizeof(GemmTask));
    }
    P->blob_bytes = o;
    P->blob.assign(o, 0);
    memcpy(P->blob.data() + P->off_mats, P->mats.data(), nmat * sizeof(EigMat));
    if (!P->mids.empty()) memcpy(P->blob.data() + P->off_mids, P->mids.data(), P->mids.size() * sizeof(int2));
    for (size_t h = 0; h < P->levels.size(); ++h) {
        memcpy(P->blob.data() + P->off_nodes[h], P->levels[h].data(), P->levels[h].size() * sizeof(Node));
        if (!P->tasks[h].empty())
            memcpy(P->blob.data() + P->off_tasks[h], P->tasks[h].data(), P->tasks[h].size() * sizeof(GemmTask));
    }
    P->off_x = o;        o += a256(P->xwords * sizeof(uint64_t));
    P->off_scratch = o;  o += a256(std::max<size_t>(scratch, 256));
    P->total = o;
    *work_bytes = o;
    return P;
}

void eig_plan_destroy(EigPlan* P) { delete P; }

hipError_t eig_plan_bind(EigPlan* P, void* work, hipStream_t st) {
    P->work = (char*)work;
    uint64_t* xbase = (uint64_t*)(P->work + P->off_x);
    for (auto& L : P->tri) {
        memset(&L.args, 0, sizeof(L.args));
        int blk = 0;
        const int cpb = L.cpb;
        for (size_t i = 0; i < L.mats.size(); ++i) {
            const EigMat& E = P->mats[L.mats[i]];
            TriMat& M = L.args.mat[i];
            M.G = E.G;
            M.d = E.d;
            M.e = E.e;
            M.tau = E.tau;
            M.x = xbase + P->xoff[L.mats[i]];
            M.m = E.m;
            M.ld = E.ld;
            M.cpb = cpb;
            M.bpm = (E.m + cpb - 1) / cpb;
            M.blk0 = blk;
            blk += M.bpm;
        }
        L.args.nmat = (int)L.mats.size();
    }
    return hipMemcpyAsync(P->work, P->blob.data(), P->blob_bytes, hipMemcpyHostToDevice, st);
}

hipError_t eig_plan_enqueue(const EigPlan* P, int* abort_w, hipStream_t st, bool cooperative) {
    hipError_t e;
    if (!P->work) return hipErrorInvalidValue;
    // 1. tridiagonalization
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<size_t>(1024, (P->xwords + 255) / 256)), dim3(256), 0,
                       st, (uint64_t*)(P->work + P->off_x), P->xwords);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (const auto& L : P->tri) {
        TriArgs ta = L.args;
        ta.abort_w = abort_w;
        const void* kf = tri_kernel(L.rpt, L.nt);
        void* args[] = {&ta};
        if (cooperative)
            e = hipLaunchCooperativeKernel(kf, dim3(L.nblocks), dim3(L.nt), args, 0, st);
        else
            e = hipLaunchKernel(kf, dim3(L.nblocks), dim3(L.nt), args, 0, st);
        if (e != hipSuccess) return e;
    }
    // 2. divide and conquer
    const EigMat* dmats = (const EigMat*)(P->work + P->off_mats);
    if (!P->mids.empty()) {
        hipLaunchKernelGGL(k_dc_modify, dim3((unsigned)((P->mids.size() + 255) / 256)), dim3(256), 0, st, dmats,
                           (const int2*)(P->work + P->off_mids), (int)P->mids.size());
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    DCArgs da{};
    da.mats = dmats;
    da.scratch = P->work + P->off_scratch;
    for (size_t h = 0; h < P->levels.size(); ++h) {
        const auto& nodes = P->levels[h];
        da.nodes = (const Node*)(P->work + P->off_nodes[h]);
        da.nnodes = (int)nodes.size();
        if (h == 0) {
            hipLaunchKernelGGL(k_dc_leaves, dim3((unsigned)nodes.size()), dim3(256), 0, st, da);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            continue;
        }
        int maxn = 0, max_tiles = 0;
        for (auto& nd : nodes) {
            const int n1 = nd.mid - nd.lo, n2 = nd.hi - nd.mid, n = nd.hi - nd.lo;
            maxn = std::max(maxn, n);
            max_tiles = std::max(max_tiles, ((std::max(n1, n2) + 63) / 64) * ((n + 63) / 64));
        }
        hipLaunchKernelGGL(k_dc_prep, dim3((unsigned)nodes.size()), dim3(256), 0, st, da);
        hipLaunchKernelGGL(k_dc_roots, dim3((unsigned)((maxn + 3) / 4), (unsigned)nodes.size()), dim3(256), 0, st, da);
        hipLaunchKernelGGL(k_dc_zhat, dim3((unsigned)((maxn + 255) / 256), (unsigned)nodes.size()), dim3(256), 0, st, da);
        hipLaunchKernelGGL(k_dc_vectors, dim3((unsigned)((maxn + 3) / 4), (unsigned)nodes.size()), dim3(256), 0, st, da);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_dc_gemm, dim3((unsigned)max_tiles, (unsigned)P->tasks[h].size()), dim3(256), 0, st, da,
                           (const GemmTask*)(P->work + P->off_tasks[h]));
        hipLaunchKernelGGL(k_dc_copyback, dim3(256, (unsigned)nodes.size()), dim3(256), 0, st, da);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t backtransform_work_doubles(int m) { return (size_t)((m + NB - 1) / NB + 1) * NB * NB; }

hipError_t launch_backtransform(const BtJob* jobs, int njobs, hipStream_t st) {
    hipError_t e;
    for (int j0 = 0; j0 < njobs; j0 += BT_MAXJOB) {
        const int cnt = std::min(BT_MAXJOB, njobs - j0);
        BtJobs J{};
        int mmax = 0, rmax = 0;
        for (int i = 0; i < cnt; ++i) {
            const BtJob& jb = jobs[j0 + i];
            if (jb.m < 1 || jb.m > MAXN || jb.nrows < jb.m || jb.ldo < jb.nrows || jb.ld < jb.m) return hipErrorInvalidValue;
            J.job[i] = jb;
            mmax = std::max(mmax, jb.m);
            rmax = std::max(rmax, jb.r);
        }
        if (rmax < 1) continue;
        const int nblk = mmax >= 3 ? (mmax - 2 + NB - 1) / NB : 0;
        if (nblk > 0) {
            hipLaunchKernelGGL(k_larft, dim3((unsigned)nblk, (unsigned)cnt), dim3(256), 0, st, J);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        const int mr = (mmax + 63) & ~63;
        const size_t sh16 = (size_t)16 * mr * sizeof(double), sh8 = sh16 / 2;
        if (sh16 <= 128 * 1024) {
            if ((e = hipFuncSetAttribute((const void*)k_apply_wy<true, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)sh16)) != hipSuccess)
                return e;
            hipLaunchKernelGGL((k_apply_wy<true, 16>), dim3((unsigned)((rmax + 15) / 16), (unsigned)cnt),
                               dim3(BT_THREADS), sh16, st, J);
        } else if (sh8 <= 128 * 1024) {
            if ((e = hipFuncSetAttribute((const void*)k_apply_wy<true, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)sh8)) != hipSuccess)
                return e;
            hipLaunchKernelGGL((k_apply_wy<true, 8>), dim3((unsigned)((rmax + 7) / 8), (unsigned)cnt),
                               dim3(BT_THREADS), sh8, st, J);
        } else {
            hipLaunchKernelGGL((k_apply_wy<false, 16>), dim3((unsigned)((rmax + 15) / 16), (unsigned)cnt),
                               dim3(BT_THREADS), 0, st, J);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

