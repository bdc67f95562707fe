// Batched reductions (rhosvd_reduce_batched): many independent Reduced HOSVD
// problems of uneven n and R in one pass over the device.
//
// Every phase is one launch over the whole batch: flattened grids for the dense
// phases, the eigensolver's tridiagonalization packed into co-resident groups
// with its divide-and-conquer levels spanning all matrices, and the Khatri-Rao
// cores as one persistent launch fed by a device-side tile counter.  Sizes are
// fixed on the host from the descriptors (rank capacities included); the ranks
// exist only on the device, so nothing in the pass waits for the host.  The
// pass is recorded into a HIP graph once per descriptor list and replayed by
// later calls with the same list.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int RPAD = 128;   // padding of the rank dimension (core tiles)

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Carve {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        T* p = base ? (T*)(base + off) : nullptr;
        off += a256(count * sizeof(T));
        return p;
    }
};

__global__ void k_init_b(const BProb* __restrict__ P, int np, int* __restrict__ abort_w) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *abort_w = 0;
    if (p >= np) return;
    for (int i = 0; i < 4; ++i) {
        P[p].flags[i] = 0;
        P[p].ranks[i] = 0;
    }
}

// result words (r1, r2, r3, status, dropped terms, core precision) and the copy of Z (status 0
// only); grid (problems, 3 modes, column groups)
__global__ __launch_bounds__(256) void k_finish_b(const BProb* __restrict__ P) {
    const BProb& q = P[blockIdx.x];
    const int l = blockIdx.y;
    const int st = q.ranks[3];
    if (l == 0 && blockIdx.z == 0 && threadIdx.x < 8) {
        int v = 0;
        if (threadIdx.x < 3) v = q.ranks[threadIdx.x];
        else if (threadIdx.x == 3) v = st;
        else if (threadIdx.x == 4) v = q.flags[1];
        else if (threadIdx.x == 5) v = q.core_prec;
        q.result[threadIdx.x] = v;
    }
    if (st != 0) return;
    const int r = q.ranks[l];
    if (q.Zo[l])
        for (int c = blockIdx.z; c < r; c += gridDim.z) {
            const double* src = q.Z[l] + (int64_t)c * q.n_pad;
            double* dst = q.Zo[l] + (int64_t)c * q.n;
            for (int i = threadIdx.x; i < q.n; i += 256) dst[i] = src[i];
        }
    // V^(l) = Z^(l)T U~^(l), the factors of the mixed Tucker-canonical format
    if (q.Vo[l])
        for (int nu = blockIdx.z; nu < q.R; nu += gridDim.z) {
            double* dst = q.Vo[l] + (int64_t)nu * q.cap_rank;
            if (q.v_f32) {
                const float* src = (const float*)q.V[l] + (int64_t)nu * q.rcap_pad;
                for (int j = threadIdx.x; j < r; j += 256) dst[j] = (double)src[j];
            } else {
                const double* src = (const double*)q.V[l] + (int64_t)nu * q.rcap_pad;
                for (int j = threadIdx.x; j < r; j += 256) dst[j] = src[j];
            }
        }
}

}  // namespace

struct BatchPlan {
    std::vector<rhosvd_problem> key;
    int prec = 0;
    int prec_key = 0;
    int core_key = 0;                    // the core's precision | beta type, + 32 when some R_pad exceeds core_flush_span()
    int core_tile = 0;                   // rows per core tile: fixed by the caller, or chosen on the first run
    bool tune_pending = false;           // the first run times the tile candidates
    std::vector<BProb> hp;
    // device memory
    char* ws = nullptr;
    size_t ws_bytes = 0;
    BProb* dP = nullptr;
    int64_t* pre[6] = {};
    int64_t nblk[6] = {};
    int64_t* core_work = nullptr;
    int* abort_w = nullptr;
    int core_grid = 256;
    // eigensolver: all Gram matrices; the R < n re-orthonormalizations
    std::vector<EigMat> em[2];
    EigPlan* eplan[2] = {nullptr, nullptr};
    void* ework[2] = {nullptr, nullptr};
    std::vector<BtJob> bt_main, bt_rside;
    struct RSide {
        int p;
        double *Wr[3], *Zraw[3], *M2[3], *P2[3], *Pf[3], *S2[3], *lam2[3];
    };
    std::vector<RSide> rs;
    // graph
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = false;
    DevAlloc alloc;                      // the handle's allocator

    ~BatchPlan() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        for (int i = 0; i < 2; ++i) {
            if (eplan[i]) eig_plan_destroy(eplan[i]);
            alloc.put(ework[i]);
        }
        alloc.put(ws);
        if (cap) hipStreamDestroy(cap);
    }
};

namespace {

// Workspace layout of the whole batch.  With base == nullptr it only measures;
// otherwise it assigns every device pointer and builds the eigensolver matrix
// lists and the back-transformation jobs.
size_t carve_batch(BatchPlan& B, char* base) {
    Carve c{base};
    const int np = (int)B.hp.size();
    B.dP = c.take<BProb>(np);
    for (int k = 0; k < 6; ++k) B.pre[k] = c.take<int64_t>(np + 1);
    B.core_work = c.take<int64_t>(np + 4);
    B.abort_w = c.take<int>(16);
    const int esz = B.prec == RHOSVD_FP64 ? 8 : 4;
    B.rs.clear();
    B.em[0].clear();
    B.em[1].clear();
    B.bt_main.clear();
    B.bt_rside.clear();
    std::vector<BtJob> bt_r1;
    for (int p = 0; p < np; ++p) {
        BProb& q = B.hp[p];
        const size_t npd = q.n_pad, Rp = q.R_pad, mp = q.m_pad, zp = q.rcap_pad;
        for (int l = 0; l < 3; ++l) q.Ut[l] = c.take<double>(npd * Rp);
        q.xip = c.take<double>(Rp);
        q.flags = c.take<int>(8);
        q.ranks = c.take<int>(8);
        q.scal = c.take<double>(16);
        const int64_t rt = Rp / 64;
        q.anorm_ntiles = rt * (rt + 1) / 2;
        q.anorm_part = c.take<double>(q.anorm_ntiles);
        q.abort_w = B.abort_w;
        q.Asplit = B.prec == RHOSVD_BF16X3 ? (void*)c.take<char>(zp * Rp * 4) : nullptr;
        BatchPlan::RSide r{};
        r.p = p;
        if (q.rside) {
            for (int l = 0; l < 3; ++l) {
                r.Wr[l] = c.take<double>(Rp * zp);
                r.Zraw[l] = c.take<double>(npd * zp);
                r.M2[l] = c.take<double>(zp * zp);
                r.P2[l] = c.take<double>(zp * zp);
                r.Pf[l] = c.take<double>(zp * zp);
                r.S2[l] = c.take<double>(zp * zp);
                r.lam2[l] = c.take<double>(zp);
                double* Qn2 = c.take<double>(zp * zp);
                double* Mg2 = c.take<double>(zp * zp);
                double* dd2 = c.take<double>(zp);
                double* ee2 = c.take<double>(zp);
                double* tau2 = c.take<double>(zp);
                double* Tw2 = c.take<double>(backtransform_work_doubles((int)zp));
                B.em[1].push_back(EigMat{r.M2[l], r.lam2[l], r.P2[l], Qn2, Mg2, dd2, ee2, tau2, (int)zp, (int)zp});
                B.bt_rside.push_back(BtJob{(int)zp, (int)zp, r.M2[l], tau2, r.P2[l], nullptr, (int)zp, nullptr,
                                           r.Pf[l], (int)zp, (int)zp, Tw2});
            }
            B.rs.push_back(r);
        }
        for (int l = 0; l < 3; ++l) {
            q.G[l] = c.take<double>(mp * mp);
            q.W[l] = c.take<double>(mp * mp);
            q.lam[l] = c.take<double>(mp);
            q.sigma[l] = c.take<double>(mp + 1);
            q.order[l] = c.take<int>(mp);
            q.tails[l] = c.take<double>(mp + 1);
            q.Z[l] = c.take<double>(npd * zp);
            q.V[l] = (void*)c.take<char>(zp * Rp * esz);
            double* Qn = c.take<double>(mp * mp);
            double* Mg = c.take<double>(mp * mp);
            double* dd = c.take<double>(mp);
            double* ee = c.take<double>(mp);
            double* ht = c.take<double>(mp);
            double* Tw = c.take<double>(backtransform_work_doubles((int)std::max(mp, zp)));
            B.em[0].push_back(EigMat{q.G[l], q.lam[l], q.W[l], Qn, Mg, dd, ee, ht, q.m, q.m_pad});
            // Z = H W[:, order] (n <= R), or W_r = H W[:, order] (R < n); the rank is read on the device
            const BtJob jb{q.m, q.m_pad, q.G[l], ht, q.W[l], q.order[l], q.rcap, q.ranks ? q.ranks + l : nullptr,
                           q.rside ? r.Wr[l] : q.Z[l], q.rside ? q.R_pad : q.n_pad, q.rside ? q.R_pad : q.n_pad, Tw};
            (q.rside ? bt_r1 : B.bt_main).push_back(jb);
        }
    }
    B.bt_main.insert(B.bt_main.end(), bt_r1.begin(), bt_r1.end());
    return c.off;
}

// everything up to and including the projection
static hipError_t enqueue_batch_pre(const BatchPlan& B, hipStream_t st, bool coop) {
    hipError_t e;
    const int np = (int)B.hp.size();
    const BProb* P = B.dP;
    hipLaunchKernelGGL(k_init_b, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, P, np, B.abort_w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_batched_dense(BK_COLNORM, P, B.pre[0], np, B.nblk[0], 0, st)) != hipSuccess) return e;
    if ((e = launch_batched_dense(BK_ANORM, P, B.pre[1], np, B.nblk[1], 0, st)) != hipSuccess) return e;
    if ((e = launch_batched_dense(BK_GRAM, P, B.pre[2], np, B.nblk[2], 0, st)) != hipSuccess) return e;
    if ((e = eig_plan_enqueue(B.eplan[0], B.abort_w, st, coop)) != hipSuccess) return e;
    if ((e = launch_truncate_b(P, np, st)) != hipSuccess) return e;
    if ((e = launch_backtransform(B.bt_main.data(), (int)B.bt_main.size(), st)) != hipSuccess) return e;
    // R < n: Z = U~ W_r Lambda_r^(-1/2), re-orthonormalized by (Z^T Z)^(-1/2)
    for (const auto& r : B.rs) {
        const BProb& q = B.hp[r.p];
        const int zp = q.rcap_pad;
        for (int l = 0; l < 3; ++l) {
            if ((e = launch_gather_scaled(q.R_pad, q.rcap, zp, r.Wr[l], nullptr, q.sigma[l], r.Wr[l], st,
                                          q.ranks + l)) != hipSuccess)
                return e;
            if ((e = launch_gemm64(false, true, q.n_pad, zp, q.R_pad, q.Ut[l], q.n_pad, r.Wr[l], q.R_pad, r.Zraw[l],
                                   q.n_pad, 1.0, st)) != hipSuccess)
                return e;
            if ((e = launch_gemm64(true, true, zp, zp, q.n_pad, r.Zraw[l], q.n_pad, r.Zraw[l], q.n_pad, r.M2[l], zp,
                                   1.0, st)) != hipSuccess)
                return e;
            if ((e = launch_pad_identity(q.rcap, zp, zp, r.M2[l], st, q.ranks + l)) != hipSuccess) return e;
        }
    }
    if (!B.rs.empty()) {
        if ((e = eig_plan_enqueue(B.eplan[1], B.abort_w, st, coop)) != hipSuccess) return e;
        if ((e = launch_backtransform(B.bt_rside.data(), (int)B.bt_rside.size(), st)) != hipSuccess) return e;
        for (const auto& r : B.rs) {
            const BProb& q = B.hp[r.p];
            const int zp = q.rcap_pad;
            for (int l = 0; l < 3; ++l) {
                if ((e = launch_scale_cols_invsqrt(zp, zp, r.lam2[l], r.Pf[l], r.S2[l], st)) != hipSuccess) return e;
                if ((e = launch_gemm64(false, false, zp, zp, zp, r.S2[l], zp, r.Pf[l], zp, r.M2[l], zp, 1.0, st)) !=
                    hipSuccess)
                    return e;
                if ((e = launch_gemm64(false, true, q.n_pad, zp, zp, r.Zraw[l], q.n_pad, r.M2[l], zp, q.Z[l], q.n_pad,
                                       1.0, st)) != hipSuccess)
                    return e;
            }
        }
    }
    if ((e = launch_batched_dense(BK_SIGN, P, B.pre[4], np, B.nblk[4], 0, st)) != hipSuccess) return e;
    if ((e = launch_batched_dense(BK_PROJECT, P, B.pre[3], np, B.nblk[3], B.prec != 0, st)) != hipSuccess) return e;
    return B.prec == RHOSVD_BF16X3 ? launch_split_b(P, B.pre[5], np, B.nblk[5], st) : hipSuccess;
}

static hipError_t enqueue_finish(const BatchPlan& B, hipStream_t st) {
    hipLaunchKernelGGL(k_finish_b, dim3((unsigned)B.hp.size(), 3, 8), dim3(256), 0, st, B.dP);
    return hipGetLastError();
}

hipError_t enqueue_batch(const BatchPlan& B, hipStream_t st, bool coop) {
    hipError_t e;
    if ((e = enqueue_batch_pre(B, st, coop)) != hipSuccess) return e;
    if ((e = launch_core_b(B.dP, (int)B.hp.size(), B.core_key, B.core_tile, B.core_work, B.core_grid, st)) !=
        hipSuccess)
        return e;
    return enqueue_finish(B, st);
}

// record the pass into a graph; on any failure the pass runs eagerly
static void capture_batch(BatchPlan* B) {
    const char* env = getenv("RHOSVD_BATCH_GRAPH");
    if (env && env[0] == '0') return;
    if (!B->cap && hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess) {
        B->cap = nullptr;
        return;
    }
    bool ok = hipStreamBeginCapture(B->cap, hipStreamCaptureModeRelaxed) == hipSuccess;
    hipError_t ee = ok ? enqueue_batch(*B, B->cap, false) : hipErrorUnknown;
    hipGraph_t g = nullptr;
    hipError_t ec = ok ? hipStreamEndCapture(B->cap, &g) : hipErrorUnknown;
    if (ok && ee == hipSuccess && ec == hipSuccess && g &&
        hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) == hipSuccess) {
        B->graph = g;
        B->use_graph = true;
    } else {
        if (g) hipGraphDestroy(g);
        B->exec = nullptr;
        hipGetLastError();
    }
}

bool same_key(const std::vector<rhosvd_problem>& k, const rhosvd_problem* probs, int count) {
    return (int)k.size() == count && memcmp(k.data(), probs, (size_t)count * sizeof(rhosvd_problem)) == 0;
}

}  // namespace

int batch_validate(const rhosvd_problem* probs, int count, std::string& msg) {
    if (count < 1) { msg = "count must be >= 1"; return RHOSVD_ERR_ARG; }
    if (!probs) { msg = "problems is NULL"; return RHOSVD_ERR_ARG; }
    for (int i = 0; i < count; ++i) {
        const rhosvd_problem& q = probs[i];
        const std::string at = "problem " + std::to_string(i) + ": ";
        if (q.n < 1 || q.R < 1) { msg = at + "n and R must be >= 1"; return RHOSVD_ERR_ARG; }
        if (!(q.eps > 0.0) || q.eps != q.eps || q.eps > 1e300) { msg = at + "eps must be finite and > 0"; return RHOSVD_ERR_ARG; }
        if (!q.U1 || !q.U2 || !q.U3 || !q.xi || !q.result) { msg = at + "null input or result pointer"; return RHOSVD_ERR_ARG; }
        if (q.cap_rank < 1) { msg = at + "cap_rank must be >= 1"; return RHOSVD_ERR_ARG; }
        const int nz = (q.Z1 != nullptr) + (q.Z2 != nullptr) + (q.Z3 != nullptr);
        if (nz != 0 && nz != 3) { msg = at + "Z1, Z2, Z3 must be all set or all NULL"; return RHOSVD_ERR_ARG; }
        const int nv = (q.V1 != nullptr) + (q.V2 != nullptr) + (q.V3 != nullptr);
        if (nv != 0 && nv != 3) { msg = at + "V1, V2, V3 must be all set or all NULL"; return RHOSVD_ERR_ARG; }
        if (q.beta && q.cap_beta < 1) { msg = at + "cap_beta must be >= 1 when beta is set"; return RHOSVD_ERR_ARG; }
        if (q.reserved0 != 0) { msg = at + "reserved0 must be zero"; return RHOSVD_ERR_ARG; }
        if (std::min(q.n, q.R) > 2048 || q.n > 65536 || q.R > ((int64_t)1 << 24)) {
            msg = at + "size not supported (min(n, R) <= 2048, n <= 65536, R <= 2^24)";
            return RHOSVD_ERR_UNSUPPORTED;
        }
    }
    return RHOSVD_OK;
}

BatchPlan* batch_plan_create(const rhosvd_problem* probs, int count, int prec, std::string& err,
                             const DevAlloc& alloc) {
    BatchPlan* B = new BatchPlan();
    B->alloc = alloc;
    // prec: the core precision, plus 16 when beta is written as float, plus the
    // caller's fixed core tile times 256 (0: tuned on the first run)
    B->key.assign(probs, probs + count);
    B->prec_key = prec;
    // one core precision serves the whole pass: BF16x3 gives way to FP32 when some
    // problem's eps lies below its floor (BF16X3_MIN_EPS)
    double eps_min = probs[0].eps;
    for (int p = 1; p < count; ++p) eps_min = std::min(eps_min, probs[p].eps);
    prec = (prec & ~3) | core_precision_for(prec & 3, eps_min);
    B->prec = prec & 3;
    B->hp.resize(count);
    for (int p = 0; p < count; ++p) {
        const rhosvd_problem& d = probs[p];
        BProb& q = B->hp[p];
        memset(&q, 0, sizeof(q));
        q.n = (int)d.n;
        q.R = (int)d.R;
        q.n_pad = (int)round_up(d.n, PAD_N);
        q.R_pad = (int)round_up(d.R, PAD_R);
        q.m = (int)std::min(d.n, d.R);
        q.rside = d.R < d.n;
        q.m_pad = q.rside ? q.R_pad : q.n_pad;
        q.cap_rank = d.cap_rank;
        q.rcap = std::min(d.cap_rank, q.m);
        q.rcap_pad = (int)round_up(std::max(q.rcap, 1), RPAD);
        q.eps = d.eps;
        q.U[0] = d.U1;
        q.U[1] = d.U2;
        q.U[2] = d.U3;
        q.xi = d.xi;
        q.Zo[0] = d.Z1;
        q.Zo[1] = d.Z2;
        q.Zo[2] = d.Z3;
        q.Vo[0] = d.V1;
        q.Vo[1] = d.V2;
        q.Vo[2] = d.V3;
        q.v_f32 = (prec & 3) != 0 ? 1 : 0;
        q.beta = d.beta;
        q.cap_beta = d.cap_beta;
        q.beta_f32 = (prec & 16) ? 1 : 0;
        q.result = d.result;
        q.core_prec = B->prec;
    }
    const size_t need = carve_batch(*B, nullptr);
    if (!(B->ws = (char*)B->alloc.get(need))) {
        err = "batch workspace allocation of " + std::to_string(need) + " bytes failed";
        delete B;
        return nullptr;
    }
    B->ws_bytes = need;
    carve_batch(*B, B->ws);
    // flattened grids
    std::vector<int64_t> pre(6 * (count + 1), 0);
    for (int p = 0; p < count; ++p) {
        const BProb& q = B->hp[p];
        const int64_t rt = q.R_pad / 64, nt = q.n_pad / 64;
        const int64_t cnt[6] = {ceil_div(q.R_pad, 4), rt * (rt + 1) / 2, q.rside ? 0 : 3 * nt * (nt + 1) / 2,
                                3 * (int64_t)(q.rcap_pad / 64) * rt, 3 * (int64_t)(q.rcap_pad / 4),
                                (int64_t)(q.rcap_pad / 64) * rt};
        for (int k = 0; k < 6; ++k) pre[k * (count + 1) + p + 1] = pre[k * (count + 1) + p] + cnt[k];
    }
    for (int k = 0; k < 6; ++k) B->nblk[k] = pre[k * (count + 1) + count];
    hipError_t e = hipMemcpy(B->dP, B->hp.data(), count * sizeof(BProb), hipMemcpyHostToDevice);
    for (int k = 0; k < 6 && e == hipSuccess; ++k)
        e = hipMemcpy(B->pre[k], pre.data() + k * (count + 1), (count + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        err = std::string("batch table upload: ") + hipGetErrorString(e);
        delete B;
        return nullptr;
    }
    // eigensolver plans
    for (int i = 0; i < 2; ++i) {
        if (B->em[i].empty()) continue;
        size_t wb = 0;
        B->eplan[i] = eig_plan_create(B->em[i].data(), (int)B->em[i].size(), &wb);
        if (!B->eplan[i]) {
            err = "eigensolver plan: matrix sizes not supported on this device";
            delete B;
            return nullptr;
        }
        if (!(B->ework[i] = B->alloc.get(wb))) {
            err = "eigensolver work allocation failed";
            delete B;
            return nullptr;
        }
        if ((e = eig_plan_bind(B->eplan[i], B->ework[i], nullptr)) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess) {
            err = std::string("eigensolver plan upload: ") + hipGetErrorString(e);
            delete B;
            return nullptr;
        }
    }
    int64_t rmax = 0;
    for (const BProb& q : B->hp) rmax = std::max<int64_t>(rmax, q.R_pad);
    B->core_key = (prec & 63) | (rmax > core_flush_span() ? 32 : 0);
    const int fixed = B->prec_key >> 8;
    bool any_beta = false;
    for (const BProb& q : B->hp) any_beta = any_beta || q.beta != nullptr;
    if (fixed || B->prec == 0 || !any_beta) {
        B->core_tile = fixed ? fixed : core_tile_default(B->prec);
        B->core_grid = core_b_max_grid(B->core_key, B->core_tile);
        capture_batch(B);
    } else {
        B->tune_pending = true;   // the first run times the candidates, then records the graph
    }
    return B;
}

bool batch_plan_matches(const BatchPlan* B, const rhosvd_problem* probs, int count, int prec) {
    return B && B->prec_key == prec && same_key(B->key, probs, count);
}

hipError_t batch_plan_run(BatchPlan* B, hipStream_t st) {
    if (B->tune_pending) {
        // first run: the pass up to the projection, then the persistent core with
        // each tile candidate (timed), then the rest; later runs use the winner
        hipError_t e;
        if ((e = enqueue_batch_pre(*B, st, true)) != hipSuccess) return e;
        const int np = (int)B->hp.size();
        int best = 0;
        const int tiles[2] = {64, 128};
        e = time_candidates(
            tiles, 2,
            [&](int tile) {
                return launch_core_b(B->dP, np, B->core_key, tile, B->core_work, core_b_max_grid(B->core_key, tile),
                                     st);
            },
            st, &best);
        if (e != hipSuccess) return e;
        if ((e = enqueue_finish(*B, st)) != hipSuccess) return e;
        B->core_tile = best;
        B->core_grid = core_b_max_grid(B->core_key, best);
        B->tune_pending = false;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        capture_batch(B);
        return hipSuccess;
    }
    if (B->use_graph) return hipGraphLaunch(B->exec, st);
    return enqueue_batch(*B, st, true);
}

int batch_plan_core_tile(const BatchPlan* B) { return B ? B->core_tile : 0; }

bool batch_plan_uses_graph(const BatchPlan* B) { return B && B->use_graph; }

void batch_plan_destroy(BatchPlan* B) { delete B; }
