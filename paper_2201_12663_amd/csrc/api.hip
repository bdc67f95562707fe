// C-ABI of the Reduced HOSVD library: handle, workspace and the reduction's
// orchestration (declared in include/rhosvd.h).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "capacity.hpp"
#include "common.hpp"
#include "kernels.hpp"

#define RHOSVD_VERSION "0.2.0"

namespace {

constexpr int NPHASE = 7;
constexpr int NEV = 9;            // 0..6 bracket the reduce phases, 7..8 the core
constexpr int DEFAULT_SWEEPS = 30;   // kept for the options ABI; the eigensolver has no sweep cap
constexpr int RPAD_CORE = 128;                                 // V row padding (core tiles)
constexpr size_t HOST_BYTES = 4096;                            // pinned host staging of a handle
constexpr int REFINE_AUTO = 0, REFINE_OFF = 3;                 // rhosvd_options.refine_tails
// auto refinement: a mode whose last kept eigenvalue of the Gram matrix lies
// within NOISE_BAND u sigma_1^2 of zero has its cut inside the FP64 Gram route's
// noise band (eigenvalues of G are exact only to about u |G|)
constexpr double NOISE_BAND = 64.0;
constexpr double U64H = 1.1102230246251565e-16;                // 2^-53

std::string g_create_error;

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct rhosvd_ctx {
    hipStream_t stream = nullptr;
    DevAlloc alloc;                      // device memory: the caller's allocator, or hipMalloc
    rhosvd_options opt{};
    std::string err;
    CoreTuner* tuner = nullptr;          // core tile per shape class (tune.hip)
    int last_tile = 0;                   // tile of the last core launch
    // workspace (grow-only)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int* host = nullptr;   // pinned host staging (ranks, flags, sweeps)
    double* hostd = nullptr;
    // layout of the last reduction
    int64_t n = 0, R = 0, n_pad = 0, R_pad = 0, m = 0, m_pad = 0, zr_pad = 0;
    bool rside = false;                  // R < n: Gram on the R side
    bool force_nside = false;            // R < n re-run on the n x n Gram (refinement)
    double* Ut[3] = {};                  // normalized side matrices (n_pad x R_pad)
    double* xip = nullptr;               // xi' (R_pad)
    int* flags = nullptr;
    double* G[3] = {};                   // Gram (m_pad^2) -> Householder vectors
    double* W[3] = {};                   // eigenvectors of the tridiagonal matrix
    double* Qn[3] = {};                  // eigensolver workspace (m_pad^2 each)
    double* Mg[3] = {};
    double* lam[3] = {};                 // eigenvalues (m_pad)
    double* dd[3] = {};
    double* ee[3] = {};
    double* htau[3] = {};                // Householder scalars
    double* Tw[3] = {};                  // compact-WY factors of the back-transformation
    // eigensolver plans (Gram matrices; R < n re-orthonormalization) and their work memory
    // [0] Gram matrices, [1] R < n re-orthonormalization, [2] sketch Grams of the
    // rank proposal, [3] range-finder matrices
    static constexpr int NPLAN = 5;     // [4]: the ALS Gram matrix (one n x n matrix)
    EigPlan* plan[NPLAN] = {};
    std::vector<EigMat> plan_mats[NPLAN];
    void* plan_w[NPLAN] = {};
    size_t plan_wbytes[NPLAN] = {};
    double* gram_part = nullptr;
    int gram_splits = 1;
    double* anorm_part = nullptr;
    int64_t anorm_ntiles = 0;
    // |A| used by the truncation: partial sums of |A|^2 (exact identity) or of
    // |beta_p|^2 (probe), and the probe's own workspace (grow-only)
    const double* a2_part = nullptr;
    int64_t a2_n = 0;
    int anorm_method = 1;
    int refine_used = 0;                 // refinement the last reduction used (0 none, 1, 2)
    double a_upper = 0;
    char* pw = nullptr;
    size_t pw_bytes = 0;
    double* sigma[3] = {};
    int* order[3] = {};
    double* tails[3] = {};
    int* ranks_dev = nullptr;
    double* scal = nullptr;
    double* Z[3] = {};                   // n_pad x zr_pad
    void* V[3] = {};                     // zr_pad x R_pad (FP64 or FP32)
    double* Vref[3] = {};                // refine_tails with a mixed core: FP64 projection
    void* Asplit = nullptr;              // BF16x3 core: hi/lo bf16 planes of V1 diag(xi') (zr_pad x R_pad each)
    double* Vc = nullptr;                // certificate on a mixed path: FP64 projection (zr_pad x R_pad)
    double* cpart = nullptr;             // certificate: column sums of squares (n_pad / 64 x R_pad)
    double* cout = nullptr;              // certificate: per-block partials of the three modes, then the sum
    double* Ud[3] = {};                  // refine_tails = 2: deflated side matrices (n_pad x R_pad)
    double* Zs[3] = {};                  //   second-pass vectors before re-orthogonalization (n_pad x zr_pad)
    double* Cz[3] = {};                  //   Z_k^T Z' (zr_pad x zr_pad)
    double* dscr = nullptr;              //   first-pass spectrum, second-pass spectrum and tails
    double* rpart[3] = {};               // refine_tails: residual partial sums
    double* Ha = nullptr;                // ALS: V_a^T V_a, then P (R_pad x R_pad)
    double* Hb = nullptr;                // ALS: V_b^T V_b (R_pad x R_pad)
    double* Tals = nullptr;              // ALS: U~_l P (n_pad x R_pad)
    double* V64a[3] = {};                // ALS on a mixed path: FP64 projections (zr_pad x R_pad)
    double* rfloor = nullptr;            // refine_tails: squared residuals (3)
    // reduced-precision Gram (gram_precision 1, 2; n <= R): the Rayleigh-Ritz step uses
    // Zraw (Q), Brr (B = Q^T U~, FP64), M2 (B B^T -> reflectors), P2 / Qn2 / Mg2 /
    // lam2 / dd2 / ee2 / tau2 (its eigensolver), Pf (selected eigenvectors of B B^T)
    double* Brr[3] = {};                 // zr_pad x R_pad
    int* rr_order[3] = {};               // order of the Ritz values (the Gram's own order stays in order)
    bool lp_gram = false;                // this reduction's Gram ran in reduced precision
    int gram_used = 0;                   // report: the Gram's arithmetic as run
    int vprec = 0;
    double eps = 0;                      // tolerance of the last reduction (the core's precision)
    // R < n: Z = U~ W_r Lambda_r^-1/2, re-orthonormalized by (Z^T Z)^-1/2
    double* Wr[3] = {};                  // R_pad x zr_pad
    double* Zraw[3] = {};                // n_pad x zr_pad
    double* M2[3] = {};                  // zr_pad^2: Z^T Z (-> reflectors), then S
    double* P2[3] = {};                  // eigenvectors of the tridiagonal of Z^T Z
    double* Qn2[3] = {};
    double* Mg2[3] = {};
    double* Pf[3] = {};                  // eigenvectors of Z^T Z
    double* S2[3] = {};
    double* lam2[3] = {};
    double* dd2[3] = {};
    double* ee2[3] = {};
    double* tau2[3] = {};
    // results
    bool have = false;
    int ranks[3] = {0, 0, 0};
    int r_pad[3] = {0, 0, 0};
    double xi_norm = 0, a_norm = 0, tau = 0;   // report values
    int sweeps = 0, dropped = 0;
    // batched reductions: the plan of the last descriptor list
    BatchPlan* batch = nullptr;
    // rank-proposal network: parameters, gradient, Adam moments (one allocation)
    float* net = nullptr;
    float* net_work = nullptr;
    size_t net_work_n = 0;
    int net_step = 0;
    bool net_set = false;
    // learned rank proposal + range finder workspace (grow-only)
    struct Learned {
        char* ws = nullptr;
        size_t bytes = 0;
        int p_cap = 0;
        double* Om32 = nullptr;
        double *Om[3] = {}, *Y[3] = {}, *Qb[3] = {}, *G2[3] = {}, *W2[3] = {}, *Qn2[3] = {}, *Mg2[3] = {}, *Pf[3] = {},
               *S2[3] = {}, *lam2[3] = {}, *dd2[3] = {}, *ee2[3] = {}, *tau2[3] = {}, *Bm[3] = {}, *Tw[3] = {},
               *part[3] = {}, *Wsel[3] = {};
        double* floor2 = nullptr;
        float* feat = nullptr;
        float* out = nullptr;
    } L;
    // Tucker-to-canonical transform: state of the last rhosvd_t2c (grow-only workspace)
    struct T2C {
        char* ws = nullptr;
        size_t bytes = 0;
        char* lw = nullptr;              // lifting scratch: padded Z, F and C
        size_t lbytes = 0;
        int r1 = 0, r2 = 0, r3 = 0;
        const double* beta = nullptr;
        int64_t R = 0;
        bool have = false;
        double *W = nullptr, *sig = nullptr, *tails = nullptr;
        int* p = nullptr;
        int64_t* off = nullptr;
        int* flags = nullptr;
    } T;
    // profiling
    hipEvent_t ev[NEV] = {};
    bool ev_ok = false;
    float phase_ms[NPHASE] = {};
    bool reduce_timed = false, get_timed = false;
};

namespace {

rhosvd_status fail(rhosvd_ctx* h, rhosvd_status s, const std::string& msg) {
    if (h) h->err = msg;
    return s;
}

#define CK(h, expr)                                                                          \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(h, RHOSVD_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

rhosvd_status check_options(const rhosvd_options* o, std::string& msg) {
    if (!o) return RHOSVD_OK;
    if (o->precision < 0 || o->precision > 2) { msg = "unknown precision"; return RHOSVD_ERR_ARG; }
    if (o->anorm < 0 || o->anorm > 2) { msg = "anorm must be 0 (auto), 1 (exact) or 2 (probe)"; return RHOSVD_ERR_ARG; }
    if (o->als_sweeps < 0 || o->als_sweeps > 4) { msg = "als_sweeps must be 0..4"; return RHOSVD_ERR_ARG; }
    if (o->refine_tails < 0 || o->refine_tails > 3) { msg = "refine_tails must be 0 (auto), 1, 2 or 3 (off)"; return RHOSVD_ERR_ARG; }
    if (o->gram_precision < 0 || o->gram_precision > 2) {
        msg = "gram_precision must be 0 (FP64), 1 (FP32) or 2 (BF16x3)";
        return RHOSVD_ERR_ARG;
    }
    if (o->core_tile != 0 && !core_tile_valid(o->precision, o->core_tile)) {
        msg = "core_tile must be 0 (tuned), 64, or 128 (128 only for the FP32 and BF16x3 cores)";
        return RHOSVD_ERR_ARG;
    }
    return RHOSVD_OK;
}

void apply_options(rhosvd_ctx* h, const rhosvd_options* o) {
    if (o) h->opt = *o;
    else memset(&h->opt, 0, sizeof(h->opt));
    if (h->opt.max_eig_sweeps <= 0) h->opt.max_eig_sweeps = DEFAULT_SWEEPS;
}

void mark(rhosvd_ctx* h, int i) {
    if (h->opt.profile && h->ev_ok) hipEventRecord(h->ev[i], h->stream);
}

// Workspace carving: the same walk runs twice, first to size, then to assign.
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

size_t carve_all(rhosvd_ctx* h, char* base) {
    Carve c{base};
    const int64_t np = h->n_pad, Rp = h->R_pad, mp = h->m_pad, zp = h->zr_pad;
    const int esz = (h->opt.precision == RHOSVD_FP64) ? 8 : 4;
    for (int l = 0; l < 3; ++l) {
        h->Ut[l] = c.take<double>((size_t)np * Rp);
        h->G[l] = c.take<double>((size_t)mp * mp);
        h->W[l] = c.take<double>((size_t)mp * mp);
        h->Qn[l] = c.take<double>((size_t)mp * mp);
        h->Mg[l] = c.take<double>((size_t)mp * mp);
        h->lam[l] = c.take<double>(mp);
        h->dd[l] = c.take<double>(mp);
        h->ee[l] = c.take<double>(mp);
        h->htau[l] = c.take<double>(mp);
        h->Tw[l] = c.take<double>(backtransform_work_doubles((int)std::max(mp, zp)));
        h->sigma[l] = c.take<double>(mp + 1);
        h->order[l] = c.take<int>(mp);
        h->tails[l] = c.take<double>(mp + 1);
        h->Z[l] = c.take<double>((size_t)np * zp);
        h->V[l] = (void*)c.take<char>((size_t)zp * Rp * esz);
    }
    const bool lp = h->lp_gram;
    for (int l = 0; l < 3; ++l) {
        const bool refine = h->opt.refine_tails != REFINE_OFF || lp;   // auto may refine
        const bool deflate = (h->opt.refine_tails == 2 || h->opt.refine_tails == REFINE_AUTO) && !h->rside;
        h->Vref[l] = (refine && esz == 4) ? c.take<double>((size_t)zp * Rp) : nullptr;
        h->rpart[l] = refine ? c.take<double>((size_t)(np / 64) * (Rp / 64)) : nullptr;
        h->Ud[l] = deflate ? c.take<double>((size_t)np * Rp) : nullptr;
        h->Zs[l] = deflate ? c.take<double>((size_t)np * zp) : nullptr;
        h->Cz[l] = deflate ? c.take<double>((size_t)zp * zp) : nullptr;
    }
    const bool als = h->opt.als_sweeps > 0 && !h->rside;
    h->Ha = als ? c.take<double>((size_t)Rp * Rp) : nullptr;
    h->Hb = als ? c.take<double>((size_t)Rp * Rp) : nullptr;
    h->Tals = als ? c.take<double>((size_t)np * Rp) : nullptr;
    for (int l = 0; l < 3; ++l) h->V64a[l] = (als && esz == 4) ? c.take<double>((size_t)zp * Rp) : nullptr;
    h->Asplit = h->opt.precision == RHOSVD_BF16X3 ? (void*)c.take<char>((size_t)zp * Rp * 4) : nullptr;
    const bool cert = h->opt.certificate != 0;
    h->Vc = (cert && esz == 4) ? c.take<double>((size_t)zp * Rp) : nullptr;
    h->cpart = cert ? c.take<double>((size_t)(np / 64) * Rp) : nullptr;
    h->cout = cert ? c.take<double>((size_t)3 * cert_blocks(Rp) + 8) : nullptr;
    h->dscr = ((h->opt.refine_tails == 2 || h->opt.refine_tails == REFINE_AUTO) && !h->rside)
                  ? c.take<double>((size_t)9 * (h->m_pad + 64)) : nullptr;
    h->rfloor = c.take<double>(4);
    h->xip = c.take<double>(Rp);
    h->flags = c.take<int>(16);
    h->gram_part = (h->gram_splits > 1) ? c.take<double>((size_t)h->gram_splits * 3 * np * np) : nullptr;
    h->anorm_part = c.take<double>(h->anorm_ntiles);
    h->ranks_dev = c.take<int>(16);
    h->scal = c.take<double>(16);
    for (int l = 0; l < 3; ++l) {
        h->Brr[l] = lp ? c.take<double>((size_t)zp * Rp) : nullptr;
        h->rr_order[l] = lp ? c.take<int>(zp) : nullptr;
    }
    if (h->rside || lp) {
        for (int l = 0; l < 3; ++l) {
            h->Wr[l] = h->rside ? c.take<double>((size_t)Rp * zp) : nullptr;
            h->Zraw[l] = c.take<double>((size_t)np * zp);
            h->M2[l] = c.take<double>((size_t)zp * zp);
            h->P2[l] = c.take<double>((size_t)zp * zp);
            h->Qn2[l] = c.take<double>((size_t)zp * zp);
            h->Mg2[l] = c.take<double>((size_t)zp * zp);
            h->Pf[l] = c.take<double>((size_t)zp * zp);
            h->S2[l] = c.take<double>((size_t)zp * zp);
            h->lam2[l] = c.take<double>(zp);
            h->dd2[l] = c.take<double>(zp);
            h->ee2[l] = c.take<double>(zp);
            h->tau2[l] = c.take<double>(zp);
        }
    }
    return c.off;
}

// lay out the workspace for (n, R, precision); grows the allocation when needed
rhosvd_status layout(rhosvd_ctx* h, int64_t n, int64_t R) {
    h->n = n;
    h->R = R;
    h->n_pad = round_up(n, PAD_N);
    h->R_pad = round_up(R, PAD_R);
    h->rside = R < n && !h->force_nside;
    h->lp_gram = h->opt.gram_precision != 0 && n <= R;
    h->gram_used = h->lp_gram ? h->opt.gram_precision : 0;
    h->m = h->rside ? R : n;                     // the Gram's size
    h->m_pad = h->rside ? h->R_pad : h->n_pad;   // Gram on the min(n, R) side
    h->zr_pad = round_up(h->m, RPAD_CORE);       // max padded rank
    const int64_t mp = h->m_pad, Rp = h->R_pad;
    // split-K for the Gram when there are few output tiles
    const int64_t tiles = 3 * (mp / 64) * (mp / 64 + 1) / 2;
    int splits = (int)ceil_div(512, tiles);
    const int64_t kmax = Rp / 256;               // keep >= 256 terms per split
    if (splits > kmax) splits = (int)kmax;
    if (splits < 1) splits = 1;
    h->gram_splits = splits;
    const int64_t rt = Rp / 64;
    h->anorm_ntiles = rt * (rt + 1) / 2;
    const size_t need = carve_all(h, nullptr);
    if (need > h->ws_bytes) {
        if (h->ws) { hipStreamSynchronize(h->stream); h->alloc.put(h->ws); h->ws = nullptr; h->ws_bytes = 0; }
        if (!(h->ws = (char*)h->alloc.get(need))) {
            return fail(h, RHOSVD_ERR_ALLOC, "workspace allocation of " + std::to_string(need) + " bytes failed");
        }
        h->ws_bytes = need;
    }
    carve_all(h, h->ws);
    h->vprec = h->opt.precision;
    return RHOSVD_OK;
}

// (Re)build eigensolver plan `which` when the matrix list changed; the plan's
// tables are uploaded once and reused by every later call with the same layout.
rhosvd_status ensure_plan(rhosvd_ctx* h, int which, const EigMat* mats, int nmat) {
    std::vector<EigMat>& key = h->plan_mats[which];
    if (h->plan[which] && (int)key.size() == nmat && memcmp(key.data(), mats, nmat * sizeof(EigMat)) == 0)
        return RHOSVD_OK;
    if (h->plan[which]) {
        hipStreamSynchronize(h->stream);   // its tables may still be in use
        eig_plan_destroy(h->plan[which]);
        h->plan[which] = nullptr;
    }
    size_t need = 0;
    EigPlan* P = eig_plan_create(mats, nmat, &need);
    if (!P) return fail(h, RHOSVD_ERR_UNSUPPORTED, "eigensolver plan: matrix sizes not supported on this device");
    if (need > h->plan_wbytes[which]) {
        if (h->plan_w[which]) { hipStreamSynchronize(h->stream); h->alloc.put(h->plan_w[which]); h->plan_w[which] = nullptr; }
        h->plan_wbytes[which] = 0;
        if (!(h->plan_w[which] = h->alloc.get(need))) {
            eig_plan_destroy(P);
            return fail(h, RHOSVD_ERR_ALLOC, "eigensolver work allocation failed");
        }
        h->plan_wbytes[which] = need;
    }
    hipError_t e = eig_plan_bind(P, h->plan_w[which], h->stream);
    if (e != hipSuccess) {
        eig_plan_destroy(P);
        return fail(h, RHOSVD_ERR_DEVICE, std::string("eigensolver plan upload: ") + hipGetErrorString(e));
    }
    h->plan[which] = P;
    key.assign(mats, mats + nmat);
    return RHOSVD_OK;
}

// workspace of the learned path for the current layout (p_cap columns of the
// test matrix); base == nullptr only measures
size_t carve_learned(rhosvd_ctx* h, char* base, int p_cap) {
    Carve c{base};
    auto& L = h->L;
    const size_t np = h->n_pad, Rp = h->R_pad, pc = p_cap, zp = h->zr_pad;
    L.Om32 = c.take<double>(Rp * 64);
    for (int l = 0; l < 3; ++l) {
        L.Om[l] = c.take<double>(Rp * pc);
        L.Y[l] = c.take<double>(np * pc);
        L.Qb[l] = c.take<double>(np * pc);
        L.G2[l] = c.take<double>(pc * pc);
        L.W2[l] = c.take<double>(pc * pc);
        L.Qn2[l] = c.take<double>(pc * pc);
        L.Mg2[l] = c.take<double>(pc * pc);
        L.Pf[l] = c.take<double>(pc * pc);
        L.S2[l] = c.take<double>(pc * pc);
        L.lam2[l] = c.take<double>(pc);
        L.dd2[l] = c.take<double>(pc);
        L.ee2[l] = c.take<double>(pc);
        L.tau2[l] = c.take<double>(pc);
        L.Bm[l] = c.take<double>(pc * Rp);
        L.Tw[l] = c.take<double>(backtransform_work_doubles((int)pc));
        L.part[l] = c.take<double>((np / 64) * (Rp / 64));
        L.Wsel[l] = c.take<double>(pc * zp);
    }
    L.floor2 = c.take<double>(4);
    L.feat = c.take<float>(3 * NET_IN);
    L.out = c.take<float>(3 * NET_OUT);
    return c.off;
}

rhosvd_status learned_layout(rhosvd_ctx* h, int p_cap) {
    const size_t need = carve_learned(h, nullptr, p_cap);
    if (need > h->L.bytes) {
        if (h->L.ws) { hipStreamSynchronize(h->stream); h->alloc.put(h->L.ws); h->L.ws = nullptr; h->L.bytes = 0; }
        if (!(h->L.ws = (char*)h->alloc.get(need))) {
            return fail(h, RHOSVD_ERR_ALLOC, "learned-path workspace allocation of " + std::to_string(need) + " bytes failed");
        }
        h->L.bytes = need;
    }
    carve_learned(h, h->L.ws, p_cap);
    h->L.p_cap = p_cap;
    return RHOSVD_OK;
}

// features of the three modes into h->L.feat (normalized side matrices in h->Ut):
// sketch Y_l = U~_l Omega[:, :32], eigenvalues of Y_l^T Y_l, log-spectrum features
rhosvd_status learned_features(rhosvd_ctx* h, const double* omega, int w, double eps) {
    hipStream_t st = h->stream;
    auto& L = h->L;
    const int64_t np = h->n_pad, Rp = h->R_pad;
    CK(h, launch_pad_omega(h->R, Rp, std::min(w, 32), 64, omega, L.Om32, st));
    EigMat em[3];
    for (int l = 0; l < 3; ++l) {
        CK(h, launch_gemm64(false, true, np, 64, Rp, h->Ut[l], np, L.Om32, Rp, L.Y[l], np, 1.0, st));
        CK(h, launch_gemm64(true, true, 64, 64, np, L.Y[l], np, L.Y[l], np, L.G2[l], 64, 1.0, st));
        em[l] = EigMat{L.G2[l], L.lam2[l], L.W2[l], L.Qn2[l], L.Mg2[l], L.dd2[l], L.ee2[l], L.tau2[l], 32, 64};
    }
    rhosvd_status ps = ensure_plan(h, 2, em, 3);
    if (ps != RHOSVD_OK) return ps;
    CK(h, eig_plan_enqueue(h->plan[2], h->flags + 2, st));
    const double* lam[3] = {L.lam2[0], L.lam2[1], L.lam2[2]};
    CK(h, launch_features(lam, (int)h->n, h->R, eps, L.feat, st));
    return RHOSVD_OK;
}

// R < n: Z = U~ W_r Lambda_r^(-1/2) (the left singular vectors from the right
// ones), then re-orthonormalized in FP64 by Z <- Z (Z^T Z)^(-1/2) (symmetric
// orthogonalization, Z^T Z = P diag(mu) P^T from the same eigensolver) and
// sign-normalized.
rhosvd_status form_z_rside(rhosvd_ctx* h) {
    hipStream_t st = h->stream;
    const int64_t np = h->n_pad, Rp = h->R_pad, zp = h->zr_pad;
    int rmp = 0;
    for (int l = 0; l < 3; ++l) rmp = h->r_pad[l] > rmp ? h->r_pad[l] : rmp;
    BtJob jobs[3];
    for (int l = 0; l < 3; ++l) {
        CK(h, hipMemsetAsync(h->Wr[l], 0, (size_t)Rp * zp * 8, st));
        jobs[l] = BtJob{(int)h->m, (int)h->m_pad, h->G[l], h->htau[l], h->W[l], h->order[l], h->ranks[l], nullptr,
                        h->Wr[l], (int)Rp, (int)Rp, h->Tw[l]};
    }
    CK(h, launch_backtransform(jobs, 3, st));
    for (int l = 0; l < 3; ++l) {
        const int r = h->ranks[l], rp = h->r_pad[l];
        CK(h, launch_gather_scaled((int)Rp, r, rp, h->Wr[l], nullptr, h->sigma[l], h->Wr[l], st));
        CK(h, hipMemsetAsync(h->Zraw[l], 0, (size_t)np * zp * 8, st));
        CK(h, launch_gemm64(false, true, np, rp, Rp, h->Ut[l], np, h->Wr[l], Rp, h->Zraw[l], np, 1.0, st));
        CK(h, launch_gemm64(true, true, rp, rp, np, h->Zraw[l], np, h->Zraw[l], np, h->M2[l], zp, 1.0, st));
        CK(h, launch_pad_identity(r, rmp, (int)zp, h->M2[l], st));
    }
    EigMat em[3];
    for (int l = 0; l < 3; ++l)
        em[l] = EigMat{h->M2[l], h->lam2[l], h->P2[l], h->Qn2[l], h->Mg2[l], h->dd2[l], h->ee2[l], h->tau2[l], rmp, (int)zp};
    rhosvd_status ps = ensure_plan(h, 1, em, 3);
    if (ps != RHOSVD_OK) return ps;
    CK(h, eig_plan_enqueue(h->plan[1], h->flags + 2, st));
    // P = H P2 (all rmp columns); S = P diag(mu^-1/2) P^T ; Z = Zraw S
    for (int l = 0; l < 3; ++l)
        jobs[l] = BtJob{rmp, (int)zp, h->M2[l], h->tau2[l], h->P2[l], nullptr, rmp, nullptr, h->Pf[l], (int)zp, rmp,
                        h->Tw[l]};
    CK(h, launch_backtransform(jobs, 3, st));
    for (int l = 0; l < 3; ++l) {
        CK(h, launch_scale_cols_invsqrt(rmp, (int)zp, h->lam2[l], h->Pf[l], h->S2[l], st));
        CK(h, launch_gemm64(false, false, rmp, rmp, rmp, h->S2[l], zp, h->Pf[l], zp, h->M2[l], zp, 1.0, st));
        CK(h, launch_gemm64(false, true, np, rmp, rmp, h->Zraw[l], np, h->M2[l], zp, h->Z[l], np, 1.0, st));
        CK(h, launch_sign_cols((int)h->n, (int)np, h->ranks[l], h->Z[l], st));
        if (h->r_pad[l] > h->ranks[l])
            CK(h, hipMemsetAsync(h->Z[l] + (int64_t)h->ranks[l] * np, 0,
                                 (size_t)(h->r_pad[l] - h->ranks[l]) * np * 8, st));
    }
    return RHOSVD_OK;
}

// truncation arguments of the Gram path for the current layout (|A| from h->a2_part)
TruncArgs trunc_args(rhosvd_ctx* h, double eps) {
    TruncArgs ta{};
    for (int l = 0; l < 3; ++l) {
        ta.lam[l] = h->lam[l];
        ta.sigma[l] = h->sigma[l];
        ta.order[l] = h->order[l];
        ta.tails[l] = h->tails[l];
    }
    ta.m = (int)h->m;
    ta.m_pad = (int)h->m_pad;
    ta.n = (int)h->n;
    ta.n_pad = (int)h->n_pad;
    ta.xip = h->xip;
    ta.R_pad = h->R_pad;
    ta.anorm_part = h->a2_part;
    ta.anorm_ntiles = h->a2_n;
    ta.eps = eps;
    ta.ranks = h->ranks_dev;
    ta.scal = h->scal;
    return ta;
}

constexpr double PROBE_TAIL = 1.0 / 30.0;   // probe ranks: t_{l,p} <= 1/30 (b_p <= |xi'| / 10)
constexpr double PROBE_GAP = 0.1;           // auto mode keeps the probe only if b_p <= L / 10
constexpr int PROBE_NPART = 256;

// |A| after the eigensolver (n <= R), for rhosvd_options.anorm = 0 or 2.  Probe
// ranks p_l = min{p : t_{l,p} <= 1/30}; Z = all m back-transformed eigenvectors
// (sign rule applied; later steps use its leading columns); V_p = Z_p^T U~ and
// beta_p = the FP64 core at the probe ranks; |beta_p|^2 partial sums become the
// truncation's |A|^2.  |beta_p| <= |A| (beta_p is the core of an orthogonal
// projection of A), and Theorem 2.3 at the probe ranks gives |A|^2 <= |beta_p|^2 +
// b_p^2 with b_p = |xi'| sum_l t_{l,p_l}.  Falls back to the exact identity in
// auto mode when the probe would cost more than half the identity's flops or
// b_p > L / 10.  *z_all is set when Z already holds every eigenvector.
rhosvd_status anorm_probe(rhosvd_ctx* h, int mode, bool* z_all) {
    hipStream_t st = h->stream;
    const int64_t np = h->n_pad, Rp = h->R_pad;
    const int m = (int)h->m;
    *z_all = false;
    auto exact = [&]() -> rhosvd_status {
        int64_t nt = 0;
        CK(h, launch_anorm_partials(h->n_pad, h->R_pad, h->Ut, h->xip, h->anorm_part, &nt, nullptr, st));
        h->a2_part = h->anorm_part;
        h->a2_n = h->anorm_ntiles;
        h->anorm_method = 1;
        h->a_upper = -1.0;
        return RHOSVD_OK;
    };
    TruncArgs tp = trunc_args(h, 1.0);
    tp.anorm_part = nullptr;
    tp.anorm_ntiles = 0;
    tp.tau_fixed = PROBE_TAIL;
    CK(h, launch_truncate(tp, st));
    CK(h, hipMemcpyAsync(h->host, h->ranks_dev, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(h, hipMemcpyAsync(h->hostd, h->scal, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(h, hipStreamSynchronize(st));
    int p[3];
    double tp_sum = 0.0;
    for (int l = 0; l < 3; ++l) {
        p[l] = std::min(h->host[l], m);
        tp_sum += h->hostd[3 + l];
    }
    const double xi_norm = h->hostd[0];
    if (p[0] < 1 || p[1] < 1 || p[2] < 1 || !(xi_norm > 0.0)) return exact();
    const double R = (double)h->R, n = (double)h->n;
    const double probe_flops = 2.0 * p[0] * p[1] * p[2] * R + 2.0 * n * (p[0] + p[1] + p[2]) * R;
    const double exact_flops = 3.0 * n * R * R;
    if (mode == 0 && 2.0 * probe_flops > exact_flops) return exact();
    int pp[3];
    for (int l = 0; l < 3; ++l) pp[l] = (int)round_up(p[l], RPAD_CORE);
    // probe workspace: V_p (FP64, three modes), beta_p, partial sums
    const size_t vbytes = a256((size_t)(pp[0] + pp[1] + pp[2]) * Rp * 8);
    const size_t bbytes = a256((size_t)p[0] * p[1] * p[2] * 8);
    const size_t need = vbytes + bbytes + a256(PROBE_NPART * 8);
    if (need > h->pw_bytes) {
        if (h->pw) { CK(h, hipStreamSynchronize(st)); h->alloc.put(h->pw); h->pw = nullptr; h->pw_bytes = 0; }
        if (!(h->pw = (char*)h->alloc.get(need))) {
            return fail(h, RHOSVD_ERR_ALLOC, "|A| probe workspace allocation of " + std::to_string(need) + " bytes failed");
        }
        h->pw_bytes = need;
    }
    double* Vp[3];
    Vp[0] = (double*)h->pw;
    Vp[1] = Vp[0] + (size_t)pp[0] * Rp;
    Vp[2] = Vp[1] + (size_t)pp[1] * Rp;
    double* beta_p = (double*)(h->pw + vbytes);
    double* part = (double*)(h->pw + vbytes + bbytes);
    // every eigenvector, back-transformed and sign-normalized, into Z
    BtJob jobs[3];
    for (int l = 0; l < 3; ++l)
        jobs[l] = BtJob{m, (int)h->m_pad, h->G[l], h->htau[l], h->W[l], h->order[l], m, nullptr, h->Z[l], (int)np,
                        (int)np, h->Tw[l]};
    CK(h, launch_backtransform(jobs, 3, st));
    for (int l = 0; l < 3; ++l) {
        CK(h, launch_sign_cols((int)h->n, (int)np, m, h->Z[l], st));
        if (h->zr_pad > m)
            CK(h, hipMemsetAsync(h->Z[l] + (int64_t)m * np, 0, (size_t)(h->zr_pad - m) * np * 8, st));
        CK(h, launch_project(np, Rp, pp[l], h->Z[l], h->Ut[l], Vp[l], nullptr, st));
    }
    *z_all = true;
    CoreArgs ca{};
    for (int l = 0; l < 3; ++l) {
        ca.r[l] = p[l];
        ca.r_pad[l] = pp[l];
        ca.V[l] = Vp[l];
    }
    ca.R_pad = Rp;
    ca.xip = h->xip;
    ca.beta = beta_p;
    ca.prec = RHOSVD_FP64;
    ca.tile = 64;
    CK(h, launch_core(ca, st));
    CK(h, launch_sumsq_partials(beta_p, (int64_t)p[0] * p[1] * p[2], part, PROBE_NPART, st));
    CK(h, hipMemcpyAsync(h->hostd + 64, part, PROBE_NPART * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(h, hipStreamSynchronize(st));
    double L2 = 0.0;
    for (int i = 0; i < PROBE_NPART; ++i) L2 += h->hostd[64 + i];
    const double L = sqrt(std::max(L2, 0.0)), bp = xi_norm * tp_sum;
    if (mode == 0 && !(bp <= PROBE_GAP * L)) return exact();
    h->a2_part = part;
    h->a2_n = PROBE_NPART;
    h->anorm_method = 2;
    h->a_upper = sqrt(L * L + bp * bp);
    return RHOSVD_OK;
}

// ALS sweeps at fixed ranks (rhosvd_options.als_sweeps; n <= R).  For mode l with
// the others a, b: P = diag(xi') (V_a^T V_a o V_b^T V_b) diag(xi'), G = U~_l P U~_l^T
// (= M_l M_l^T for the contracted unfolding M_l = U~_l diag(xi') (V_b (.) V_a)^T),
// Z_l = its r_l leading eigenvectors (same eigensolver, sign rule), V_l = Z_l^T U~_l.
// Modes are updated in the order 0, 1, 2, each with the others' latest V.  Uses the
// mode-0 eigensolver buffers for every mode; leaves V in the path's precision.
rhosvd_status als_refine(rhosvd_ctx* h) {
    hipStream_t st = h->stream;
    const int64_t np = h->n_pad, Rp = h->R_pad, mp = h->m_pad;
    const int m = (int)h->m;
    const bool f64 = h->vprec == RHOSVD_FP64;
    double* V64[3];
    for (int l = 0; l < 3; ++l) {
        V64[l] = f64 ? (double*)h->V[l] : h->V64a[l];
        if (!f64) CK(h, launch_project(np, Rp, h->r_pad[l], h->Z[l], h->Ut[l], V64[l], nullptr, st));
    }
    EigMat em{h->G[0], h->lam[0], h->W[0], h->Qn[0], h->Mg[0], h->dd[0], h->ee[0], h->htau[0], m, (int)mp};
    rhosvd_status s = ensure_plan(h, 4, &em, 1);
    if (s != RHOSVD_OK) return s;
    for (int sweep = 0; sweep < h->opt.als_sweeps; ++sweep) {
        for (int l = 0; l < 3; ++l) {
            const int a = l == 0 ? 1 : 0, b = l == 2 ? 1 : 2;
            CK(h, launch_gemm64(true, true, Rp, Rp, h->r_pad[a], V64[a], h->r_pad[a], V64[a], h->r_pad[a], h->Ha, Rp,
                                1.0, st));
            CK(h, launch_gemm64(true, true, Rp, Rp, h->r_pad[b], V64[b], h->r_pad[b], V64[b], h->r_pad[b], h->Hb, Rp,
                                1.0, st));
            CK(h, launch_als_hadamard(Rp, h->Ha, h->Hb, h->xip, st));
            CK(h, launch_gemm64(false, true, np, Rp, Rp, h->Ut[l], np, h->Ha, Rp, h->Tals, np, 1.0, st));
            CK(h, launch_gemm64(false, false, np, np, Rp, h->Tals, np, h->Ut[l], np, h->G[0], mp, 1.0, st));
            CK(h, eig_plan_enqueue(h->plan[4], h->flags + 2, st));
            CK(h, launch_order_desc(h->lam[0], m, h->order[0], st));
            const int r = h->ranks[l];
            BtJob jb{m, (int)mp, h->G[0], h->htau[0], h->W[0], h->order[0], r, nullptr, h->Z[l], (int)np, (int)np,
                     h->Tw[0]};
            CK(h, launch_backtransform(&jb, 1, st));
            CK(h, launch_sign_cols((int)h->n, (int)np, r, h->Z[l], st));
            if (h->r_pad[l] > r)
                CK(h, hipMemsetAsync(h->Z[l] + (int64_t)r * np, 0, (size_t)(h->r_pad[l] - r) * np * 8, st));
            CK(h, launch_project(np, Rp, h->r_pad[l], h->Z[l], h->Ut[l], V64[l], nullptr, st));
        }
    }
    if (!f64)
        for (int l = 0; l < 3; ++l)
            CK(h, launch_project(np, Rp, h->r_pad[l], h->Z[l], h->Ut[l], nullptr, (float*)h->V[l], st));
    return RHOSVD_OK;
}

// refine_tails = 2 (n <= R): a second, deflated Gram pass.  The leading k_l
// eigenvectors of the first pass (sigma >= 2^-13 sigma_1, where the FP64 Gram
// route is accurate) form Z_k; the side matrix is deflated twice,
// U'' = (I - Z_k Z_k^T)^2 U~, so that its Gram has norm ~sigma_{k+1}^2 and
// resolves singular values down to ~u^(1/2) sigma_{k+1} instead of ~u^(1/2)
// sigma_1.  The cut is taken on the deflated spectrum with the same tau (the
// tails of U~ beyond Z_k are those of U''); Z = [Z_k, Z'] with Z' the leading
// deflated eigenvectors, projected once more against Z_k.
rhosvd_status deflate_pass(rhosvd_ctx* h, double eps) {
    hipStream_t st = h->stream;
    const int64_t np = h->n_pad, Rp = h->R_pad, mp = h->m_pad, zp = h->zr_pad;
    const int m = (int)h->m;
    std::vector<double> sg((size_t)3 * m);
    for (int l = 0; l < 3; ++l)
        CK(h, hipMemcpyAsync(sg.data() + (size_t)l * m, h->sigma[l], (size_t)m * 8, hipMemcpyDeviceToHost, st));
    CK(h, hipStreamSynchronize(st));
    int k[3];
    double *sig1[3], *sig2[3], *tl2[3];
    for (int l = 0; l < 3; ++l) {
        const double s1 = sg[(size_t)l * m];
        int kk = 0;
        while (kk < m && sg[(size_t)l * m + kk] >= s1 * 0x1p-13) ++kk;
        k[l] = std::max(0, std::min(kk, h->ranks[l] - 1));
        sig1[l] = h->dscr + (size_t)l * 3 * (mp + 64);
        sig2[l] = sig1[l] + (mp + 64);
        tl2[l] = sig2[l] + (mp + 64);
        CK(h, hipMemcpyAsync(sig1[l], h->sigma[l], (size_t)m * 8, hipMemcpyDeviceToDevice, st));
    }
    // Z_k from the first pass (its Householder vectors are still in G)
    BtJob jobs[3];
    for (int l = 0; l < 3; ++l) {
        CK(h, hipMemsetAsync(h->Z[l], 0, (size_t)np * zp * 8, st));
        jobs[l] = BtJob{m, (int)mp, h->G[l], h->htau[l], h->W[l], h->order[l], k[l], nullptr, h->Z[l], (int)np,
                        (int)np, h->Tw[l]};
    }
    CK(h, launch_backtransform(jobs, 3, st));
    int kp[3];
    for (int l = 0; l < 3; ++l) {
        kp[l] = (int)round_up(std::max(k[l], 1), 64);
        double* V64 = h->vprec == RHOSVD_FP64 ? (double*)h->V[l] : h->Vref[l];
        CK(h, launch_project(np, Rp, kp[l], h->Z[l], h->Ut[l], V64, nullptr, st));
        CK(h, launch_residual(np, Rp, kp[l], h->Z[l], V64, h->Ut[l], h->Ud[l], st));
        CK(h, launch_project(np, Rp, kp[l], h->Z[l], h->Ud[l], V64, nullptr, st));
        CK(h, launch_residual(np, Rp, kp[l], h->Z[l], V64, h->Ud[l], h->Ud[l], st));
    }
    // the deflated Grams through the same eigensolver plan (same buffers)
    CK(h, launch_gram_nt(np, Rp, h->Ud, h->G, h->gram_part, h->gram_splits, st));
    CK(h, eig_plan_enqueue(h->plan[0], h->flags + 2, st));
    TruncArgs ta{};
    for (int l = 0; l < 3; ++l) {
        ta.lam[l] = h->lam[l];
        ta.sigma[l] = h->sigma[l];
        ta.order[l] = h->order[l];
        ta.tails[l] = h->tails[l];
    }
    ta.m = m;
    ta.m_pad = (int)mp;
    ta.n = (int)h->n;
    ta.n_pad = (int)np;
    ta.xip = h->xip;
    ta.R_pad = Rp;
    ta.anorm_part = h->a2_part;
    ta.anorm_ntiles = h->a2_n;
    ta.eps = eps;
    ta.ranks = h->ranks_dev;
    ta.scal = h->scal;
    CK(h, launch_truncate(ta, st));
    CK(h, hipMemcpyAsync(h->host, h->ranks_dev, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(h, hipMemcpyAsync(h->host + 6, h->flags + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(h, hipStreamSynchronize(st));
    if (h->host[6]) return fail(h, RHOSVD_ERR_DEVICE, "eigensolver: a cross-workgroup wait ran out");
    for (int l = 0; l < 3; ++l) {
        const int r2 = std::max(1, std::min(h->host[l], m - k[l]));
        // combined spectrum and tails
        CK(h, hipMemcpyAsync(sig2[l], h->sigma[l], (size_t)m * 8, hipMemcpyDeviceToDevice, st));
        CK(h, hipMemcpyAsync(tl2[l], h->tails[l], (size_t)(m + 1) * 8, hipMemcpyDeviceToDevice, st));
        CK(h, launch_combine_spectrum(k[l], m, sig1[l], sig2[l], tl2[l], h->sigma[l], h->tails[l], st));
        // Z' = the leading r2 deflated eigenvectors, projected against Z_k once more
        CK(h, hipMemsetAsync(h->Zs[l], 0, (size_t)np * zp * 8, st));
        BtJob jb{m, (int)mp, h->G[l], h->htau[l], h->W[l], h->order[l], r2, nullptr, h->Zs[l], (int)np, (int)np,
                 h->Tw[l]};
        CK(h, launch_backtransform(&jb, 1, st));
        CK(h, launch_project(np, zp, kp[l], h->Z[l], h->Zs[l], h->Cz[l], nullptr, st));
        CK(h, launch_residual(np, zp, kp[l], h->Z[l], h->Cz[l], h->Zs[l], h->Zs[l], st));
        CK(h, hipMemcpyAsync(h->Z[l] + (int64_t)k[l] * np, h->Zs[l], (size_t)r2 * np * 8, hipMemcpyDeviceToDevice,
                             st));
        const int r = k[l] + r2;
        CK(h, launch_sign_cols((int)h->n, (int)np, r, h->Z[l], st));
        h->ranks[l] = r;
        h->r_pad[l] = (int)round_up(r, RPAD_CORE);
        if (zp > r) CK(h, hipMemsetAsync(h->Z[l] + (int64_t)r * np, 0, (size_t)(zp - r) * np * 8, st));
    }
    return RHOSVD_OK;
}

// Reduced-precision Gram (rhosvd_options.gram_precision): the Rayleigh-Ritz step.
// Q = the leading p eigenvectors of that Gram (its own cut r, p = min(m, r + r/8 + 16)),
// B = Q^T U~ in FP64, the residual |U~ - Q B|_F^2 formed directly and B B^T
// eigendecomposed by the FP64 eigensolver.  For orthonormal Q, with B B^T = Y S^2 Y^T,
// |(I - (QY)_r (QY)_r^T) U~|_F^2 = sum_{k>r} s_k^2 + |U~ - Q B|_F^2, so the cut on those
// tails is certified by Theorem 2.3 for Z = Q Y[:, 0:r], whatever the accuracy of Q.
// Where no r <= p certifies (the residual alone exceeds tau), p grows (2p + 64, at
// most m) and the step repeats.
rhosvd_status rr_pass(rhosvd_ctx* h, double eps) {
    hipStream_t st = h->stream;
    const int64_t np = h->n_pad, Rp = h->R_pad, zp = h->zr_pad;
    const int m = (int)h->m;
    const int64_t ntl = (np / 64) * (Rp / 64);
    int p[3], pp[3];
    for (int l = 0; l < 3; ++l) p[l] = std::min(m, std::max(1, h->ranks[l]) + h->ranks[l] / 8 + 16);
    for (;;) {
        BtJob jobs[3];
        for (int l = 0; l < 3; ++l) {
            pp[l] = (int)round_up(p[l], RPAD_CORE);
            jobs[l] = BtJob{m, (int)h->m_pad, h->G[l], h->htau[l], h->W[l], h->order[l], p[l], nullptr, h->Zraw[l],
                            (int)np, (int)np, h->Tw[l]};
        }
        CK(h, launch_backtransform(jobs, 3, st));
        EigMat em[3];
        for (int l = 0; l < 3; ++l) {
            if (pp[l] > p[l])
                CK(h, hipMemsetAsync(h->Zraw[l] + (int64_t)p[l] * np, 0, (size_t)(pp[l] - p[l]) * np * 8, st));
            CK(h, launch_project(np, Rp, pp[l], h->Zraw[l], h->Ut[l], h->Brr[l], nullptr, st));
            CK(h, launch_resid_partials(np, Rp, pp[l], h->Zraw[l], h->Brr[l], h->Ut[l], h->rpart[l], st));
            CK(h, launch_floor_sum(h->rpart[l], ntl, h->rfloor + l, st));
            CK(h, launch_gemm64(false, false, pp[l], pp[l], Rp, h->Brr[l], pp[l], h->Brr[l], pp[l], h->M2[l], zp, 1.0,
                                st));
            em[l] = EigMat{h->M2[l], h->lam2[l], h->P2[l], h->Qn2[l], h->Mg2[l], h->dd2[l], h->ee2[l], h->tau2[l], p[l],
                           (int)zp};
        }
        rhosvd_status ps = ensure_plan(h, 1, em, 3);
        if (ps != RHOSVD_OK) return ps;
        CK(h, eig_plan_enqueue(h->plan[1], h->flags + 2, st));
        TruncArgs ta = trunc_args(h, eps);
        for (int l = 0; l < 3; ++l) {
            ta.lam[l] = h->lam2[l];
            ta.m_mode[l] = p[l];
            ta.order[l] = h->rr_order[l];
            CK(h, hipMemsetAsync(h->sigma[l], 0, (size_t)(h->m_pad + 1) * 8, st));
        }
        ta.floor2 = h->rfloor;
        CK(h, launch_truncate(ta, st));
        CK(h, hipMemcpyAsync(h->host, h->ranks_dev, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
        CK(h, hipMemcpyAsync(h->host + 6, h->flags + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        CK(h, hipStreamSynchronize(st));
        if (h->host[6]) return fail(h, RHOSVD_ERR_DEVICE, "eigensolver: a cross-workgroup wait ran out");
        bool again = false;
        for (int l = 0; l < 3; ++l) {
            if (h->host[l] < 1 || h->host[l] > p[l] + 1)
                return fail(h, RHOSVD_ERR_DEVICE, "Rayleigh-Ritz cut returned rank " + std::to_string(h->host[l]) +
                                                      " (internal error)");
            if (h->host[l] > p[l] && p[l] < m) {
                p[l] = (int)std::min<int64_t>(m, 2 * (int64_t)p[l] + 64);
                again = true;
            }
        }
        if (!again) break;
    }
    // Z = Q Y[:, order[0..r)], sign rule, zero padding
    BtJob jobs[3];
    for (int l = 0; l < 3; ++l) {
        // p + 1 at p = m: not even the full basis certifies (tau below the residual's
        // rounding); keep m, as the refined cut does
        const int r = std::min(h->host[l], p[l]);
        h->ranks[l] = r;
        h->r_pad[l] = (int)round_up(r, RPAD_CORE);
        jobs[l] = BtJob{p[l], (int)zp, h->M2[l], h->tau2[l], h->P2[l], h->rr_order[l], r, nullptr, h->Pf[l], (int)zp,
                        (int)zp, h->Tw[l]};
    }
    CK(h, launch_backtransform(jobs, 3, st));
    for (int l = 0; l < 3; ++l) {
        const int r = h->ranks[l];
        CK(h, launch_gemm64(false, true, np, h->r_pad[l], pp[l], h->Zraw[l], np, h->Pf[l], zp, h->Z[l], np, 1.0, st));
        CK(h, launch_sign_cols((int)h->n, (int)np, r, h->Z[l], st));
        if (h->r_pad[l] > r)
            CK(h, hipMemsetAsync(h->Z[l] + (int64_t)r * np, 0, (size_t)(h->r_pad[l] - r) * np * 8, st));
    }
    return RHOSVD_OK;
}

}  // namespace

extern "C" {

const char* rhosvd_version(void) { return RHOSVD_VERSION; }

const char* rhosvd_last_error(rhosvd_handle h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

rhosvd_status rhosvd_create(rhosvd_handle* out, void* hip_stream, const rhosvd_options* opt) {
    return rhosvd_create_with_allocator(out, hip_stream, nullptr, opt);
}

rhosvd_status rhosvd_create_with_allocator(rhosvd_handle* out, void* hip_stream, const rhosvd_allocator* allocator,
                                           const rhosvd_options* opt) {
    if (!out) { g_create_error = "out is NULL"; return RHOSVD_ERR_ARG; }
    if (allocator && (!allocator->alloc || !allocator->free)) {
        g_create_error = "allocator needs both alloc and free";
        return RHOSVD_ERR_ARG;
    }
    *out = nullptr;
    std::string msg;
    rhosvd_status s = check_options(opt, msg);
    if (s != RHOSVD_OK) { g_create_error = msg; return s; }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        g_create_error = "no HIP device";
        return RHOSVD_ERR_DEVICE;
    }
    rhosvd_ctx* h = new rhosvd_ctx();
    h->stream = (hipStream_t)hip_stream;
    if (allocator) h->alloc.a = *allocator;
    apply_options(h, opt);
    h->tuner = core_tuner_create();
    if (hipHostMalloc((void**)&h->host, HOST_BYTES, hipHostMallocDefault) != hipSuccess) {
        delete h;
        g_create_error = "pinned host allocation failed";
        return RHOSVD_ERR_ALLOC;
    }
    // host staging words: 0..2 ranks, 4..6 flags, 8 abort word (report), 32.. doubles
    // (0..2 norms, 3..5 probe tails, 4..6 tails, 8..10 range-finder residuals;
    // 64 .. 64 + PROBE_NPART probe partial sums), 56..61 network outputs
    h->hostd = (double*)(h->host + 32);
    h->ev_ok = true;
    for (int i = 0; i < NEV; ++i)
        if (hipEventCreate(&h->ev[i]) != hipSuccess) h->ev_ok = false;
    *out = h;
    return RHOSVD_OK;
}

rhosvd_status rhosvd_destroy(rhosvd_handle h) {
    if (!h) return RHOSVD_ERR_ARG;
    hipStreamSynchronize(h->stream);
    h->alloc.put(h->ws);
    h->alloc.put(h->pw);
    if (h->batch) batch_plan_destroy(h->batch);
    h->alloc.put(h->net);
    h->alloc.put(h->L.ws);
    h->alloc.put(h->T.ws);
    h->alloc.put(h->T.lw);
    h->alloc.put(h->net_work);
    for (int i = 0; i < rhosvd_ctx::NPLAN; ++i) {
        if (h->plan[i]) eig_plan_destroy(h->plan[i]);
        h->alloc.put(h->plan_w[i]);
    }
    if (h->host) hipHostFree(h->host);
    for (int i = 0; i < NEV; ++i)
        if (h->ev[i]) hipEventDestroy(h->ev[i]);
    core_tuner_destroy(h->tuner);
    delete h;
    return RHOSVD_OK;
}

rhosvd_status rhosvd_set_options(rhosvd_handle h, const rhosvd_options* opt) {
    if (!h) return RHOSVD_ERR_ARG;
    std::string msg;
    rhosvd_status s = check_options(opt, msg);
    if (s != RHOSVD_OK) return fail(h, s, msg);
    apply_options(h, opt);
    h->have = false;
    return RHOSVD_OK;
}

rhosvd_status rhosvd_reduce(rhosvd_handle h, int64_t n, int64_t R, const double* U1, const double* U2,
                            const double* U3, const double* xi, double eps, int32_t ranks[3]) {
    if (!h) return RHOSVD_ERR_ARG;
    h->have = false;
    h->err.clear();
    if (!U1 || !U2 || !U3 || !xi || !ranks) return fail(h, RHOSVD_ERR_ARG, "null pointer argument");
    if (n < 1 || R < 1) return fail(h, RHOSVD_ERR_ARG, "n and R must be >= 1");
    if (!(eps > 0.0) || !isfinite(eps)) return fail(h, RHOSVD_ERR_ARG, "eps must be finite and > 0");
    if ((n < R ? n : R) > 2048) return fail(h, RHOSVD_ERR_UNSUPPORTED, "min(n, R) > 2048 is not supported by this library");
    if (n > 65536) return fail(h, RHOSVD_ERR_UNSUPPORTED, "n > 65536 is not supported by this library");
    if (h->opt.als_sweeps > 0 && (R < n || R > 16384))
        return fail(h, RHOSVD_ERR_UNSUPPORTED, "ALS sweeps need n <= R <= 16384");
    rhosvd_status s = layout(h, n, R);
    if (s != RHOSVD_OK) return s;
    h->eps = eps;
    hipStream_t st = h->stream;
    const double* U[3] = {U1, U2, U3};
    mark(h, 0);
    CK(h, hipMemsetAsync(h->flags, 0, 64, st));
    CK(h, launch_colnorm(n, R, h->n_pad, h->R_pad, U, xi, h->Ut, h->xip, h->flags, st));
    mark(h, 1);
    // |A|: the exact identity now (when R < n its tiles are the Grams U~^T U~ on the
    // R side), or after the eigensolver by the probe (rhosvd_options.anorm)
    const bool probe = !h->rside && h->opt.anorm != 1 && !h->lp_gram;
    h->a2_part = h->anorm_part;
    h->a2_n = h->anorm_ntiles;
    h->anorm_method = 1;
    h->a_upper = -1.0;
    if (!probe) {
        int64_t nt = 0;
        CK(h, launch_anorm_partials(h->n_pad, h->R_pad, h->Ut, h->xip, h->anorm_part, &nt,
                                    h->rside ? h->G : nullptr, st));
    }
    mark(h, 2);
    if (h->lp_gram)
        CK(h, launch_gram_lp(h->opt.gram_precision, h->n_pad, h->R_pad, h->Ut, h->G, h->gram_part, h->gram_splits,
                             st));
    else if (!h->rside)
        CK(h, launch_gram_nt(h->n_pad, h->R_pad, h->Ut, h->G, h->gram_part, h->gram_splits, st));
    mark(h, 3);
    EigMat em[3];
    for (int l = 0; l < 3; ++l)
        em[l] = EigMat{h->G[l], h->lam[l], h->W[l], h->Qn[l], h->Mg[l], h->dd[l], h->ee[l], h->htau[l], (int)h->m,
                       (int)h->m_pad};
    s = ensure_plan(h, 0, em, 3);
    if (s != RHOSVD_OK) return s;
    CK(h, eig_plan_enqueue(h->plan[0], h->flags + 2, st));
    mark(h, 4);
    bool z_all = false;   // the probe leaves every eigenvector in Z
    if (probe) {
        s = anorm_probe(h, h->opt.anorm, &z_all);
        if (s != RHOSVD_OK) return s;
    }
    {
        // a reduced-precision Gram's cut only sizes the Rayleigh-Ritz basis: its small
        // eigenvalues are noise of either sign, summed with their signs
        TruncArgs ta = trunc_args(h, eps);
        ta.signed_tails = h->lp_gram ? 1 : 0;
        CK(h, launch_truncate(ta, st));
    }
    // the one host synchronization: ranks, flags, sweeps and norms
    CK(h, hipMemcpyAsync(h->host, h->ranks_dev, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(h, hipMemcpyAsync(h->host + 4, h->flags, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(h, hipMemcpyAsync(h->hostd, h->scal, 12 * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(h, hipStreamSynchronize(st));
    if (h->host[4]) return fail(h, RHOSVD_ERR_NONFINITE, "input contains NaN or Inf");
    if (h->host[6]) return fail(h, RHOSVD_ERR_DEVICE, "eigensolver: a cross-workgroup wait ran out");
    for (int l = 0; l < 3; ++l)
        if (h->host[l] < 0 || h->host[l] > h->m)
            return fail(h, RHOSVD_ERR_DEVICE, "truncation returned rank " + std::to_string(h->host[l]) + " (internal error)");
    // refine_tails = 0 (auto): refined tails (mode 1) when some mode's cut lies in the
    // Gram route's noise band, lambda_r <= NOISE_BAND u lambda_1; else none
    // (the deflated pass, mode 2, when tau^2 itself lies in that band: the first pass's
    // vectors near such a cut are inaccurate, and only the deflated Gram resolves it)
    // (a reduced-precision Gram takes its own Rayleigh-Ritz step instead)
    int refine_mode = h->lp_gram ? REFINE_OFF : h->opt.refine_tails;
    if (refine_mode == REFINE_AUTO) {
        const double tau2 = h->hostd[2] * h->hostd[2];
        int want = 0;
        for (int l = 0; l < 3; ++l) {
            const double band = NOISE_BAND * U64H * h->hostd[6 + l];
            if (h->host[l] >= 1 && h->hostd[9 + l] <= band)
                want = std::max(want, tau2 <= band && !h->rside ? 2 : 1);
        }
        refine_mode = want ? want : REFINE_OFF;
    }
    if (refine_mode != REFINE_OFF && h->rside) {
        // The R-side route forms Z = U~ W Sigma^-1: its columns whose sigma^2 lies at
        // the Gram's rounding level lose orthonormality, and the refined tails (which
        // need orthonormal Z_p) would be wrong there.  The reduction runs again on the
        // n x n Gram, whose eigenvectors are orthonormal to working precision, with the
        // same refinement choice; beyond the eigensolver's size the plain cut stays.
        if (n <= 2048) {
            const rhosvd_options keep = h->opt;
            h->force_nside = true;
            h->opt.anorm = 1;
            rhosvd_status rs = rhosvd_reduce(h, n, R, U1, U2, U3, xi, eps, ranks);
            h->opt = keep;
            h->force_nside = false;
            if (rs == RHOSVD_OK) h->refine_used |= 4;
            return rs;
        }
        refine_mode = REFINE_OFF;
    }
    h->refine_used = refine_mode == REFINE_OFF ? 0 : refine_mode;
    h->sweeps = 0;
    h->dropped = h->host[5];
    h->xi_norm = h->hostd[0];
    h->a_norm = h->hostd[1];
    h->tau = h->hostd[2];
    for (int l = 0; l < 3; ++l) {
        h->ranks[l] = h->host[l];
        h->r_pad[l] = (int)round_up(h->ranks[l] > 0 ? h->ranks[l] : 1, RPAD_CORE);
    }
    // reduced-precision Gram: the Rayleigh-Ritz step cuts again and forms Z itself
    bool z_done = false;
    if (h->lp_gram && h->ranks[0] > 0) {
        rhosvd_status rs = rr_pass(h, eps);
        if (rs != RHOSVD_OK) return rs;
        z_done = true;
    }
    // refine_tails = 2: the deflated second pass forms Z itself
    if (refine_mode == 2 && !h->rside && h->ranks[0] > 0) {
        rhosvd_status ds = deflate_pass(h, eps);
        if (ds != RHOSVD_OK) return ds;
        z_done = true;
    }
    // refine_tails = 1: Z and V first at the wider p_l = min(m, r + r/8 + 16); where
    // even p_l does not certify on the refined tails, p_l grows (2 p_l + 64, at most m)
    // and the pass repeats, so the refined cut always ends certified
    const bool refine = refine_mode == 1 && h->ranks[0] > 0;
    int p_ref[3] = {0, 0, 0};
    if (refine)
        for (int l = 0; l < 3; ++l) p_ref[l] = (int)std::min<int64_t>(h->m, h->ranks[l] + h->ranks[l] / 8 + 16);
    for (int pass = 0;; ++pass) {
        if (refine)
            for (int l = 0; l < 3; ++l) {
                h->ranks[l] = p_ref[l];
                h->r_pad[l] = (int)round_up(p_ref[l], RPAD_CORE);
            }
        // a5/a6: Z and the projections V = Z^T U~ (FP64 MFMA; rounded to FP32 for the mixed core)
        if (z_done) {
        } else if (z_all && pass == 0) {
            for (int l = 0; l < 3; ++l) {
                const int r = h->ranks[l];
                if (r >= 1 && h->r_pad[l] > r)
                    CK(h, hipMemsetAsync(h->Z[l] + (int64_t)r * h->n_pad, 0,
                                         (size_t)(h->r_pad[l] - r) * h->n_pad * 8, st));
            }
        } else if (!h->rside) {
            // Z = H W[:, order[0..r-1]]: back-transformed eigenvectors, sign rule, zero padding
            BtJob jobs[3];
            for (int l = 0; l < 3; ++l)
                jobs[l] = BtJob{(int)h->m, (int)h->m_pad, h->G[l], h->htau[l], h->W[l], h->order[l], h->ranks[l],
                                nullptr, h->Z[l], (int)h->n_pad, (int)h->n_pad, h->Tw[l]};
            CK(h, launch_backtransform(jobs, 3, st));
            for (int l = 0; l < 3; ++l) {
                const int r = h->ranks[l];
                if (r < 1) continue;
                CK(h, launch_sign_cols((int)n, (int)h->n_pad, r, h->Z[l], st));
                if (h->r_pad[l] > r)
                    CK(h, hipMemsetAsync(h->Z[l] + (int64_t)r * h->n_pad, 0,
                                         (size_t)(h->r_pad[l] - r) * h->n_pad * 8, st));
            }
        } else if (h->ranks[0] > 0) {
            rhosvd_status zs = form_z_rside(h);
            if (zs != RHOSVD_OK) return zs;
        }
        if (pass == 0) mark(h, 5);
        for (int l = 0; l < 3; ++l) {
            if (h->ranks[l] < 1) continue;
            if (h->vprec == RHOSVD_FP64)
                CK(h, launch_project(h->n_pad, h->R_pad, h->r_pad[l], h->Z[l], h->Ut[l], (double*)h->V[l], nullptr,
                                     st));
            else if (refine)
                CK(h, launch_project(h->n_pad, h->R_pad, h->r_pad[l], h->Z[l], h->Ut[l], h->Vref[l], nullptr, st));
            else
                CK(h, launch_project(h->n_pad, h->R_pad, h->r_pad[l], h->Z[l], h->Ut[l], nullptr, (float*)h->V[l], st));
        }
        if (!refine) break;
        // the cut again on tails computed from V, not from G: for orthonormal Z_p,
        // |(I - Z_r Z_r^T) U~|_F^2 = sum_{r<=k<p} |V[k, :]|^2 + |U~ - Z_p V_p|_F^2 exactly,
        // in the order of Z's columns; both parts are formed directly in FP64
        const int64_t ntl = (h->n_pad / 64) * (h->R_pad / 64);
        for (int l = 0; l < 3; ++l) {
            const double* V64 = h->vprec == RHOSVD_FP64 ? (const double*)h->V[l] : h->Vref[l];
            CK(h, launch_resid_partials(h->n_pad, h->R_pad, h->r_pad[l], h->Z[l], V64, h->Ut[l], h->rpart[l], st));
            CK(h, launch_floor_sum(h->rpart[l], ntl, h->rfloor + l, st));
            CK(h, launch_row_norms2(p_ref[l], h->r_pad[l], h->R_pad, V64, h->Qn[l], st));
        }
        TruncArgs tb = trunc_args(h, eps);
        for (int l = 0; l < 3; ++l) {
            tb.lam[l] = h->Qn[l];
            tb.m_mode[l] = p_ref[l];
        }
        tb.floor2 = h->rfloor;
        tb.presorted = 1;
        CK(h, launch_truncate(tb, st));
        CK(h, hipMemcpyAsync(h->host, h->ranks_dev, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
        CK(h, hipStreamSynchronize(st));
        bool again = false;
        for (int l = 0; l < 3; ++l)
            if (h->host[l] > p_ref[l] && p_ref[l] < h->m) {
                p_ref[l] = (int)std::min<int64_t>(h->m, 2 * (int64_t)p_ref[l] + 64);
                again = true;
            }
        if (again) continue;
        for (int l = 0; l < 3; ++l) {
            // p_l + 1 with p_l = m: not even the full basis certifies (tau below the
            // residual's rounding); keep m (the report's tail says so)
            const int r = std::max(1, std::min(h->host[l], p_ref[l]));
            h->ranks[l] = r;
            if (h->r_pad[l] > r)
                CK(h, hipMemsetAsync(h->Z[l] + (int64_t)r * h->n_pad, 0, (size_t)(h->r_pad[l] - r) * h->n_pad * 8, st));
            if (h->vprec == RHOSVD_FP64)
                CK(h, launch_v_finalize(r, h->r_pad[l], h->R_pad, (const double*)h->V[l], (double*)h->V[l], nullptr,
                                        st));
            else
                CK(h, launch_v_finalize(r, h->r_pad[l], h->R_pad, h->Vref[l], nullptr, (float*)h->V[l], st));
        }
        break;
    }
    if (h->opt.als_sweeps > 0 && h->ranks[0] > 0 && h->ranks[1] > 0 && h->ranks[2] > 0) {
        rhosvd_status as = als_refine(h);
        if (as != RHOSVD_OK) return as;
        CK(h, hipMemcpyAsync(h->host + 6, h->flags + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        CK(h, hipStreamSynchronize(st));
        if (h->host[6]) return fail(h, RHOSVD_ERR_DEVICE, "eigensolver: a cross-workgroup wait ran out");
    }
    mark(h, 6);
    h->reduce_timed = true;
    h->get_timed = false;
    for (int l = 0; l < 3; ++l) ranks[l] = h->ranks[l];
    h->have = true;
    return RHOSVD_OK;
}

rhosvd_status rhosvd_get(rhosvd_handle h, double* Z1, double* Z2, double* Z3, void* beta, double* sigma,
                         rhosvd_report* report) {
    if (!h) return RHOSVD_ERR_ARG;
    if (!h->have) return fail(h, RHOSVD_ERR_STATE, "no successful rhosvd_reduce on this handle");
    hipStream_t st = h->stream;
    const bool any = h->ranks[0] > 0 && h->ranks[1] > 0 && h->ranks[2] > 0;
    // the core's arithmetic: as the handle's precision, except BF16x3 below its
    // tolerance floor (BF16X3_MIN_EPS), where the FP32 core runs on the same FP32 V
    const int cprec = core_precision_for(h->vprec, h->eps);
    if (h->opt.profile && h->ev_ok) hipEventRecord(h->ev[7], st);
    if (beta && any) {
        CoreArgs ca{};
        for (int l = 0; l < 3; ++l) {
            ca.r[l] = h->ranks[l];
            ca.r_pad[l] = h->r_pad[l];
            ca.V[l] = h->V[l];
        }
        ca.R_pad = h->R_pad;
        ca.xip = h->xip;
        ca.beta = beta;
        ca.prec = cprec;
        ca.beta_f32 = h->opt.beta_fp32 != 0;
        if (cprec == RHOSVD_BF16X3) {
            CK(h, launch_split_a(h->r_pad[0], h->R_pad, h->r_pad[0], (const float*)h->V[0], h->xip, h->Asplit, st));
            ca.Asplit = h->Asplit;
        }
        if (h->opt.core_tile) {
            ca.tile = h->opt.core_tile;
            CK(h, launch_core(ca, st));
            h->last_tile = ca.tile;
        } else {
            CK(h, launch_core_tuned(h->tuner, ca, st, &h->last_tile));
        }
    }
    if (h->opt.profile && h->ev_ok) hipEventRecord(h->ev[8], st);
    h->get_timed = true;
    double* Zo[3] = {Z1, Z2, Z3};
    int64_t off = 0;
    for (int l = 0; l < 3; ++l) {
        const int r = h->ranks[l];
        if (Zo[l] && r > 0)
            CK(h, hipMemcpy2DAsync(Zo[l], (size_t)h->n * 8, h->Z[l], (size_t)h->n_pad * 8, (size_t)h->n * 8, (size_t)r,
                                   hipMemcpyDeviceToDevice, st));
        if (sigma && r > 0)
            CK(h, hipMemcpyAsync(sigma + off, h->sigma[l], (size_t)r * 8, hipMemcpyDeviceToDevice, st));
        off += r;
    }
    const bool cert = report && h->opt.certificate && any;
    if (cert) {
        const int64_t nb = cert_blocks(h->R_pad);
        for (int l = 0; l < 3; ++l) {
            const double* V64 = (const double*)h->V[l];
            if (h->vprec != RHOSVD_FP64) {
                CK(h, launch_project(h->n_pad, h->R_pad, h->r_pad[l], h->Z[l], h->Ut[l], h->Vc, nullptr, st));
                V64 = h->Vc;
            }
            CK(h, launch_cert_mode(h->n_pad, h->R_pad, h->r_pad[l], h->Z[l], V64, h->Ut[l], h->xip, h->cpart,
                                   h->cout + l * nb, st));
        }
        CK(h, launch_floor_sum(h->cout, 3 * nb, h->cout + 3 * nb, st));
        CK(h, hipMemcpyAsync(h->hostd + 8, h->cout + 3 * nb, 8, hipMemcpyDeviceToHost, st));
    }
    if (report) {
        // tails at the ranks need one small read; only done when a report is requested
        double tl[3] = {0, 0, 0};
        // (a mode cut to rank 0 discards its whole tail, tails[0])
        for (int l = 0; l < 3; ++l)
            CK(h, hipMemcpyAsync(h->hostd + 4 + l, h->tails[l] + h->ranks[l], 8, hipMemcpyDeviceToHost, st));
        CK(h, hipMemcpyAsync(h->host + 8, h->flags + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        CK(h, hipStreamSynchronize(st));
        if (h->host[8]) return fail(h, RHOSVD_ERR_DEVICE, "eigensolver: a cross-workgroup wait ran out");
        for (int l = 0; l < 3; ++l) tl[l] = h->hostd[4 + l];
        memset(report, 0, sizeof(*report));
        report->xi_norm = h->xi_norm;
        report->a_norm = h->a_norm;
        report->tau = h->tau;
        for (int l = 0; l < 3; ++l) {
            report->tail[l] = tl[l];
            report->ranks[l] = h->ranks[l];
        }
        report->bound = h->xi_norm * (tl[0] + tl[1] + tl[2]);
        report->m = (int)std::min(h->n, h->R);
        report->eig_sweeps = h->sweeps;
        report->dropped = h->dropped;
        report->certificate = cert ? h->hostd[8] : -1.0;
        report->anorm_method = h->anorm_method;
        report->refine_used = h->refine_used;
        report->a_norm_upper = h->anorm_method == 2 ? h->a_upper : h->a_norm;
        report->core_precision = cprec;
        report->gram_precision = h->gram_used;
    }
    return RHOSVD_OK;
}

rhosvd_status rhosvd_get_xi(rhosvd_handle h, double* xip) {
    if (!h) return RHOSVD_ERR_ARG;
    if (!h->have) return fail(h, RHOSVD_ERR_STATE, "no successful rhosvd_reduce on this handle");
    if (!xip) return fail(h, RHOSVD_ERR_ARG, "null pointer");
    CK(h, hipMemcpyAsync(xip, h->xip, (size_t)h->R * 8, hipMemcpyDeviceToDevice, h->stream));
    return RHOSVD_OK;
}

rhosvd_status rhosvd_get_spectrum(rhosvd_handle h, int32_t l, double* sigma_all) {
    if (!h) return RHOSVD_ERR_ARG;
    if (!h->have) return fail(h, RHOSVD_ERR_STATE, "no successful rhosvd_reduce on this handle");
    if (l < 0 || l > 2 || !sigma_all) return fail(h, RHOSVD_ERR_ARG, "mode must be 0..2, pointer non-null");
    // min(n, R) values (the n-side re-run of R < n has n, the rest rounding noise)
    CK(h, hipMemcpyAsync(sigma_all, h->sigma[l], (size_t)std::min(h->n, h->R) * 8, hipMemcpyDeviceToDevice,
                         h->stream));
    return RHOSVD_OK;
}

__global__ void k_v_to_f64(int r, int ldv, int64_t R, const float* __restrict__ V, double* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)r * R; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = e % r, nu = e / r;
        out[e] = (double)V[j + nu * ldv];
    }
}

rhosvd_status rhosvd_get_v(rhosvd_handle h, int32_t l, double* V) {
    if (!h) return RHOSVD_ERR_ARG;
    if (!h->have) return fail(h, RHOSVD_ERR_STATE, "no successful rhosvd_reduce on this handle");
    if (l < 0 || l > 2 || !V) return fail(h, RHOSVD_ERR_ARG, "mode must be 0..2, pointer non-null");
    const int r = h->ranks[l];
    if (r < 1) return RHOSVD_OK;
    if (h->vprec == RHOSVD_FP64) {
        CK(h, hipMemcpy2DAsync(V, (size_t)r * 8, h->V[l], (size_t)h->r_pad[l] * 8, (size_t)r * 8, (size_t)h->R,
                               hipMemcpyDeviceToDevice, h->stream));
    } else {
        hipLaunchKernelGGL(k_v_to_f64, dim3(1024), dim3(256), 0, h->stream, r, h->r_pad[l], h->R,
                           (const float*)h->V[l], V);
        CK(h, hipGetLastError());
    }
    return RHOSVD_OK;
}

rhosvd_status rhosvd_reduce_batched(rhosvd_handle h, int32_t count, const rhosvd_problem* problems) {
    if (!h) return RHOSVD_ERR_ARG;
    h->err.clear();
    std::string msg;
    const int vs = batch_validate(problems, count, msg);
    if (vs != RHOSVD_OK) return fail(h, (rhosvd_status)vs, msg);
    const int prec_key = h->opt.precision | (h->opt.beta_fp32 ? 16 : 0) | (h->opt.core_tile << 8);
    if (!batch_plan_matches(h->batch, problems, count, prec_key)) {
        // earlier work on the stream may still use the old plan's memory
        CK(h, hipStreamSynchronize(h->stream));
        if (h->batch) {
            batch_plan_destroy(h->batch);
            h->batch = nullptr;
        }
        std::string err;
        h->batch = batch_plan_create(problems, count, prec_key, err, h->alloc);
        if (!h->batch) return fail(h, RHOSVD_ERR_ALLOC, err);
    }
    CK(h, batch_plan_run(h->batch, h->stream));
    h->last_tile = batch_plan_core_tile(h->batch);
    return RHOSVD_OK;
}

// ---------------------------------------------------------------------------
// rank-proposal network
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
rhosvd_status net_alloc(rhosvd_ctx* h, int batch) {
    if (!h->net) {
        if (!(h->net = (float*)h->alloc.get(4 * (size_t)NET_PARAMS * sizeof(float)))) {
            return fail(h, RHOSVD_ERR_ALLOC, "network parameter allocation failed");
        }
    }
    const size_t need = net_work_floats(std::max(batch, 1));
    if (need > h->net_work_n) {
        if (h->net_work) { hipStreamSynchronize(h->stream); h->alloc.put(h->net_work); h->net_work = nullptr; }
        h->net_work_n = 0;
        if (!(h->net_work = (float*)h->alloc.get(need * sizeof(float)))) {
            return fail(h, RHOSVD_ERR_ALLOC, "network workspace allocation failed");
        }
        h->net_work_n = need;
    }
    return RHOSVD_OK;
}
}  // namespace

extern "C" {

int32_t rhosvd_net_num_params(void) { return NET_PARAMS; }

rhosvd_status rhosvd_net_set_params(rhosvd_handle h, const float* params) {
    if (!h) return RHOSVD_ERR_ARG;
    if (!params) return fail(h, RHOSVD_ERR_ARG, "params is NULL");
    rhosvd_status s = net_alloc(h, 1);
    if (s != RHOSVD_OK) return s;
    CK(h, hipMemcpyAsync(h->net, params, (size_t)NET_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    // new parameters restart the optimizer: gradient and both moments zero
    CK(h, hipMemsetAsync(h->net + NET_PARAMS, 0, 3 * (size_t)NET_PARAMS * sizeof(float), h->stream));
    h->net_step = 0;
    h->net_set = true;
    return RHOSVD_OK;
}

rhosvd_status rhosvd_net_get_params(rhosvd_handle h, float* params) {
    if (!h) return RHOSVD_ERR_ARG;
    if (!h->net_set) return fail(h, RHOSVD_ERR_STATE, "no network parameters on this handle");
    if (!params) return fail(h, RHOSVD_ERR_ARG, "params is NULL");
    CK(h, hipMemcpyAsync(params, h->net, (size_t)NET_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return RHOSVD_OK;
}

rhosvd_status rhosvd_net_forward(rhosvd_handle h, int32_t count, const float* x, float* y) {
    if (!h) return RHOSVD_ERR_ARG;
    if (!h->net_set) return fail(h, RHOSVD_ERR_STATE, "no network parameters on this handle");
    if (count < 1 || !x || !y) return fail(h, RHOSVD_ERR_ARG, "count >= 1 and non-null x, y required");
    rhosvd_status s = net_alloc(h, count);
    if (s != RHOSVD_OK) return s;
    CK(h, net_forward(h->net, count, x, y, h->net_work, h->stream));
    return RHOSVD_OK;
}

rhosvd_status rhosvd_net_train_step(rhosvd_handle h, int32_t count, const float* x, const float* target, float lr,
                                    float* loss, float* grad) {
    if (!h) return RHOSVD_ERR_ARG;
    if (!h->net_set) return fail(h, RHOSVD_ERR_STATE, "no network parameters on this handle");
    if (count < 1 || !x || !target) return fail(h, RHOSVD_ERR_ARG, "count >= 1 and non-null x, target required");
    if (!(lr >= 0.0f)) return fail(h, RHOSVD_ERR_ARG, "lr must be >= 0");
    rhosvd_status s = net_alloc(h, count);
    if (s != RHOSVD_OK) return s;
    float* G = h->net + NET_PARAMS;
    if (lr > 0.0f) ++h->net_step;
    CK(h, net_train_step(h->net, G, G + NET_PARAMS, G + 2 * NET_PARAMS, std::max(h->net_step, 1), lr, count, x,
                         target, loss, h->net_work, h->stream));
    if (grad)
        CK(h, hipMemcpyAsync(grad, G, (size_t)NET_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return RHOSVD_OK;
}

// ---------------------------------------------------------------------------
// learned rank proposal + randomized range finder
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// argument checks, layout, normalization and the |A| identity (the part of a
// reduction both paths share)
rhosvd_status prologue(rhosvd_ctx* h, int64_t n, int64_t R, const double* U1, const double* U2, const double* U3,
                       const double* xi, double eps) {
    if (!U1 || !U2 || !U3 || !xi) return fail(h, RHOSVD_ERR_ARG, "null pointer argument");
    if (n < 1 || R < 1) return fail(h, RHOSVD_ERR_ARG, "n and R must be >= 1");
    if (!(eps > 0.0) || !isfinite(eps)) return fail(h, RHOSVD_ERR_ARG, "eps must be finite and > 0");
    if ((n < R ? n : R) > 2048) return fail(h, RHOSVD_ERR_UNSUPPORTED, "min(n, R) > 2048 is not supported by this library");
    if (n > 65536) return fail(h, RHOSVD_ERR_UNSUPPORTED, "n > 65536 is not supported by this library");
    rhosvd_status s = layout(h, n, R);
    if (s != RHOSVD_OK) return s;
    hipStream_t st = h->stream;
    const double* U[3] = {U1, U2, U3};
    CK(h, hipMemsetAsync(h->flags, 0, 64, st));
    CK(h, launch_colnorm(n, R, h->n_pad, h->R_pad, U, xi, h->Ut, h->xip, h->flags, st));
    int64_t nt = 0;
    CK(h, launch_anorm_partials(h->n_pad, h->R_pad, h->Ut, h->xip, h->anorm_part, &nt, h->rside ? h->G : nullptr, st));
    h->a2_part = h->anorm_part;
    h->a2_n = h->anorm_ntiles;
    h->anorm_method = 1;
    h->a_upper = -1.0;
    return RHOSVD_OK;
}

}  // namespace

extern "C" {

rhosvd_status rhosvd_sketch_features(rhosvd_handle h, int64_t n, int64_t R, const double* U1, const double* U2,
                                     const double* U3, const double* xi, double eps, const double* omega,
                                     int32_t omega_cols, float* feat) {
    if (!h) return RHOSVD_ERR_ARG;
    h->have = false;
    h->err.clear();
    if (!omega || !feat || omega_cols < 32) return fail(h, RHOSVD_ERR_ARG, "omega (>= 32 columns) and feat required");
    rhosvd_status s = prologue(h, n, R, U1, U2, U3, xi, eps);
    if (s != RHOSVD_OK) return s;
    s = learned_layout(h, 64);
    if (s != RHOSVD_OK) return s;
    s = learned_features(h, omega, omega_cols, eps);
    if (s != RHOSVD_OK) return s;
    CK(h, hipMemcpyAsync(feat, h->L.feat, 3 * NET_IN * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return RHOSVD_OK;
}

rhosvd_status rhosvd_reduce_learned(rhosvd_handle h, int64_t n, int64_t R, const double* U1, const double* U2,
                                    const double* U3, const double* xi, double eps, const double* omega,
                                    int32_t omega_cols, int32_t ranks[3], rhosvd_learned_info* info) {
    if (!h) return RHOSVD_ERR_ARG;
    h->have = false;
    h->err.clear();
    if (!ranks) return fail(h, RHOSVD_ERR_ARG, "ranks is NULL");
    if (!omega || omega_cols < 64) return fail(h, RHOSVD_ERR_ARG, "omega with >= 64 columns required");
    if (!h->net_set) return fail(h, RHOSVD_ERR_STATE, "no network parameters on this handle");
    rhosvd_learned_info li;
    memset(&li, 0, sizeof(li));
    if (R < n || std::min(n, R) < 192) {
        // the range finder is built for the n-side Gram path, and below m = 192 no
        // width (a multiple of 64) satisfies 3p < m: the full method runs
        rhosvd_status s = rhosvd_reduce(h, n, R, U1, U2, U3, xi, eps, ranks);
        for (int l = 0; l < 3; ++l) li.fallback[l] = R < n ? 3 : 1;
        if (info) *info = li;
        return s;
    }
    rhosvd_status s = prologue(h, n, R, U1, U2, U3, xi, eps);
    if (s != RHOSVD_OK) return s;
    h->eps = eps;
    hipStream_t st = h->stream;
    const int m = (int)h->m;
    const int p_cap = (int)std::min<int64_t>(round_up(m, 64), (int64_t)(omega_cols / 64) * 64);
    if ((s = learned_layout(h, std::max(p_cap, 64))) != RHOSVD_OK) return s;
    auto& L = h->L;
    mark(h, 0);
    if ((s = learned_features(h, omega, omega_cols, eps)) != RHOSVD_OK) return s;
    if ((s = net_alloc(h, 3)) != RHOSVD_OK) return s;
    CK(h, net_forward(h->net, 3, L.feat, L.out, h->net_work, st));
    float* hout = (float*)(h->host + 56);   // host words 56..61 (see rhosvd_create)
    CK(h, hipMemcpyAsync(hout, L.out, 3 * NET_OUT * sizeof(float), hipMemcpyDeviceToHost, st));
    CK(h, hipMemcpyAsync(h->host + 4, h->flags, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(h, hipStreamSynchronize(st));
    if (h->host[4]) return fail(h, RHOSVD_ERR_NONFINITE, "input contains NaN or Inf");
    if (h->host[6]) return fail(h, RHOSVD_ERR_DEVICE, "eigensolver: a cross-workgroup wait ran out");
    // proposals: rank r = out0 * m, sketch width p = out1 * m (at least r + 8), in
    // multiples of 64; the range finder is used where it saves eigensolver work (3p < m)
    int width[3] = {0, 0, 0};
    bool rf[3] = {false, false, false};
    for (int l = 0; l < 3; ++l) {
        const double o0 = std::isfinite(hout[2 * l]) ? hout[2 * l] : 1.0;
        const double o1 = std::isfinite(hout[2 * l + 1]) ? hout[2 * l + 1] : 1.0;
        const int rh = (int)std::min<double>(m, std::max(1.0, std::round(o0 * m)));
        int p = (int)std::min<double>(m, std::max<double>(rh + 8, std::round(o1 * m)));
        const int pp = (int)std::min<int64_t>(round_up(p, 64), p_cap);
        li.proposal[l] = rh;
        rf[l] = pp >= 64 && 3 * pp < m;
        width[l] = rf[l] ? pp : 0;
        li.width[l] = width[l];
        li.fallback[l] = rf[l] ? 0 : 1;
    }
    const int64_t np = h->n_pad, Rp = h->R_pad;
    CK(h, hipMemsetAsync(L.floor2, 0, 4 * sizeof(double), st));
    std::vector<EigMat> em;
    auto rf_eig = [&]() -> rhosvd_status {
        rhosvd_status ps = ensure_plan(h, 3, em.data(), (int)em.size());
        if (ps != RHOSVD_OK) return ps;
        CK(h, eig_plan_enqueue(h->plan[3], h->flags + 2, st));
        return RHOSVD_OK;
    };
    std::vector<int> rfl;
    for (int l = 0; l < 3; ++l)
        if (rf[l]) rfl.push_back(l);
    if (!rfl.empty()) {
        // Y = U~ Omega_p, orthonormal basis Q by two Lowdin passes, B = Q^T U~
        for (int l : rfl) {
            const int p = width[l];
            CK(h, launch_pad_omega(h->R, Rp, omega_cols, p, omega, L.Om[l], st));
            CK(h, launch_gemm64(false, true, np, p, Rp, h->Ut[l], np, L.Om[l], Rp, L.Y[l], np, 1.0, st));
            em.push_back(EigMat{L.G2[l], L.lam2[l], L.W2[l], L.Qn2[l], L.Mg2[l], L.dd2[l], L.ee2[l], L.tau2[l], p, p});
        }
        for (int pass = 0; pass < 2; ++pass) {
            for (int l : rfl) {
                const int p = width[l];
                const double* X = pass == 0 ? L.Y[l] : L.Qb[l];
                CK(h, launch_gemm64(true, true, p, p, np, X, np, X, np, L.G2[l], p, 1.0, st));
            }
            if ((s = rf_eig()) != RHOSVD_OK) return s;
            std::vector<BtJob> jobs;
            for (int l : rfl) {
                const int p = width[l];
                jobs.push_back(BtJob{p, p, L.G2[l], L.tau2[l], L.W2[l], nullptr, p, nullptr, L.Pf[l], p, p, L.Tw[l]});
            }
            CK(h, launch_backtransform(jobs.data(), (int)jobs.size(), st));
            for (int l : rfl) {
                const int p = width[l];
                CK(h, launch_lowdin(p, p, L.lam2[l], L.Pf[l], L.S2[l], 1e-15, st));
                // pass 0: Qb = Y S;  pass 1: Y = Qb S (the orthonormal basis ends in Y)
                if (pass == 0)
                    CK(h, launch_gemm64(false, true, np, p, p, L.Y[l], np, L.S2[l], p, L.Qb[l], np, 1.0, st));
                else
                    CK(h, launch_gemm64(false, true, np, p, p, L.Qb[l], np, L.S2[l], p, L.Y[l], np, 1.0, st));
            }
        }
        for (int l : rfl) {
            const int p = width[l];
            CK(h, launch_project(np, Rp, p, L.Y[l], h->Ut[l], L.Bm[l], nullptr, st));
            CK(h, launch_resid_partials(np, Rp, p, L.Y[l], L.Bm[l], h->Ut[l], L.part[l], st));
            CK(h, launch_floor_sum(L.part[l], (np / 64) * (Rp / 64), L.floor2 + l, st));
            CK(h, launch_gemm64(false, false, p, p, Rp, L.Bm[l], p, L.Bm[l], p, L.G2[l], p, 1.0, st));
        }
        if ((s = rf_eig()) != RHOSVD_OK) return s;
    }
    // the Gram path for the other modes (all three Grams are formed; the
    // eigensolver runs only for the modes that need it)
    bool gram_done = false;
    auto gram_modes = [&](const bool* which) -> rhosvd_status {
        if (!(which[0] || which[1] || which[2])) return RHOSVD_OK;
        if (!gram_done) {
            CK(h, launch_gram_nt(h->n_pad, h->R_pad, h->Ut, h->G, h->gram_part, h->gram_splits, st));
            gram_done = true;
        }
        std::vector<EigMat> eg;
        for (int l = 0; l < 3; ++l)
            if (which[l])
                eg.push_back(EigMat{h->G[l], h->lam[l], h->W[l], h->Qn[l], h->Mg[l], h->dd[l], h->ee[l], h->htau[l], m,
                                    (int)h->m_pad});
        if (eg.empty()) return RHOSVD_OK;
        rhosvd_status ps = ensure_plan(h, 0, eg.data(), (int)eg.size());
        if (ps != RHOSVD_OK) return ps;
        CK(h, eig_plan_enqueue(h->plan[0], h->flags + 2, st));
        return RHOSVD_OK;
    };
    bool gm[3] = {!rf[0], !rf[1], !rf[2]};
    if ((s = gram_modes(gm)) != RHOSVD_OK) return s;
    auto truncate = [&]() -> rhosvd_status {
        TruncArgs ta{};
        for (int l = 0; l < 3; ++l) {
            ta.lam[l] = rf[l] ? L.lam2[l] : h->lam[l];
            ta.m_mode[l] = rf[l] ? width[l] : m;
            ta.sigma[l] = h->sigma[l];
            ta.order[l] = h->order[l];
            ta.tails[l] = h->tails[l];
            if (rf[l]) CK(h, hipMemsetAsync(h->sigma[l], 0, (size_t)(h->m_pad + 1) * 8, st));
        }
        ta.m = m;
        ta.m_pad = (int)h->m_pad;
        ta.n = (int)n;
        ta.n_pad = (int)h->n_pad;
        ta.xip = h->xip;
        ta.R_pad = h->R_pad;
        ta.anorm_part = h->anorm_part;
        ta.anorm_ntiles = h->anorm_ntiles;
        ta.eps = eps;
        ta.ranks = h->ranks_dev;
        ta.scal = h->scal;
        ta.floor2 = L.floor2;
        CK(h, launch_truncate(ta, st));
        CK(h, hipMemcpyAsync(h->host, h->ranks_dev, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
        CK(h, hipMemcpyAsync(h->host + 4, h->flags, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
        CK(h, hipMemcpyAsync(h->hostd, h->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
        CK(h, hipMemcpyAsync(h->hostd + 8, L.floor2, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
        CK(h, hipStreamSynchronize(st));
        if (h->host[6]) return fail(h, RHOSVD_ERR_DEVICE, "eigensolver: a cross-workgroup wait ran out");
        return RHOSVD_OK;
    };
    if ((s = truncate()) != RHOSVD_OK) return s;
    // certificate: a range-finder mode whose tails never reach tau (rank m + 1) falls back
    bool again[3] = {false, false, false};
    bool any = false;
    for (int l = 0; l < 3; ++l) {
        li.residual[l] = rf[l] ? sqrt(std::max(h->hostd[8 + l], 0.0)) : 0.0;
        if (rf[l] && h->host[l] > width[l]) {
            again[l] = true;
            any = true;
            rf[l] = false;
            li.fallback[l] = 2;
        }
    }
    if (any) {
        // the Gram path has no residual: clear the floor of the modes that fall back
        for (int l = 0; l < 3; ++l)
            if (again[l]) CK(h, hipMemsetAsync(L.floor2 + l, 0, sizeof(double), st));
        if ((s = gram_modes(again)) != RHOSVD_OK) return s;
        if ((s = truncate()) != RHOSVD_OK) return s;
    }
    for (int l = 0; l < 3; ++l)
        if (h->host[l] < 0 || h->host[l] > (rf[l] ? width[l] : m))
            return fail(h, RHOSVD_ERR_DEVICE, "truncation returned rank " + std::to_string(h->host[l]) + " for mode " +
                                                  std::to_string(l) + " (internal error)");
    mark(h, 4);
    h->sweeps = 0;
    h->dropped = h->host[5];
    h->xi_norm = h->hostd[0];
    h->a_norm = h->hostd[1];
    h->tau = h->hostd[2];
    for (int l = 0; l < 3; ++l) {
        h->ranks[l] = h->host[l];
        h->r_pad[l] = (int)round_up(h->ranks[l] > 0 ? h->ranks[l] : 1, 128);
        const int bad = learned_mode_fits(m, (int)h->zr_pad, L.p_cap, rf[l], width[l], h->ranks[l], h->r_pad[l]);
        if (bad)
            return fail(h, RHOSVD_ERR_DEVICE, "learned path: rank " + std::to_string(h->ranks[l]) + " of mode " +
                                                  std::to_string(l) + " exceeds its buffers (check " +
                                                  std::to_string(bad) + ", internal error)");
    }
    // Z: range-finder modes Z = Q W_B[:, order[0..r-1]]; Gram modes as in rhosvd_reduce
    std::vector<BtJob> jobs;
    for (int l = 0; l < 3; ++l) {
        const int r = h->ranks[l];
        if (r < 1) continue;
        if (rf[l]) {
            const int p = width[l];
            CK(h, hipMemsetAsync(L.Wsel[l], 0, (size_t)p * h->r_pad[l] * 8, st));
            jobs.push_back(BtJob{p, p, L.G2[l], L.tau2[l], L.W2[l], h->order[l], r, nullptr, L.Wsel[l], p, p, L.Tw[l]});
        } else {
            jobs.push_back(BtJob{m, (int)h->m_pad, h->G[l], h->htau[l], h->W[l], h->order[l], r, nullptr, h->Z[l],
                                 (int)np, (int)np, h->Tw[l]});
        }
    }
    CK(h, launch_backtransform(jobs.data(), (int)jobs.size(), st));
    for (int l = 0; l < 3; ++l) {
        const int r = h->ranks[l];
        if (r < 1) continue;
        if (rf[l])
            CK(h, launch_gemm64(false, true, np, h->r_pad[l], width[l], L.Y[l], np, L.Wsel[l], width[l], h->Z[l], np,
                                1.0, st));
        CK(h, launch_sign_cols((int)n, (int)np, r, h->Z[l], st));
        if (h->r_pad[l] > r)
            CK(h, hipMemsetAsync(h->Z[l] + (int64_t)r * np, 0, (size_t)(h->r_pad[l] - r) * np * 8, st));
    }
    mark(h, 5);
    for (int l = 0; l < 3; ++l) {
        if (h->ranks[l] < 1) continue;
        if (h->vprec == RHOSVD_FP64)
            CK(h, launch_project(np, Rp, h->r_pad[l], h->Z[l], h->Ut[l], (double*)h->V[l], nullptr, st));
        else
            CK(h, launch_project(np, Rp, h->r_pad[l], h->Z[l], h->Ut[l], nullptr, (float*)h->V[l], st));
    }
    mark(h, 6);
    // phases 1..3 are not separated on this path: the events between them coincide
    for (int i = 1; i <= 3; ++i) mark(h, i);
    h->reduce_timed = true;
    h->get_timed = false;
    for (int l = 0; l < 3; ++l) ranks[l] = h->ranks[l];
    if (info) *info = li;
    h->have = true;
    return RHOSVD_OK;
}

// ---------------------------------------------------------------------------
// Tucker-to-canonical transform (Remark 2.6)
// ---------------------------------------------------------------------------
rhosvd_status rhosvd_t2c(rhosvd_handle h, int32_t r1, int32_t r2, int32_t r3, const double* beta, double eps,
                         int64_t* R, double* bound) {
    if (!h) return RHOSVD_ERR_ARG;
    h->err.clear();
    auto& T = h->T;
    T.have = false;
    if (!beta || !R) return fail(h, RHOSVD_ERR_ARG, "beta and R are required");
    if (r1 < 1 || r2 < 1 || r3 < 1) return fail(h, RHOSVD_ERR_ARG, "core dimensions must be >= 1");
    if (!(eps > 0.0) || !isfinite(eps)) return fail(h, RHOSVD_ERR_ARG, "eps must be finite and > 0");
    if (std::min(r1, r2) > T2C_MAXC || t2c_lds_bytes(r1, r2) > T2C_MAX_LDS)
        return fail(h, RHOSVD_ERR_UNSUPPORTED, "core slices too large for the one-workgroup Jacobi SVD "
                                               "(min(r1, r2) <= 256 and r1 r2 <= 19456)");
    hipStream_t st = h->stream;
    const int L = std::max(r1, r2), c = std::min(r1, r2);
    Carve cv{nullptr};
    auto carve = [&](Carve& k) {
        T.W = k.take<double>((size_t)r3 * L * c);
        T.sig = k.take<double>((size_t)r3 * c);
        T.tails = k.take<double>(r3);
        T.p = k.take<int>(r3);
        T.off = k.take<int64_t>((size_t)r3 + 1);
        T.flags = k.take<int>(4);
    };
    carve(cv);
    if (cv.off > T.bytes) {
        if (T.ws) { CK(h, hipStreamSynchronize(st)); h->alloc.put(T.ws); T.ws = nullptr; T.bytes = 0; }
        if (!(T.ws = (char*)h->alloc.get(cv.off))) {
            return fail(h, RHOSVD_ERR_ALLOC, "T2C workspace allocation of " + std::to_string(cv.off) + " bytes failed");
        }
        T.bytes = cv.off;
    }
    Carve ck{T.ws};
    carve(ck);
    const double thr = eps / ((double)r3 * sqrt((double)c));
    CK(h, hipMemsetAsync(T.flags, 0, 4 * sizeof(int), st));
    CK(h, launch_t2c_jacobi(beta, r1, r2, r3, thr, 60, T.W, T.sig, T.p, T.tails, T.flags, st));
    std::vector<int> p(r3);
    std::vector<double> tl(r3);
    int flag = 0;
    CK(h, hipMemcpyAsync(p.data(), T.p, (size_t)r3 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(h, hipMemcpyAsync(tl.data(), T.tails, (size_t)r3 * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(h, hipMemcpyAsync(&flag, T.flags, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(h, hipStreamSynchronize(st));
    if (flag) return fail(h, RHOSVD_ERR_NOCONV, "T2C: a slice's Jacobi sweeps did not converge");
    std::vector<int64_t> off((size_t)r3 + 1, 0);
    double b = 0.0;
    for (int m = 0; m < r3; ++m) {
        if (p[m] < 0 || p[m] > c) return fail(h, RHOSVD_ERR_DEVICE, "T2C: invalid slice rank (internal error)");
        off[m + 1] = off[m] + p[m];
        b += tl[m];
    }
    CK(h, hipMemcpy(T.off, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    T.r1 = r1;
    T.r2 = r2;
    T.r3 = r3;
    T.beta = beta;
    T.R = off[r3];
    T.have = true;
    *R = T.R;
    if (bound) *bound = b;
    return RHOSVD_OK;
}

rhosvd_status rhosvd_t2c_get(rhosvd_handle h, double* weights, double* F1, double* F2, int32_t* slice,
                             double* sigma, int64_t n, const double* Z1, const double* Z2, const double* Z3,
                             double* C1, double* C2, double* C3) {
    if (!h) return RHOSVD_ERR_ARG;
    auto& T = h->T;
    if (!T.have) return fail(h, RHOSVD_ERR_STATE, "no successful rhosvd_t2c on this handle");
    const bool lift_any = Z1 || Z2 || Z3 || C1 || C2 || C3;
    const bool lift = lift_any && n >= 1 && Z1 && Z2 && Z3 && C1 && C2 && C3;
    if (lift_any && !lift) return fail(h, RHOSVD_ERR_ARG, "lifting needs n >= 1 and all of Z1..Z3, C1..C3");
    if (T.R > 0 && (!weights || !F1 || !F2 || !slice))
        return fail(h, RHOSVD_ERR_ARG, "weights, F1, F2 and slice are required");
    hipStream_t st = h->stream;
    const int c = std::min(T.r1, T.r2);
    if (sigma) CK(h, hipMemcpyAsync(sigma, T.sig, (size_t)T.r3 * c * 8, hipMemcpyDeviceToDevice, st));
    if (T.R < 1) return RHOSVD_OK;
    CK(h, launch_t2c_terms(T.beta, T.r1, T.r2, T.r3, T.W, T.sig, T.off, T.R, weights, F1, T.r1, F2, T.r2, slice, st));
    if (!lift) return RHOSVD_OK;
    // C_l = Z_l F_l through the FP64 MFMA GEMM on zero-padded copies
    const int64_t np = round_up(n, 64), Rp = round_up(T.R, 64);
    const int64_t kp = round_up(std::max(T.r1, T.r2), 64);
    const size_t need = a256((size_t)np * kp * 8) + a256((size_t)kp * Rp * 8) + a256((size_t)np * Rp * 8);
    if (need > T.lbytes) {
        if (T.lw) { CK(h, hipStreamSynchronize(st)); h->alloc.put(T.lw); T.lw = nullptr; T.lbytes = 0; }
        if (!(T.lw = (char*)h->alloc.get(need))) {
            return fail(h, RHOSVD_ERR_ALLOC, "T2C lifting workspace allocation of " + std::to_string(need) +
                                                 " bytes failed");
        }
        T.lbytes = need;
    }
    double* Zp = (double*)T.lw;
    double* Fp = (double*)(T.lw + a256((size_t)np * kp * 8));
    double* Cp = (double*)(T.lw + a256((size_t)np * kp * 8) + a256((size_t)kp * Rp * 8));
    const double* Zs[2] = {Z1, Z2};
    const double* Fs[2] = {F1, F2};
    double* Cs[2] = {C1, C2};
    const int rs[2] = {T.r1, T.r2};
    for (int l = 0; l < 2; ++l) {
        CK(h, hipMemsetAsync(Zp, 0, (size_t)np * kp * 8, st));
        CK(h, hipMemsetAsync(Fp, 0, (size_t)kp * Rp * 8, st));
        CK(h, hipMemcpy2DAsync(Zp, (size_t)np * 8, Zs[l], (size_t)n * 8, (size_t)n * 8, (size_t)rs[l],
                               hipMemcpyDeviceToDevice, st));
        CK(h, hipMemcpy2DAsync(Fp, (size_t)kp * 8, Fs[l], (size_t)rs[l] * 8, (size_t)rs[l] * 8, (size_t)T.R,
                               hipMemcpyDeviceToDevice, st));
        CK(h, launch_gemm64(false, true, np, Rp, kp, Zp, np, Fp, kp, Cp, np, 1.0, st));
        CK(h, hipMemcpy2DAsync(Cs[l], (size_t)n * 8, Cp, (size_t)np * 8, (size_t)n * 8, (size_t)T.R,
                               hipMemcpyDeviceToDevice, st));
    }
    CK(h, launch_t2c_gather_cols((int)n, T.R, Z3, n, slice, C3, n, st));
    return RHOSVD_OK;
}

int32_t rhosvd_batch_uses_graph(rhosvd_handle h) { return (h && batch_plan_uses_graph(h->batch)) ? 1 : 0; }

int32_t rhosvd_last_core_tile(rhosvd_handle h) { return h ? h->last_tile : 0; }

double rhosvd_phase_ms(rhosvd_handle h, int32_t phase) {
    if (!h || !h->opt.profile || !h->ev_ok || phase < 0 || phase >= NPHASE) return -1.0;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return -1.0;
    float ms = -1.0f;
    if (phase < 6) {
        if (!h->reduce_timed) return -1.0;
        if (hipEventElapsedTime(&ms, h->ev[phase], h->ev[phase + 1]) != hipSuccess) return -1.0;
    } else {
        if (!h->get_timed) return -1.0;
        if (hipEventElapsedTime(&ms, h->ev[7], h->ev[8]) != hipSuccess) return -1.0;
    }
    return (double)ms;
}

}  // extern "C"
