// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <stdint.h>

#include <string>

#include "../../include/rhosvd.h"

// Device memory of a handle and its batch plans: the caller's allocator
// (rhosvd_create_with_allocator), or hipMalloc / hipFree when it has none.
struct DevAlloc {
    rhosvd_allocator a{};
    void* get(size_t bytes) const {
        if (bytes == 0) bytes = 256;
        if (a.alloc) return a.alloc(bytes, a.ctx);
        void* p = nullptr;
        return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    }
    void put(void* p) const {
        if (!p) return;
        if (a.free) a.free(p, a.ctx);
        else hipFree(p);
    }
};

// Padding granularities shared by the workspace layout and the kernels.
constexpr int PAD_N = 64;    // rows of U~, Z and the Gram side (n, m)
constexpr int PAD_R = 64;    // canonical terms (columns of U~, K of the core)
// The BF16x3 core runs for eps >= BF16X3_MIN_EPS only; below it the FP32 core runs
// in its place.  Its error, about 2e-6 |A| (n = 1024, R = 4096 and R = 90000), lies
// inside the Tucker subspace and so adds to the truncation error (orthogonal to
// that subspace) in quadrature: the total stays within (eps + 1e-6) |A| when the
// core error is below (2 eps 1e-6 + 1e-12)^(1/2) |A|, 4.6e-6 at eps = 1e-5 (2.3x the
// measured error) but 1.7e-6 at eps = 1e-6.
constexpr double BF16X3_MIN_EPS = 1e-5;
inline int core_precision_for(int prec, double eps) { return (prec == 2 && eps < BF16X3_MIN_EPS) ? 1 : prec; }

// a1: scaled column norms, xi' and normalized side matrices (all three modes).
// U_l: n x R (ld n); Ut_l: n_pad x R_pad (ld n_pad), zero padded; xip: R_pad.
// flags[0] |= 1 on a non-finite input; flags[1] += number of dropped terms.
hipError_t launch_colnorm(int64_t n, int64_t R, int64_t n_pad, int64_t R_pad,
                          const double* const U[3], const double* xi,
                          double* const Ut[3], double* xip, int* flags, hipStream_t st);

// a2: G_l = U~_l U~_l^T (n_pad x n_pad, col-major) for l = 0..2, split over K.
// part: workspace of splits * 3 * n_pad^2 doubles (unused when splits == 1).
hipError_t launch_gram_nt(int64_t n_pad, int64_t R_pad, double* const Ut[3], double* const G[3],
                          double* part, int splits, hipStream_t st);
// split-K partials of the Gram (splits x 3 x n_pad^2) summed in a fixed order into
// the lower triangle and mirrored
hipError_t launch_gram_reduce(int64_t n_pad, const double* part, int splits, double* const G[3], hipStream_t st);
// a2 in reduced precision (k_gram_lp.hip): prec 1 FP32 MFMA, 2 BF16x3; FP32
// accumulation restarted every 4096 terms and summed in FP64; same split-K and
// partial buffer as launch_gram_nt
hipError_t launch_gram_lp(int prec, int64_t n_pad, int64_t R_pad, double* const Ut[3], double* const G[3],
                          double* part, int splits, hipStream_t st);

// |A|^2 = xi'^T (G1 o G2 o G3) xi' with G_l = U~_l^T U~_l, per-tile partial sums
// written to part (ntiles doubles); the caller reduces them in a fixed order.
// When Gr is non-null the three R_pad x R_pad Grams U~_l^T U~_l are written too
// (the Gram on the R side, used when R < n).
hipError_t launch_anorm_partials(int64_t n_pad, int64_t R_pad, double* const Ut[3],
                                 const double* xip, double* part, int64_t* ntiles, double* const Gr[3],
                                 hipStream_t st);

// |U~ - Q B|_F^2 partial sums per 64 x 64 tile (R_pad/64 * n_pad/64 doubles in part)
hipError_t launch_resid_partials(int64_t n_pad, int64_t R_pad, int64_t p_pad, const double* Q, const double* B,
                                 const double* Ut, double* part, hipStream_t st);

// Generic FP64 MFMA GEMM on padded operands, C = alpha A B (col-major C).
//   a_kcontig: A(i,k) = A[k + i*lda], else A[i + k*lda]
//   b_kcontig: B(k,j) = B[k + j*ldb], else B[j + k*ldb]
// out = T - Q B (n_pad x N_pad, ld n_pad; Q n_pad x p_pad ld n_pad; B p_pad x N_pad
// ld p_pad); out may be T
// The certificate inside the proof of Theorem 2.3 for one mode: per 256 columns,
// sum_nu |xi'_nu| |U~[:, nu] - Z V[:, nu]| -> out[0 .. cert_blocks(R_pad)) (Z: n_pad x
// p_pad, V: p_pad x R_pad FP64 = Z^T U~).  part: n_pad / 64 x R_pad doubles of scratch.
int64_t cert_blocks(int64_t R_pad);
hipError_t launch_cert_mode(int64_t n_pad, int64_t R_pad, int64_t p_pad, const double* Z, const double* V64,
                            const double* Ut, const double* xip, double* part, double* out, hipStream_t st);
hipError_t launch_residual(int64_t n_pad, int64_t N_pad, int64_t p_pad, const double* Q, const double* B,
                           const double* T, double* out, hipStream_t st);
// deflated spectrum: sigma = [sig1[0..k), sig2[0..m-k)], tails from tails2 plus sig1
hipError_t launch_combine_spectrum(int k, int m, const double* sig1, const double* sig2, const double* tails2,
                                   double* sigma, double* tails, hipStream_t st);
hipError_t launch_gemm64(bool a_kcontig, bool b_kcontig, int64_t M, int64_t N, int64_t K, const double* A,
                         int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, double alpha,
                         hipStream_t st);
// R < n helpers (Z = U~ W Lambda^-1/2 and its re-orthonormalization)
// r_dev (nullable): the rank is min(*r_dev, r) (known only on the device)
hipError_t launch_gather_scaled(int m_pad, int r, int r_pad, const double* W, const int* order,
                                const double* sigma, double* Wr, hipStream_t st, const int* r_dev = nullptr);
hipError_t launch_pad_identity(int r, int mp, int ld, double* M, hipStream_t st, const int* r_dev = nullptr);
hipError_t launch_scale_cols_invsqrt(int mp, int ld, const double* mu, const double* P, double* out, hipStream_t st);
hipError_t launch_sign_cols(int n, int n_pad, int r, double* Z, hipStream_t st);

// a6: V_l = Z_l^T U~_l (r_pad x R_pad, col-major ld r_pad); Z_l: n_pad x r_pad (ld n_pad).
// out_f64 or out_f32 (one of them non-null).
hipError_t launch_project(int64_t n_pad, int64_t R_pad, int64_t r_pad, const double* Z,
                          const double* Ut, double* out_f64, float* out_f32, hipStream_t st);

// a3: FP64 eigensolver (Householder tridiagonalization + divide and conquer) for
// a list of symmetric matrices of order m <= 2048 (each its own m and ld).  G is
// overwritten by the Householder vectors (column k holds v_k in rows k+1..m-1);
// lam receives the eigenvalues (unsorted) and Q the eigenvectors of the
// tridiagonal matrix T (eigenvectors of G = H Q, see launch_backtransform).
struct EigMat {
    double* G;      // m x m (ld)
    double* lam;    // m
    double* Q;      // ld x m
    double* Qn;     // ld x m workspace
    double* M;      // ld x m workspace
    double* d;      // m
    double* e;      // m
    double* tau;    // m
    int m, ld;
};
// A plan fixes the launches and device tables for one list of matrices:
// create (host only; returns the bytes of device work memory it needs), bind
// (assigns that memory and enqueues the upload of its tables on st; the plan
// keeps the host copy alive), enqueue (kernel launches only, so it may be
// recorded into a graph once bound).  abort_w: a device int set to 1 when a
// cross-workgroup wait of the tridiagonalization ran out (results invalid).
struct EigPlan;
EigPlan* eig_plan_create(const EigMat* mats, int nmat, size_t* work_bytes);
hipError_t eig_plan_bind(EigPlan* plan, void* work, hipStream_t st);
// cooperative: launch the tridiagonalization cooperatively (the runtime checks that
// all workgroups are resident); otherwise residency rests on the plan's packing,
// which never exceeds the device's occupancy for the launch.
hipError_t eig_plan_enqueue(const EigPlan* plan, int* abort_w, hipStream_t st, bool cooperative = true);
void eig_plan_destroy(EigPlan* plan);

// Back-transformation jobs: out[:, k] = H Q[:, order[k]] for k < r (order NULL:
// identity), H = H_0 ... H_{m-3} from the reflectors left in Hv by launch_eig,
// rows m .. nrows-1 of out set to zero.  r = min(*r_dev, r) when r_dev is set
// (the rank is then known only on the device; r is the capacity).
// Tw: backtransform_work_doubles(m) doubles per job (the compact-WY T factors).
struct BtJob {
    int m, ld;
    const double* Hv;
    const double* tau;
    const double* Q;
    const int* order;
    int r;
    const int* r_dev;
    double* out;
    int ldo, nrows;
    double* Tw;
};
constexpr int BT_MAXJOB = 16;
struct BtJobs {
    BtJob job[BT_MAXJOB];
};
size_t backtransform_work_doubles(int m);
hipError_t launch_backtransform(const BtJob* jobs, int njobs, hipStream_t st);

// a4/a5: norms finalize, sort, tails, ranks (per mode).
struct TruncArgs {
    const double* lam[3];   // eigenvalues (any order)
    int m;                  // valid eigenpairs (min(n, R))
    int m_pad;
    int n;
    int n_pad;
    const double* xip;      // R_pad
    int64_t R_pad;
    const double* anorm_part;
    int64_t anorm_ntiles;
    double eps;
    // outputs
    double* sigma[3];       // m each, descending
    int* order[3];          // m each: column of W for the k-th largest
    double* tails[3];       // m + 1 each
    int* ranks;             // 3 ints (m + 1 when no r certifies, see floor2)
    double* scal;           // 16 doubles: [0] xi_norm, [1] a_norm, [2] tau, [3 + l] tail at mode l's
                            // rank, [6 + l] largest eigenvalue, [9 + l] eigenvalue at the rank
    int m_mode[3];          // per-mode number of eigenvalues (0: m)
    const double* floor2;   // per-mode squared tail floor (device, 3 doubles) or null
    int presorted;          // nonzero: keep the given order (no sort; order = identity)
    double tau_fixed;       // > 0: use this tau instead of eps |A| / (3 |xi'|)
    int signed_tails;       // nonzero: tails from the signed eigenvalues (clamped at zero)
};
hipError_t launch_truncate(const TruncArgs& a, hipStream_t st);
// Sums of squares of x[0 .. count) into part[0 .. nparts), each over a fixed
// strided subset in a fixed order (nparts <= 1024).
hipError_t launch_sumsq_partials(const double* x, int64_t count, double* part, int nparts, hipStream_t st);

// a7: beta[j1 + r1 (j2 + r2 j3)] = sum_nu xi'_nu V1[j1,nu] V2[j2,nu] V3[j3,nu].
// V_l: col-major (r_pad_l x R_pad), xip: R_pad.  prec 0 = f64, 1 = f32, 2 = bf16x3.
struct CoreArgs {
    int r[3];
    int r_pad[3];
    int64_t R_pad;
    const void* V[3];
    const double* xip;
    void* beta;       // double, or float when beta_f32
    int prec;
    int beta_f32;
    int tile;         // rows of j1 per workgroup tile: 64 or 128 (FP32, BF16x3), 64 (FP64); 0: default
    const void* Asplit;   // BF16x3: V1 diag(xi') as bf16 hi and lo planes (launch_split_a), r_pad[0] x R_pad each
};
hipError_t launch_core(const CoreArgs& a, hipStream_t st);
// A operand of the BF16x3 core: x = V1[j1, nu] * xi'_nu (FP32), hi = bf16(x), lo =
// bf16(x - hi), as two planes of rows_pad x R_pad bf16 with nu contiguous
// (plane[j1 * R_pad + nu]; lo plane right after hi).  V1: FP32, ld >= rows_pad.
hipError_t launch_split_a(int64_t rows_pad, int64_t R_pad, int64_t ld, const float* V1, const double* xip,
                          void* planes, hipStream_t st);
int core_tile_default(int prec);
bool core_tile_valid(int prec, int tile);

// Autotuner of the core tile (tune.hip).  launch_core_tuned launches with the
// cached tile of the shape class, or times the candidates first (synchronizing
// the stream; the output then holds the winner's result); *used: tile launched.
struct CoreTuner;
CoreTuner* core_tuner_create();
void core_tuner_destroy(CoreTuner* T);
hipError_t launch_core_tuned(CoreTuner* T, CoreArgs a, hipStream_t st, int* used);
// times launch(tile) for each candidate (two alternating rounds, fastest launch
// of each), leaves the winner's result in place, synchronizes st
hipError_t time_candidates(const int* tiles, int ncand, const std::function<hipError_t(int)>& launch,
                           hipStream_t st, int* best);

// ---------------------------------------------------------------------------
// Batched reductions: one descriptor per problem in device memory.  Sizes are
// fixed on the host; the ranks exist only on the device (ranks[0..2]), and the
// status word ranks[3] (0, or a negative rhosvd_status) gates the later phases.
// ---------------------------------------------------------------------------
struct BProb {
    int n, R, n_pad, R_pad;
    int m, m_pad, rside, rcap, rcap_pad, cap_rank;   // rcap = min(cap_rank, m)
    double eps;
    const double* U[3];
    const double* xi;
    double* Ut[3];         // n_pad x R_pad
    double* xip;           // R_pad
    int* flags;            // [0] non-finite input, [1] dropped terms
    const int* abort_w;    // eigensolver abort word of the batch
    double* G[3];          // m_pad x m_pad Gram (n or R side) -> reflectors
    double* lam[3];        // m_pad eigenvalues
    double* W[3];          // eigenvectors of the tridiagonal matrices
    double* anorm_part;
    int64_t anorm_ntiles;
    double* sigma[3];      // m_pad + 1
    int* order[3];         // m_pad
    double* tails[3];      // m_pad + 1
    double* scal;          // xi_norm, a_norm, tau
    int* ranks;            // [0..2] ranks, [3] status
    double* Z[3];          // n_pad x rcap_pad
    void* V[3];            // rcap_pad x R_pad (FP64, or FP32 for the mixed cores)
    void* Asplit;          // BF16x3: hi and lo planes of V1 diag(xi') (rcap_pad x R_pad bf16 each)
    double* Zo[3];         // caller outputs, n x cap_rank (ld n), or null
    double* Vo[3];         // caller outputs V^(l), r_l x R (ld cap_rank, FP64), or null
    int v_f32;             // V is held in FP32 (mixed cores)
    void* beta;            // caller output (double, or float when beta_f32) or null
    int64_t cap_beta;
    int beta_f32;
    int* result;           // caller's int32[8]: r1, r2, r3, status, dropped, core precision
    int core_prec;         // the core's arithmetic for the whole pass (rhosvd_precision)
};
enum { BK_COLNORM = 0, BK_ANORM = 1, BK_GRAM = 2, BK_PROJECT = 3, BK_SIGN = 4, BK_SPLIT = 5 };
// the BF16x3 A planes of every problem (blocks: rcap_pad / 64 x R_pad / 64 each)
hipError_t launch_split_b(const BProb* P, const int64_t* pre, int np, int64_t nblocks, hipStream_t st);
// Flattened launch of one batched dense phase: pre (device, np + 1 entries) holds
// each problem's first block, nblocks = pre[np].  f32: V in FP32 (projection).
hipError_t launch_batched_dense(int which, const BProb* P, const int64_t* pre, int np, int64_t nblocks, int f32,
                                hipStream_t st);
// truncation of every problem and mode (grid 3 x np), then the per-problem status:
// non-finite input, eigensolver abort, or ranks beyond the capacities.
hipError_t launch_truncate_b(const BProb* P, int np, hipStream_t st);
// Khatri-Rao cores of every problem with status 0 and a beta output, as one
// persistent launch: a device-side plan counts each problem's tiles from its
// ranks, workgroups take tiles from a shared counter.  work: np + 4 int64.
// prec: core precision (0..2), plus 16 when beta is written as float, plus 32
// when some problem's R_pad exceeds core_flush_span() (the FP32-accumulating
// cores then hand their partial sums to beta periodically).
hipError_t launch_core_b(const BProb* P, int np, int prec, int tile, int64_t* work, int grid, hipStream_t st);
// workgroups of the persistent core that fit on the device at once (prec, tile as above)
int core_b_max_grid(int prec, int tile);
int64_t core_flush_span();
// copy Z to the caller's buffers and write the result words (ranks, status)
hipError_t launch_finish_b(const BProb* P, int np, hipStream_t st);

// Batch plans (batch.hip): validation, layout + uploads + graph capture, replay.
struct BatchPlan;
int batch_validate(const rhosvd_problem* probs, int count, std::string& msg);   // rhosvd_status
// prec: core precision (0..2), plus 16 when beta is written as float
BatchPlan* batch_plan_create(const rhosvd_problem* probs, int count, int prec, std::string& err,
                             const DevAlloc& alloc);
bool batch_plan_matches(const BatchPlan* plan, const rhosvd_problem* probs, int count, int prec);
hipError_t batch_plan_run(BatchPlan* plan, hipStream_t st);
bool batch_plan_uses_graph(const BatchPlan* plan);
// rows per core tile of the plan's batched core (0 until the first run has chosen)
int batch_plan_core_tile(const BatchPlan* plan);
void batch_plan_destroy(BatchPlan* plan);

// ---------------------------------------------------------------------------
// Rank-proposal network (k_net.hip): FP32 MLP NET_IN -> NET_HID -> NET_HID -> NET_OUT.
// ---------------------------------------------------------------------------
constexpr int NET_IN = 67, NET_HID = 128, NET_OUT = 2;
constexpr int NET_PARAMS = NET_HID * NET_IN + NET_HID + NET_HID * NET_HID + NET_HID + NET_OUT * NET_HID + NET_OUT;
size_t net_work_floats(int batch);
// Y (B x NET_OUT) = net(X (B x NET_IN)); work: net_work_floats(B) floats
hipError_t net_forward(const float* params, int B, const float* X, float* Y, float* work, hipStream_t st);
// gradient G of the MSE loss at (X, T); loss (nullable) receives the mean loss; when
// lr > 0, one Adam step (step = 1, 2, ...) updates params with moments M, V
hipError_t net_train_step(float* params, float* G, float* M, float* V, int step, float lr, int B, const float* X,
                          const float* T, float* loss, float* work, hipStream_t st);

// Learned rank proposal (k_learned.hip)
// feat (3 x NET_IN floats) from the 32 eigenvalues of each mode's sketch Gram
hipError_t launch_features(const double* const lam[3], int n, int64_t R, double eps, float* feat, hipStream_t st);
// out (R_pad x cols, ld R_pad) = omega (R x w, ld R) zero padded (columns >= w zero)
hipError_t launch_pad_omega(int64_t R, int64_t R_pad, int w, int cols, const double* omega, double* out,
                            hipStream_t st);
// out[:, j] = P[:, j] / sqrt(mu_j) for mu_j > rel * max(mu), else 0 (mp x mp, leading dimension ld)
hipError_t launch_lowdin(int mp, int ld, const double* mu, const double* P, double* out, double rel, hipStream_t st);
hipError_t launch_floor_sum(const double* part, int64_t ntiles, double* out, hipStream_t st);
// out[k] = |V[k, :]|^2 for k < p (V: ld x R_pad, column-major, FP64)
hipError_t launch_row_norms2(int p, int ld, int64_t R_pad, const double* V, double* out, hipStream_t st);
// refinement of the Gram-route cut: out[k] = sigma[k]^2 (k < r); V rows >= keep zeroed
// (dst64 may equal src) or converted to FP32 (dst32)
hipError_t launch_square_prefix(int r, const double* sigma, double* out, hipStream_t st);
hipError_t launch_v_finalize(int keep, int ld, int64_t R_pad, const double* src, double* dst64, float* dst32,
                             hipStream_t st);

// Tucker-to-canonical transform (k_t2c.hip).  Slices B_m = beta[:, :, m] of an
// r1 x r2 x r3 FP64 core (Fortran order); min(r1, r2) <= T2C_MAXC and r1 r2
// doubles within T2C_MAX_LDS bytes (the slice lives in one workgroup's LDS).
constexpr int T2C_MAXC = 256;
constexpr size_t T2C_MAX_LDS = 152 * 1024;
size_t t2c_lds_bytes(int r1, int r2);
// one-sided Jacobi SVD of every slice: Wout (r3 x L x c: unit singular vectors on
// the side of length L = max(r1, r2), by descending sigma), sig_out (r3 x c,
// descending), p_out (r3: sigma > thr), tail_out (r3: dropped tail norms);
// flags |= 1 when a slice did not converge within max_sweeps
hipError_t launch_t2c_jacobi(const double* beta, int r1, int r2, int r3, double thr, int max_sweeps, double* Wout,
                             double* sig_out, int* p_out, double* tail_out, int* flags, hipStream_t st);
// the R kept terms (off: r3 + 1 prefix offsets of p): weights, u_k into F1 (ld1),
// v_k into F2 (ld2), slice index of each term
// (R_lim, nullable: device word; terms t >= *R_lim are skipped, so R may be a capacity)
hipError_t launch_t2c_terms(const double* beta, int r1, int r2, int r3, const double* Wj, const double* sig,
                            const int64_t* off, int64_t R, double* weights, double* F1, int64_t ld1, double* F2,
                            int64_t ld2, int* slice_of, hipStream_t st, const int64_t* R_lim = nullptr);
// counts to offsets, R, bound and a status word on the device (no host round trip)
hipError_t launch_t2c_offsets(const int* p, const double* tails, int r3, int64_t cap, const int* flags, int64_t* off,
                              int64_t* R_lim, int64_t* R_out, double* bound_out, int* status, hipStream_t st);
hipError_t launch_t2c_clear_flags(int* flags, hipStream_t st);
// C[:, t] = Z[:, slice_of[t]]
hipError_t launch_t2c_gather_cols(int n, int64_t R, const double* Z, int64_t ldz, const int* slice_of, double* C,
                                  int64_t ldc, hipStream_t st);

// ALS refinement (k_als.hip): Ha <- diag(xi') (Ha o Hb) diag(xi') on R_pad x R_pad,
// and the descending order of m eigenvalues
hipError_t launch_als_hadamard(int64_t R_pad, double* Ha, const double* Hb, const double* xip, hipStream_t st);
hipError_t launch_order_desc(const double* lam, int m, int* order, hipStream_t st);
