/*
 * rhosvd.h — C-ABI of the MI355X (gfx950) Reduced HOSVD library.
 *
 * The Reduced HOSVD (Khoromskaia & Khoromskij, Section 2.1, Definition 2.1)
 * turns a d=3 canonical tensor
 *     A = sum_nu xi_nu u1_nu (x) u2_nu (x) u3_nu            (eq. eqn:can_A3)
 * with side matrices U^(l) = [u^(l)_1 .. u^(l)_R] (n x R) into a rank-(r1,r2,r3)
 * orthogonal Tucker tensor  A_r = beta x_1 Z^(1) x_2 Z^(2) x_3 Z^(3):
 *   1. each side matrix is normalized column by column and its singular value
 *      decomposition U^(l) = Z D V^T is truncated at epsilon   (eqs. eqn:SVD_Ul, eq:svdr)
 *   2. V^(l) = Z^(l)T U^(l) projects the side matrices     (Definition 2.1, Proposition 2.2)
 *   3. the core beta_(1) = V^(1) diag(xi') (V^(3) (.) V^(2))^T  (Proposition 2.2)
 *
 * Truncation rule (the paper leaves it open): tau = eps * |A|_F / (3 |xi'|_2),
 * r_l = min{ r >= 1 : (sum_{k>r} sigma_{l,k}^2)^(1/2) <= tau }.  Theorem 2.3 then
 * guarantees |A - A_r|_F <= eps |A|_F.  |A|_F is exact or a certified lower bound
 * (rhosvd_options.anorm); a lower bound only lowers tau, so the guarantee holds.
 *
 * Conventions
 *   - All matrices are column-major.  U^(l): n x R, leading dimension n, column nu
 *     is the canonical vector u^(l)_nu.  Z^(l): n x r_l, leading dimension n.
 *     beta: r1*r2*r3 doubles, entry (j1,j2,j3) at j1 + r1*(j2 + r2*j3).
 *   - Every data pointer is a DEVICE pointer unless marked "host".  Inputs are
 *     read-only and must stay valid until the stream has finished the call.
 *   - All work is enqueued on the stream given at rhosvd_create.  rhosvd_reduce
 *     synchronizes with that stream once (to return the ranks on the host);
 *     rhosvd_get does not synchronize.
 *   - A handle owns its device workspace (grown on demand, reused across
 *     calls, released by rhosvd_destroy), drawn from the caller's allocator
 *     (rhosvd_create_with_allocator) or hipMalloc.  A handle is not thread-safe and must
 *     not be used by two calls at once.
 *   - Functions never throw; they return a status.  rhosvd_last_error gives a
 *     human-readable message for the last failing call on a handle.
 */
#ifndef RHOSVD_H
#define RHOSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RHOSVD_OK = 0,
    RHOSVD_ERR_ARG = -1,        /* bad size, null pointer, eps <= 0, unknown option */
    RHOSVD_ERR_NONFINITE = -2,  /* an input entry (U or xi) is NaN or infinite */
    RHOSVD_ERR_ALLOC = -3,      /* device workspace allocation failed */
    RHOSVD_ERR_DEVICE = -4,     /* a HIP runtime call failed */
    RHOSVD_ERR_NOCONV = -5,     /* the eigensolver hit its sweep cap */
    RHOSVD_ERR_STATE = -6,      /* rhosvd_get/inspection without a successful rhosvd_reduce */
    RHOSVD_ERR_UNSUPPORTED = -7, /* size or option outside what the library supports */
    RHOSVD_ERR_CAPACITY = -8     /* batched: a rank exceeds cap_rank, or r1 r2 r3 exceeds cap_beta */
} rhosvd_status;

/* Arithmetic of the Khatri-Rao core contraction.  The column norms, the Gram
 * matrix, the eigensolver, the truncation decision and Z are FP64 in every
 * mode; the projection V = Z^T U~ is an FP64 MFMA product, rounded to FP32 for
 * the FP32 and BF16x3 cores. */
typedef enum {
    RHOSVD_FP64 = 0,    /* FP64 MFMA */
    RHOSVD_FP32 = 1,    /* FP32 MFMA, FP32 accumulation */
    RHOSVD_BF16X3 = 2   /* a = a_hi + a_lo in bf16, a*b ~ hi*hi + hi*lo + lo*hi, FP32
                           accumulation (bf16 MFMA).  Its error, about 2e-6 |A|, keeps the
                           total within (eps + 1e-6) |A| only for eps >= 1e-5: below that
                           the FP32 core runs in its place (the report's core_precision,
                           word 5 of a batched result) */
} rhosvd_precision;

typedef struct {
    int32_t precision;       /* rhosvd_precision */
    int32_t max_eig_sweeps;  /* unused (the eigensolver is not iterative); any value */
    int32_t profile;         /* nonzero: time each phase with HIP events (see rhosvd_phase_ms) */
    int32_t beta_fp32;       /* nonzero: beta is written as float (r1*r2*r3 floats) instead of
                                double, halving its size; meant for the FP32 and BF16x3 cores.
                                When R (padded to 64) exceeds 8192 these cores add their
                                partial sums over each 8192 terms into beta, in float here */
    int32_t refine_tails;    /* 0 (auto), 1, 2 or 3 (off) (rhosvd_reduce; other values:
                                RHOSVD_ERR_ARG).
                                0 (default): when the Gram-route cut of some mode lies
                                in the FP64 noise band of its Gram matrix, lambda_r <=
                                64 u lambda_1 (u = 2^-53: there the discarded and even
                                the last kept eigenvalues carry noise of about u |G|),
                                2 if tau^2 itself lies in that band, else 1; none
                                otherwise.  The report's refine_used says which.
                                When R < n (Gram on the R side, Z = U~ W Sigma^-1, whose
                                columns at the Gram's rounding level are not
                                orthonormal) a refinement re-runs the whole reduction
                                on the n x n Gram with the exact |A| (n <= 2048; beyond
                                that the plain cut stays), at the cost of that larger
                                eigensolve.
                                With 1, where even the wider p does not certify on the
                                refined tails, p grows (2p + 64, at most m) and the
                                refined cut is taken again.
                                3: the plain Gram-route cut.
                                1: after the Gram-route cut r, with
                                Z_p the leading p = min(m, r + r/8 + 16) eigenvectors and
                                V_p = Z_p^T U~, the cut is taken again on the tails
                                t_r^2 = sum_{r<=k<p} |V_p[k,:]|^2 + |U~ - Z_p V_p|_F^2
                                (= |(I - Z_r Z_r^T) U~|_F^2 exactly, in Z's column order),
                                both parts formed directly in FP64.  The Gram route's
                                small eigenvalues carry FP64 noise of about u |G|; where
                                tau^2 lies below that floor the refined ranks are the
                                smaller, still certified ones (Theorem 2.3); the
                                spectrum then holds |V_p[k,:]| for k < p.
                                2: a deflated second
                                Gram pass.  With Z_k the leading k eigenvectors of the
                                first pass whose singular values are >= 2^-13 sigma_1
                                (k < r), U'' = (I - Z_k Z_k^T)^2 U~ is formed in FP64 and
                                its Gram eigendecomposed again; its spectrum resolves
                                values down to about u^(1/2) sigma_(k+1) instead of
                                u^(1/2) sigma_1.  The cut is taken on that spectrum with
                                the same tau, r = k + r'; Z = [Z_k, Z'] with Z' the leading
                                r' deflated eigenvectors projected once more against Z_k;
                                the spectrum reported is sigma_1..k of the first pass
                                followed by the deflated one, the tails those of U''.
                                Costs one more Gram, eigensolve and two projections. */
    int32_t core_tile;       /* rows of j1 per workgroup tile of the FP32 / BF16x3 core: 64 or
                                128; 0 (default): chosen by the library's autotuner, which
                                times both on the first core of each shape class (precision,
                                beta type, r1 in steps of 32, r2*r3 and R in quarter octaves)
                                on the caller's stream and keeps the faster.  That first
                                rhosvd_get synchronizes the stream (and its beta is written
                                up to four times, the last by the winner); batched: the
                                first rhosvd_reduce_batched of a plan does the same with
                                the persistent core before recording its graph.  The FP64
                                core has one tile (64).  See rhosvd_last_core_tile. */
    int32_t certificate;     /* nonzero: rhosvd_get with a report also forms the certificate
                                inside the proof of Theorem 2.3,
                                c = sum_l sum_nu |xi'_nu| |(I - Z_l Z_l^T) u~_nu^(l)| <= bound,
                                each residual column formed directly in FP64 (from an FP64
                                projection in every precision: one more n x r x R product per
                                mode on the mixed paths).  Not formed by rhosvd_reduce_batched. */
    int32_t anorm;           /* how rhosvd_reduce obtains |A|_F for tau (other values: RHOSVD_ERR_ARG):
                                1 exact: |A|^2 = xi'^T (G1 o G2 o G3) xi' with G_l = U~_l^T U~_l
                                  (R x R, 3 n R^2 flops).
                                2 probe: a certified lower bound L <= |A|, the norm of the
                                  core at probe ranks p_l (the smallest ranks whose tails
                                  t_{l,p} are <= 1/30): |beta_p| = |A x_1 Z_p1^T x_2 Z_p2^T
                                  x_3 Z_p3^T| <= |A| (an orthogonal projection of A), formed
                                  with the FP64 core after the eigensolver (2 p1 p2 p3 R
                                  flops).  Theorem 2.3 applied at p gives the upper bound
                                  U = (L^2 + b_p^2)^(1/2), b_p = |xi'| sum_l t_{l,p_l}; tau
                                  from L is at most the exact one (so the result stays
                                  certified: bound <= eps L <= eps |A|) and differs from it
                                  by at most 1 - L/U relatively.
                                0 (default): the probe where n <= R, its flops are under
                                  half the exact identity's and b_p <= L / 10; else exact.
                                When R < n the identity's tiles are the Gram matrices
                                themselves, so it is always exact there.  Batched and
                                learned reductions use the exact identity. */
    int32_t als_sweeps;      /* 0..4: sweeps of the canonical-to-Tucker ALS iteration started from
                                the RHOSVD factors (Section 2.1 after Definition 2.1, eq.
                                eqn:can_A_Tuck_als), run by rhosvd_reduce after Z at fixed
                                ranks.  For mode l (others a, b, modes taken 1, 2, 3 in turn,
                                each with the others' latest factors) Z_l becomes the r_l
                                leading left singular vectors of the contracted unfolding
                                M_l = U~_l diag(xi') (V_b (.) V_a)^T, computed as the leading
                                eigenvectors of M_l M_l^T = U~_l diag(xi') (V_a^T V_a o
                                V_b^T V_b) diag(xi') U~_l^T in FP64.  Each update maximizes
                                |beta| given the others, so |A - A_r| only decreases and the
                                Theorem 2.3 bound of the RHOSVD factors (the report's) still
                                holds.  n <= R <= 16384 (the R x R FP64 products);
                                otherwise RHOSVD_ERR_UNSUPPORTED.  Not used by batched or
                                learned reductions. */
    int32_t gram_precision;  /* arithmetic of the Gram matrix (n <= R; other values: RHOSVD_ERR_ARG):
                                0 (default) FP64 MFMA.
                                1 FP32 MFMA or 2 BF16x3 (a_hi + a_lo split, three bf16 products),
                                both accumulating in FP32 (summed in FP64 every 4096 terms).
                                Its eigenvalues then carry noise of about u_32 |G| (2^-17 |G|
                                for BF16x3), far above the FP64 route's, and a Rayleigh-Ritz
                                step in FP64 recovers the accuracy: with Q the leading p
                                eigenvectors of that Gram (p = min(m, r + r/8 + 16), r its
                                own cut on tails that sum its eigenvalues with their signs,
                                so that the noise largely cancels), B = Q^T U~ (FP64 MFMA),
                                the residual |U~ - Q B|_F^2
                                formed directly, and B B^T = Y S^2 Y^T (the FP64
                                eigensolver), the cut is taken on
                                t_r^2 = sum_{k>r} s_k^2 + |U~ - Q B|_F^2 and
                                Z = Q Y[:, 0:r] (Theorem 2.3 holds for this orthonormal Z).
                                Where no r <= p certifies, p grows (2p + 64, at most m) and
                                the step repeats; at p = m the step is exact, at about the
                                cost of the FP64 route twice.  The reduced-precision Gram pays
                                where tau^2 lies well above its noise (loose eps, large R);
                                the spectrum then holds the p Ritz values.  |A| comes from the
                                exact identity and refine_tails is not used.  When R < n, and
                                for batched and learned reductions, the Gram is FP64; the
                                report's gram_precision says which ran. */
} rhosvd_options;

typedef struct {
    double xi_norm;      /* |xi'|_2 after normalization */
    double a_norm;       /* |A|_F as used for tau: exact (Gram identity), or the probe's certified
                            lower bound (anorm_method) */
    double tau;          /* truncation threshold on the tails, eps * a_norm / (3 |xi'|) */
    double bound;        /* Theorem 2.3: |xi'| * sum_l tail[l] */
    double tail[3];      /* t_{l, r_l} = (sum_{k > r_l} sigma_{l,k}^2)^(1/2) */
    int32_t ranks[3];
    int32_t m;           /* min(n, R): number of singular values per mode */
    int32_t eig_sweeps;  /* eigensolver sweeps used */
    int32_t dropped;     /* terms dropped because xi = 0 or a column is zero */
    double certificate;  /* with the certificate option: sum_l sum_nu |xi'_nu| |(I - Z_l Z_l^T)
                            u~_nu^(l)| (proof of Theorem 2.3), |A - A_r| <= certificate <= bound;
                            -1 when not formed */
    double a_norm_upper; /* an upper bound of |A|_F: equal to a_norm when that is exact,
                            (a_norm^2 + b_p^2)^(1/2) with the probe (see rhosvd_options.anorm) */
    int32_t anorm_method;  /* 1 exact identity, 2 probe lower bound */
    int32_t refine_used;   /* the refinement rhosvd_reduce ran: 0 none, 1 refined tails, 2 deflated
                              pass; plus 4 when R < n and it ran on the n x n Gram */
    int32_t core_precision; /* rhosvd_precision of the core contraction (see RHOSVD_BF16X3) */
    int32_t gram_precision; /* the Gram's arithmetic (rhosvd_options.gram_precision) as run: 0 FP64,
                               1 FP32 or 2 BF16x3 followed by the FP64 Rayleigh-Ritz step */
} rhosvd_report;

typedef struct rhosvd_ctx* rhosvd_handle;

/* A caller's device-memory allocator (for example a framework's caching
 * allocator).  alloc returns device memory of at least `bytes` bytes, aligned to
 * 256 bytes and usable on the handle's stream, or NULL; free releases a pointer
 * alloc returned.  Both are called from the thread that calls the library, only
 * inside library calls (create, reduce, get, the batched, learned, network and
 * transform calls, set_options, destroy), and a pointer is freed only after the
 * handle's stream has finished the work that used it. */
typedef struct {
    void* (*alloc)(size_t bytes, void* ctx);
    void (*free)(void* ptr, void* ctx);
    void* ctx;
} rhosvd_allocator;

/* Create a handle bound to a HIP stream (hipStream_t passed as void*; NULL is
 * the default stream).  opt may be NULL (FP64, default sweep cap).
 * Errors: RHOSVD_ERR_ARG (out == NULL, bad option), RHOSVD_ERR_DEVICE. */
rhosvd_status rhosvd_create(rhosvd_handle* out, void* hip_stream, const rhosvd_options* opt);

/* rhosvd_create with the handle's device memory drawn from `allocator` (copied;
 * NULL: hipMalloc / hipFree): the reduction workspace, the eigensolver plans'
 * work memory, batch plans, the learned path's and the network's memory, the |A|
 * probe's and the Tucker-to-canonical transform's workspace.  (The handle's 4 KiB
 * of pinned host staging is separate.)  Errors: as rhosvd_create, ARG when the
 * allocator lacks alloc or free. */
rhosvd_status rhosvd_create_with_allocator(rhosvd_handle* out, void* hip_stream, const rhosvd_allocator* allocator,
                                           const rhosvd_options* opt);

/* Release the handle and its workspace (waits for the handle's stream). */
rhosvd_status rhosvd_destroy(rhosvd_handle h);

/* Change the options of an existing handle (same rules as rhosvd_create). */
rhosvd_status rhosvd_set_options(rhosvd_handle h, const rhosvd_options* opt);

/*
 * Phase 1 of a reduction (Definition 2.1 up to the ranks): normalization, the
 * |A| identity or probe (rhosvd_options.anorm), Gram matrices on the min(n,R)
 * side, FP64 eigensolver, truncation, Z and the projections V^(l).
 *   n, R     : grid size and canonical rank, 1 <= n <= 2048, R >= 1
 *   U1..U3   : device, n x R each (column-major, ld = n)
 *   xi       : device, R weights
 *   eps      : relative accuracy, > 0
 *   ranks    : HOST int32[3], receives (r1, r2, r3); (0,0,0) when every term is dropped
 * Synchronizes with the handle's stream once (the probe adds two more, its
 * fallback to the exact identity one more).  On error nothing is retained.
 * Errors: ARG, NONFINITE, ALLOC, DEVICE, NOCONV, UNSUPPORTED.
 */
rhosvd_status rhosvd_reduce(rhosvd_handle h, int64_t n, int64_t R,
                            const double* U1, const double* U2, const double* U3,
                            const double* xi, double eps, int32_t ranks[3]);

/*
 * Phase 2: the Khatri-Rao core and the copy-out into caller buffers sized from
 * the ranks of the last successful rhosvd_reduce on this handle.
 *   Z1..Z3 : device, n x r_l each (column-major), or NULL to skip
 *   beta   : device, r1*r2*r3 doubles (floats with the beta_fp32 option), Fortran
 *            order, or NULL to skip the core
 *   sigma  : device, r1+r2+r3 doubles (kept singular values, mode by mode), or NULL
 *   report : HOST, or NULL
 * Enqueued on the handle's stream; does not synchronize.
 * Errors: STATE (no reduction), DEVICE.
 */
rhosvd_status rhosvd_get(rhosvd_handle h, double* Z1, double* Z2, double* Z3,
                         void* beta, double* sigma, rhosvd_report* report);

/*
 * Inspection of the last reduction (for tests and the mixed Tucker-canonical
 * format of Proposition 2.2, whose core is the rank-R canonical tensor with
 * factors V^(l)).  All outputs are device pointers; these calls enqueue copies.
 *   rhosvd_get_xi       : xi' (R doubles; zero for dropped terms)
 *   rhosvd_get_spectrum : all m singular values of mode l, descending (m doubles)
 *   rhosvd_get_v        : V^(l) = Z^(l)T U~^(l) as an r_l x R column-major matrix
 *                         (converted to FP64 when the projection ran in FP32)
 * Errors: STATE, ARG (l outside 0..2), DEVICE.
 */
rhosvd_status rhosvd_get_xi(rhosvd_handle h, double* xip);
rhosvd_status rhosvd_get_spectrum(rhosvd_handle h, int32_t l, double* sigma_all);
rhosvd_status rhosvd_get_v(rhosvd_handle h, int32_t l, double* V);

/*
 * Batched reductions: many independent problems of uneven n and R in one pass.
 * The reductions of a batch are the same as rhosvd_reduce + rhosvd_get would
 * compute one by one (same options and precision as the handle), but no call
 * waits for the host: every phase is one launch over the whole batch, the
 * ranks stay on the device, and the Khatri-Rao cores of all problems run as one
 * persistent launch.  The first call with a given descriptor list (the bytes
 * of the array) lays out the workspace, uploads its tables and records the pass
 * into a HIP graph; later calls with an identical list replay that graph with
 * one launch on the handle's stream.  A new list replaces the cached plan
 * (synchronizing with the stream first).
 *
 * Per problem (all pointers DEVICE pointers; caller-owned; valid until the
 * stream has finished the call):
 *   n, R       : 1 <= n, R; min(n, R) <= 2048
 *   U1..U3, xi : inputs as for rhosvd_reduce
 *   eps        : > 0
 *   cap_rank   : >= 1, the columns available in each Z output (rows of each V); ranks above it
 *                give RHOSVD_ERR_CAPACITY for that problem (Z, beta not written)
 *   cap_beta   : entries available in beta (>= 1 when beta is set)
 *   Z1..Z3     : n x cap_rank outputs (ld n, first r_l columns written), or all NULL
 *   beta       : r1*r2*r3 output (Fortran order; doubles, or floats with the handle's
 *                beta_fp32 option), or NULL (ranks and Z only)
 *   V1..V3     : r_l x R outputs V^(l) = Z^(l)T U~^(l) (ld cap_rank, FP64, converted from FP32
 *                on the mixed paths): with xi' (the normalized weights) they are the
 *                factors of the mixed Tucker-canonical format of Proposition 2.2, whose core
 *                is the rank-R canonical tensor sum_nu xi'_nu V1[:,nu] (x) V2[:,nu] (x) V3[:,nu]
 *                (R (r1 + r2 + r3) numbers instead of r1 r2 r3), or all NULL.  Set with
 *                beta NULL to skip the Khatri-Rao core altogether.  xi' is not an output of
 *                the batch; it is xi times the three column norms of each term.
 *   result     : int32[8]: r1, r2, r3, status (rhosvd_status of this problem:
 *                OK, ERR_NONFINITE, ERR_CAPACITY, or ERR_DEVICE when an
 *                eigensolver wait ran out), dropped terms, the core's
 *                rhosvd_precision (one for the whole pass: FP32 in place of
 *                BF16x3 when some problem's eps is below 1e-5), 2 reserved
 *   reserved0  : must be zero
 * Returns (host): OK once the pass is enqueued (per-problem outcomes are in
 * result), ARG for a bad descriptor (message names the problem), UNSUPPORTED,
 * ALLOC, DEVICE.  A handle serves one batch at a time.
 */
typedef struct {
    int64_t n, R;
    const double* U1;
    const double* U2;
    const double* U3;
    const double* xi;
    double eps;
    int32_t cap_rank;
    int32_t reserved0;
    int64_t cap_beta;
    double* Z1;
    double* Z2;
    double* Z3;
    void* beta;
    int32_t* result;
    double* V1;
    double* V2;
    double* V3;
} rhosvd_problem;

rhosvd_status rhosvd_reduce_batched(rhosvd_handle h, int32_t count, const rhosvd_problem* problems);

/* 1 when the last batched call ran as a graph replay, 0 when it ran eagerly. */
int32_t rhosvd_batch_uses_graph(rhosvd_handle h);

/* Tile height (rows of j1) used by the last core launch on this handle
 * (rhosvd_get or rhosvd_reduce_batched): 64 or 128, 0 before any core. */
int32_t rhosvd_last_core_tile(rhosvd_handle h);

/*
 * Rank-proposal network (learned rank proposal for the randomized range
 * finder; not part of the paper's method, an addition on top of it).  A small
 * FP32 multilayer perceptron
 *     x (67) -> relu(W1 x + b1) (128) -> relu(W2 h1 + b2) (128) -> W3 h2 + b3 (2)
 * held on the handle.  Parameters are one float vector, W1 | b1 | W2 | b2 | W3 | b3,
 * each W row-major (out x in), rhosvd_net_num_params() floats in total.  Inputs
 * x are the per-mode features of rhosvd_sketch_features; rows of x, y, target
 * are samples.  All pointers are DEVICE pointers; calls are enqueued on the
 * handle's stream and do not synchronize.
 *   rhosvd_net_set_params : copy params in (and reset the Adam optimizer)
 *   rhosvd_net_get_params : copy params out
 *   rhosvd_net_forward    : y (count x 2) = net(x (count x 67))
 *   rhosvd_net_train_step : gradient of L = 1/(2 count) sum (y - target)^2 at the
 *                           current params into grad (nullable), L into loss
 *                           (nullable, one float), then one Adam step with
 *                           learning rate lr (lr = 0: gradient only, no update)
 * Errors: ARG, STATE (no parameters set), ALLOC, DEVICE.
 */
int32_t rhosvd_net_num_params(void);
rhosvd_status rhosvd_net_set_params(rhosvd_handle h, const float* params);
rhosvd_status rhosvd_net_get_params(rhosvd_handle h, float* params);
rhosvd_status rhosvd_net_forward(rhosvd_handle h, int32_t count, const float* x, float* y);
rhosvd_status rhosvd_net_train_step(rhosvd_handle h, int32_t count, const float* x, const float* target, float lr,
                                    float* loss, float* grad);

/*
 * Learned rank proposal with a randomized range finder (an addition on top of
 * the paper's method; Halko, Martinsson & Tropp 2011 for the range finder).
 *
 * rhosvd_sketch_features: normalizes the side matrices (as rhosvd_reduce) and
 *   writes the network's input for each mode into feat (DEVICE, 3 x 67 floats):
 *   from the 32 singular values s_k of the sketch Y_l = U~_l Omega[:, 0:32]
 *   (via the eigenvalues of Y_l^T Y_l), log10(s_k / s_1) / 16 clamped at -1,
 *   then 32 zeros, ln(n)/10, ln(R)/10, ln(eps)/10.
 *   omega: DEVICE, R x omega_cols Gaussian test matrix (ld R), omega_cols >= 32.
 *   Does not synchronize.  Errors: as rhosvd_reduce, ARG.
 *
 * rhosvd_reduce_learned: rhosvd_reduce with the network's proposals (the
 *   handle needs network parameters; omega_cols >= 64).  Per mode the network
 *   proposes a rank r^ and a sketch width p (out0 * m, out1 * m; p >= r^ + 8,
 *   rounded up to a multiple of 64, at most omega_cols).  Where 3p < m the mode
 *   runs the range finder: Y = U~ Omega[:, 0:p]; an orthonormal basis Q of Y in
 *   FP64 (two symmetric orthogonalizations); B = Q^T U~; eigenpairs of B B^T;
 *   tails t_r^2 = sum_{k>r} sigma_k(B)^2 + |U~ - Q B|_F^2 (the residual computed
 *   directly); r_l = min{r : t_r <= tau}; Z_l = Q times the top r_l eigenvectors.
 *   Theorem 2.3's bound holds for any orthonormal Z with these tails.  A mode
 *   whose residual alone exceeds tau (no r <= p certifies) falls back to the
 *   Gram path, as does every mode where 3p >= m (always when m < 192: the
 *   network is then not consulted), and every mode when R < n.
 *   Ranks, Z, beta and the report come out as for rhosvd_reduce (rhosvd_get);
 *   for a range-finder mode the spectrum holds the p Ritz values.
 *   info (HOST, nullable): per mode the proposed rank, the width used (0 on the
 *   Gram path), the path (0 range finder, 1 Gram path chosen up front, 2 Gram
 *   path after a failed certificate, 3 Gram path because R < n) and the residual.
 *   Synchronizes with the stream two or three times.
 */
typedef struct {
    int32_t proposal[3];
    int32_t width[3];
    int32_t fallback[3];
    int32_t reserved;
    double residual[3];
} rhosvd_learned_info;

rhosvd_status rhosvd_sketch_features(rhosvd_handle h, int64_t n, int64_t R, const double* U1, const double* U2,
                                     const double* U3, const double* xi, double eps, const double* omega,
                                     int32_t omega_cols, float* feat);
rhosvd_status rhosvd_reduce_learned(rhosvd_handle h, int64_t n, int64_t R, const double* U1, const double* U2,
                                    const double* U3, const double* xi, double eps, const double* omega,
                                    int32_t omega_cols, int32_t ranks[3], rhosvd_learned_info* info);

/*
 * Tucker-to-canonical transform (T2C) of a 3rd-order core (Section 2.3,
 * Remark 2.6, eqs. T2C_slice, T2C_SVD, beta_R).  The core is written as the sum
 * of its third-mode slices, beta = sum_m B_m (x) e_m with B_m = beta[:, :, m]
 * (r1 x r2); each slice's SVD keeps its p_m singular values above the threshold
 *     thr = eps / (r3 sqrt(min(r1, r2)))     (eps / r^(3/2) for an r x r x r core)
 * and the kept terms of all slices give the canonical tensor
 *     beta_(R) = sum_m sum_{k <= p_m} sigma_k^(m) u_k^(m) (x) v_k^(m) (x) e_m,
 * of rank R = p_1 + ... + p_r3 <= r3 min(r1, r2), with
 *     |beta - beta_(R)|_F <= sum_m (sum_{k > p_m} sigma_k^(m)^2)^(1/2) <= eps.
 * eps is absolute (as in the remark); a relative accuracy is eps_rel |beta|_F.
 * With orthonormal Tucker factors Z^(l) the same holds for the full tensors:
 * lifting the factors, A_(R) = sum sigma (Z1 u) (x) (Z2 v) (x) z3_m, leaves
 * |A_r - A_(R)| = |beta - beta_(R)|.
 *
 * Each slice is decomposed by a one-sided Jacobi SVD in one workgroup's LDS:
 * min(r1, r2) <= 256 and r1 * r2 * 8 bytes <= 152 KiB (a 139 x 139 core, or
 * 64 x 304 ...); larger cores give RHOSVD_ERR_UNSUPPORTED.
 *
 * rhosvd_t2c: phase 1, the slice SVDs and the counts.
 *   r1, r2, r3 : core dimensions (>= 1)
 *   beta       : DEVICE, r1*r2*r3 doubles, Fortran order (index j1 + r1 (j2 + r2 j3)),
 *                for example rhosvd_get's FP64 output; read again by rhosvd_t2c_get,
 *                so it must stay valid and unchanged until then
 *   eps        : absolute accuracy, > 0
 *   R          : HOST, receives the canonical rank R
 *   bound      : HOST, nullable, receives sum_m (sum_{k > p_m} sigma_k^2)^(1/2)
 * Synchronizes with the handle's stream once.  Errors: ARG, UNSUPPORTED,
 * NOCONV (a slice's Jacobi sweeps did not converge), ALLOC, DEVICE.
 *
 * rhosvd_t2c_get: phase 2, the R terms of the last rhosvd_t2c on this handle.
 *   weights : DEVICE, R doubles (sigma_k^(m), slices in order, descending within one)
 *   F1, F2  : DEVICE, r1 x R and r2 x R (column-major, ld r1 / r2): unit u_k, v_k
 *   slice   : DEVICE, R int32: m of each term (its third factor is e_m)
 *   n, Z1, Z2, Z3, C1, C2, C3 : optional lifting (all non-NULL and n >= 1, or
 *             all NULL): Z_l DEVICE n x r_l (ld n, orthonormal columns), C_l DEVICE
 *             n x R (ld n) receive Z1 F1, Z2 F2 and the columns Z3[:, slice]
 *   sigma   : DEVICE, nullable, r3 * min(r1, r2) doubles: every slice's singular
 *             values, slice by slice, descending
 * Enqueued on the handle's stream; does not synchronize.  Errors: STATE, ARG, DEVICE.
 */
rhosvd_status rhosvd_t2c(rhosvd_handle h, int32_t r1, int32_t r2, int32_t r3, const double* beta, double eps,
                         int64_t* R, double* bound);
rhosvd_status rhosvd_t2c_get(rhosvd_handle h, double* weights, double* F1, double* F2, int32_t* slice,
                             double* sigma, int64_t n, const double* Z1, const double* Z2, const double* Z3,
                             double* C1, double* C2, double* C3);

/*
 * rhosvd_t2c_noalloc: rhosvd_t2c and rhosvd_t2c_get in one call that allocates
 * nothing (no hipMalloc, hipFree or allocating library call), for callers that
 * cannot allocate device memory: code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid allocation.  It needs no handle and never
 * waits for the GPU: everything, the status included, is written to device memory.
 *
 * Workspace: one static device array of 8 MiB per GPU (created with the code
 * object, held until the process ends), shared by every call on that GPU: calls
 * that overlap on one GPU (different streams, or threads) race and must not be
 * made.  The core must fit it: r3 (max(r1, r2) min(r1, r2) + min(r1, r2) + 3) doubles
 * plus a few hundred bytes (for example a 64 x 64 x 64 or 90 x 90 x 60 core), and
 * the limits of rhosvd_t2c; larger cores return RHOSVD_ERR_UNSUPPORTED.
 *
 *   hip_stream : hipStream_t as void* (NULL: the default stream); all work is enqueued on it
 *   r1, r2, r3, beta, eps : as rhosvd_t2c (beta DEVICE, read during the call's kernels)
 *   cap        : capacity of the outputs in terms (>= 0); R above it writes no term
 *   weights, F1, F2, slice : DEVICE outputs as rhosvd_t2c_get, each sized for cap terms
 *                (F1 r1 x cap, F2 r2 x cap, ld r1 / r2); may be NULL when cap = 0
 *   R          : DEVICE int64, receives the canonical rank
 *   bound      : DEVICE double, nullable, receives the error estimate (as rhosvd_t2c)
 *   status     : DEVICE int32, receives RHOSVD_OK, RHOSVD_ERR_NOCONV (a slice's Jacobi
 *                sweeps did not converge) or RHOSVD_ERR_CAPACITY (R > cap); the terms
 *                are written only with RHOSVD_OK
 * Returns (host): OK once enqueued, ARG, UNSUPPORTED, DEVICE.
 */
rhosvd_status rhosvd_t2c_noalloc(void* hip_stream, int32_t r1, int32_t r2, int32_t r3, const double* beta,
                                 double eps, int64_t cap, double* weights, double* F1, double* F2, int32_t* slice,
                                 int64_t* R, double* bound, int32_t* status);

/* Phase times in milliseconds of the last rhosvd_reduce / rhosvd_get when the
 * handle was created with profile != 0 (synchronizes with the stream):
 *   0 norms, 1 |A| identity, 2 Gram, 3 eigensolver, 4 truncation + Z (with the
 *   |A| probe, which runs after the eigensolver), 5 projection, 6 core.  Returns -1 for an unknown phase or when profiling is off. */
double rhosvd_phase_ms(rhosvd_handle h, int32_t phase);

/* Message describing the last error on this handle ("" if none); valid until
 * the next call on the handle.  h may be NULL (message of the last failed create). */
const char* rhosvd_last_error(rhosvd_handle h);

/* Library version string. */
const char* rhosvd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RHOSVD_H */
