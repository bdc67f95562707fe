/*
 * TEST INFRASTRUCTURE ONLY.  Part of the CPU oracle for the Reduced HOSVD:
 * only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code with the GPU path.
 *
 * Left singular vectors and singular values of a side matrix X (p x q,
 * column-major), computed the slow and obviously correct way:
 *
 *   1. Householder QR of the tall orientation Y (Y = X^T when p <= q, else Y = X):
 *      Y = Q1 R1 with R1 (m x m) upper triangular, m = min(p, q).
 *   2. One-sided (Hestenes) Jacobi on the columns of B (B = R1 when p <= q,
 *      B = R1^T otherwise): plane rotations J are applied until all columns of
 *      B J are mutually orthogonal; then B J = P diag(sigma) and J holds the
 *      right singular vectors of B.
 *   3. p <= q: X = R1^T Q1^T, so the left singular vectors of X are J.
 *      p >  q: X = Q1 R1, so they are Q1 J.
 *
 * This is the SVD of each side matrix U^(l) = Z D V^T that the method is built
 * on (Section 2.1, eqs. eqn:SVD_Ul and eq:svdr).  The QR step only
 * preconditions the Jacobi iteration; it does not change the result.
 *
 * Jacobi pairs are visited in round-robin ("tournament") order so that the
 * m/2 pairs of one round are disjoint and can run in parallel (OpenMP).
 * Convergence: a full sweep in which every pair already satisfies
 * |b_i . b_j| <= tol * |b_i| |b_j|, tol = m * 2^-53.
 *
 * Error codes: 0 ok, -1 bad argument, -2 allocation failure, -5 sweep cap hit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

static double dot(const double* a, const double* b, int64_t len) {
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += a[i] * b[i];
    return s;
}

/* Householder QR of Y (N x m, N >= m, column-major, ld = N), in place:
 * R1 in the upper triangle, reflector k stored as v_k = [1; Y[k+1:N, k]] with
 * scalar tau[k], so that H_k = I - tau_k v_k v_k^T and Q1 = H_0 H_1 ... H_{m-1}. */
static void householder_qr(int64_t N, int64_t m, double* Y, double* tau) {
    for (int64_t k = 0; k < m; ++k) {
        double* x = Y + IDX(k, k, N);
        int64_t len = N - k;
        double normx = 0.0, scale = 0.0;
        for (int64_t i = 0; i < len; ++i) scale = fmax(scale, fabs(x[i]));
        if (scale == 0.0) { tau[k] = 0.0; continue; }
        for (int64_t i = 0; i < len; ++i) { double t = x[i] / scale; normx += t * t; }
        normx = scale * sqrt(normx);
        double alpha = x[0];
        double beta = (alpha >= 0.0) ? -normx : normx;   /* new diagonal entry */
        /* v = x - beta e1, scaled so v[0] = 1 */
        double v0 = alpha - beta;
        for (int64_t i = 1; i < len; ++i) x[i] /= v0;
        tau[k] = (beta - alpha) / beta;
        x[0] = beta;
        /* apply H_k to the trailing columns */
#pragma omp parallel for schedule(static)
        for (int64_t j = k + 1; j < m; ++j) {
            double* y = Y + IDX(k, j, N);
            double s = y[0];
            for (int64_t i = 1; i < len; ++i) s += x[i] * y[i];
            s *= tau[k];
            y[0] -= s;
            for (int64_t i = 1; i < len; ++i) y[i] -= s * x[i];
        }
    }
}

/* M (N x c) <- Q1 M, with Q1 from householder_qr (reflectors applied last-first). */
static void apply_q(int64_t N, int64_t m, const double* Y, const double* tau,
                    int64_t c, double* M) {
    for (int64_t k = m - 1; k >= 0; --k) {
        if (tau[k] == 0.0) continue;
        const double* v = Y + IDX(k, k, N);
        int64_t len = N - k;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < c; ++j) {
            double* y = M + IDX(k, j, N);
            double s = y[0];
            for (int64_t i = 1; i < len; ++i) s += v[i] * y[i];
            s *= tau[k];
            y[0] -= s;
            for (int64_t i = 1; i < len; ++i) y[i] -= s * v[i];
        }
    }
}

/* One-sided Jacobi on the columns of B (m x m, ld = m); J (m x m) accumulates
 * the rotations starting from the identity.  Returns sweeps used, or -1 if the
 * cap was hit before convergence.
 * A pair (p, q) is orthogonal enough when |b_p . b_q| <= m u |b_p| |b_q|, or
 * when |b_p . b_q| <= (2 m u |B|_F)^2: below that floor a rotation cannot move
 * any singular value above about 2 m u |B|_F, the part of the spectrum that FP64
 * data determines at all; without the floor, pairs of columns that are pure
 * rounding noise can keep failing the relative test forever. */
static int jacobi_columns(int64_t m, double* B, double* J, int max_sweeps) {
    memset(J, 0, sizeof(double) * (size_t)m * (size_t)m);
    for (int64_t i = 0; i < m; ++i) J[IDX(i, i, m)] = 1.0;
    if (m < 2) return 0;
    const double tol = (double)m * ldexp(1.0, -53);
    double fro2 = 0.0;                  /* |B|_F^2 (rotations preserve it) */
    for (int64_t j = 0; j < m; ++j) fro2 += dot(B + IDX(0, j, m), B + IDX(0, j, m), m);
    const double floor_g = 4.0 * tol * tol * fro2;
    int64_t slots = (m % 2 == 0) ? m : m + 1;     /* odd m: one dummy slot */
    int64_t* ring = (int64_t*)malloc(sizeof(int64_t) * (size_t)slots);
    if (!ring) return -2;
    for (int64_t i = 0; i < slots; ++i) ring[i] = i;
    int sweeps = 0;
    for (;;) {
        if (sweeps >= max_sweeps) { free(ring); return -1; }
        ++sweeps;
        int64_t rotated = 0;
        for (int64_t round = 0; round < slots - 1; ++round) {
            /* pairs (ring[k], ring[slots-1-k]), k = 0..slots/2-1 */
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : rotated)
            for (int64_t k = 0; k < slots / 2; ++k) {
                int64_t p = ring[k], q = ring[slots - 1 - k];
                if (p >= m || q >= m) continue;
                if (p > q) { int64_t t = p; p = q; q = t; }
                double* bp = B + IDX(0, p, m);
                double* bq = B + IDX(0, q, m);
                double a = dot(bp, bp, m), b = dot(bq, bq, m), g = dot(bp, bq, m);
                if (a == 0.0 || b == 0.0) continue;
                if (fabs(g) <= tol * sqrt(a) * sqrt(b) || fabs(g) <= floor_g) continue;
                /* rotation [bp bq] <- [bp bq] [[c, s], [-s, c]] zeroing bp.bq */
                double zeta = (b - a) / (2.0 * g);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int64_t i = 0; i < m; ++i) {
                    double x = bp[i], y = bq[i];
                    bp[i] = c * x - s * y;
                    bq[i] = s * x + c * y;
                }
                double* jp = J + IDX(0, p, m);
                double* jq = J + IDX(0, q, m);
                for (int64_t i = 0; i < m; ++i) {
                    double x = jp[i], y = jq[i];
                    jp[i] = c * x - s * y;
                    jq[i] = s * x + c * y;
                }
                rotated += 1;
            }
            /* tournament rotation: keep ring[0], shift the rest by one */
            int64_t last = ring[slots - 1];
            for (int64_t i = slots - 1; i > 1; --i) ring[i] = ring[i - 1];
            ring[1] = last;
        }
        if (rotated == 0) break;
    }
    free(ring);
    return sweeps;
}

/*
 * orc_svd_left: X (p x q, column-major, ld = p, read only).
 * Outputs: sigma[m] descending, Z (p x m, column-major) left singular vectors,
 * m = min(p, q).  *sweeps_out = Jacobi sweeps used.
 */
int orc_svd_left(int64_t p, int64_t q, const double* X, double* sigma, double* Z,
                 int max_sweeps, int* sweeps_out) {
    if (p < 1 || q < 1 || !X || !sigma || !Z) return -1;
    int wide = (p <= q);
    int64_t N = wide ? q : p;          /* rows of the tall orientation */
    int64_t m = wide ? p : q;
    double* Y = (double*)malloc(sizeof(double) * (size_t)N * (size_t)m);
    double* tau = (double*)malloc(sizeof(double) * (size_t)m);
    double* B = (double*)malloc(sizeof(double) * (size_t)m * (size_t)m);
    double* J = (double*)malloc(sizeof(double) * (size_t)m * (size_t)m);
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    double* nrm = (double*)malloc(sizeof(double) * (size_t)m);
    if (!Y || !tau || !B || !J || !order || !nrm) {
        free(Y); free(tau); free(B); free(J); free(order); free(nrm);
        return -2;
    }
    /* tall orientation */
    if (wide) {
        for (int64_t j = 0; j < m; ++j)
            for (int64_t i = 0; i < N; ++i) Y[IDX(i, j, N)] = X[IDX(j, i, p)];
    } else {
        memcpy(Y, X, sizeof(double) * (size_t)N * (size_t)m);
    }
    householder_qr(N, m, Y, tau);
    /* B = R1 (wide) or R1^T (tall) */
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double r = (i <= j) ? Y[IDX(i, j, N)] : 0.0;   /* R1[i][j] */
            if (wide) B[IDX(i, j, m)] = r;
            else      B[IDX(j, i, m)] = r;
        }
    int sw = jacobi_columns(m, B, J, max_sweeps);
    if (sweeps_out) *sweeps_out = sw;
    if (sw < 0) {
        free(Y); free(tau); free(B); free(J); free(order); free(nrm);
        return sw == -2 ? -2 : -5;
    }
    for (int64_t j = 0; j < m; ++j) {
        double s2 = 0.0, sc = 0.0;
        const double* b = B + IDX(0, j, m);
        for (int64_t i = 0; i < m; ++i) sc = fmax(sc, fabs(b[i]));
        if (sc > 0.0)
            for (int64_t i = 0; i < m; ++i) { double t = b[i] / sc; s2 += t * t; }
        nrm[j] = sc * sqrt(s2);
        order[j] = j;
    }
    /* sort descending by sigma (stable insertion sort: ties keep index order) */
    for (int64_t i = 1; i < m; ++i) {
        int64_t o = order[i];
        int64_t k = i;
        while (k > 0 && nrm[order[k - 1]] < nrm[o]) { order[k] = order[k - 1]; --k; }
        order[k] = o;
    }
    for (int64_t j = 0; j < m; ++j) sigma[j] = nrm[order[j]];
    if (wide) {
        for (int64_t j = 0; j < m; ++j)
            memcpy(Z + IDX(0, j, p), J + IDX(0, order[j], m), sizeof(double) * (size_t)m);
    } else {
        /* Z = Q1 [J; 0] */
        double* M = (double*)calloc((size_t)N * (size_t)m, sizeof(double));
        if (!M) { free(Y); free(tau); free(B); free(J); free(order); free(nrm); return -2; }
        for (int64_t j = 0; j < m; ++j)
            memcpy(M + IDX(0, j, N), J + IDX(0, order[j], m), sizeof(double) * (size_t)m);
        apply_q(N, m, Y, tau, m, M);
        memcpy(Z, M, sizeof(double) * (size_t)N * (size_t)m);
        free(M);
    }
    free(Y); free(tau); free(B); free(J); free(order); free(nrm);
    return 0;
}

/* Number of OpenMP threads this library runs with (reported by the CPU baseline). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
