"""Seeded synthetic canonical tensors shaped like the paper's workloads.

This module only *builds inputs*: side matrices U^(l) (n x R, column-major,
column nu = canonical vector u_nu^(l)) and weights xi.  It holds none of the
reduction's arithmetic (no norms, Grams, SVDs, projections or cores), so both
the HIP path and the CPU oracle may draw their inputs from it.

Workload shapes follow the paper's own sources of large-rank canonical tensors:
  * sums of Gaussians sampled on a uniform grid (Section 4.1, the sinc /
    Laplace-Gauss route to radial kernels, eqs. eqn:laplace, eqn:sinc_Newt);
  * the Newton kernel 1/|x| as a Gaussian sum, from the Laplace-Gauss identity
    1/z = (2/sqrt(pi)) int_0^inf exp(-z^2 t^2) dt (eq. eqn:Laplace_Newton);
  * Hadamard products of canonical tensors, whose rank is the product of the
    factors' ranks (Section 4.2, Lemma 4.3; Section 3, eq. eq:rho_ten).

Grid: cell centres x_i = -b + (i + 1/2) * 2b/n, i = 0..n-1 (the paper samples
at "centers of discretization intervals", Section 3; mesh h = 2b/n, Section 4.1).

Random numbers come from numpy's counter-based Philox generator keyed by
(workload id, seed), so every machine draws the same stream.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# workload ids used as the first Philox key word
WL_SMALL_GAUSS = 0      # n=64, R=200 Gaussian sum
WL_NEWTON_CENTRES = 1   # n=1024, R=4096: 128 charges x 32-term 1/|x| sum
WL_HADAMARD = 2         # n=512, R=90000 Hadamard product of two 300-term sums
WL_BATCH = 3            # 256 uneven (n, R) problems
WL_RANKNET = 4          # rank-proposal training / evaluation draws
WL_LOWRANK = 10         # exactly-low-rank test inputs
WL_RANDOM = 11          # dense random test inputs
WL_CORE = 13            # synthetic Tucker cores (Tucker-to-canonical tests)
WL_RS = 14              # range-separated workloads (multi-Slater amplitudes)


def rng(workload: int, seed: int) -> np.random.Generator:
    """Philox stream keyed by (workload, seed)."""
    return np.random.Generator(np.random.Philox(key=[int(workload), int(seed)]))


def grid(n: int, b: float = 10.0) -> np.ndarray:
    """Cell centres of a uniform n-cell grid on [-b, b]."""
    h = 2.0 * b / n
    return -b + (np.arange(n, dtype=np.float64) + 0.5) * h


@dataclass
class CanonicalInput:
    """A d=3 canonical tensor A = sum_nu xi_nu u1_nu (x) u2_nu (x) u3_nu."""
    U: list            # three float64 arrays, shape (n, R), Fortran order
    xi: np.ndarray     # float64, shape (R,)
    eps: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.U[0].shape[0])

    @property
    def R(self) -> int:
        return int(self.U[0].shape[1])


def gaussian_side_matrices(x: np.ndarray, alpha: np.ndarray, centres: np.ndarray) -> list:
    """u_nu^(l)(i) = exp(-alpha_nu (x_i - c_{nu,l})^2) for l = 0, 1, 2.

    alpha: (R,), centres: (R, 3).  Returns three (n, R) Fortran-ordered arrays.
    """
    out = []
    for l in range(3):
        d = x[:, None] - centres[None, :, l]
        out.append(np.asfortranarray(np.exp(-alpha[None, :] * d * d)))
    return out


def small_gaussian_sum(seed: int = 0, n: int = 64, R: int = 200, b: float = 10.0,
                       eps: float = 1e-6) -> CanonicalInput:
    """n=64 grid on [-10,10]^3, R Gaussians exp(-a_k |x-c_k|^2) factored per axis,
    a_k log-uniform in [0.5, 50], c_k uniform in [-5,5]^3, xi_k uniform in [0.5, 1.5]."""
    g = rng(WL_SMALL_GAUSS, seed)
    alpha = np.exp(g.uniform(math.log(0.5), math.log(50.0), size=R))
    centres = g.uniform(-5.0, 5.0, size=(R, 3))
    xi = g.uniform(0.5, 1.5, size=R)
    U = gaussian_side_matrices(grid(n, b), alpha, centres)
    return CanonicalInput(U, xi, eps, name=f"gauss-n{n}-R{R}",
                          meta=dict(alpha=alpha, centres=centres, b=b))


def newton_gaussian_sum(K: int = 32, lo: float = 1e-2, hi: float = 1e4):
    """K-term Gaussian sum for 1/|x| with exponents log-spaced in [lo, hi].

    From 1/z = (1/sqrt(pi)) int exp(-z^2 e^s) e^{s/2} ds (substitute t^2 = e^s in
    the Laplace-Gauss identity for the Newton kernel) and the trapezoid rule in
    s with step h: alpha_k = e^{s_k}, w_k = h sqrt(alpha_k) / sqrt(pi).
    All weights are positive.
    """
    s = np.linspace(math.log(lo), math.log(hi), K)
    h = s[1] - s[0]
    alpha = np.exp(s)
    w = h * np.sqrt(alpha) / math.sqrt(math.pi)
    return alpha, w


def newton_centres(seed: int = 0, n: int = 1024, n_centres: int = 128, K: int = 32,
                   b: float = 10.0, box: float = 6.0, eps: float = 1e-5,
                   workload: int = WL_NEWTON_CENTRES) -> CanonicalInput:
    """sum_c q_c / |x - c| over n_centres random centres in [-box, box]^3 with
    random charges q_c = +-1, each 1/|x-c| a K-term Gaussian sum: R = n_centres*K."""
    g = rng(workload, seed)
    centres_c = g.uniform(-box, box, size=(n_centres, 3))
    q = np.where(g.uniform(size=n_centres) < 0.5, -1.0, 1.0)
    alpha_k, w_k = newton_gaussian_sum(K)
    alpha = np.tile(alpha_k, n_centres)
    centres = np.repeat(centres_c, K, axis=0)
    xi = np.repeat(q, K) * np.tile(w_k, n_centres)
    U = gaussian_side_matrices(grid(n, b), alpha, centres)
    return CanonicalInput(U, xi, eps, name=f"newton-n{n}-R{n_centres * K}",
                          meta=dict(alpha=alpha, centres=centres, q=q, b=b))


def hadamard_product(seed: int = 0, n: int = 512, R_each: int = 300, b: float = 10.0,
                     eps: float = 1e-4) -> CanonicalInput:
    """Pointwise product of two Gaussian sums of R_each terms (each drawn like
    small_gaussian_sum): columns u_a * w_b for all (a, b), weights xi_a * eta_b,
    so R = R_each^2 (the rank-multiplying Hadamard product of canonical tensors)."""
    g = rng(WL_HADAMARD, seed)
    x = grid(n, b)
    parts = []
    for _ in range(2):
        alpha = np.exp(g.uniform(math.log(0.5), math.log(50.0), size=R_each))
        centres = g.uniform(-5.0, 5.0, size=(R_each, 3))
        xi = g.uniform(0.5, 1.5, size=R_each)
        parts.append((gaussian_side_matrices(x, alpha, centres), xi))
    (Ua, xa), (Ub, xb) = parts
    U = []
    for l in range(3):
        P = (Ua[l][:, :, None] * Ub[l][:, None, :]).reshape(n, R_each * R_each)
        U.append(np.asfortranarray(P))
    xi = (xa[:, None] * xb[None, :]).reshape(-1)
    return CanonicalInput(U, xi, eps, name=f"hadamard-n{n}-R{R_each * R_each}",
                          meta=dict(factors=((Ua, xa), (Ub, xb))))


def batch_shapes(seed: int = 0, count: int = 256):
    """(n, R) for the uneven batch: n uniform in {128,...,2048}, R log-uniform in [64, 8192]."""
    g = rng(WL_BATCH, seed)
    ns = g.choice(np.array([128, 256, 512, 1024, 2048]), size=count)
    Rs = np.rint(np.exp(g.uniform(math.log(64), math.log(8192), size=count))).astype(int)
    return [(int(a), int(c)) for a, c in zip(ns, Rs)]


def batch_problem(seed: int, index: int, n: int, R: int, eps: float = 1e-5) -> CanonicalInput:
    """One problem of the uneven batch: the first R terms of ceil(R/32) charges x 32
    Gaussian terms (the n=1024, R=4096 construction at another size)."""
    nc = (R + 31) // 32
    full = newton_centres(seed=seed * 4096 + index, n=n, n_centres=nc, eps=eps,
                          workload=WL_BATCH)
    U = [np.asfortranarray(u[:, :R]) for u in full.U]
    return CanonicalInput(U, full.xi[:R].copy(), eps, name=f"batch{index}-n{n}-R{R}")


def batch_problem_params(seed: int, index: int, n: int, R: int, eps: float = 1e-5):
    """The random draws of batch_problem (alpha, centres (R, 3), xi) without
    sampling the side matrices: the same Philox stream, so the tensors built from
    them on any device are the ones batch_problem returns."""
    nc = (R + 31) // 32
    g = rng(WL_BATCH, seed * 4096 + index)
    centres_c = g.uniform(-6.0, 6.0, size=(nc, 3))
    q = np.where(g.uniform(size=nc) < 0.5, -1.0, 1.0)
    alpha_k, w_k = newton_gaussian_sum(32)
    alpha = np.tile(alpha_k, nc)[:R]
    centres = np.repeat(centres_c, 32, axis=0)[:R]
    xi = (np.repeat(q, 32) * np.tile(w_k, nc))[:R]
    return alpha, centres, xi


def gaussian_side_matrices_torch(n: int, alpha: np.ndarray, centres: np.ndarray, b: float = 10.0,
                                 device: str = "cuda") -> list:
    """gaussian_side_matrices sampled with torch on `device`: three (n, R)
    column-major float64 tensors (for inputs too large to build on the host)."""
    import torch
    x = torch.from_numpy(grid(n, b)).to(device)
    a = torch.from_numpy(np.ascontiguousarray(alpha)).to(device)
    out = []
    for l in range(3):
        c = torch.from_numpy(np.ascontiguousarray(centres[:, l])).to(device)
        d = x[None, :] - c[:, None]                   # (R, n): row nu is column nu of U
        out.append(torch.exp(-a[:, None] * d * d).t())
    return out


def gaussian_test_matrix(seed: int, R: int, w: int) -> np.ndarray:
    """R x w standard Gaussian test matrix (Fortran order) for the sketches of the
    learned rank proposal and its randomized range finder."""
    g = rng(WL_RANKNET, seed)
    return np.asfortranarray(g.standard_normal(size=(R, w)))


def smooth_problem_params(seed: int, index: int, n: int, R: int):
    """A smooth Gaussian sum (the low-rank end of the rank-proposal workloads):
    exponents log-uniform in [1e-2, 1], centres uniform in [-6, 6]^3, weights
    uniform in [-1, 1].  Returns (alpha, centres (R, 3), xi)."""
    g = rng(WL_RANKNET, 2_000_000 + seed * 4096 + index)
    alpha = np.exp(g.uniform(math.log(1e-2), math.log(1.0), size=R))
    centres = g.uniform(-6.0, 6.0, size=(R, 3))
    xi = g.uniform(-1.0, 1.0, size=R)
    return alpha, centres, xi


def ranknet_shapes(seed: int, count: int):
    """(family, n, R, eps) of the rank-proposal training and evaluation problems:
    the uneven batch's size distribution (n uniform in {128,...,2048}, R
    log-uniform in [64, 8192]), eps uniform over {1e-6, 1e-5, 1e-4, 1e-3}, and
    the family ("newton": charges x 32-term 1/|x| sums, ranks about 0.6 m;
    "smooth": smooth_problem_params, ranks about 0.1 m) with equal odds."""
    g = rng(WL_RANKNET, 1_000_000 + seed)
    ns = g.choice(np.array([128, 256, 512, 1024, 2048]), size=count)
    Rs = np.rint(np.exp(g.uniform(math.log(64), math.log(8192), size=count))).astype(int)
    es = g.choice(np.array([1e-6, 1e-5, 1e-4, 1e-3]), size=count)
    fam = np.where(g.uniform(size=count) < 0.5, "newton", "smooth")
    return [(str(f), int(a), int(c), float(e)) for f, a, c, e in zip(fam, ns, Rs, es)]


def exactly_low_rank(seed: int, n: int, R: int, ranks=(3, 4, 5), eps: float = 1e-8,
                     signed: bool = True) -> CanonicalInput:
    """U^(l) = Q_l C_l with Q_l (n x r_l) orthonormal and C_l (r_l x R) Gaussian, so
    every side matrix has rank exactly r_l (up to rounding)."""
    g = rng(WL_LOWRANK, seed)
    U = []
    for r in ranks:
        Q, _ = np.linalg.qr(g.standard_normal((n, r)))
        C = g.standard_normal((r, R))
        U.append(np.asfortranarray(Q @ C))
    xi = g.standard_normal(R) if signed else g.uniform(0.5, 1.5, size=R)
    return CanonicalInput(U, xi, eps, name=f"lowrank-n{n}-R{R}-r{ranks}")


def random_dense(seed: int, n: int, R: int, eps: float = 1e-3) -> CanonicalInput:
    """Gaussian random side matrices and weights (no structure, slow singular decay)."""
    g = rng(WL_RANDOM, seed)
    U = [np.asfortranarray(g.standard_normal((n, R))) for _ in range(3)]
    xi = g.standard_normal(R)
    return CanonicalInput(U, xi, eps, name=f"random-n{n}-R{R}")


def core_with_slice_spectra(seed: int, r1: int, r2: int, r3: int, spectra) -> np.ndarray:
    """An r1 x r2 x r3 core (Fortran order) whose third-mode slice m is
    Q_m diag(spectra[m]) P_m^T with random orthonormal Q_m (r1 x k), P_m (r2 x k),
    k = min(r1, r2): the slices' singular values are spectra[m] exactly (up to
    rounding)."""
    g = rng(WL_CORE, seed)
    k = min(r1, r2)
    beta = np.zeros((r1, r2, r3), order="F")
    for m in range(r3):
        Q, _ = np.linalg.qr(g.standard_normal((r1, k)))
        P, _ = np.linalg.qr(g.standard_normal((r2, k)))
        beta[:, :, m] = (Q * np.asarray(spectra[m])[None, :]) @ P.T
    return beta


def random_core(seed: int, r1: int, r2: int, r3: int) -> np.ndarray:
    """Gaussian random core (Fortran order)."""
    return np.asfortranarray(rng(WL_CORE, 100_000 + seed).standard_normal((r1, r2, r3)))


# ---------------------------------------------------------------------------
# range-separated (RS) workloads of Section 4: sinc-quadrature Gaussian sums for
# radial functions, split into long-range (t_k <= 1) and short-range terms
# (eq. eqn:RS_repres), the Hadamard cube of the Newton kernel (the 1/|x|^3 example
# of Section 5) and sums of Slater functions on lattices (Section 4.5)
# ---------------------------------------------------------------------------
def collocation_grid(n: int, b: float = 10.0) -> np.ndarray:
    """n equispaced points on [-b, b] including both ends (and the origin for odd
    n): the collocation discretization of Section 4.1 for continuous or singular
    radial functions."""
    return np.linspace(-b, b, n)


def _sinc_rule(M: int, h: float, logweight):
    """Trapezoid rule in s over nodes s_k = k h, k = -M..M, of int f(s) ds with
    f = exp(logweight(s)) times a Gaussian factor: returns (s_k, log w_k)."""
    s = h * np.arange(-M, M + 1, dtype=np.float64)
    return s, math.log(h) + logweight(s)


def newton_sinc_terms(R: int = 19, n: int = 257, b: float = 10.0):
    """R-term (R = 2M + 1) Gaussian sum for 1/z, 1/z ~ sum_k w_k exp(-t_k^2 z^2):
    the Laplace-Gauss identity 1/z = (2/sqrt(pi)) int_0^inf exp(-z^2 t^2) dt
    (eq. eqn:Laplace_Newton) with t = e^s and the trapezoid rule at s_k = k h,
    k = -M..M (eq. eqn:sinc_Newt): t_k = e^{s_k}, w_k = (2/sqrt(pi)) h e^{s_k}.
    The step h is the one (on a fine scan) with the smallest relative error on
    z in [grid step, 2 b sqrt(3)], the range the grid's differences span.
    Long-range terms are those with t_k <= 1 (k <= 0): M + 1 of them."""
    assert R % 2 == 1
    M = (R - 1) // 2
    z = np.geomspace(2.0 * b / (n - 1), 2.0 * b * math.sqrt(3.0), 400)
    best = None
    for h in np.linspace(0.05, 2.5, 491):
        s, lw = _sinc_rule(M, h, lambda s: math.log(2.0 / math.sqrt(math.pi)) + s)
        t2 = np.exp(2.0 * s)
        approx = np.exp(lw)[None, :] * np.exp(-z[:, None] ** 2 * t2[None, :])
        err = float(np.max(np.abs(approx.sum(axis=1) * z - 1.0)))
        if best is None or err < best[0]:
            best = (err, h)
    s, lw = _sinc_rule(M, best[1], lambda s: math.log(2.0 / math.sqrt(math.pi)) + s)
    return np.exp(s), np.exp(lw), dict(h=best[1], rel_err=best[0])


def newton_kernel(n: int = 257, R: int = 19, b: float = 10.0, long_range: bool = False):
    """Side matrices and weights of the collocated Newton kernel P_R (eq.
    eqn:sinc_general): columns exp(-t_k^2 x_i^2) on the collocation grid, weights
    w_k; with long_range only the terms t_k <= 1 (P_{R_l} of eq. eqn:RS_repres)."""
    t, w, info = newton_sinc_terms(R, n, b)
    keep = t <= 1.0 if long_range else np.ones_like(t, dtype=bool)
    x = collocation_grid(n, b)
    V = np.exp(-(x[:, None] ** 2) * (t[keep] ** 2)[None, :])
    return V, w[keep], info


def newton_cubed(n: int = 257, R: int = 19, b: float = 10.0, long_range: bool = False,
                 eps: float = 1e-5) -> CanonicalInput:
    """P (.) P (.) P, the discretized 1/|x|^3 of Section 5 (the Newton kernel's
    Gaussian sum cubed pointwise, Lemma 4.3 for its long-range part): columns
    p_a (.) p_b (.) p_c in each mode for all (a, b, c), weights w_a w_b w_c, so
    R' = R^3 (6859 for R = 19; 1000 for the long-range part, R_l = 10)."""
    V, w, info = newton_kernel(n, R, b, long_range)
    K = V.shape[1]
    col = (V[:, :, None, None] * V[:, None, :, None] * V[:, None, None, :]).reshape(n, K ** 3)
    xi = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
    U = [np.asfortranarray(col) for _ in range(3)]
    name = f"newton-cubed{'-long' if long_range else ''}-n{n}-R{K ** 3}"
    return CanonicalInput(U, xi, eps, name=name, meta=dict(terms=K, sinc=info, b=b))


def slater_sinc_terms(lam: float = 0.5, R: int = 8, R_l: int = 3, n: int = 384, b: float = 10.0):
    """R-term Gaussian sum for the Slater function exp(-lam |x|) = G(rho),
    rho = |x|^2, from its Laplace transform G(rho) = int_0^inf Ghat(tau)
    exp(-rho tau) dtau with Ghat(tau) = sqrt(alpha/pi) tau^{-3/2} exp(-alpha/tau),
    alpha = lam^2 / 4 (eq. Slater_Laplace_tr): tau = e^s, trapezoid nodes
    s_k = (k - R_l + 1) h, k = 0..R-1, so that exactly R_l terms have tau_k <= 1
    (the long-range part).  Weights w_k = h sqrt(alpha/pi) e^{-s_k/2}
    exp(-alpha e^{-s_k}).  h minimizes the max error on rho in
    [grid step^2, 12 b^2] (a scan)."""
    alpha = lam * lam / 4.0
    rho = np.geomspace((2.0 * b / (n - 1)) ** 2, 12.0 * b * b, 400)
    exact = np.exp(-lam * np.sqrt(rho))

    def rule(h):
        s = h * (np.arange(R, dtype=np.float64) - (R_l - 1))
        lw = math.log(h) + 0.5 * math.log(alpha / math.pi) - 0.5 * s - alpha * np.exp(-s)
        return np.exp(s), np.exp(lw)

    best = None
    for h in np.linspace(0.05, 3.0, 591):
        tau, w = rule(h)
        err = float(np.max(np.abs((w[None, :] * np.exp(-rho[:, None] * tau[None, :])).sum(axis=1) - exact)))
        if best is None or err < best[0]:
            best = (err, h)
    tau, w = rule(best[1])
    return tau, w, dict(h=best[1], max_err=best[0])


def lattice_nodes(L, spacing: float = 1.0) -> np.ndarray:
    """Nodes of an L1 x L2 x L3 lattice with the given spacing, centred at the origin."""
    axes = [spacing * (np.arange(Lk, dtype=np.float64) - (Lk - 1) / 2.0) for Lk in L]
    X, Y, Zc = np.meshgrid(*axes, indexing="ij")
    return np.stack([X.ravel(order="F"), Y.ravel(order="F"), Zc.ravel(order="F")], axis=1)


def slater_amplitude_function(nodes: np.ndarray, c1: float = 6.0, c2: float = 0.1) -> np.ndarray:
    """F(x,y,z) = c1 cos(x + 2y + 4z) exp(-c2 sqrt(x^2 + 2y^2 + 4z^2)) (eq. eq:func2)."""
    x, y, z = nodes[:, 0], nodes[:, 1], nodes[:, 2]
    return c1 * np.cos(x + 2 * y + 4 * z) * np.exp(-c2 * np.sqrt(x * x + 2 * y * y + 4 * z * z))


def multi_slater(L=(4, 4, 4), n: int = 384, lam: float = 0.5, R: int = 8, R_l: int = 3, b: float = 10.0,
                 spacing: float = 1.0, amplitudes: str = "random", seed: int = 0, long_range: bool = True,
                 eps: float = 1e-3) -> CanonicalInput:
    """Long-range part of a sum of Slater functions c_j exp(-lam |x - x_j|) over
    the nodes x_j of an L1 x L2 x L3 lattice (Section 4.5, eq.
    eqn:Slater_interp_multi): each Slater function is the Gaussian sum of
    slater_sinc_terms, and its long-range terms (tau_k <= 1; all terms when
    long_range is False) are shifted to the node, so the canonical rank is
    N R_l.  Amplitudes: uniform in [-5, 5] ("random", Table 4.1) or
    slater_amplitude_function at the nodes ("function", Table 4.2).
    Collocation grid on [-b, b]."""
    tau, w, info = slater_sinc_terms(lam, R, R_l, n, b)
    keep = tau <= 1.0 if long_range else np.ones_like(tau, dtype=bool)
    tau, w = tau[keep], w[keep]
    nodes = lattice_nodes(L, spacing)
    N = nodes.shape[0]
    if amplitudes == "random":
        c = rng(WL_RS, seed).uniform(-5.0, 5.0, size=N)
    else:
        c = slater_amplitude_function(nodes)
    x = collocation_grid(n, b)
    K = len(tau)
    U = []
    for l in range(3):
        d = x[:, None] - nodes[None, :, l]                     # n x N
        U.append(np.asfortranarray(np.exp(-(d[:, :, None] ** 2) * tau[None, None, :]).reshape(n, N * K)))
    xi = (c[:, None] * w[None, :]).reshape(-1)
    tag = "x".join(str(v) for v in L)
    return CanonicalInput(U, xi, eps, name=f"multi-slater-{amplitudes}-{tag}-n{n}-R{N * K}",
                          meta=dict(nodes=nodes, c=c, tau=tau, w=w, sinc=info, b=b, terms=K))
