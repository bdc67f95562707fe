"""CPU oracle for the Reduced HOSVD (RHOSVD) canonical-to-Tucker reduction.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check (__graft_entry__.smoke)
and the benchmark's cpu_baseline leg may import this package.  The product
path never calls it, and it shares no code with the GPU path (the two meet only
in the seeded input generators, which hold no arithmetic of the method).

Plain, slow, FP64.  Every step follows the paper (Khoromskaia & Khoromskij,
"Reduced Higher Order SVD: ubiquitous rank-reduction method in tensor-based
scientific computing", Section 2.1) in its own order and notation:

  normalize   canonical vectors scaled to unit norm, norms folded into xi
              (the format of eq. eqn:can_A3 assumes |u_nu^(l)| = 1)
  svd_left    SVD of each side matrix U^(l) = Z D V^T (eq. eqn:SVD_Ul), by our
              own QR-preconditioned one-sided Jacobi (jacobi_svd.c)
  truncate    epsilon-truncation to rank r_l (eq. eq:svdr; the threshold rule is
              the reading stated in truncation_threshold)
  project     V^(l) = Z0^(l)T U^(l) (= D_{l,0} V_0^(l)T, Definition 2.1 and
              Proposition 2.2)
  core        beta_0 = xi x_1 V^(1) x_2 V^(2) x_3 V^(3) (Proposition 2.2),
              i.e. beta[j1,j2,j3] = sum_nu xi_nu V1[j1,nu] V2[j2,nu] V3[j3,nu]
  error       |A - A_r| exactly (brute force, or an exact Gram identity)
  bound       Theorem 2.3: |A - A_r| <= |xi| sum_l (sum_{k>r_l} sigma_{l,k}^2)^(1/2)

Library primitives used as single steps: numpy matmul, sort.  No blocking,
fusion or reordering beyond what each formula states.

Parity is pinned (tests/test_oracle_pins.py) against closed forms, exactly
low-rank inputs, brute force on small grids, the textbook truncated HOSVD in
a special case, invariances and Theorem 2.3.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi_svd.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_svd.so")
_lib = None

D = 3   # tensor order handled here


def build(force: bool = True) -> str:
    """Compile the oracle's C part (plain gcc -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_svd_left.restype = ctypes.c_int
        lib.orc_svd_left.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int)]
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ---------------------------------------------------------------------------
# a1: normalization
# ---------------------------------------------------------------------------
def column_norms(U: np.ndarray) -> np.ndarray:
    """Euclidean norm of every column, computed scaled (max-abs first) so that
    neither tiny nor huge entries under/overflow when squared."""
    M = np.max(np.abs(U), axis=0)
    safe = np.where(M > 0, M, 1.0)
    return np.where(M > 0, M * np.sqrt(np.sum((U / safe) ** 2, axis=0)), 0.0)


def normalize(U: list, xi: np.ndarray):
    """Bring the input to the normalized canonical form of eq. eqn:can_A3:
    u~_nu^(l) = u_nu^(l) / s_{l,nu}, xi'_nu = xi_nu * prod_l s_{l,nu}.

    A term with xi_nu = 0 or any zero column contributes nothing to A and is
    dropped: its normalized columns and xi' are set to zero.
    Returns (Ut list of (n,R) arrays, xip (R,), keep mask (R,), scales (3,R)).
    """
    s = np.stack([column_norms(u) for u in U])          # (3, R)
    keep = (xi != 0) & np.all(s > 0, axis=0)
    xip = np.where(keep, xi * s[0] * s[1] * s[2], 0.0)
    Ut = []
    for l in range(D):
        safe = np.where(keep, s[l], 1.0)
        Ut.append(np.asfortranarray(np.where(keep[None, :], U[l] / safe[None, :], 0.0)))
    return Ut, xip, keep, s


# ---------------------------------------------------------------------------
# a2/a3: SVD of a side matrix (own one-sided Jacobi)
# ---------------------------------------------------------------------------
def svd_left(X: np.ndarray, max_sweeps: int = 60):
    """Singular values (descending) and left singular vectors of X (p x q),
    eq. eqn:SVD_Ul.  Returns (sigma (m,), Z (p, m), sweeps), m = min(p, q)."""
    lib = _load()
    X = np.asfortranarray(X, dtype=np.float64)
    p, q = X.shape
    m = min(p, q)
    sigma = np.zeros(m)
    Z = np.zeros((p, m), order="F")
    sw = ctypes.c_int(0)
    rc = lib.orc_svd_left(p, q, X.ctypes.data, sigma.ctypes.data, Z.ctypes.data,
                          int(max_sweeps), ctypes.byref(sw))
    if rc != 0:
        raise RuntimeError(f"oracle Jacobi SVD failed (code {rc}, sweeps {sw.value})")
    return sigma, Z, int(sw.value)


# ---------------------------------------------------------------------------
# |A|_F, exactly
# ---------------------------------------------------------------------------
def full_tensor(Ut: list, xip: np.ndarray) -> np.ndarray:
    """Materialize A = sum_nu xi'_nu u1 (x) u2 (x) u3 (n^3 entries; small n only)."""
    n = Ut[0].shape[0]
    A = np.zeros((n, n, n))
    for nu in np.nonzero(xip)[0]:
        A += xip[nu] * np.einsum("i,j,k->ijk", Ut[0][:, nu], Ut[1][:, nu], Ut[2][:, nu])
    return A


def full_tensor_slabs(Ut: list, xip: np.ndarray) -> np.ndarray:
    """The same A, one k-slab at a time: A[:, :, k] = U~1 diag(xi' * U~3[k, :]) U~2^T
    (Fortran order; any n the memory allows)."""
    n = Ut[0].shape[0]
    A = np.empty((n, n, n), order="F")
    for k in range(n):
        A[:, :, k] = (Ut[0] * (xip * Ut[2][k])) @ Ut[1].T
    return A


def anorm_gram(Ut: list, xip: np.ndarray) -> float:
    """|A|_F^2 = sum_{nu,mu} xi'_nu xi'_mu prod_l <u~_nu^(l), u~_mu^(l)>
    = xi'^T (G1 o G2 o G3) xi', with G_l = U~^(l)T U~^(l) (R x R): the inner
    product of two canonical sums, expanded term by term."""
    H = np.ones((len(xip), len(xip)))
    for l in range(D):
        H *= Ut[l].T @ Ut[l]
    val = float(xip @ H @ xip)
    return math.sqrt(max(val, 0.0))


def anorm_hadamard(factors) -> float:
    """|A|_F of the pointwise (Hadamard) product A = B o C of two canonical
    tensors (Section 4.3, Lemma 4.3), by definition: B and C are formed slab by slab on the
    grid, B[:, :, k] = U_a0 diag(x_a * U_a2[k, :]) U_a1^T, and the squares of
    B o C summed.  factors = ((U_a, x_a), (U_b, x_b)) with U_* three n x R_* arrays."""
    (Ua, xa), (Ub, xb) = factors
    n = Ua[0].shape[0]
    s = 0.0
    for k in range(n):
        Bk = (Ua[0] * (xa * Ua[2][k])) @ Ua[1].T
        Ck = (Ub[0] * (xb * Ub[2][k])) @ Ub[1].T
        s += float(np.sum((Bk * Ck) ** 2))
    return float(np.sqrt(s))


def hadamard_full(factors) -> np.ndarray:
    """The pointwise product A = B o C of two canonical tensors materialized on
    the n^3 grid (Section 4.3): slab k is B[:, :, k] * C[:, :, k], each slab of
    a canonical tensor formed as U_0 diag(x * U_2[k, :]) U_1^T."""
    (Ua, xa), (Ub, xb) = factors
    n = Ua[0].shape[0]
    A = np.empty((n, n, n), order="F")
    for k in range(n):
        A[:, :, k] = ((Ua[0] * (xa * Ua[2][k])) @ Ua[1].T) * ((Ub[0] * (xb * Ub[2][k])) @ Ub[1].T)
    return A


def anorm(Ut: list, xip: np.ndarray, brute_max_n: int = 64) -> float:
    n = Ut[0].shape[0]
    if n <= brute_max_n:
        return float(np.linalg.norm(full_tensor(Ut, xip).ravel()))
    return anorm_gram(Ut, xip)


# ---------------------------------------------------------------------------
# a4: truncation
# ---------------------------------------------------------------------------
def tails(sigma: np.ndarray) -> np.ndarray:
    """t_r = (sum_{k>r} sigma_k^2)^(1/2) for r = 0..m, summed from the smallest
    sigma upwards (the tail sums of Theorem 2.3, eq. error bound CtoT)."""
    sq = sigma[::-1] ** 2
    acc = np.concatenate([[0.0], np.cumsum(sq)])[::-1]   # acc[r] = sum_{k>=r} (0-based)
    return np.sqrt(acc)


def truncation_threshold(eps: float, a_norm: float, xi_norm: float) -> float:
    """tau = eps |A| / (d |xi'|).

    The paper controls accuracy by an epsilon threshold on the truncated SVDs
    (Section 2.1, after Proposition 2.2) without fixing the rule.  With this tau
    and every mode truncated so that its tail t_{l,r_l} <= tau, Theorem 2.3
    gives |A - A_r| <= |xi'| sum_l t_{l,r_l} <= eps |A|: a relative Frobenius
    guarantee.
    """
    if xi_norm == 0.0:
        return 0.0
    return eps * a_norm / (D * xi_norm)


def choose_rank(t: np.ndarray, tau: float) -> int:
    """r = min{ r >= 1 : t_r <= tau } (non-strict at a tie)."""
    m = len(t) - 1
    for r in range(1, m + 1):
        if t[r] <= tau:
            return r
    return m


def sign_normalize(Z: np.ndarray) -> np.ndarray:
    """Fix each singular vector's sign: its largest-magnitude entry is positive
    (ties: the lowest index)."""
    Z = Z.copy()
    for k in range(Z.shape[1]):
        i = int(np.argmax(np.abs(Z[:, k])))
        if Z[i, k] < 0:
            Z[:, k] = -Z[:, k]
    return Z


# ---------------------------------------------------------------------------
# a6/a7: projection and core
# ---------------------------------------------------------------------------
def project(Z: np.ndarray, Ut: np.ndarray) -> np.ndarray:
    """V^(l) = Z0^(l)T U~^(l) (r_l x R): the side matrices projected onto the
    kept left singular vectors (Definition 2.1; equal to D_{l,0} V_0^(l)T)."""
    return Z.T @ Ut


def core(V: list, xip: np.ndarray) -> np.ndarray:
    """beta[j1,j2,j3] = sum_nu xi'_nu V1[j1,nu] V2[j2,nu] V3[j3,nu]
    (Proposition 2.2), one j3-slab at a time:
    beta[:,:,j3] = V1 diag(xi' * V3[j3,:]) V2^T."""
    V1, V2, V3 = V
    r1, r2, r3 = V1.shape[0], V2.shape[0], V3.shape[0]
    beta = np.zeros((r1, r2, r3), order="F")
    for j3 in range(r3):
        w = xip * V3[j3, :]
        beta[:, :, j3] = (V1 * w[None, :]) @ V2.T
    return beta


def reconstruct(beta: np.ndarray, Z: list) -> np.ndarray:
    """A_r = beta x_1 Z1 x_2 Z2 x_3 Z3 (materialized, n^3 entries), one mode
    product at a time: c with Z3, then a with Z1, then b with Z2.  Returned as
    an (i, j, k) view of a (k, j, i) array (Fortran order, like hadamard_full)."""
    T = np.tensordot(Z[2], beta, axes=([1], [2]))          # (k, a, b)
    T = np.tensordot(T, Z[1], axes=([2], [1]))             # (k, a, j)
    T = np.tensordot(T, Z[0], axes=([1], [1]))             # (k, j, i)
    return T.transpose(2, 1, 0)


# ---------------------------------------------------------------------------
# exact error of the reduction and the Theorem 2.3 bound
# ---------------------------------------------------------------------------
def error_brute(Ut: list, xip: np.ndarray, beta: np.ndarray, Z: list) -> float:
    return float(np.linalg.norm((full_tensor(Ut, xip) - reconstruct(beta, Z)).ravel()))


def error_dense(A: np.ndarray, beta: np.ndarray, Z: list) -> float:
    """|A - beta x_1 Z1 x_2 Z2 x_3 Z3|_F against a materialized A (any n the
    memory allows; A - A_r formed entry by entry)."""
    return float(np.linalg.norm((A - reconstruct(beta, Z)).ravel(order="K")))


def error_gram(Ut: list, xip: np.ndarray, Z: list) -> float:
    """|A - A_r|_F from Gram matrices, without forming A.

    A - A_r = sum_nu xi'_nu [u1 u2 u3 - P1u1 P2u2 P3u3] splits into three
    mutually orthogonal parts (I-P1)u1 u2 u3, P1u1 (I-P2)u2 u3,
    P1u1 P2u2 (I-P3)u3 (P_l = Z_l Z_l^T), so
    err^2 = xi'^T (E1 o G2 o G3 + H1 o E2 o G3 + H1 o H2 o E3) xi'
    with G_l = U~^T U~, H_l = (Z^T U~)^T (Z^T U~), E_l = G_l - ... computed
    directly as Delta_l^T Delta_l, Delta_l = U~ - Z_l Z_l^T U~ (every term is a
    Schur product of PSD matrices, so nothing cancels)."""
    G, H, E = [], [], []
    for l in range(D):
        Vl = Z[l].T @ Ut[l]
        Dl = Ut[l] - Z[l] @ Vl
        G.append(Ut[l].T @ Ut[l])
        H.append(Vl.T @ Vl)
        E.append(Dl.T @ Dl)
    M = E[0] * G[1] * G[2] + H[0] * E[1] * G[2] + H[0] * H[1] * E[2]
    return math.sqrt(max(float(xip @ M @ xip), 0.0))


def theorem23_bound(xi_norm: float, tail_at_rank: list) -> float:
    """Theorem 2.3: |A - A_r| <= |xi'| sum_l (sum_{k>r_l} sigma_{l,k}^2)^(1/2)."""
    return xi_norm * float(sum(tail_at_rank))


def certificate(Ut: list, xip: np.ndarray, Z: list) -> float:
    """The bound reached inside the proof of Theorem 2.3 (Section 2.1) before its
    final Cauchy-Schwarz step:
        |A - A_r| <= sum_l sum_nu |xi'_nu| |(I - Z_l Z_l^T) u~_nu^(l)|,
    each residual column formed directly (not from 1 - |Z^T u~|^2).  It is at
    most |xi'| sum_l t_{l, r_l} and, like that bound, holds for any orthonormal
    Z_l (the proof uses only |u~_nu| = 1 and |Z_l Z_l^T u~_nu| <= 1)."""
    c = 0.0
    for l in range(D):
        Dl = Ut[l] - Z[l] @ (Z[l].T @ Ut[l])
        c += float(np.abs(xip) @ np.sqrt(np.sum(Dl * Dl, axis=0)))
    return c


# ---------------------------------------------------------------------------
# the whole reduction
# ---------------------------------------------------------------------------
@dataclass
class OracleResult:
    ranks: tuple
    sigma: list        # full singular value lists, one per mode (descending)
    Z: list            # kept left singular vectors, n x r_l, sign-normalized
    V: list            # projected side matrices r_l x R
    beta: np.ndarray   # r1 x r2 x r3 (Fortran order)
    xip: np.ndarray
    xi_norm: float
    a_norm: float
    tau: float
    tails: list        # tail arrays t_0..t_m per mode
    bound: float
    sweeps: list


def rhosvd(U: list, xi: np.ndarray, eps: float, a_norm: float | None = None,
           with_core: bool = True, max_sweeps: int = 60) -> OracleResult:
    """Reduced HOSVD of a d=3 canonical tensor (Definition 2.1)."""
    Ut, xip, keep, _ = normalize(U, xi)
    xi_norm = float(np.linalg.norm(xip))
    n = Ut[0].shape[0]
    if xi_norm == 0.0:
        z = [np.zeros((n, 0)) for _ in range(D)]
        return OracleResult((0, 0, 0), [np.zeros(0)] * 3, z, [np.zeros((0, len(xi)))] * 3,
                            np.zeros((0, 0, 0)), xip, 0.0, 0.0, 0.0, [np.zeros(1)] * 3, 0.0,
                            [0, 0, 0])
    if a_norm is None:
        a_norm = anorm(Ut, xip)
    tau = truncation_threshold(eps, a_norm, xi_norm)
    sig, Zs, ts, ranks, sweeps = [], [], [], [], []
    for l in range(D):
        s, Zf, sw = svd_left(Ut[l], max_sweeps=max_sweeps)
        t = tails(s)
        r = choose_rank(t, tau)
        sig.append(s)
        ts.append(t)
        ranks.append(r)
        sweeps.append(sw)
        Zs.append(sign_normalize(Zf[:, :r]))
    V = [project(Zs[l], Ut[l]) for l in range(D)]
    beta = core(V, xip) if with_core else None
    bound = theorem23_bound(xi_norm, [ts[l][ranks[l]] for l in range(D)])
    return OracleResult(tuple(ranks), sig, Zs, V, beta, xip, xi_norm, a_norm, tau, ts,
                        bound, sweeps)
