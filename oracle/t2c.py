"""Oracle of the Tucker-to-canonical (T2C) transform of a 3rd-order core.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): tests/, the smoke check and
the benchmark's cpu_baseline leg may use it; the product path never does.

Follows Remark 2.6 of Section 2.3 (Khoromskaia & Khoromskij): the core beta
(r1 x r2 x r3) is written as a sum of its matrix slices in one fixed mode,
beta = sum_m B_m (x) e_m (eq. T2C_slice, here the third mode: B_m =
beta[:, :, m], r1 x r2), each slice is truncated by its SVD (eq. T2C_SVD),
keeping the p_m singular values above a threshold, and the kept rank-one terms
of all slices form the canonical tensor beta_(R) (eq. beta_R), of rank
R = p_1 + ... + p_r3 <= r3 min(r1, r2).

Threshold (the remark states it for a cube r x r x r as eps / r^(3/2), with the
error estimate |beta - beta_(R)| <= sum_m |B_m - B_{p_m}| <= eps): for a general
core each of the r3 slices has min(r1, r2) singular values, and the same
argument gives |beta - beta_(R)| <= eps with the threshold
thr = eps / (r3 sqrt(min(r1, r2))), which is eps / r^(3/2) for a cube.
p_m = #{k : sigma_k^(m) > thr} (the singular values at or below thr are
dropped; p_m = 0 drops the whole slice).  eps is absolute, as in the remark.

Plain FP64.  The slice SVDs use the oracle's own one-sided Jacobi (svd_left);
the right factors are v_k = B_m^T u_k / sigma_k.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class T2CResult:
    weights: np.ndarray   # (R,) sigma_k^(m) of the kept terms, slice by slice, descending within a slice
    U: np.ndarray         # (r1, R) left factors u_k (unit)
    V: np.ndarray         # (r2, R) right factors v_k (unit)
    slice: np.ndarray     # (R,) slice index m of each term (the third factor is e_m)
    p: np.ndarray         # (r3,) kept terms per slice
    sigma: list           # per slice, all min(r1, r2) singular values (descending)
    tails: np.ndarray     # (r3,) |B_m - B_{p_m}|_F = (sum_{k > p_m} sigma_k^2)^(1/2)
    threshold: float
    bound: float          # sum_m tails[m] (Remark 2.6), <= eps


def t2c_threshold(eps: float, r1: int, r2: int, r3: int) -> float:
    """eps / (r3 sqrt(min(r1, r2))): eps / r^(3/2) for an r x r x r core."""
    return eps / (r3 * math.sqrt(min(r1, r2)))


def t2c(beta: np.ndarray, eps: float) -> T2CResult:
    """Remark 2.6: slice-wise SVD truncation of the core in its third mode."""
    from . import svd_left
    r1, r2, r3 = beta.shape
    thr = t2c_threshold(eps, r1, r2, r3)
    w, Us, Vs, sl, p, sig, tails = [], [], [], [], [], [], []
    for m in range(r3):
        B = np.asarray(beta[:, :, m], dtype=np.float64)
        s, Ul, _ = svd_left(B)                      # B = sum_k s_k u_k v_k^T
        pm = int(np.sum(s > thr))
        p.append(pm)
        sig.append(s)
        tails.append(math.sqrt(float(np.sum(s[pm:] ** 2))))
        for k in range(pm):
            u = Ul[:, k]
            v = (B.T @ u) / s[k]
            w.append(s[k])
            Us.append(u)
            Vs.append(v)
            sl.append(m)
    R = len(w)
    U = np.array(Us).T if R else np.zeros((r1, 0))
    V = np.array(Vs).T if R else np.zeros((r2, 0))
    tails = np.array(tails)
    return T2CResult(np.array(w), U.reshape(r1, R), V.reshape(r2, R), np.array(sl, dtype=np.int64),
                     np.array(p, dtype=np.int64), sig, tails, thr, float(np.sum(tails)))


def canonical_core(res: T2CResult, r3: int) -> np.ndarray:
    """beta_(R) = sum_k w_k u_k (x) v_k (x) e_{slice_k} as a dense r1 x r2 x r3 array."""
    r1, r2 = res.U.shape[0], res.V.shape[0]
    out = np.zeros((r1, r2, r3), order="F")
    for k in range(len(res.weights)):
        out[:, :, res.slice[k]] += res.weights[k] * np.outer(res.U[:, k], res.V[:, k])
    return out


def lift(res: T2CResult, Z: list):
    """The canonical tensor in the full space: A_(R) = sum_k w_k (Z1 u_k) (x)
    (Z2 v_k) (x) z3_{slice_k} (Z_l orthonormal, so the error is the core's).
    Returns (weights, C1 n x R, C2 n x R, C3 n x R)."""
    return res.weights, Z[0] @ res.U, Z[1] @ res.V, Z[2][:, res.slice]
