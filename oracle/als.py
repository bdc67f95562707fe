"""Oracle of the canonical-to-Tucker ALS refinement started from the RHOSVD.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Section 2.1 after Definition 2.1 (Khoromskaia & Khoromskij): the RHOSVD
subspaces are the initial guess of the alternating least-squares iteration for
the best rank-(r1, r2, r3) Tucker approximation, and one step for a mode
contracts the canonical tensor with the current orthogonal factors of the other
two modes (eq. eqn:can_A_Tuck_als: A_2 = xi x_1 V^(1)T x_3 V^(3)T for the second
mode) and takes the best rank-r_l approximation of the resulting n x (r r')
unfolding: its r_l dominant left singular vectors become the new Z^(l).  A sweep
updates the modes in the order 1, 2, 3, each with the others' latest factors
(reading: the paper describes the step for one mode only).  The ranks stay
those of the RHOSVD.

In the canonical format the contracted unfolding is explicit:
    M_l = U~_l diag(xi') (V_b (.) V_a)^T   (n x r_a r_b), V_a = Z_a^T U~_a,
formed here column by column (the Khatri-Rao product), then decomposed by the
oracle's own Jacobi SVD.  Sign rule as for the RHOSVD.
"""
from __future__ import annotations

import numpy as np


def contracted_unfolding(Ut_l: np.ndarray, xip: np.ndarray, Va: np.ndarray, Vb: np.ndarray) -> np.ndarray:
    """M = U~_l diag(xi') (V_b (.) V_a)^T: column (ja + ra jb) is
    sum_nu xi'_nu Va[ja, nu] Vb[jb, nu] u~_nu."""
    ra, rb = Va.shape[0], Vb.shape[0]
    KR = (Va[:, None, :] * Vb[None, :, :]).reshape(ra * rb, -1, order="F")   # row ja + ra jb
    return (Ut_l * xip[None, :]) @ KR.T


def als_sweeps(Ut: list, xip: np.ndarray, Z: list, sweeps: int):
    """Sweeps of the ALS iteration from the factors Z (n x r_l each).  Returns
    (Z, V, history) with history the core norms |beta| after every mode update."""
    from . import core, project, sign_normalize, svd_left
    Z = [z.copy() for z in Z]
    V = [project(Z[l], Ut[l]) for l in range(3)]
    hist = [float(np.linalg.norm(core(V, xip).ravel()))]
    for _ in range(sweeps):
        for l in range(3):
            a, b = [k for k in range(3) if k != l]
            M = contracted_unfolding(Ut[l], xip, V[a], V[b])
            _, Zf, _ = svd_left(M)
            Z[l] = sign_normalize(Zf[:, :Z[l].shape[1]])
            V[l] = project(Z[l], Ut[l])
            hist.append(float(np.linalg.norm(core(V, xip).ravel())))
    return Z, V, hist
