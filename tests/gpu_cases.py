"""Helpers for the GPU parity tests: run the HIP path through the C-ABI on a
seeded input and compare with the oracle to the tolerances derived from the
arithmetic (see the comparison functions)."""
from __future__ import annotations

import math

import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24
ETA64 = 2.0 ** -52     # relative error of the FP64 Gram matrix (a few ulps)


def eig_tol(n, R):
    """Bound on |sigma_gpu^2 - sigma^2| / sigma_1^2 for the Gram route: the FP64
    Gram's rounding (~sqrt(K) u per entry relative to |G|, K = max(n, R) the
    contraction length) plus a backward-stable eigensolver's error (~m u |G|,
    m the padded Gram size), with a safety factor of 16."""
    K = max(n, R)
    m = -(-min(n, R) // 64) * 64
    return 16.0 * (math.sqrt(K) + m) * U64


def run_gpu(ci, precision="fp64", want_beta=True, profile=False, **kw):
    import torch
    from paper_2201_12663_amd import rhosvd
    U = [rhosvd.to_device(u) for u in ci.U]
    xi = torch.from_numpy(np.ascontiguousarray(ci.xi)).cuda()
    red = rhosvd.Reducer(precision=precision, profile=profile, **kw)
    ranks = red.reduce(U[0], U[1], U[2], xi, ci.eps)
    res = red.get(beta=want_beta)
    spectra = [red.spectrum(l) for l in range(3)]
    Vs = [red.V(l) for l in range(3)]
    xip = red.xi_prime()
    torch.cuda.synchronize()
    out = dict(
        ranks=tuple(ranks),
        Z=[z.cpu().numpy() for z in res.Z],
        beta=None if res.beta is None else res.beta.cpu().numpy(),
        sigma=res.sigma.cpu().numpy(),
        spectra=[s.cpu().numpy() for s in spectra],
        V=[v.cpu().numpy() for v in Vs],
        xip=xip.cpu().numpy(),
        report=res.report,
        phases=red.phase_ms() if profile else None,
    )
    red.close()
    return out


def cut_margin_ok(tails, rank, tau, sigma1, eta=ETA64):
    """Rank-parity rule: ranks must agree when the cut's margin in the tail sums
    exceeds 10x the path's tail error e_t ~ eta * sigma1^2 / (2 tau)."""
    if tau <= 0:
        return False
    e_t = eta * sigma1 ** 2 / (2.0 * tau)
    lo = tails[rank - 1] - tau if rank >= 1 else math.inf
    hi = tau - tails[rank]
    return min(lo, hi) > 10.0 * e_t


def tails_of(sigma):
    """t_r = (sum_{k >= r} sigma_k^2)^(1/2), r = 0..m, summed smallest first."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    return np.sqrt(np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]]))


def cut_margin_ok_measured(t_path, t_orc, rank, tau, factor=10.0):
    """Rank-parity rule with the path's tail error measured instead of modelled:
    the path's tails t_path (from its own spectrum) differ from the oracle's by
    d = max |t_path - t_orc| at r - 1 and r; ranks must agree when the oracle's
    cut margin exceeds factor * d.  (For Gram matrices of order ~2000 the
    eigensolver's own backward error, tens of u |G|, exceeds the 2^-52 |G| of
    the modelled rule.)"""
    if tau <= 0 or rank < 1:
        return False
    d = max(abs(t_path[rank - 1] - t_orc[rank - 1]), abs(t_path[rank] - t_orc[rank]))
    margin = min(t_orc[rank - 1] - tau, tau - t_orc[rank])
    return margin > factor * d


def separated(sigma, r, rel_gap=1e-4):
    s2 = sigma ** 2
    out = []
    for k in range(r):
        lo = s2[k - 1] - s2[k] if k > 0 else np.inf
        hi = s2[k] - s2[k + 1] if k + 1 < len(s2) else np.inf
        if min(lo, hi) > rel_gap * s2[0]:
            out.append(k)
    return out


def align_signs(Zg, Zo):
    """Sign of each GPU column relative to the oracle's (both follow the same
    sign rule, so this is +1 except at ties of the largest entry)."""
    return np.sign(np.sum(Zg * Zo, axis=0) + 1e-300)


def check_anorm(rep, a_exact, tau_exact):
    """|A| as the path used it: the exact identity (equal to the oracle's to 1e-11),
    or the probe's certified bracket a_norm <= |A| <= a_norm_upper, which puts the
    path's tau at or below the oracle's.  Returns the tau the path cut with."""
    if rep["anorm_method"] == 1:
        assert abs(rep["a_norm"] - a_exact) <= 1e-11 * a_exact
        assert abs(rep["tau"] - tau_exact) <= 1e-11 * tau_exact
    else:
        assert rep["anorm_method"] == 2
        assert rep["a_norm"] <= a_exact * (1 + 1e-12), (rep["a_norm"], a_exact)
        assert a_exact <= rep["a_norm_upper"] * (1 + 1e-12), (a_exact, rep["a_norm_upper"])
        assert rep["tau"] <= tau_exact * (1 + 1e-12)
    return rep["tau"]


def compare_fp64(g, o, ci, check_beta=True):
    """GPU FP64 result g (run_gpu) vs oracle result o (oracle.rhosvd).  Ranks are
    compared with the oracle's cut at the tau the path used (the same as the
    oracle's with the exact |A|; at most it with the probe's lower bound)."""
    import oracle as orc
    # xi' elementwise
    assert np.allclose(g["xip"], o.xip, rtol=1e-13, atol=0.0)
    # norms
    rep = g["report"]
    assert abs(rep["xi_norm"] - o.xi_norm) <= 1e-13 * o.xi_norm
    tau = check_anorm(rep, o.a_norm, o.tau)
    o_ranks = tuple(orc.choose_rank(o.tails[l], tau) for l in range(3))
    if o_ranks != tuple(o.ranks):
        o = orc.rhosvd(ci.U, ci.xi, ci.eps, a_norm=o.a_norm * tau / o.tau)
    for l in range(3):
        s1 = o.sigma[l][0]
        m = len(o.sigma[l])
        sg = g["spectra"][l]
        assert sg.shape == (m,)
        # eigenvalues of the FP64 Gram: absolute accuracy a few ulps of |G|
        d2 = np.abs(sg ** 2 - o.sigma[l] ** 2)
        assert np.all(d2 <= eig_tol(ci.n, ci.R) * s1 ** 2), (l, d2.max() / s1 ** 2)
        # ranks: equal unless the cut is a knife edge for FP64
        if cut_margin_ok(o.tails[l], o.ranks[l], o.tau, s1):
            assert g["ranks"][l] == o.ranks[l], (l, g["ranks"], o.ranks)
        r = g["ranks"][l]
        Z = g["Z"][l]
        assert Z.shape == (ci.n, r)
        assert np.max(np.abs(Z.T @ Z - np.eye(r))) <= 10 * m * U64 * 10
        rside = ci.R < ci.n
        if rside:
            # R < n: Z = U~ W Lambda^-1/2 re-orthonormalized, so Z spans the kept left
            # singular subspace but is only defined up to a rotation inside it:
            # compare projectors (Davis-Kahan: angle <~ eta sigma1^2 / gap at the cut)
            if g["ranks"][l] == o.ranks[l] and r < m:
                gap = o.sigma[l][r - 1] ** 2 - o.sigma[l][r] ** 2
                if gap > 0:
                    dk = 10 * eig_tol(ci.n, ci.R) * s1 ** 2 / gap
                    if dk < 0.1:
                        Po = o.Z[l] @ o.Z[l].T
                        assert np.linalg.norm(Z @ Z.T - Po, 2) <= dk, (l, dk)
            continue
        # V V^T = diag(sigma^2) (projection identity)
        V = g["V"][l]
        assert np.allclose(V @ V.T, np.diag(sg[:r] ** 2), atol=1e-12 * s1 ** 2)
        # well-separated singular vectors agree
        if g["ranks"][l] == o.ranks[l]:
            sep = separated(o.sigma[l], r)
            if sep:
                sgn = align_signs(Z[:, sep], o.Z[l][:, sep])
                assert np.allclose(Z[:, sep] * sgn, o.Z[l][:, sep], atol=1e-9)
    if check_beta and ci.R >= ci.n and g["beta"] is not None and g["ranks"] == tuple(o.ranks):
        seps = [separated(o.sigma[l], o.ranks[l]) for l in range(3)]
        if all(len(s) for s in seps):
            sg = [align_signs(g["Z"][l][:, seps[l]], o.Z[l][:, seps[l]]) for l in range(3)]
            bg = g["beta"][np.ix_(*seps)] * sg[0][:, None, None] * sg[1][None, :, None] * sg[2][None, None, :]
            bo = o.beta[np.ix_(*seps)]
            assert np.max(np.abs(bg - bo)) <= 1e-9 * o.xi_norm, np.max(np.abs(bg - bo))


def recon_error(orc, ci, Z, beta=None):
    """|A - A_r| for the GPU's Z (and optionally its beta): brute force for small
    n, else the Gram identity plus |beta - beta_exact| (orthogonal parts)."""
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    if ci.n <= 64 and beta is not None:
        A = orc.full_tensor(Ut, xip)
        return float(np.linalg.norm((A - orc.reconstruct(beta, Z)).ravel()))
    return orc.error_gram(Ut, xip, Z)


def pad64(x):
    return -(-int(x) // 64) * 64


def v_abs_error(n):
    """Bound on the absolute error of one entry of the FP64 projection
    V[j, nu] = z_j . u~_nu of unit vectors: the FP64 MFMA (16x16x4) accumulates
    the n_pad products in n_pad/4 rounded steps, each partial sum at most
    sum_i |z_i||u_i| <= 1 (Cauchy-Schwarz); doubled for safety."""
    return 2.0 * (pad64(n) / 4 + 16) * U64


def core_rel_const(prec, R, beta_fp32=False):
    """c_p: |beta_gpu[j] - beta_exact[j]| <= c_p * S_j per entry, where
    S_j = sum_nu |xi'_nu| |V1[j1,nu]| |V2[j2,nu]| |V3[j3,nu]| and the V are the
    exact projections (their own error is added separately).  Per product:
    FP64: two roundings (xi' V1 and V2 V3); FP32: the three V and xi' rounded to
    float and the two products (6 u32); BF16x3: those plus the split (bf16 keeps
    8 significant bits, so hi = bf16(a) is within 2^-8 |a| and lo = bf16(a - hi)
    leaves |a - hi - lo| <= 2^-16 |a| for each operand, and the dropped lo*lo is
    <= 2^-16 |ab|: 3 * 2^-16 in all).  Then one rounding per accumulation step:
    R_pad/4 MFMA steps (16x16x4 FP64 / FP32), 3 R_pad / 32 for BF16x3 (three
    16x16x32 products per 32 terms).  A float beta adds its final rounding."""
    Rp = pad64(R)
    if prec == "fp64":
        c = (Rp / 4 + 8) * U64
    elif prec == "fp32":
        c = (Rp / 4 + 12) * U32
    else:
        c = 3 * 2.0 ** -16 + (3 * Rp / 32 + 12) * U32
    return c + (U32 if beta_fp32 else 0.0)


def check_core_slabs(orc, Ut, xip, Z, beta, j3s, prec, beta_fp32=False, what="", beta_is_slabs=False):
    """Element-by-element check of the core on the j3-slabs j3s (Proposition 2.2):
    the oracle forms V = Z^T U~ from its own normalized side matrices and the
    returned (orthonormal) Z, and beta[:, :, j3] = V1 diag(xi' V3[j3, :]) V2^T.
    Each entry must lie within c_p S_j + (S^d_j - S_j) of it, S^d the same sum
    with every |V| raised by the projection's error bound d (v_abs_error).
    With beta_is_slabs, beta holds only the slabs j3s (sorted, no repeats).
    Returns the largest ratio |error| / tolerance over the slabs."""
    n = Ut[0].shape[0]
    R = Ut[0].shape[1]
    V = [orc.project(Z[l], Ut[l]) for l in range(3)]
    d = v_abs_error(n)
    j3s = sorted(set(int(j) for j in j3s))
    ref = orc.core([V[0], V[1], V[2][j3s, :]], xip)
    aV = [np.abs(v) for v in V]
    ax = np.abs(xip)
    S = orc.core([aV[0], aV[1], aV[2][j3s, :]], ax)
    Sd = orc.core([aV[0] + d, aV[1] + d, aV[2][j3s, :] + d], ax)
    tol = core_rel_const(prec, R, beta_fp32) * S + (Sd - S) + 1e-300
    got = np.asarray(beta if beta_is_slabs else beta[:, :, j3s], dtype=np.float64)
    err = np.abs(got - ref)
    worst = float(np.max(err / tol))
    assert worst <= 1.0, (what, prec, "slab", j3s[int(np.argmax(np.max(err / tol, axis=(0, 1))))], worst)
    return worst


def boundary_slabs(r3, extra=()):
    """j3 slabs at the core's tile edges (16-wide j2/j3 tiles, 64/128-row j1
    tiles), the first and the ragged last slab, and any extra ones."""
    js = {0, r3 - 1, min(15, r3 - 1), min(16, r3 - 1), r3 // 2}
    for j in extra:
        if 0 <= j < r3:
            js.add(int(j))
    return sorted(js)
