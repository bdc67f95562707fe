"""Pins of the Tucker-to-canonical oracle (oracle/t2c.py, Remark 2.6), on the
CPU: closed-form slice spectra, LAPACK's singular values, the remark's error
estimate, the rank bound, brute force through the whole canonical-to-canonical
chain on a small grid, and planted mistakes that each fail a pin."""
import math

import numpy as np
import pytest

from paper_2201_12663_amd import inputs

WL = 12   # seeded stream of these tests


def _orth(g, n, k):
    Q, _ = np.linalg.qr(g.standard_normal((n, k)))
    return Q


@pytest.fixture(scope="module")
def t2c():
    from oracle import t2c as mod
    return mod


def known_slices(r1, r2, r3, eps, seed=0):
    """Core whose slice m is Q diag(s_m) P^T with q_m values far above the
    threshold (1 ... 1e-3) and the rest far below it (thr / 10 ... thr / 100)."""
    g = inputs.rng(WL, seed)
    thr = eps / (r3 * math.sqrt(min(r1, r2)))
    k = min(r1, r2)
    beta = np.zeros((r1, r2, r3), order="F")
    q = []
    spectra = []
    for m in range(r3):
        qm = int(g.integers(0, k + 1))
        s = np.concatenate([np.geomspace(1.0, 1e-3, qm), np.geomspace(thr / 10, thr / 100, k - qm)])
        beta[:, :, m] = _orth(g, r1, k) @ np.diag(s) @ _orth(g, r2, k).T
        q.append(qm)
        spectra.append(s)
    return beta, np.array(q), spectra


def pin_known_slice_ranks(t2c):
    for shape in [(9, 9, 9), (12, 7, 5), (6, 11, 8)]:
        eps = 1e-4
        beta, q, spectra = known_slices(*shape, eps, seed=sum(shape))
        res = t2c.t2c(beta, eps)
        assert np.array_equal(res.p, q), (res.p, q)
        for m in range(shape[2]):
            assert np.allclose(res.sigma[m], spectra[m], rtol=1e-10, atol=1e-14)
            assert abs(res.tails[m] - math.sqrt(np.sum(spectra[m][q[m]:] ** 2))) <= 1e-12
        # kept slices reproduce the above-threshold part of each slice
        approx = t2c.canonical_core(res, shape[2])
        assert np.linalg.norm((beta - approx).ravel()) <= res.bound * (1 + 1e-9) + 1e-13
        assert res.bound <= eps


def pin_threshold_closed_form(t2c):
    """r x r x r: the remark's eps / r^(3/2); a slice whose r singular values all
    sit just above eps / r^(3/2) keeps them all, one just below drops them all,
    and the error estimate sum_m |B_m - B_pm| <= eps then holds with equality
    up to the factor (1 - 1e-9)."""
    r = 6
    eps = 1e-3
    assert t2c.t2c_threshold(eps, r, r, r) == pytest.approx(eps / r ** 1.5, rel=1e-15)
    g = inputs.rng(WL, 7)
    for scale, kept in ((1 + 1e-9, r), (1 - 1e-9, 0)):
        beta = np.zeros((r, r, r), order="F")
        for m in range(r):
            beta[:, :, m] = _orth(g, r, r) @ np.diag(np.full(r, scale * eps / r ** 1.5)) @ _orth(g, r, r).T
        res = t2c.t2c(beta, eps)
        assert np.all(res.p == kept), (res.p, kept)
        if kept == 0:
            err = np.linalg.norm(beta.ravel())
            # every slice has norm sqrt(r) * thr: the sum of the r slice norms is eps (1 - 1e-9)
            assert res.bound == pytest.approx(eps * (1 - 1e-9), rel=1e-9)
            assert err <= res.bound <= eps


def pin_sigma_vs_lapack(t2c):
    g = inputs.rng(WL, 3)
    for shape in [(10, 14, 4), (15, 8, 3)]:
        beta = np.asfortranarray(g.standard_normal(shape))
        res = t2c.t2c(beta, 1e-2)
        for m in range(shape[2]):
            s = np.linalg.svd(beta[:, :, m], compute_uv=False)
            assert np.allclose(res.sigma[m], s, rtol=1e-12, atol=1e-14)


def pin_error_estimate_and_rank_bound(t2c):
    """Remark 2.6: |beta - beta_(R)| <= sum_m |B_m - B_pm| <= eps and
    R = sum p_m <= r3 min(r1, r2), on random cores with decaying spectra."""
    g = inputs.rng(WL, 5)
    for shape in [(8, 8, 8), (10, 6, 9), (5, 12, 7)]:
        r1, r2, r3 = shape
        core = np.zeros(shape, order="F")
        k = min(r1, r2)
        for m in range(r3):
            core[:, :, m] = _orth(g, r1, k) @ np.diag(np.geomspace(1, 1e-8, k) * g.uniform(0.5, 2)) @ _orth(g, r2, k).T
        for eps in (1e-2, 1e-5, 1e-7):
            res = t2c.t2c(core, eps)
            err = np.linalg.norm((core - t2c.canonical_core(res, r3)).ravel())
            assert err <= res.bound * (1 + 1e-9) + 1e-14
            assert res.bound <= eps
            assert len(res.weights) == int(np.sum(res.p)) <= r3 * k
            assert np.all(res.weights > res.threshold)


def pin_c2c_brute_force(t2c):
    """The chain canonical -> Tucker (RHOSVD) -> canonical (T2C) on a 20^3 grid:
    the lifted canonical tensor is within |A - A_r| + sum_m |B_m - B_pm| of A."""
    import oracle
    ci = inputs.small_gaussian_sum(4, n=20, R=60, eps=1e-4)
    o = oracle.rhosvd(ci.U, ci.xi, ci.eps)
    Ut, xip, _, _ = oracle.normalize(ci.U, ci.xi)
    A = oracle.full_tensor(Ut, xip)
    a = float(np.linalg.norm(A.ravel()))
    Ar = oracle.reconstruct(o.beta, o.Z)
    e_tucker = float(np.linalg.norm((A - Ar).ravel()))
    eps2 = 1e-5 * a
    res = t2c.t2c(o.beta, eps2)
    w, C1, C2, C3 = t2c.lift(res, o.Z)
    AR = np.einsum("k,ik,jk,lk->ijl", w, C1, C2, C3)
    e_can = float(np.linalg.norm((A - AR).ravel()))
    assert e_can <= e_tucker + res.bound * (1 + 1e-9) + 1e-12 * a
    assert e_can <= (ci.eps + 1e-5) * a
    assert len(w) <= o.ranks[2] * min(o.ranks[0], o.ranks[1])


PINS = [pin_known_slice_ranks, pin_threshold_closed_form, pin_sigma_vs_lapack,
        pin_error_estimate_and_rank_bound, pin_c2c_brute_force]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_t2c_pin(t2c, pin):
    pin(t2c)


def _fails(mod, pins):
    for p in pins:
        try:
            p(mod)
        except (AssertionError, ValueError, IndexError):
            return True
    return False


def test_planted_threshold_eps_over_r(t2c, monkeypatch):
    """eps / r instead of eps / r^(3/2) (the sqrt(r) of the per-slice tail forgotten)"""
    monkeypatch.setattr(t2c, "t2c_threshold", lambda eps, r1, r2, r3: eps / r3)
    assert _fails(t2c, PINS)


def test_planted_threshold_eps(t2c, monkeypatch):
    monkeypatch.setattr(t2c, "t2c_threshold", lambda eps, r1, r2, r3: eps)
    assert _fails(t2c, PINS)


def test_planted_transposed_right_factor(t2c, monkeypatch):
    """v_k = B u_k / sigma_k instead of B^T u_k / sigma_k (square slices only)"""
    real = t2c.t2c

    def bad(beta, eps):
        res = real(beta, eps)
        for k in range(len(res.weights)):
            B = beta[:, :, res.slice[k]]
            if B.shape[0] == B.shape[1]:
                res.V[:, k] = B @ res.U[:, k] / res.weights[k]
        return res
    monkeypatch.setattr(t2c, "t2c", bad)
    assert _fails(t2c, PINS)


def test_planted_slices_in_the_wrong_mode(t2c, monkeypatch):
    """slices taken along the second mode but placed as third-mode slices"""
    real = t2c.t2c
    monkeypatch.setattr(t2c, "t2c", lambda beta, eps: real(np.asfortranarray(beta.transpose(0, 2, 1)), eps))
    assert _fails(t2c, PINS)


def test_planted_strict_ge_keeps_ties(t2c, monkeypatch):
    """a threshold one ulp-scale too high (keeps only sigma > thr (1 + 1e-6))"""
    real_thr = t2c.t2c_threshold
    monkeypatch.setattr(t2c, "t2c_threshold", lambda eps, r1, r2, r3: real_thr(eps, r1, r2, r3) * (1 + 1e-6))
    assert _fails(t2c, PINS)
