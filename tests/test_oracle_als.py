"""Pins of the ALS oracle (oracle/als.py, Section 2.1 after Definition 2.1), on
the CPU: the textbook higher-order orthogonal iteration on the materialized
tensor (SVDs of dense unfoldings by LAPACK), the iteration's monotone core norm,
the Pythagorean error identity against brute force, the exact-Tucker fixed
point, and planted mistakes that each fail a pin."""
import numpy as np
import pytest

from paper_2201_12663_amd import inputs


@pytest.fixture(scope="module")
def als():
    from oracle import als as mod
    return mod


def _proj(Z):
    return Z @ Z.T


def dense_hooi_step(A, Z, l):
    """Textbook: Y = A x_a Z_a^T x_b Z_b^T, mode-l unfolding, LAPACK SVD."""
    Zs = [Z[0], Z[1], Z[2]]
    Y = A
    for k in range(3):
        if k != l:
            Y = np.moveaxis(np.tensordot(Y, Zs[k], axes=([k], [0])), -1, k)
    Yl = np.moveaxis(Y, l, 0).reshape(A.shape[l], -1)
    Uf, _, _ = np.linalg.svd(Yl, full_matrices=False)
    return Uf[:, :Z[l].shape[1]]


def _case(seed=3, n=16, R=60, eps=1e-3):
    import oracle
    ci = inputs.small_gaussian_sum(seed, n=n, R=R, eps=eps)
    o = oracle.rhosvd(ci.U, ci.xi, ci.eps)
    Ut, xip, _, _ = oracle.normalize(ci.U, ci.xi)
    return ci, o, Ut, xip


def pin_dense_hooi(als):
    """Low Tucker ranks (eps = 0.3), where a sweep moves the subspaces visibly and
    the order of the mode updates matters (updating every mode from the previous
    sweep's factors moves the third mode's subspace by ~3e-5 here)."""
    import oracle
    ci, o, Ut, xip = _case(seed=7, eps=0.3)
    A = oracle.full_tensor(Ut, xip)
    Zd = [z.copy() for z in o.Z]
    for sweeps in (1, 2):
        Z, V, _ = als.als_sweeps(Ut, xip, o.Z, sweeps)
        if sweeps == 1:
            for l in range(3):
                Zd[l] = dense_hooi_step(A, Zd, l)
        else:
            for l in range(3):
                Zd[l] = dense_hooi_step(A, Zd, l)
        for l in range(3):
            assert np.linalg.norm(_proj(Z[l]) - _proj(Zd[l]), 2) <= 1e-8, (sweeps, l)


def pin_monotone_and_pythagoras(als):
    import oracle
    for seed in (1, 2):
        ci, o, Ut, xip = _case(seed=seed, n=18, R=70, eps=1e-2)
        A = oracle.full_tensor(Ut, xip)
        a2 = float(np.sum(A * A))
        Z, V, hist = als.als_sweeps(Ut, xip, o.Z, 2)
        assert all(b >= a * (1 - 1e-13) for a, b in zip(hist, hist[1:])), hist
        beta = oracle.core(V, xip)
        err = float(np.linalg.norm((A - oracle.reconstruct(beta, Z)).ravel()))
        err0 = float(np.linalg.norm((A - oracle.reconstruct(o.beta, o.Z)).ravel()))
        assert err <= err0 * (1 + 1e-12) + 1e-14
        assert abs(err ** 2 - (a2 - hist[-1] ** 2)) <= 1e-10 * a2


def pin_fixed_point(als):
    """Exactly low-rank side matrices: the RHOSVD is exact, and the iteration
    keeps its subspaces."""
    import oracle
    ci = inputs.exactly_low_rank(6, 20, 40, ranks=(3, 4, 5), eps=1e-6)
    o = oracle.rhosvd(ci.U, ci.xi, ci.eps)
    Ut, xip, _, _ = oracle.normalize(ci.U, ci.xi)
    Z, V, hist = als.als_sweeps(Ut, xip, o.Z, 1)
    for l in range(3):
        assert np.linalg.norm(_proj(Z[l]) - _proj(o.Z[l]), 2) <= 1e-10


def pin_unfolding_entries(als):
    """The contracted unfolding equals the dense contraction's mode-1 unfolding."""
    import oracle
    ci, o, Ut, xip = _case(seed=5, n=12, R=30)
    A = oracle.full_tensor(Ut, xip)
    V = [oracle.project(o.Z[l], Ut[l]) for l in range(3)]
    M = als.contracted_unfolding(Ut[0], xip, V[1], V[2])
    Y = np.einsum("ijk,ja,kb->iab", A, o.Z[1], o.Z[2])
    assert np.allclose(M, Y.reshape(A.shape[0], -1, order="F"), atol=1e-12 * np.abs(A).max())


PINS = [pin_dense_hooi, pin_monotone_and_pythagoras, pin_fixed_point, pin_unfolding_entries]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_als_pin(als, pin):
    pin(als)


def _fails(mod, pins):
    for p in pins:
        try:
            p(mod)
        except (AssertionError, ValueError, IndexError):
            return True
    return False


def test_planted_unweighted_terms(als, monkeypatch):
    real = als.contracted_unfolding
    monkeypatch.setattr(als, "contracted_unfolding", lambda U, x, a, b: real(U, np.ones_like(x), a, b))
    assert _fails(als, PINS)


def test_planted_jacobi_order(als, monkeypatch):
    """every mode of a sweep updated from the previous sweep's factors"""
    import oracle

    def bad(Ut, xip, Z, sweeps):
        Z = [z.copy() for z in Z]
        V = [oracle.project(Z[l], Ut[l]) for l in range(3)]
        hist = [float(np.linalg.norm(oracle.core(V, xip).ravel()))]
        for _ in range(sweeps):
            Vold = [v.copy() for v in V]
            for l in range(3):
                a, b = [k for k in range(3) if k != l]
                _, Zf, _ = oracle.svd_left(als.contracted_unfolding(Ut[l], xip, Vold[a], Vold[b]))
                Z[l] = oracle.sign_normalize(Zf[:, :Z[l].shape[1]])
                V[l] = oracle.project(Z[l], Ut[l])
                hist.append(float(np.linalg.norm(oracle.core(V, xip).ravel())))
        return Z, V, hist
    monkeypatch.setattr(als, "als_sweeps", bad)
    assert _fails(als, PINS)


def test_planted_own_mode_projection(als, monkeypatch):
    """the mode's own old projection used in place of one of the others"""
    real = als.contracted_unfolding
    monkeypatch.setattr(als, "contracted_unfolding",
                        lambda U, x, a, b: real(U, x, a, a) if a.shape == b.shape else real(U, x, b, b))
    assert _fails(als, PINS)
