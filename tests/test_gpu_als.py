"""GPU tests of the canonical-to-Tucker ALS refinement (rhosvd_options.als_sweeps,
Section 2.1 after Definition 2.1, eq. eqn:can_A_Tuck_als) through the C-ABI,
against the ALS oracle (oracle/als.py): the subspaces after one and two sweeps,
the error decrease against the RHOSVD's, the core of the refined factors element
by element, and the size limits."""
import numpy as np
import pytest

import gpu_cases as gc
from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu


def flush(msg):
    print(msg, flush=True)


def run(ci, sweeps, prec="fp64"):
    return gc.run_gpu(ci, prec, als_sweeps=sweeps, anorm="exact")


CASES = [("gauss n64 R200 eps0.3", lambda: inputs.small_gaussian_sum(7, n=64, R=200, eps=0.3)),
         ("newton n160 R640 eps1e-2", lambda: inputs.newton_centres(2, n=160, n_centres=20, eps=1e-2)),
         ("gauss n100 R333 eps1e-3", lambda: inputs.small_gaussian_sum(1, n=100, R=333, eps=1e-3))]


@pytest.mark.parametrize("sweeps", [1, 2])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_als_subspaces_match_oracle(orc, name, make, sweeps):
    from oracle import als
    ci = make()
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    g = run(ci, sweeps)
    assert g["ranks"] == tuple(o.ranks)
    Zo, Vo, hist = als.als_sweeps(Ut, xip, o.Z, sweeps)
    for l in range(3):
        r = g["ranks"][l]
        Z = g["Z"][l]
        assert np.max(np.abs(Z.T @ Z - np.eye(r))) <= 1e-12
        # Davis-Kahan: the last update of mode l took the leading r singular
        # vectors of its contracted unfolding; the tolerance follows its gap
        a, b = [k for k in range(3) if k != l]
        Vl = [orc.project(Zo[k], Ut[k]) for k in range(3)]
        s = np.linalg.svd(als.contracted_unfolding(Ut[l], xip, Vl[a], Vl[b]), compute_uv=False)
        gap = (s[r - 1] ** 2 - (s[r] ** 2 if r < len(s) else 0.0)) / s[0] ** 2
        d = np.linalg.norm(Z @ Z.T - Zo[l] @ Zo[l].T, 2)
        flush(f"{name} sweeps={sweeps} mode {l}: projector distance {d:.2e}, relative gap {gap:.2e}")
        if gap > 1e-8:
            assert d <= 1e-12 / gap + 1e-10, (l, d, gap)
    # the core of the refined factors, every slab element by element
    gc.check_core_slabs(orc, Ut, xip, g["Z"], g["beta"], range(g["ranks"][2]), "fp64", what=name)
    # |beta| grew as in the oracle's iteration (an orthogonal projection of A, so
    # the error fell): |A - A_r|^2 = |A|^2 - |beta|^2
    nb = float(np.linalg.norm(g["beta"].ravel()))
    assert nb >= hist[0] * (1 - 1e-12)
    assert abs(nb - hist[-1]) <= 1e-10 * hist[-1]


def test_als_error_decreases_and_mixed_cores(orc):
    """n=256, R=1024, eps=1e-3: the exact error of the ALS factors is at most the
    RHOSVD's (and within the RHOSVD's Theorem 2.3 bound, which the report keeps);
    the FP32 path's refined factors equal the FP64 path's bit for bit (the
    iteration runs in FP64 on both), its core within its own bound.  After the
    first sweep (here 39x below the RHOSVD's error) the iteration has converged
    below what its FP64 Gram route resolves: the subspaces move within the
    eigenvalue noise of the contracted Grams, about 64 sqrt(m) u |A|^2, so the
    second sweep's error is bounded by that noise, not by the first's."""
    ci = inputs.batch_problem(5, 3, 256, 1024, eps=1e-3)
    g0 = gc.run_gpu(ci, "fp64", want_beta=False, anorm="exact")
    g1 = run(ci, 1)
    g2 = run(ci, 2)
    g2f = run(ci, 2, prec="fp32")
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    a = orc.anorm_gram(Ut, xip)
    e0, e1, e2 = (orc.error_gram(Ut, xip, g["Z"]) for g in (g0, g1, g2))
    flush(f"errors / |A|: RHOSVD {e0 / a:.4e}, ALS 1 sweep {e1 / a:.4e}, 2 sweeps {e2 / a:.4e}")
    assert e1 <= e0 * (1 + 1e-9)
    noise = 64.0 * np.sqrt(min(ci.n, ci.R)) * 2.0 ** -53 * a * a
    assert e2 ** 2 <= e1 ** 2 * (1 + 1e-9) + noise, (e1, e2, noise)
    assert e2 <= g2["report"]["bound"] * (1 + 1e-9)
    for l in range(3):
        assert np.array_equal(g2f["Z"][l], g2["Z"][l])
    gc.check_core_slabs(orc, Ut, xip, g2f["Z"], g2f["beta"], gc.boundary_slabs(g2f["ranks"][2]), "fp32")


def test_als_limits():
    import torch
    from paper_2201_12663_amd import rhosvd
    for n, R in ((200, 90), (64, 17000)):
        ci = inputs.small_gaussian_sum(3, n=n, R=R)
        U = [rhosvd.to_device(u) for u in ci.U]
        red = rhosvd.Reducer(als_sweeps=1)
        with pytest.raises(rhosvd.RhosvdError) as e:
            red.reduce(U[0], U[1], U[2], torch.from_numpy(ci.xi).cuda(), 1e-3)
        assert e.value.status == -7
        red.close()
    with pytest.raises(rhosvd.RhosvdError):
        rhosvd.Reducer(als_sweeps=5)
