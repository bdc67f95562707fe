"""The Gram matrix in reduced precision (rhosvd_options.gram_precision: FP32 MFMA
or BF16x3) followed by the FP64 Rayleigh-Ritz step, through the C-ABI, against
the CPU oracle.

What is fixed whatever the accuracy of the reduced-precision Gram:
  * Z is orthonormal and the result is certified: the exact error (oracle, from
    Gram matrices) is within the reported Theorem 2.3 bound, itself within
    eps |A| (|A| from the exact identity, equal to the oracle's);
  * the Ritz values s_k of B = Q^T U~ interlace with the oracle's singular values:
    0 <= sigma_k^2 - s_k^2 <= |U~ - Q B|_2^2 <= t_r^2 (Weyl on U~^T U~ = B^T B +
    C^T C, C = Q_perp^T U~), with t_r the path's reported tail at its rank;
  * the rank is at least the oracle's (the SVD's tails are the smallest of any
    orthonormal Z), and equal where the oracle's cut margin exceeds 10x the
    difference between the path's tails and the oracle's;
  * beta equals the oracle's core of the path's own Z, slab by slab.
"""
import numpy as np
import pytest

from paper_2201_12663_amd import inputs
import gpu_cases as gc

pytestmark = pytest.mark.gpu

GP = {"fp32": 1, "bf16x3": 2}

CASES = [
    ("gauss n200 R700 eps1e-3", lambda: inputs.small_gaussian_sum(4, n=200, R=700, eps=1e-3)),
    ("newton n256 R1024 eps1e-4", lambda: inputs.newton_centres(5, n=256, n_centres=32, eps=1e-4)),
    # tau^2 far below the reduced-precision Gram's noise: the step widens p
    ("newton n160 R640 eps1e-5", lambda: inputs.newton_centres(2, n=160, n_centres=20, eps=1e-5)),
]


def _flush(msg):
    print(msg, flush=True)


def path_tails(spec, tail_r, r):
    """The path's tails at r - 1 and r from its Ritz values and its reported t_r."""
    return np.sqrt(tail_r ** 2 + spec[r - 1] ** 2), tail_r


@pytest.mark.parametrize("gp", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_reduced_precision_gram_is_certified_and_matches_the_oracle(orc, name, make, gp):
    ci = make()
    _flush(f"case {name} gram {gp}: n={ci.n} R={ci.R} eps={ci.eps}")
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g = gc.run_gpu(ci, "fp64", gram_precision=gp)
    rep = g["report"]
    assert rep["gram_precision"] == GP[gp]
    assert rep["refine_used"] == 0 and rep["anorm_method"] == 1
    assert abs(rep["a_norm"] - o.a_norm) <= 1e-12 * o.a_norm
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    for l in range(3):
        Z = g["Z"][l]
        assert np.max(np.abs(Z.T @ Z - np.eye(Z.shape[1]))) <= 1e-12, l
    err = orc.error_gram(Ut, xip, g["Z"])
    assert err <= rep["bound"] * (1 + 1e-9) + 1e-12 * o.a_norm
    assert rep["bound"] <= ci.eps * o.a_norm * (1 + 1e-9)
    for l in range(3):
        r, ro = g["ranks"][l], o.ranks[l]
        so = np.asarray(o.sigma[l])
        spec = g["spectra"][l]
        s1 = so[0]
        t_r = rep["tail"][l]
        # interlacing of the Ritz values with the singular values
        dl = so[:r] ** 2 - spec[:r] ** 2
        assert np.all(dl >= -1e-12 * s1 ** 2), (l, float(dl.min()))
        assert np.all(dl <= t_r ** 2 * (1 + 1e-9) + 1e-12 * s1 ** 2), (l, float(dl.max()), t_r ** 2)
        # ranks: the path's tails are those of an orthonormal Z, never below the
        # SVD's (up to rounding), so its rank is never below the oracle's; equal
        # where the oracle's margin is clear of the measured tail difference
        t_orc = np.asarray(o.tails[l])
        t_prev, t_cur = path_tails(spec, t_r, r)
        assert t_cur >= t_orc[r] - 1e-9 * t_orc[0], (l, t_cur, t_orc[r])
        assert r >= ro or t_orc[r] - t_cur <= 1e-9 * t_orc[0], (l, r, ro)
        d = max(abs(t_prev - t_orc[r - 1]), abs(t_cur - t_orc[r]))
        margin = min(t_orc[ro - 1] - o.tau, o.tau - t_orc[ro])
        if margin > 10 * d:
            assert r == ro, (l, r, ro, margin, d)
        _flush(f"  mode {l}: rank {r} (oracle {ro}), leading Ritz rel. diff {float(dl[0]) / s1 ** 2:.2e}, "
               f"t_r {t_r:.3e} tau {o.tau:.3e}")
    slabs = gc.boundary_slabs(g["ranks"][2])
    gc.check_core_slabs(orc, Ut, xip, g["Z"], g["beta"], slabs, "fp64", what=name)


@pytest.mark.parametrize("gp", ["fp32", "bf16x3"])
def test_loose_eps_reaches_the_oracle_ranks(orc, gp):
    """A larger loose-eps problem (n = 512, R = 2000, eps = 1e-3): the step lands on
    the oracle's ranks wherever the oracle's cut margin is clear of the path's
    tail difference."""
    ci = inputs.small_gaussian_sum(7, n=512, R=2000, eps=1e-3)
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g = gc.run_gpu(ci, "fp64", gram_precision=gp)
    g64 = gc.run_gpu(ci, "fp64")
    rep = g["report"]
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    assert orc.error_gram(Ut, xip, g["Z"]) <= rep["bound"] * (1 + 1e-9) + 1e-12 * o.a_norm
    assert rep["bound"] <= ci.eps * o.a_norm * (1 + 1e-9)
    for l in range(3):
        r, ro = g["ranks"][l], o.ranks[l]
        t_orc = o.tails[l]
        t_prev, t_r = path_tails(g["spectra"][l], g["report"]["tail"][l], r)
        d = max(abs(t_prev - t_orc[r - 1]), abs(t_r - t_orc[r]))
        margin = min(t_orc[ro - 1] - o.tau, o.tau - t_orc[ro])
        _flush(f"{gp} mode {l}: rank {r} (oracle {ro}, FP64 Gram {g64['ranks'][l]}), tail diff {d:.2e}, "
               f"margin {margin:.2e}")
        if margin > 10 * d:
            assert r == ro, (l, r, ro)


def test_r_less_than_n_keeps_the_fp64_gram(orc):
    """R < n: the Gram lives on the R side and stays FP64 (the report says so);
    the result equals the default path's."""
    ci = inputs.small_gaussian_sum(11, n=200, R=90, eps=1e-5)
    g = gc.run_gpu(ci, "fp64", gram_precision="fp32")
    g64 = gc.run_gpu(ci, "fp64")
    assert g["report"]["gram_precision"] == 0
    assert g["ranks"] == g64["ranks"]
    for l in range(3):
        assert np.array_equal(g["Z"][l], g64["Z"][l])


def test_with_the_bf16x3_core(orc):
    """The reduced-precision Gram with a mixed core: the Rayleigh-Ritz Z, then the
    BF16x3 core (eps = 1e-4, above its floor) within its bound of the oracle's
    core of that Z, and the total within (eps + 1e-6) |A|."""
    ci = inputs.newton_centres(5, n=256, n_centres=32, eps=1e-4)
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g = gc.run_gpu(ci, "bf16x3", gram_precision="bf16x3")
    assert g["report"]["gram_precision"] == 2 and g["report"]["core_precision"] == 2
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    gc.check_core_slabs(orc, Ut, xip, g["Z"], g["beta"], range(g["ranks"][2]), "bf16x3", what="gram bf16x3")
    err = gc.recon_error(orc, ci, g["Z"], g["beta"])
    assert err <= (ci.eps + 1e-6) * o.a_norm


def test_gram_precision_option_is_checked():
    from paper_2201_12663_amd import rhosvd
    with pytest.raises(rhosvd.RhosvdError):
        rhosvd.Reducer(gram_precision=3)


def test_with_als_sweeps_and_certificate(orc):
    """ALS sweeps start from the Rayleigh-Ritz Z at its ranks and only lower the
    error; the certificate (formed on the final Z) equals the oracle's certificate
    of that Z and stays within the reported bound."""
    ci = inputs.newton_centres(5, n=256, n_centres=32, eps=1e-4)
    g0 = gc.run_gpu(ci, "fp64", gram_precision="fp32")
    g1 = gc.run_gpu(ci, "fp64", gram_precision="fp32", als_sweeps=1, certificate=True)
    assert g1["ranks"] == g0["ranks"]
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    e0 = orc.error_gram(Ut, xip, g0["Z"])
    e1 = orc.error_gram(Ut, xip, g1["Z"])
    a = g1["report"]["a_norm"]
    _flush(f"ALS after the Rayleigh-Ritz Z: error {e0 / a:.4e} -> {e1 / a:.4e} |A|")
    assert e1 <= e0 * (1 + 1e-9) + 1e-12 * a
    c = g1["report"]["certificate"]
    co = orc.certificate(Ut, xip, g1["Z"])
    assert abs(c - co) <= 1e-8 * co + 1e-13 * float(np.sum(np.abs(xip)))
    assert c <= g1["report"]["bound"] * (1 + 1e-9)
