"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Sizes span several tiles with ragged tails (n, R not multiples of 64; ranks not
multiples of the core tiles).  Full-size n=1024, R=4096 parity is against stored
oracle values (tests/golden/newton1024_seed0.json, written by make_golden.py)
plus properties that hold at any size.
"""
import json
import os

import numpy as np
import pytest

from paper_2201_12663_amd import inputs
import gpu_cases as gc

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    from paper_2201_12663_amd import rhosvd
    assert torch.cuda.is_available()
    rhosvd.load()


CASES = [
    ("gauss n64 R200", lambda: inputs.small_gaussian_sum(0)),
    ("gauss n100 R333", lambda: inputs.small_gaussian_sum(1, n=100, R=333, eps=1e-5)),
    ("newton n160 R640", lambda: inputs.newton_centres(2, n=160, n_centres=20, eps=1e-5)),
    ("lowrank n70 R150", lambda: inputs.exactly_low_rank(3, 70, 150, ranks=(3, 7, 12), eps=1e-8)),
    # R < n: Gram on the R side, Z = U~ W Lambda^-1/2 re-orthonormalized in FP64
    ("gauss n200 R90 (R<n)", lambda: inputs.small_gaussian_sum(11, n=200, R=90, eps=1e-5)),
    ("newton n300 R160 (R<n)", lambda: inputs.newton_centres(12, n=300, n_centres=5, eps=1e-5)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fp64_parity(orc, name, make):
    ci = make()
    _flush(f"case {name}: n={ci.n} R={ci.R} eps={ci.eps}")
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g = gc.run_gpu(ci, "fp64")
    gc.compare_fp64(g, o, ci)
    err = gc.recon_error(orc, ci, g["Z"], g["beta"])
    assert err <= ci.eps * o.a_norm * (1 + 1e-9)
    assert err <= g["report"]["bound"] * (1 + 1e-9) + 1e-12 * o.a_norm


def test_exactly_low_rank_r_side(orc):
    ci = inputs.exactly_low_rank(5, 130, 40, ranks=(4, 6, 3), eps=1e-4)
    g = gc.run_gpu(ci, "fp64")
    assert g["ranks"] == (4, 6, 3)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    a = orc.anorm_gram(Ut, xip)
    assert gc.recon_error(orc, ci, g["Z"]) <= 1e-11 * a


def test_exactly_low_rank_reconstruction(orc):
    # eps well above the FP64 Gram's noise floor: tau^2 >> (m - r) u |G|, so the
    # exact ranks must come out (at eps = 1e-8 the noise eigenvalues of the Gram
    # exceed tau^2 and the ranks may only grow, see the parity case above)
    ci = inputs.exactly_low_rank(4, 48, 90, ranks=(2, 5, 9), eps=1e-4)
    g = gc.run_gpu(ci, "fp64")
    assert g["ranks"] == (2, 5, 9)
    err = gc.recon_error(orc, ci, g["Z"], g["beta"])
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    a = float(np.linalg.norm(orc.full_tensor(Ut, xip).ravel()))
    assert err <= 1e-12 * a


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_parity(orc, prec):
    ci = inputs.small_gaussian_sum(5, n=96, R=300, eps=1e-5)
    _flush(f"mixed {prec}")
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g64 = gc.run_gpu(ci, "fp64")
    g = gc.run_gpu(ci, prec)
    # Gram, eigensolver and truncation are FP64 in every mode: identical ranks and Z
    assert g["ranks"] == g64["ranks"]
    for l in range(3):
        assert np.array_equal(g["Z"][l], g64["Z"][l])
    err = gc.recon_error(orc, ci, g["Z"], g["beta"])
    assert err <= (ci.eps + 1e-6) * o.a_norm
    db = np.linalg.norm((g["beta"] - g64["beta"]).ravel()) / o.a_norm
    assert db <= (1e-5 if prec == "bf16x3" else 1e-6), db
    # every entry of every slab against the oracle's core of Z (Proposition 2.2)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    for gg, p in ((g, prec), (g64, "fp64")):
        w = gc.check_core_slabs(orc, Ut, xip, gg["Z"], gg["beta"], range(gg["ranks"][2]), p, what="n96 R300")
        _flush(f"{p}: worst entry at {w:.3f} of its bound")
    assert g["report"]["core_precision"] == (1 if prec == "fp32" else 2)


def test_bf16x3_below_its_floor_runs_the_fp32_core(orc):
    """eps < 1e-5 with the BF16x3 precision: the split's own error (~2e-6 |A|)
    would exceed the 1e-6 allowance, so the FP32 core runs on the same FP32 V.
    Its beta equals the FP32 path's bit for bit (same kernel and tile), the report
    says FP32, and the total error is within (eps + 1e-6) |A|; in a batch, one
    problem below the floor moves the whole pass to the FP32 core."""
    import torch
    from paper_2201_12663_amd import rhosvd
    ci = inputs.small_gaussian_sum(5, n=96, R=300, eps=1e-6)
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g32 = gc.run_gpu(ci, "fp32", core_tile=64)
    g = gc.run_gpu(ci, "bf16x3", core_tile=64)
    assert g["report"]["core_precision"] == 1 and g32["report"]["core_precision"] == 1
    assert g["ranks"] == g32["ranks"]
    assert np.array_equal(g["beta"], g32["beta"])
    assert gc.recon_error(orc, ci, g["Z"], g["beta"]) <= (ci.eps + 1e-6) * o.a_norm
    # batched: eps 1e-5 and 1e-6 together -> FP32 core for both; 1e-5 alone -> BF16x3
    cj = inputs.small_gaussian_sum(6, n=80, R=250, eps=1e-5)
    dev = []
    for c in (ci, cj):
        U = [rhosvd.to_device(u) for u in c.U]
        dev.append((U[0], U[1], U[2], torch.from_numpy(np.ascontiguousarray(c.xi)).cuda(), c.eps))
    red = rhosvd.Reducer(precision="bf16x3", core_tile=64)
    both, _, _, _ = red.reduce_batched(dev)
    alone, _, _, _ = red.reduce_batched(dev[1:])
    torch.cuda.synchronize()
    assert [b["core_precision"] for b in both] == [1, 1]
    assert alone[0]["core_precision"] == 2
    assert both[0]["ranks"] == g["ranks"]
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    Zb = [z.cpu().numpy() for z in both[0]["Z"]]
    gc.check_core_slabs(orc, Ut, xip, Zb, both[0]["beta"].cpu().numpy(), range(g["ranks"][2]), "fp32",
                        what="batched n96 R300")
    red.close()


def test_degenerate_single_term(orc):
    g0 = np.random.default_rng(1)
    U = [np.asfortranarray(g0.standard_normal((37, 1))) for _ in range(3)]
    ci = inputs.CanonicalInput(U, np.array([-2.5]), 1e-6)
    g = gc.run_gpu(ci, "fp64")
    assert g["ranks"] == (1, 1, 1)
    nrm = np.prod([np.linalg.norm(u) for u in U])
    assert abs(abs(g["beta"][0, 0, 0]) - 2.5 * nrm) <= 1e-12 * 2.5 * nrm


def test_dropped_terms_and_all_dropped(orc):
    ci = inputs.small_gaussian_sum(6, n=40, R=80, eps=1e-5)
    U = [u.copy() for u in ci.U]
    U[2][:, 5] = 0.0
    xi = ci.xi.copy()
    xi[9] = 0.0
    ci2 = inputs.CanonicalInput(U, xi, ci.eps)
    o = orc.rhosvd(U, xi, ci.eps)
    g = gc.run_gpu(ci2, "fp64")
    assert g["report"]["dropped"] == 2
    assert g["xip"][5] == 0.0 and g["xip"][9] == 0.0
    gc.compare_fp64(g, o, ci2)
    ci3 = inputs.CanonicalInput(U, np.zeros(80), ci.eps)
    g3 = gc.run_gpu(ci3, "fp64")
    assert g3["ranks"] == (0, 0, 0)


def test_tiny_and_huge_columns_are_normalized_not_dropped(orc):
    """Columns whose largest entry is subnormal (1/max overflows) or above 2^1000
    are nonzero: their terms stay in the normalized side matrices, as in the
    oracle (their unit columns shape the Gram even where xi' rounds to almost
    nothing).  The subnormal columns keep 40+ bits, so both sides' normalized
    columns agree to ~1e-13."""
    ci = inputs.small_gaussian_sum(6, n=40, R=80, eps=1e-5)
    U = [u.copy() for u in ci.U]
    xi = ci.xi.copy()
    U[0][:, 3] *= 1e-310
    U[1][:, 7] *= 3e-309
    U[2][:, 11] *= 1e305
    xi[11] *= 1e-305
    ci2 = inputs.CanonicalInput(U, xi, ci.eps)
    o = orc.rhosvd(U, xi, ci.eps)
    g = gc.run_gpu(ci2, "fp64")
    assert g["report"]["dropped"] == 0
    tiny = [3, 7]
    for k in tiny + [11]:
        assert g["xip"][k] != 0.0
        assert abs(g["xip"][k] - o.xip[k]) <= 1e-12 * abs(o.xip[k]) + 8 * 2.0 ** -1074
    g["xip"][tiny] = o.xip[tiny]        # subnormal: compared above to their own precision
    gc.compare_fp64(g, o, ci2)


def test_nonfinite_input_is_rejected():
    import torch
    from paper_2201_12663_amd import rhosvd
    ci = inputs.small_gaussian_sum(7, n=32, R=50)
    U = [u.copy() for u in ci.U]
    U[1][3, 4] = np.nan
    Ud = [rhosvd.to_device(u) for u in U]
    xi = torch.from_numpy(ci.xi).cuda()
    red = rhosvd.Reducer()
    with pytest.raises(rhosvd.RhosvdError) as e:
        red.reduce(Ud[0], Ud[1], Ud[2], xi, 1e-6)
    assert e.value.status == -2
    with pytest.raises(rhosvd.RhosvdError) as e:
        red.reduce(Ud[0], Ud[1], Ud[2], xi, -1.0)
    assert e.value.status == -1
    with pytest.raises(rhosvd.RhosvdError) as e:
        red.get()
    assert e.value.status == -6
    red.close()


def test_deterministic_repeat():
    ci = inputs.small_gaussian_sum(8, n=128, R=400, eps=1e-5)
    a = gc.run_gpu(ci, "fp64")
    b = gc.run_gpu(ci, "fp64")
    assert a["ranks"] == b["ranks"]
    assert np.array_equal(a["beta"], b["beta"])
    for l in range(3):
        assert np.array_equal(a["Z"][l], b["Z"][l])


def test_full_size_newton1024_vs_golden(orc):
    """n=1024, R=4096, eps=1e-5: the configuration the benchmark times."""
    gold = json.load(open(os.path.join(HERE, "golden", "newton1024_seed0.json")))
    ci = inputs.newton_centres(0)
    _flush("full size n=1024 R=4096")
    g = gc.run_gpu(ci, "fp64")
    rep = g["report"]
    assert abs(rep["a_norm"] - gold["a_norm"]) <= 1e-10 * gold["a_norm"]
    assert abs(rep["xi_norm"] - gold["xi_norm"]) <= 1e-12 * gold["xi_norm"]
    for l in range(3):
        so = np.array(gold["sigma"][l])
        s1 = so[0]
        d2 = np.abs(g["spectra"][l] ** 2 - so ** 2)
        assert np.all(d2 <= gc.eig_tol(ci.n, ci.R) * s1 ** 2), (l, d2.max() / s1 ** 2)
        tails = np.sqrt(np.concatenate([np.cumsum((so ** 2)[::-1])[::-1], [0.0]]))
        if gc.cut_margin_ok(tails, gold["ranks"][l], gold["tau"], s1):
            assert g["ranks"][l] == gold["ranks"][l]
        r = g["ranks"][l]
        Z = g["Z"][l]
        assert np.max(np.abs(Z.T @ Z - np.eye(r))) <= 1e-11
    # sampled core entries of the oracle's own reduction (its sign convention; indices
    # of well-separated singular vectors).  beta[j1,j2,j3] depends only on columns
    # j1, j2, j3 of the Z's, not on the ranks, so a knife-edge rank difference in
    # one mode leaves every sample below both ranks comparable
    checked = 0
    for j1, j2, j3, v in gold["beta_samples"]:
        if j1 < g["ranks"][0] and j2 < g["ranks"][1] and j3 < g["ranks"][2]:
            assert abs(g["beta"][j1, j2, j3] - v) <= 1e-9 * gold["xi_norm"], (j1, j2, j3)
            checked += 1
    assert checked >= len(gold["beta_samples"]) - 2, checked
    # whole slabs element by element: the oracle's core of the returned Z at the
    # tile edges, the ragged last slab and a few more (Proposition 2.2)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    slabs = gc.boundary_slabs(g["ranks"][2], extra=(127, 128, 255, 256, 511, 512))
    w = gc.check_core_slabs(orc, Ut, xip, g["Z"], g["beta"], slabs, "fp64", what="newton1024")
    err = gc.recon_error(orc, ci, g["Z"])
    assert err <= ci.eps * gold["a_norm"]
    assert err <= rep["bound"] * (1 + 1e-9)
    _flush(f"full size: ranks {g['ranks']} rel err {err / gold['a_norm']:.3e}, "
           f"{checked} oracle samples, slabs {slabs}: worst entry at {w:.3f} of its bound")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_full_size_newton1024_mixed(orc, prec):
    import torch
    ci = inputs.newton_centres(0)
    _flush(f"full size mixed {prec}")
    g64 = gc.run_gpu(ci, "fp64")
    g = gc.run_gpu(ci, prec)
    assert g["ranks"] == g64["ranks"]
    err_z = gc.recon_error(orc, ci, g["Z"])
    a = g64["report"]["a_norm"]
    # whole slabs element by element against the oracle's core of Z, each entry
    # within the mixed core's own bound (and the FP64 core's within its own)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    slabs = gc.boundary_slabs(g["ranks"][2], extra=(127, 128, 255, 256))
    w = gc.check_core_slabs(orc, Ut, xip, g["Z"], g["beta"], slabs, prec, what="newton1024")
    w64 = gc.check_core_slabs(orc, Ut, xip, g64["Z"], g64["beta"], slabs, "fp64", what="newton1024")
    # the mixed core's whole distance from the exact core of Z, through the FP64
    # core (same Z): |beta' - beta_e| <= |beta' - beta_64| + |beta_64 - beta_e|, the
    # last at most the FP64 per-entry bound (below 1e-10 |xi'| here, checked on the
    # slabs above).  The total error: A - A_r is orthogonal to the Tucker subspace
    # and the core error lies inside it
    db = float(np.linalg.norm((g["beta"] - g64["beta"]).ravel())) + 1e-10 * g64["report"]["xi_norm"]
    err = float(np.sqrt(err_z ** 2 + db ** 2))
    _flush(f"{prec}: worst slab entry at {w:.3f} of its bound (FP64 core {w64:.2e}); rel err {err / a:.3e} "
           f"(core part {db / a:.3e})")
    assert err <= (ci.eps + 1e-6) * a


@pytest.mark.parametrize("refine", [1, 2, "auto"])
@pytest.mark.parametrize("prec,shape", [("fp64", (512, 1024, 1e-5)), ("fp32", (512, 1024, 1e-5)),
                                        ("fp64", (256, 2048, 1e-6)), ("fp32", (512, 2048, 1e-6)),
                                        # R < n: the R-side Gram, re-run on the n side to refine
                                        ("fp64", (512, 382, 1e-6, 10_007, 44)),
                                        ("fp32", (1024, 455, 1e-6, 10_007, 125))])
def test_refined_tails_recover_the_oracle_ranks(orc, prec, shape, refine):
    """Smooth low-rank inputs: where the sum of the Gram route's noise eigenvalues
    (about u |G| each) exceeds tau^2 its ranks come out above the oracle's; with
    refine_tails the cut uses tails formed from V and the exact residual and lands
    on the oracle's ranks, with orthonormal Z, beta the exact core of Z and the
    error within the bound.  (Below tau^2 ~ u |G| itself the Gram route's vectors
    near the cut are inaccurate and no refinement of its cut can recover them;
    refine_tails = 2, the deflated second pass, is meant for that case.)  With
    R < n the refinement runs on the n x n Gram (refine_used + 4)."""
    import torch
    from paper_2201_12663_amd import rhosvd
    n, R, eps = shape[:3]
    seed, index = shape[3:] if len(shape) > 3 else (9, 0)
    _flush(f"refined tails {prec} n={n} R={R} eps={eps} refine={refine}")
    a, c, xi = inputs.smooth_problem_params(seed, index, n, R)
    ci = inputs.CanonicalInput(inputs.gaussian_side_matrices(inputs.grid(n), a, c), xi, eps)
    o = orc.rhosvd(ci.U, ci.xi, ci.eps, with_core=False)
    U = [rhosvd.to_device(u) for u in ci.U]
    xd = torch.from_numpy(ci.xi).cuda()
    plain = rhosvd.Reducer(precision=prec, refine_tails="off")
    ref = rhosvd.Reducer(precision=prec, refine_tails=refine)
    rp = plain.reduce(U[0], U[1], U[2], xd, ci.eps)
    rr = ref.reduce(U[0], U[1], U[2], xd, ci.eps)
    res = ref.get()
    torch.cuda.synchronize()
    print("oracle", o.ranks, "gram route", rp, f"refined ({refine})", rr, "used", res.report["refine_used"], flush=True)
    if refine == "auto":
        # the default refines exactly where the Gram route's cut sits in its noise
        # band (its ranks then far above the oracle's), and there with the deflated
        # pass when tau^2 is in the band too; elsewhere it keeps the plain cut
        used = res.report["refine_used"]
        if any(rp[l] > o.ranks[l] + 2 for l in range(3)):
            assert used & 3 in (1, 2)
        if used == 0:
            assert tuple(rr) == tuple(rp)
    if R < n and refine != "auto":
        assert res.report["refine_used"] == refine + 4
    for l in range(3):
        assert abs(rr[l] - o.ranks[l]) <= 2, (rr, o.ranks)
        assert rr[l] <= rp[l]
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    Z = [z.cpu().numpy() for z in res.Z]
    for l in range(3):
        assert np.max(np.abs(Z[l].T @ Z[l] - np.eye(rr[l]))) <= 1e-12
    be = orc.core([orc.project(Z[l], Ut[l]) for l in range(3)], xip)
    tol = 1e-10 if prec == "fp64" else 2e-6
    assert np.linalg.norm((res.beta.cpu().numpy() - be).ravel()) <= tol * o.xi_norm
    err = orc.error_gram(Ut, xip, Z)
    assert err <= res.report["bound"] * (1 + 1e-9)
    assert res.report["bound"] <= ci.eps * o.a_norm * (1 + 1e-9)
    plain.close()
    ref.close()


def test_refined_tails_keep_accurate_gram_ranks(orc):
    """Where the Gram route's tails are accurate (the Newton-type input), the
    refinement keeps the same ranks."""
    import torch
    from paper_2201_12663_amd import rhosvd
    ci = inputs.newton_centres(seed=2, n=160, n_centres=20, eps=1e-5)
    U = [rhosvd.to_device(u) for u in ci.U]
    xd = torch.from_numpy(ci.xi).cuda()
    a = rhosvd.Reducer(precision="fp64", refine_tails="off")
    b = rhosvd.Reducer(precision="fp64", refine_tails=True)
    ra = a.reduce(U[0], U[1], U[2], xd, ci.eps)
    rb = b.reduce(U[0], U[1], U[2], xd, ci.eps)
    torch.cuda.synchronize()
    o = orc.rhosvd(ci.U, ci.xi, ci.eps, with_core=False)
    print("oracle", o.ranks, "gram", ra, "refined", rb, flush=True)
    for l in range(3):
        assert abs(rb[l] - ra[l]) <= 1 and abs(rb[l] - o.ranks[l]) <= 1
    a.close()
    b.close()


def test_deflated_pass_on_rank_one_and_on_the_r_side(orc):
    """refine_tails = 2 edge cases: a rank-1 tensor (k = 0, nothing deflated, the
    second pass repeats the first: same ranks and Z), and R < n, where the option
    re-runs on the n x n Gram with either choice."""
    import torch
    from paper_2201_12663_amd import rhosvd
    rng = np.random.default_rng(41)
    n, R = 96, 150
    u = [rng.standard_normal(n) for _ in range(3)]
    U = [np.ascontiguousarray(np.outer(v, rng.uniform(0.5, 2.0, R))) for v in u]
    xi = rng.uniform(0.1, 1.0, R)
    ci = inputs.CanonicalInput([np.asfortranarray(m) for m in U], xi, 1e-3)
    outs = {}
    for refine in (3, 2):
        red = rhosvd.Reducer(precision="fp64", refine_tails=refine)
        Ud = [rhosvd.to_device(m) for m in ci.U]
        r = red.reduce(Ud[0], Ud[1], Ud[2], torch.from_numpy(xi).cuda(), ci.eps)
        res = red.get()
        torch.cuda.synchronize()
        outs[refine] = (tuple(r), [z.cpu().numpy() for z in res.Z], res.report)
        red.close()
    assert outs[3][0] == outs[2][0] == (1, 1, 1)
    for l in range(3):
        assert np.array_equal(outs[3][1][l], outs[2][1][l])
    o = orc.rhosvd(ci.U, ci.xi, ci.eps, with_core=False)
    assert tuple(o.ranks) == (1, 1, 1)
    # R < n
    ci = inputs.small_gaussian_sum(seed=42, n=300, R=120, eps=1e-6)
    got = {}
    for refine in (1, 2):
        red = rhosvd.Reducer(precision="fp64", refine_tails=refine)
        Ud = [rhosvd.to_device(m) for m in ci.U]
        r = red.reduce(Ud[0], Ud[1], Ud[2], torch.from_numpy(ci.xi).cuda(), ci.eps)
        res = red.get()
        torch.cuda.synchronize()
        got[refine] = (tuple(r), [z.cpu().numpy() for z in res.Z], res.beta.cpu().numpy(), res.report)
        red.close()
    o = orc.rhosvd(ci.U, ci.xi, ci.eps, with_core=False)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    for refine in (1, 2):
        r, Z, beta, rep = got[refine]
        assert rep["refine_used"] == refine + 4 and rep["m"] == 120
        assert all(abs(r[l] - o.ranks[l]) <= 2 for l in range(3)), (r, o.ranks)
        for l in range(3):
            assert np.max(np.abs(Z[l].T @ Z[l] - np.eye(r[l]))) <= 1e-12
        assert orc.error_gram(Ut, xip, Z) <= rep["bound"] * (1 + 1e-9)
        assert rep["bound"] <= ci.eps * o.a_norm * (1 + 1e-9)


def test_refine_tails_values_are_checked():
    from paper_2201_12663_amd import rhosvd
    with pytest.raises(rhosvd.RhosvdError):
        rhosvd.Reducer(precision="fp64", refine_tails=4)


@pytest.mark.parametrize("n,R", [(1, 4), (2, 5), (3, 2), (2, 2), (5, 3), (65, 1), (65, 129)])
def test_tiny_and_ragged_sizes(orc, n, R):
    """The smallest shapes (one- to five-row side matrices, R = 1 .. 5: Gram
    matrices of size 1 to 5, eigensolver without a tridiagonalization step) and
    shapes one past a 64-row tile, against the oracle."""
    rng = np.random.default_rng(1000 + 7 * n + R)
    U = [np.asfortranarray(rng.standard_normal((n, R))) for _ in range(3)]
    xi = rng.uniform(0.5, 1.5, R)
    ci = inputs.CanonicalInput(U, xi, 1e-8)
    _flush(f"tiny case n={n} R={R}")
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g = gc.run_gpu(ci, "fp64")
    gc.compare_fp64(g, o, ci)
    err = gc.recon_error(orc, ci, g["Z"], g["beta"])
    assert err <= ci.eps * o.a_norm * (1 + 1e-9) + 1e-12 * o.a_norm


def test_argument_and_size_limits():
    """Empty inputs, eps <= 0 or not finite, and sizes beyond the library's
    limits (min(n, R) > 2048, n > 65536) are errors, raised before any kernel runs;
    an all-zero input reduces to ranks (0, 0, 0)."""
    import torch
    from paper_2201_12663_amd import rhosvd
    red = rhosvd.Reducer(precision="fp64")

    def call(n, R, eps=1e-6):
        U = [torch.zeros((R, n), dtype=torch.float64, device="cuda").t() for _ in range(3)]
        xi = torch.zeros(R, dtype=torch.float64, device="cuda")
        return red.reduce(U[0], U[1], U[2], xi, eps)

    for args in [(0, 5), (5, 0), (4, 4, 0.0), (4, 4, -1.0), (4, 4, float("nan")), (4, 4, float("inf"))]:
        with pytest.raises((rhosvd.RhosvdError, ValueError)):
            call(*args)
    for args in [(2049, 2049), (65537, 1)]:
        with pytest.raises(rhosvd.RhosvdError) as ei:
            call(*args)
        assert ei.value.status == -7
    assert call(4, 4) == (0, 0, 0)
    red.close()


CERT_CASES = [("newton n160 R640", lambda: inputs.newton_centres(2, n=160, n_centres=20, eps=1e-5)),
              ("gauss n200 R90 (R<n)", lambda: inputs.small_gaussian_sum(11, n=200, R=90, eps=1e-5)),
              ("gauss n100 R333", lambda: inputs.small_gaussian_sum(1, n=100, R=333, eps=1e-3))]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("name,make", CERT_CASES, ids=[c[0] for c in CERT_CASES])
def test_certificate(orc, name, make, prec):
    """The certificate from the proof of Theorem 2.3 (certificate option): equal to
    the oracle's certificate of the GPU's own Z, the same in every precision (it
    uses an FP64 projection), and err <= c <= bound."""
    import torch
    from paper_2201_12663_amd import rhosvd
    ci = make()
    U = [rhosvd.to_device(u) for u in ci.U]
    xi = torch.from_numpy(np.ascontiguousarray(ci.xi)).cuda()
    red = rhosvd.Reducer(precision=prec, certificate=True)
    red.reduce(U[0], U[1], U[2], xi, ci.eps)
    res = red.get()
    torch.cuda.synchronize()
    Z = [z.cpu().numpy() for z in res.Z]
    red.close()
    c = res.report["certificate"]
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    co = orc.certificate(Ut, xip, Z)
    _flush(f"{name} {prec}: certificate {c:.6e} (oracle {co:.6e}), bound {res.report['bound']:.6e}")
    assert abs(c - co) <= 1e-8 * co + 1e-13 * float(np.sum(np.abs(xip)))
    assert c <= res.report["bound"] * (1 + 1e-9)
    if prec == "fp64":
        err = orc.error_gram(Ut, xip, Z)
        assert err <= c * (1 + 1e-9) + 1e-12 * res.report["a_norm"]
    plain = rhosvd.Reducer(precision=prec)
    plain.reduce(U[0], U[1], U[2], xi, ci.eps)
    assert plain.get(beta=False, Z=False, sigma=False).report["certificate"] == -1.0
    plain.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_certificate_after_deflated_pass(orc, prec):
    """The certificate also covers the Z of the deflated second pass (A9: any
    orthonormal Z), and stays below that path's bound."""
    import torch
    from paper_2201_12663_amd import rhosvd
    n, R, eps = 256, 2048, 1e-6
    a, c, xi = inputs.smooth_problem_params(9, 0, n, R)
    ci = inputs.CanonicalInput(inputs.gaussian_side_matrices(inputs.grid(n), a, c), xi, eps)
    U = [rhosvd.to_device(u) for u in ci.U]
    xd = torch.from_numpy(ci.xi).cuda()
    red = rhosvd.Reducer(precision=prec, refine_tails=2, certificate=True)
    red.reduce(U[0], U[1], U[2], xd, eps)
    res = red.get()
    torch.cuda.synchronize()
    Z = [z.cpu().numpy() for z in res.Z]
    red.close()
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    co = orc.certificate(Ut, xip, Z)
    cg = res.report["certificate"]
    _flush(f"deflated {prec}: ranks {res.ranks} certificate {cg:.6e} (oracle {co:.6e}) bound {res.report['bound']:.6e}")
    assert abs(cg - co) <= 1e-8 * co + 1e-13 * float(np.sum(np.abs(xip)))
    assert cg <= res.report["bound"] * (1 + 1e-9)
    assert orc.error_gram(Ut, xip, Z) <= cg * (1 + 1e-9) + 1e-12 * res.report["a_norm"]


def smooth_wide(seed, n, R, eps, pairs=False):
    """Wide Gaussians (alpha log-uniform in [0.05, 0.5]), centres in [-4, 4]^3, so the
    side matrices have low numerical rank; with pairs, every term is followed by a
    copy whose centre moved by 1e-3 and whose weight has the opposite sign, so that
    |A| is about 1e-3 |xi'| (heavy cancellation)."""
    g = np.random.default_rng(9000 + seed)
    k = R // 2 if pairs else R
    a = np.exp(g.uniform(np.log(0.05), np.log(0.5), k))
    c = g.uniform(-4, 4, (k, 3))
    xi = g.uniform(0.5, 1.5, k)
    if pairs:
        a = np.repeat(a, 2)
        c = np.repeat(c, 2, axis=0)
        c[1::2] += 1e-3
        xi = np.repeat(xi, 2) * np.tile([1.0, -1.0], k)
    U = inputs.gaussian_side_matrices(inputs.grid(n), a, c)
    return inputs.CanonicalInput(U, xi, eps, name=f"smooth-wide n{n} R{R}{' pairs' if pairs else ''}")


PROBE_CASES = [
    ("gauss n64 R200", lambda: inputs.small_gaussian_sum(0)),
    ("newton n160 R640", lambda: inputs.newton_centres(2, n=160, n_centres=20, eps=1e-5)),
    ("smooth n96 R3000", lambda: smooth_wide(1, 96, 3000, 1e-6)),
    ("lowrank n70 R150", lambda: inputs.exactly_low_rank(3, 70, 150, ranks=(3, 7, 12), eps=1e-8)),
]


@pytest.mark.parametrize("name,make", PROBE_CASES, ids=[c[0] for c in PROBE_CASES])
def test_anorm_probe_certified_lower_bound(orc, name, make):
    """rhosvd_options.anorm = probe: |A| from the FP64 core at the probe ranks
    (tails <= 1/30).  Its value L = |beta_p| is a lower bound of the oracle's exact
    |A| and (L^2 + b_p^2)^(1/2) an upper bound (Theorem 2.3 at the probe ranks);
    tau is at most the oracle's; the ranks are the oracle's cut at that tau
    (margin rule); the error stays within the bound, and the bound within
    eps |A| with the exact |A|."""
    ci = make()
    _flush(f"probe case {name}")
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g = gc.run_gpu(ci, "fp64", anorm="probe")
    rep = g["report"]
    assert rep["anorm_method"] == 2
    tau = gc.check_anorm(rep, o.a_norm, o.tau)
    _flush(f"  L/|A| = {rep['a_norm'] / o.a_norm:.9f}, U/|A| = {rep['a_norm_upper'] / o.a_norm:.9f}")
    for l in range(3):
        r_ref = orc.choose_rank(o.tails[l], tau)
        if gc.cut_margin_ok(o.tails[l], r_ref, tau, o.sigma[l][0]):
            assert g["ranks"][l] == r_ref, (l, g["ranks"], r_ref)
    err = gc.recon_error(orc, ci, g["Z"], g["beta"])
    assert err <= rep["bound"] * (1 + 1e-9) + 1e-12 * o.a_norm
    assert rep["bound"] <= ci.eps * o.a_norm * (1 + 1e-9)
    # the same reduction with the exact identity: same spectrum, ranks no larger
    g1 = gc.run_gpu(ci, "fp64", want_beta=False, anorm="exact")
    assert g1["report"]["anorm_method"] == 1
    assert all(a >= b for a, b in zip(g["ranks"], g1["ranks"]))
    for l in range(3):
        assert np.array_equal(g["spectra"][l], g1["spectra"][l])


def test_anorm_auto_mode_choices(orc):
    """Default |A| (anorm auto): the probe where n << R and the spectra are low
    (its flops well under the identity's 3 n R^2), the exact identity where the
    probe would cost more (n160 R640 here) and where heavy cancellation makes the
    probe's bracket wide (|A| ~ 1e-3 |xi'|, so b_p > L / 10).  Every result is
    certified against the oracle's exact |A|; two wide cases (R = 60000, beyond
    the oracle's reach) against the library's own exact identity."""
    for ci, want in ((smooth_wide(1, 96, 3000, 1e-6), 2),
                     (inputs.newton_centres(2, n=160, n_centres=20, eps=1e-5), 1),
                     (smooth_wide(2, 64, 2000, 1e-6, pairs=True), 1)):
        o = orc.rhosvd(ci.U, ci.xi, ci.eps, with_core=False)
        g = gc.run_gpu(ci, "fp64")
        rep = g["report"]
        _flush(f"{ci.name}: anorm method {rep['anorm_method']} (want {want}), |A|/|xi'| {o.a_norm / o.xi_norm:.3e}")
        assert rep["anorm_method"] == want, ci.name
        gc.check_anorm(rep, o.a_norm, o.tau)
        assert rep["bound"] <= ci.eps * o.a_norm * (1 + 1e-9)
        err = gc.recon_error(orc, ci, g["Z"])
        # rounding scale: |xi'| (the terms' own size), not |A|, under cancellation
        assert err <= rep["bound"] * (1 + 1e-9) + 1e-10 * o.xi_norm
    for ci, want in ((smooth_wide(3, 64, 60000, 1e-6), 2), (smooth_wide(4, 64, 60000, 1e-6, pairs=True), 1)):
        g = gc.run_gpu(ci, "fp64", want_beta=False)
        ge = gc.run_gpu(ci, "fp64", want_beta=False, anorm="exact")
        rep, rex = g["report"], ge["report"]
        _flush(f"{ci.name}: anorm method {rep['anorm_method']} (want {want}), |A|/|xi'| {rex['a_norm'] / rex['xi_norm']:.3e}")
        assert rep["anorm_method"] == want, ci.name
        gc.check_anorm(rep, rex["a_norm"], rex["tau"])
        assert rep["bound"] <= ci.eps * rex["a_norm"] * (1 + 1e-9)
    # the forced probe under heavy cancellation is still certified (its tau only smaller)
    ci = smooth_wide(2, 64, 2000, 1e-6, pairs=True)
    o = orc.rhosvd(ci.U, ci.xi, ci.eps, with_core=False)
    g = gc.run_gpu(ci, "fp64", anorm="probe")
    gc.check_anorm(g["report"], o.a_norm, o.tau)
    assert g["report"]["bound"] <= ci.eps * o.a_norm * (1 + 1e-9)
