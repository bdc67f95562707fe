"""GPU tests of the batched entry point (rhosvd_reduce_batched) through the C-ABI:
a batch of uneven problems (both Gram sides, several tiles, ragged tails) is
compared problem by problem with the oracle, the recorded graph is replayed on
live inputs, and the per-problem error paths (capacity, non-finite input, all
terms dropped) are checked inside a batch of good problems."""
import math

import numpy as np
import pytest

from gpu_cases import U64, check_core_slabs, cut_margin_ok, cut_margin_ok_measured, eig_tol, tails_of
from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu

# (kind, n, R): n <= R and R < n, sizes that are not multiples of the tiles
SHAPES = [("gauss", 48, 150), ("newton", 64, 200), ("gauss", 100, 333), ("newton", 72, 40),
          ("gauss", 130, 90), ("newton", 160, 640), ("gauss", 90, 90), ("newton", 33, 500),
          ("gauss", 200, 257), ("newton", 129, 64)]


def make_problem(kind, n, R, idx):
    if kind == "gauss":
        return inputs.small_gaussian_sum(seed=100 + idx, n=n, R=R)
    return inputs.batch_problem(seed=7, index=idx, n=n, R=R, eps=1e-5)


def to_dev(ci):
    import torch
    from paper_2201_12663_amd import rhosvd
    U = [rhosvd.to_device(u) for u in ci.U]
    return (U[0], U[1], U[2], torch.from_numpy(np.ascontiguousarray(ci.xi)).cuda(), ci.eps)


def check_against_oracle(orc, ci, ranks, Z, beta, eta=2.0 ** -52, beta_tol=1e-10):
    """One problem's batched result vs the oracle: ranks under the margin rule,
    orthonormal Z, the kept subspaces (Davis-Kahan), beta equal to the exact core
    of the GPU's own Z, and the reconstruction error within eps |A|."""
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    m = min(ci.n, ci.R)
    for l in range(3):
        s1 = o.sigma[l][0]
        if cut_margin_ok(o.tails[l], o.ranks[l], o.tau, s1, eta=eta):
            assert ranks[l] == o.ranks[l], (ci.name, l, ranks, o.ranks)
        r = ranks[l]
        Zl = Z[l]
        assert Zl.shape == (ci.n, r)
        assert np.max(np.abs(Zl.T @ Zl - np.eye(r))) <= 100 * m * U64, ci.name
        if ranks[l] == o.ranks[l] and r < m:
            gap = o.sigma[l][r - 1] ** 2 - o.sigma[l][r] ** 2
            if gap > 0:
                dk = 10 * max(eig_tol(ci.n, ci.R), eta) * s1 ** 2 / gap
                if dk < 0.1:
                    Po = o.Z[l] @ o.Z[l].T
                    assert np.linalg.norm(Zl @ Zl.T - Po, 2) <= dk, (ci.name, l, dk)
    V = [orc.project(Z[l], Ut[l]) for l in range(3)]
    be = orc.core(V, xip)
    assert beta.shape == be.shape
    assert np.max(np.abs(beta - be)) <= beta_tol * o.xi_norm, (ci.name, np.max(np.abs(beta - be)))
    err = orc.error_gram(Ut, xip, Z)
    assert err <= ci.eps * o.a_norm * (1 + 1e-9) + 1e-300, (ci.name, err / o.a_norm)
    return o


@pytest.fixture(scope="module")
def batch_inputs():
    cis = [make_problem(k, n, R, i) for i, (k, n, R) in enumerate(SHAPES)]
    return cis


def test_batched_fp64_matches_oracle(orc, batch_inputs):
    import torch
    from paper_2201_12663_amd import rhosvd
    cis = batch_inputs
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision="fp64")
    out, desc, res, outs = red.reduce_batched(probs)
    torch.cuda.synchronize()
    print("batched fp64: graph", red.batch_uses_graph(), [o["ranks"] for o in out], flush=True)
    for ci, o in zip(cis, out):
        assert o["status"] == 0, (ci.name, o["status"])
        Z = [z.cpu().numpy() for z in o["Z"]]
        check_against_oracle(orc, ci, o["ranks"], Z, o["beta"].cpu().numpy())
    red.close()


def test_batched_equals_single_path_ranks(batch_inputs):
    """The batched pass and rhosvd_reduce compute the same ranks on every problem."""
    import torch
    from paper_2201_12663_amd import rhosvd
    cis = batch_inputs
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision="fp64")
    out, _, _, _ = red.reduce_batched(probs, beta=False)
    single = rhosvd.Reducer(precision="fp64", anorm="exact", refine_tails="off")
    for ci, p, o in zip(cis, probs, out):
        r = single.reduce(*p)
        assert tuple(r) == o["ranks"], (ci.name, r, o["ranks"])
    torch.cuda.synchronize()
    red.close()
    single.close()


def test_graph_replay_reads_live_inputs(batch_inputs):
    """Replays of the recorded pass, with eager work in between, give identical
    results; scaling xi in place (same pointers) scales beta and keeps the ranks
    (the truncation threshold is scale-invariant)."""
    import torch
    from paper_2201_12663_amd import rhosvd
    cis = batch_inputs[:6]
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision="fp64")
    out, desc, res, outs = red.reduce_batched(probs)
    torch.cuda.synchronize()
    ref = [o["beta"].clone() for o in out]
    ref_ranks = [o["ranks"] for o in out]
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        red.reduce_batched_raw(desc)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        rr = res.cpu().numpy()
        for i, o in enumerate(out):
            assert tuple(int(x) for x in rr[i, :3]) == ref_ranks[i]
            assert torch.equal(o["beta"], ref[i]), (rep, i)
    assert red.batch_uses_graph()
    for p in probs:
        p[3].mul_(2.0)
    red.reduce_batched_raw(desc)
    torch.cuda.synchronize()
    rr = res.cpu().numpy()
    for i, o in enumerate(out):
        assert tuple(int(x) for x in rr[i, :3]) == ref_ranks[i]
        assert torch.allclose(o["beta"], 2.0 * ref[i], rtol=1e-12, atol=1e-12 * float(ref[i].abs().max()))
    red.close()


def test_batch_error_paths_do_not_disturb_neighbours(orc, batch_inputs):
    import torch
    from paper_2201_12663_amd import rhosvd
    good = batch_inputs[1]          # newton n=64 R=200
    bad_nan = inputs.small_gaussian_sum(seed=5, n=40, R=60)
    bad_nan.U[1][3, 7] = np.nan
    zero = inputs.small_gaussian_sum(seed=6, n=40, R=60)
    zero.xi[:] = 0.0
    capped = batch_inputs[2]        # gauss n=100 R=333, rank far above 5
    cis = [good, bad_nan, zero, capped, good]
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision="fp64")
    res = torch.zeros((len(cis), 8), dtype=torch.int32, device="cuda")
    outs = []
    caps = [80, 40, 40, 5, 80]
    for ci, cap in zip(cis, caps):
        Zs = [rhosvd.colmajor_empty(ci.n, cap).fill_(7.0) for _ in range(3)]
        b = torch.full((cap ** 3,), 7.0, dtype=torch.float64, device="cuda")
        outs.append((Zs[0], Zs[1], Zs[2], b))
    desc = red.batch_descriptors(probs, res, outputs=outs)
    red.reduce_batched_raw(desc)
    torch.cuda.synchronize()
    rr = res.cpu().numpy()
    assert rr[1, 3] == -2                          # non-finite input
    assert tuple(rr[2, :4]) == (0, 0, 0, 0)        # every term dropped: ranks 0, status OK
    assert rr[2, 4] == 60
    assert rr[3, 3] == -8 and min(rr[3, :3]) > 5   # ranks above cap_rank: capacity
    assert torch.all(outs[3][0] == 7.0) and torch.all(outs[3][3] == 7.0)   # nothing written
    for i in (0, 4):
        assert rr[i, 3] == 0
        r = tuple(int(x) for x in rr[i, :3])
        Z = [outs[i][l][:, :r[l]].cpu().numpy() for l in range(3)]
        beta = outs[i][3][: r[0] * r[1] * r[2]].view(r[2], r[1], r[0]).permute(2, 1, 0).cpu().numpy()
        check_against_oracle(orc, good, r, Z, beta)
    red.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batched_mixed_precision(orc, batch_inputs, prec):
    """Mixed cores: ranks and Z as in FP64 (those phases are FP64) and beta within
    the core's precision of the exact core of Z: FP32 within 2e-6 |xi'|, BF16x3
    (two bf16 terms per operand, about 2^-17 per product) within 2^-15 |xi'|.
    The total error stays within (eps + 1e-6) |A|.  The BF16x3 run takes every
    problem at eps = 1e-5: one problem below that (the Gaussian ones' 1e-6) would
    move the whole pass to the FP32 core."""
    import dataclasses
    import torch
    from paper_2201_12663_amd import rhosvd
    cis = batch_inputs
    if prec == "bf16x3":
        cis = [dataclasses.replace(ci, eps=max(ci.eps, 1e-5)) for ci in cis]
    probs = [to_dev(ci) for ci in cis]
    r64 = rhosvd.Reducer(precision="fp64")
    o64, _, _, _ = r64.reduce_batched(probs)
    rm = rhosvd.Reducer(precision=prec)
    om, _, _, _ = rm.reduce_batched(probs)
    torch.cuda.synchronize()
    for ci, a, b in zip(cis, o64, om):
        assert a["ranks"] == b["ranks"], ci.name
        assert b["core_precision"] == (1 if prec == "fp32" else 2), ci.name
        for l in range(3):
            assert torch.equal(a["Z"][l], b["Z"][l]), (ci.name, l)
        Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
        Z = [z.cpu().numpy() for z in b["Z"]]
        bb = b["beta"].cpu().numpy()
        check_core_slabs(orc, Ut, xip, Z, bb, range(bb.shape[2]), prec, what=ci.name)
        be = orc.core([orc.project(Z[l], Ut[l]) for l in range(3)], xip)
        db = np.linalg.norm((b["beta"].cpu().numpy() - be).ravel())
        xin = float(np.linalg.norm(xip))
        assert db <= (2e-6 if prec == "fp32" else 2.0 ** -15) * xin, (ci.name, db / xin)
        a_norm = orc.anorm_gram(Ut, xip)
        err = math.hypot(orc.error_gram(Ut, xip, Z), db)
        assert err <= (ci.eps + 1e-6) * a_norm, (ci.name, err / a_norm)
    r64.close()
    rm.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_long_contraction_hands_over_partial_sums(orc, batch_inputs, prec):
    """R = 20000 (R_pad above 8192): the FP32-accumulating cores hand their
    partial sums to beta every 8192 terms, on the single path and in a batch
    that also holds a short problem (whose core then runs in the same kernel
    variant with a single final store).  Every beta is within the core's
    precision of the exact core of its own Z, and the total error is within
    (eps + 1e-6) |A| against the materialized tensor.  The BF16x3 run takes
    eps = 1e-5 (below that the library would run the FP32 core in its place)."""
    import dataclasses
    import torch
    from paper_2201_12663_amd import rhosvd
    long_ci = inputs.small_gaussian_sum(seed=21, n=96, R=20000, eps=1e-6 if prec == "fp32" else 1e-5)
    cis = [long_ci, batch_inputs[2] if prec == "fp32" else dataclasses.replace(batch_inputs[2], eps=1e-5)]
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision=prec)
    out, _, _, _ = red.reduce_batched(probs)
    single = rhosvd.Reducer(precision=prec, anorm="exact", refine_tails="off")
    # |beta - beta_exact| against |A|: FP32 accumulation of up to 8192 terms
    # (2048 sequential MFMA steps) per hand-over, u32 sqrt(2048) ~ 3e-6 of the
    # running sums for positive terms; BF16x3 adds its split error (~2^-17)
    tol = 3e-6 if prec == "fp32" else 1e-5
    for k, (ci, p, o) in enumerate(zip(cis, probs, out)):
        assert o["status"] == 0
        assert o["core_precision"] == (1 if prec == "fp32" else 2)
        r = single.reduce(*p)
        res = single.get(sigma=False)
        torch.cuda.synchronize()
        assert tuple(r) == o["ranks"], ci.name
        assert res.report["core_precision"] == o["core_precision"], ci.name
        Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
        A = orc.full_tensor_slabs(Ut, xip)
        a_norm = float(np.linalg.norm(A.ravel(order="K")))
        for Zt, bt, where in ((o["Z"], o["beta"], "batched"), (res.Z, res.beta, "single")):
            Z = [z.cpu().numpy() for z in Zt]
            beta = bt.cpu().numpy()
            be = orc.core([orc.project(Z[l], Ut[l]) for l in range(3)], xip)
            db = float(np.linalg.norm((beta - be).ravel()))
            err = orc.error_dense(A, beta, Z)
            print(f"{prec} {ci.name} {where}: ranks {o['ranks']} core error {db / a_norm:.3e} |A|, "
                  f"total error {err / a_norm:.3e} |A|", flush=True)
            assert db <= tol * a_norm, (ci.name, where, db / a_norm)
            assert err <= (ci.eps + 1e-6) * a_norm
        del A
    red.close()
    single.close()


def test_batched_uneven_config_sample():
    """Problems of the uneven batch at their real sizes (n up to 2048, R up to
    8192, one R < n): ranks equal the single path's, Z is orthonormal, its
    well-separated columns equal the single path's, and |beta| agrees."""
    import torch
    from gpu_cases import separated
    from paper_2201_12663_amd import rhosvd
    shapes = inputs.batch_shapes(seed=0, count=256)
    pick = sorted(range(256), key=lambda i: -shapes[i][0] * min(shapes[i][1], 4096))[:2]
    pick += [next(i for i in range(256) if shapes[i][1] < shapes[i][0] and shapes[i][0] >= 1024)]
    pick += [min(range(256), key=lambda i: shapes[i][0] * shapes[i][1])]
    cis = [inputs.batch_problem(0, i, *shapes[i]) for i in pick]
    print("config sample:", [(ci.n, ci.R) for ci in cis], flush=True)
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision="fp32")
    out, _, _, _ = red.reduce_batched(probs)
    single = rhosvd.Reducer(precision="fp32", anorm="exact", refine_tails="off")
    for ci, p, o in zip(cis, probs, out):
        assert o["status"] == 0
        r = single.reduce(*p)
        res = single.get(Z=True, sigma=False)
        assert tuple(r) == o["ranks"], (ci.name, r, o["ranks"])
        for l in range(3):
            Zb = o["Z"][l]
            I = Zb.T @ Zb
            assert float((I - torch.eye(I.shape[0], device="cuda", dtype=I.dtype)).abs().max()) <= 1e-11
            if ci.R < ci.n:
                continue   # R < n: Z is fixed only up to a rotation of the kept subspace
            sig = single.spectrum(l).cpu().numpy()
            sep = separated(sig, r[l])
            Zs = res.Z[l]
            d = Zb[:, sep] - Zs[:, sep] * torch.sign((Zb[:, sep] * Zs[:, sep]).sum(0))
            assert float(d.abs().max()) <= 1e-8, (ci.name, l)
        nb = float(torch.linalg.vector_norm(o["beta"]))
        ns = float(torch.linalg.vector_norm(res.beta))
        assert abs(nb - ns) <= 1e-5 * ns, (ci.name, nb, ns)
        del res
    torch.cuda.synchronize()
    red.close()
    single.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_beta_fp32_output_is_the_rounded_core(batch_inputs, prec):
    """With the beta_fp32 option the core (accumulated in FP32) is stored as float:
    exactly the double output rounded to float, on the single path and batched."""
    import torch
    from paper_2201_12663_amd import rhosvd
    ci = batch_inputs[5]
    p = to_dev(ci)
    a = rhosvd.Reducer(precision=prec)
    b = rhosvd.Reducer(precision=prec, beta_fp32=True)
    a.reduce(*p)
    b.reduce(*p)
    ra, rb = a.get(Z=False, sigma=False), b.get(Z=False, sigma=False)
    torch.cuda.synchronize()
    assert rb.beta.dtype == torch.float32
    assert torch.equal(rb.beta, ra.beta.float())
    oa, _, _, _ = a.reduce_batched([p])
    ob, _, _, _ = b.reduce_batched([p])
    torch.cuda.synchronize()
    assert torch.equal(ob[0]["beta"], oa[0]["beta"].float())
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_real_sizes_vs_golden(orc, prec):
    """The uneven batch's largest n <= R problem (n=2048, R=7115) and largest R < n
    problem (n=2048, R=2041) in one batched pass with two small ones, against the
    oracle's stored values (tests/golden/batch_seed0.json): ranks under the margin
    rule, every singular value within the Gram route's accuracy, the oracle's core
    samples (entries of well-separated singular vectors, FP64 cores), whole slabs
    of the core element by element against the oracle's core of the returned Z,
    and the exact error within eps |A| and the Theorem 2.3 bound."""
    import json
    import os
    import torch
    from gpu_cases import boundary_slabs, separated
    from paper_2201_12663_amd import rhosvd
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_seed0.json")))
    shapes = inputs.batch_shapes(seed=0, count=256)
    big = [inputs.batch_problem(0, p["index"], *shapes[p["index"]]) for p in gold["problems"]]
    small = [make_problem(k, n, R, i) for i, (k, n, R) in enumerate(SHAPES[:2])]
    cis = big + small
    print(f"real-size batch {prec}:", [(ci.n, ci.R) for ci in cis], flush=True)
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision=prec)
    out, _, _, _ = red.reduce_batched(probs)
    torch.cuda.synchronize()
    # the single path on the same problems gives the spectrum the batched pass cut
    # (the two form the same Gram matrices and tridiagonalize them identically, up
    # to the Gram's summation order): its tails measure the path's tail error
    single = rhosvd.Reducer(precision=prec, anorm="exact", refine_tails="off")
    for ci, g, o in zip(big, gold["problems"], out):
        assert o["status"] == 0
        r = o["ranks"]
        m = min(ci.n, ci.R)
        Z = [z.cpu().numpy() for z in o["Z"]]
        rs = single.reduce(*to_dev(ci))
        for l in range(3):
            so = np.array(g["sigma"][l])
            sg = single.spectrum(l).cpu().numpy()
            assert np.all(np.abs(sg ** 2 - so ** 2) <= eig_tol(ci.n, ci.R) * so[0] ** 2), (ci.name, l)
            t_o, t_g = tails_of(so), tails_of(sg)
            ok = cut_margin_ok_measured(t_g, t_o, g["ranks"][l], g["tau"])
            print(f"  {ci.name} mode {l}: batched {r[l]}, single {rs[l]}, oracle {g['ranks'][l]}, "
                  f"margin ok {ok}", flush=True)
            if ok:
                assert r[l] == g["ranks"][l], (ci.name, l, r, g["ranks"])
            assert abs(r[l] - rs[l]) <= 1
            assert np.max(np.abs(Z[l].T @ Z[l] - np.eye(r[l]))) <= 100 * m * U64
        Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
        beta = o["beta"]
        if prec == "fp64":
            checked = 0
            for j1, j2, j3, v in g["beta_samples"]:
                if j1 < r[0] and j2 < r[1] and j3 < r[2]:
                    assert abs(float(beta[j1, j2, j3]) - v) <= 1e-9 * g["xi_norm"], (ci.name, j1, j2, j3)
                    checked += 1
            assert checked >= len(g["beta_samples"]) - 2
        slabs = boundary_slabs(r[2], extra=(127, 128, 511, 512, 1023, 1024))
        bs = beta[:, :, slabs].cpu().numpy()
        w = check_core_slabs(orc, Ut, xip, Z, bs, slabs, prec, what=ci.name, beta_is_slabs=True)
        err = orc.error_gram(Ut, xip, Z)
        print(f"  {ci.name}: ranks {r} (oracle {g['ranks']}), worst core entry at {w:.3f} of its bound, "
              f"rel err {err / g['a_norm']:.3e}", flush=True)
        assert err <= ci.eps * g["a_norm"] * (1 + 1e-9)
        del beta
    for ci, o in zip(small, out[2:]):
        assert o["status"] == 0
        Z = [z.cpu().numpy() for z in o["Z"]]
        check_against_oracle(orc, ci, o["ranks"], Z, o["beta"].cpu().numpy(),
                             beta_tol=1e-10 if prec == "fp64" else 2e-6)
    del out
    red.close()
    single.close()
    torch.cuda.empty_cache()
