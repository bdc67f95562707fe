"""GPU tests of the Tucker-to-canonical transform (rhosvd_t2c / rhosvd_t2c_get,
Section 2.3, Remark 2.6) through the C-ABI, against the oracle (oracle/t2c.py):
per-slice singular values and kept counts, the kept terms, the error estimate,
lifting by the Tucker factors, and the whole canonical-to-canonical chain on the
small Gaussian-sum workload against the materialized tensor."""
import math

import numpy as np
import pytest

from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def flush(msg):
    print(msg, flush=True)


def fortran_dev(beta):
    """numpy (r1, r2, r3) -> CUDA float64 tensor in Fortran order."""
    import torch
    r1, r2, r3 = beta.shape
    flat = torch.from_numpy(np.asfortranarray(beta).ravel(order="F")).cuda()
    return flat.view(r3, r2, r1).permute(2, 1, 0)


def run_t2c(beta, eps, Z=None):
    import torch
    from paper_2201_12663_amd import rhosvd
    red = rhosvd.Reducer()
    out = red.t2c(fortran_dev(beta), eps, Z=Z)
    torch.cuda.synchronize()
    red.close()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def sigma_tol(L, s1):
    """One-sided Jacobi: singular values to a few L u of the slice's largest."""
    return 16.0 * L * U64 * s1


def compare_with_oracle(o, g, beta, eps, core_tol=0.0):
    """Slice counts under the margin rule, all singular values, the kept slice
    approximations (unique where the cut has a gap) and the error estimate.
    core_tol > 0: the oracle transformed its own core, which equals beta only to
    within core_tol (entrywise, up to column signs of the Tucker factors), so the
    singular values carry that much more and slices are not compared entrywise."""
    from oracle import t2c as ot
    r1, r2, r3 = beta.shape
    L = max(r1, r2)
    assert g["R"] == int(np.sum(g["weights"].shape[0]))
    p_g = np.bincount(g["slice"], minlength=r3) if g["R"] else np.zeros(r3, dtype=int)
    for m in range(r3):
        so = o.sigma[m]
        tol = sigma_tol(L, so[0] if len(so) else 0.0) + core_tol * math.sqrt(r1 * r2)
        assert np.all(np.abs(g["sigma"][m] - so) <= tol + 1e-300), (m, np.max(np.abs(g["sigma"][m] - so)))
        # margin rule: the count must agree where no singular value lies within tol of thr
        if np.all(np.abs(so - o.threshold) > 10 * tol):
            assert p_g[m] == o.p[m], (m, p_g[m], o.p[m])
    # the canonical core reproduces each slice's kept part (equal to the oracle's
    # where the counts agree, as the truncated SVD is unique there up to rounding)
    res = ot.T2CResult(g["weights"], g["F1"], g["F2"], g["slice"].astype(np.int64), p_g, list(g["sigma"]),
                       None, o.threshold, g["bound"])
    approx = ot.canonical_core(res, r3)
    ref = ot.canonical_core(o, r3)
    err = float(np.linalg.norm((beta - approx).ravel()))
    assert err <= g["bound"] * (1 + 1e-9) + 1e-12 * float(np.linalg.norm(beta.ravel()))
    assert g["bound"] <= eps * (1 + 1e-12)
    same = [m for m in range(r3) if p_g[m] == o.p[m]] if core_tol == 0.0 else []
    for m in same:
        d = np.abs(approx[:, :, m] - ref[:, :, m]).max()
        assert d <= 1e-10 * max(1.0, o.sigma[m][0]), (m, d)
    # factors are unit vectors
    if g["R"]:
        assert np.allclose(np.linalg.norm(g["F1"], axis=0), 1.0, atol=1e-12)
        assert np.allclose(np.linalg.norm(g["F2"], axis=0), 1.0, atol=1e-10)
        assert np.all(g["weights"] > o.threshold)
    return err


SHAPES = [(9, 9, 9), (12, 7, 5), (6, 11, 8), (33, 33, 33), (64, 40, 17), (17, 100, 3), (1, 5, 4), (139, 139, 3)]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{a}x{b}x{c}" for a, b, c in SHAPES])
def test_known_slice_spectra(orc, shape):
    """Cores whose slices have chosen spectra: some values far above the threshold,
    the rest far below it (counts exact), every slice within its own scale."""
    from oracle import t2c as ot
    r1, r2, r3 = shape
    eps = 1e-6
    thr = ot.t2c_threshold(eps, r1, r2, r3)
    g0 = np.random.default_rng(sum(shape))
    k = min(r1, r2)
    spectra, q = [], []
    for m in range(r3):
        qm = int(g0.integers(0, k + 1))
        spectra.append(np.concatenate([np.geomspace(3.0, 1e-4, qm), np.geomspace(thr / 10, thr / 1e3, k - qm)]))
        q.append(qm)
    beta = inputs.core_with_slice_spectra(sum(shape), r1, r2, r3, spectra)
    o = ot.t2c(beta, eps)
    g = run_t2c(beta, eps)
    flush(f"{shape}: R {g['R']} (oracle {len(o.weights)}), bound {g['bound']:.3e}")
    assert np.array_equal(np.bincount(g["slice"], minlength=r3) if g["R"] else np.zeros(r3), q)
    compare_with_oracle(o, g, beta, eps)


@pytest.mark.parametrize("shape", [(20, 20, 20), (48, 31, 9), (31, 48, 9)])
def test_random_cores(orc, shape):
    from oracle import t2c as ot
    beta = inputs.random_core(sum(shape), *shape)
    for eps in (1.0, 1e-1):
        o = ot.t2c(beta, eps)
        g = run_t2c(beta, eps)
        compare_with_oracle(o, g, beta, eps)


def test_edges_and_limits():
    """All terms dropped (R = 0), a single slice, and the LDS size limit."""
    import torch
    from paper_2201_12663_amd import rhosvd
    beta = inputs.random_core(1, 8, 8, 4) * 1e-12
    g = run_t2c(beta, 1.0)
    assert g["R"] == 0 and g["bound"] <= 1.0
    red = rhosvd.Reducer()
    with pytest.raises(rhosvd.RhosvdError) as e:
        red.t2c(fortran_dev(np.zeros((200, 200, 2))), 1e-3)
    assert e.value.status == -7
    # no successful transform on the handle: phase 2 is refused
    assert red.lib.rhosvd_t2c_get(red.h, None, None, None, None, None, 0, None, None, None, None, None, None) == -6
    with pytest.raises(rhosvd.RhosvdError) as e:
        red.t2c(fortran_dev(np.ones((3, 3, 3))), -1.0)
    assert e.value.status == -1
    red.close()


def test_c2c_chain_small_workload(orc):
    """The small Gaussian-sum workload (n=64, R=200, eps=1e-6): the GPU's
    reduction, then its Tucker-to-canonical transform at eps_T2C = 1e-6 |beta| and
    the lifting by Z, against the materialized tensor (brute force) and against
    the oracle's transform of the oracle's own core (same slice spectra: the cores
    differ only by column signs of the Z's)."""
    import torch
    from oracle import t2c as ot
    from paper_2201_12663_amd import rhosvd
    ci = inputs.small_gaussian_sum(0)
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    U = [rhosvd.to_device(u) for u in ci.U]
    red = rhosvd.Reducer()
    red.reduce(U[0], U[1], U[2], torch.from_numpy(ci.xi).cuda(), ci.eps)
    res = red.get()
    bnorm = float(torch.linalg.vector_norm(res.beta))
    eps2 = 1e-6 * bnorm
    out = red.t2c(res.beta, eps2, Z=res.Z)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    assert tuple(res.ranks) == tuple(o.ranks)
    ot_res = ot.t2c(o.beta, eps2)
    flush(f"small workload: Tucker ranks {res.ranks}, canonical rank {g['R']} (oracle {len(ot_res.weights)}), "
          f"bound {g['bound'] / bnorm:.3e} |beta|")
    compare_with_oracle(ot_res, g, res.beta.cpu().numpy(), eps2, core_tol=1e-10 * bnorm)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    A = orc.full_tensor(Ut, xip)
    a = float(np.linalg.norm(A.ravel()))
    Z = [z.cpu().numpy() for z in res.Z]
    assert np.allclose(g["C1"], Z[0] @ g["F1"], atol=1e-13)
    assert np.allclose(g["C2"], Z[1] @ g["F2"], atol=1e-13)
    assert np.array_equal(g["C3"], Z[2][:, g["slice"]])
    AR = np.einsum("k,ik,jk,lk->ijl", g["weights"], g["C1"], g["C2"], g["C3"], optimize=True)
    e_can = float(np.linalg.norm((A - AR).ravel()))
    e_tucker = float(np.linalg.norm((A - orc.reconstruct(res.beta.cpu().numpy(), Z)).ravel()))
    flush(f"  |A - A_r| = {e_tucker / a:.3e} |A|, |A - A_(R)| = {e_can / a:.3e} |A|")
    assert e_can <= e_tucker + g["bound"] * (1 + 1e-9) + 1e-12 * a
    assert e_can <= (ci.eps + 1e-6) * a
    red.close()
