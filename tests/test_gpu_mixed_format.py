"""GPU tests of the mixed Tucker-canonical output (Proposition 2.2) through the
C-ABI: the factors V^(l) = Z^(l)T U~^(l) of the single path (rhosvd_get_v) and of
the batched pass (the V1..V3 outputs of rhosvd_problem, with the core skipped),
against the oracle's projections element by element, the oracle's own V on rows
of well-separated singular vectors, and the materialized tensor."""
import numpy as np
import pytest

import gpu_cases as gc
from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def to_dev(ci):
    import torch
    from paper_2201_12663_amd import rhosvd
    U = [rhosvd.to_device(u) for u in ci.U]
    return (U[0], U[1], U[2], torch.from_numpy(np.ascontiguousarray(ci.xi)).cuda(), ci.eps)


def check_v(orc, Ut, Z, V, prec, what):
    """V against the oracle's projection of the returned Z, entry by entry: the
    FP64 projection's error bound (gpu_cases.v_abs_error), plus the rounding to
    float on the mixed paths."""
    d = gc.v_abs_error(Ut.shape[0])
    ref = orc.project(Z, Ut)
    tol = d + (U32 * np.abs(ref) if prec != "fp64" else 0.0)
    assert V.shape == ref.shape, what
    assert np.all(np.abs(V - ref) <= tol), (what, float(np.max(np.abs(V - ref))))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_path_factors(orc, prec):
    ci = inputs.small_gaussian_sum(0)                      # n=64, R=200, eps=1e-6
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    g = gc.run_gpu(ci, prec)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    assert g["ranks"] == tuple(o.ranks)
    for l in range(3):
        check_v(orc, Ut[l], g["Z"][l], g["V"][l], prec, f"mode {l}")
        # rows of well-separated singular vectors equal the oracle's own V rows
        sep = gc.separated(o.sigma[l], o.ranks[l])
        assert len(sep) > o.ranks[l] // 2
        sgn = gc.align_signs(g["Z"][l][:, sep], o.Z[l][:, sep])
        assert np.allclose(g["V"][l][sep] * sgn[:, None], o.V[l][sep], atol=1e-9)
    # the mixed format itself: A_r = sum_nu xi'_nu (Z1 V1[:,nu]) (x) (Z2 V2[:,nu]) (x) (Z3 V3[:,nu])
    A = orc.full_tensor(Ut, xip)
    W = [g["Z"][l] @ g["V"][l] for l in range(3)]
    Ar = np.einsum("k,ik,jk,lk->ijl", g["xip"], W[0], W[1], W[2], optimize=True)
    a = float(np.linalg.norm(A.ravel()))
    err = float(np.linalg.norm((A - Ar).ravel()))
    assert err <= g["report"]["bound"] * (1 + 1e-9) + (1e-12 if prec == "fp64" else 1e-6) * a
    assert err <= (ci.eps + 1e-6) * a


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_batched_factors_without_core(orc, prec):
    """Batched, V outputs with beta NULL (the core is skipped): every problem's V
    against the oracle's projection of its Z, and the single path's V."""
    import torch
    from paper_2201_12663_amd import rhosvd
    shapes = [("gauss", 48, 150), ("newton", 64, 200), ("gauss", 100, 333), ("newton", 72, 40), ("gauss", 130, 90)]
    cis = [inputs.small_gaussian_sum(seed=100 + i, n=n, R=R) if k == "gauss" else
           inputs.batch_problem(seed=7, index=i, n=n, R=R, eps=1e-5) for i, (k, n, R) in enumerate(shapes)]
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision=prec)
    res = torch.zeros((len(cis), 8), dtype=torch.int32, device="cuda")
    outs, vouts, caps = [], [], []
    for ci in cis:
        cap = min(ci.n, ci.R)
        caps.append(cap)
        outs.append(tuple(rhosvd.colmajor_empty(ci.n, cap) for _ in range(3)) + (None,))
        vouts.append(tuple(rhosvd.colmajor_empty(cap, ci.R).fill_(7.0) for _ in range(3)))
    desc = red.batch_descriptors(probs, res, outputs=outs, v_outputs=vouts)
    red.reduce_batched_raw(desc)
    torch.cuda.synchronize()
    rr = res.cpu().numpy()
    single = rhosvd.Reducer(precision=prec, anorm="exact", refine_tails="off")
    for i, ci in enumerate(cis):
        assert rr[i, 3] == 0, (ci.name, rr[i])
        r = [int(x) for x in rr[i, :3]]
        Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
        single.reduce(*probs[i])
        for l in range(3):
            Z = outs[i][l][:, :r[l]].cpu().numpy()
            V = vouts[i][l][:r[l]].cpu().numpy()
            check_v(orc, Ut[l], Z, V, prec, f"{ci.name} mode {l}")
            assert torch.all(vouts[i][l][r[l]:] == 7.0)          # rows beyond the rank untouched
            Vs = single.V(l).cpu().numpy()
            if Vs.shape == V.shape:
                assert np.allclose(V, Vs, atol=1e-10), (ci.name, l)
    red.close()
    single.close()
