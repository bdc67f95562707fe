"""CPU tests of the element-by-element core check used by the GPU parity tests
(gpu_cases.check_core_slabs): cores formed with the mixed paths' roundings pass
it, and plausible kernel mistakes (a tile edge that drops one K chunk, a wrong
slab, a ragged row off by 2^-15 |xi'|) fail it."""
import numpy as np
import pytest

import gpu_cases as gc
from paper_2201_12663_amd import inputs


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), kept as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def split(x):
    hi = bf16(x)
    lo = bf16((x.astype(np.float32) - hi).astype(np.float32))
    return hi, lo


@pytest.fixture(scope="module")
def case(orc):
    ci = inputs.small_gaussian_sum(3, n=40, R=300, eps=1e-6)
    o = orc.rhosvd(ci.U, ci.xi, ci.eps)
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    V = [orc.project(o.Z[l], Ut[l]) for l in range(3)]
    return ci, o, Ut, xip, V


def mixed_core(V, xip, prec):
    """Slab by slab: x = V1 diag(xi') and y = V2[j2] V3[j3] in float32, products
    of float32 (or of the bf16 hi/lo parts, lo*lo dropped), float32 sums."""
    V1, V2, V3 = [v.astype(np.float32) for v in V]
    x = (V1 * xip.astype(np.float32)[None, :]).astype(np.float32)
    r1, r2, r3 = V1.shape[0], V2.shape[0], V3.shape[0]
    out = np.zeros((r1, r2, r3))
    for j3 in range(r3):
        y = (V2 * V3[j3][None, :]).astype(np.float32)       # r2 x R
        if prec == "fp32":
            out[:, :, j3] = x @ y.T
        else:
            xh, xl = split(x)
            yh, yl = split(y)
            out[:, :, j3] = (xh @ yh.T) + (xh @ yl.T) + (xl @ yh.T)
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_roundings_pass(orc, case, prec):
    ci, o, Ut, xip, V = case
    beta = mixed_core(V, xip, prec)
    w = gc.check_core_slabs(orc, Ut, xip, o.Z, beta, range(beta.shape[2]), prec)
    assert w <= 1.0


def test_exact_core_passes_fp64(orc, case):
    ci, o, Ut, xip, V = case
    w = gc.check_core_slabs(orc, Ut, xip, o.Z, o.beta, range(o.beta.shape[2]), "fp64")
    assert w <= 1e-2


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_planted_core_mistakes_fail(orc, case, prec):
    ci, o, Ut, xip, V = case
    base = o.beta if prec == "fp64" else mixed_core(V, xip, prec)
    r1, r2, r3 = base.shape
    # a tile edge that drops one chunk of 32 terms for the last row of j1
    V1 = V[0].copy()
    V1[r1 - 1, 64:96] = 0.0
    dropped = orc.core([V1, V[1], V[2]], xip)
    b1 = base.copy()
    b1[r1 - 1] = dropped[r1 - 1]
    # a slab written from its neighbour
    b2 = base.copy()
    b2[:, :, r3 - 1] = base[:, :, r3 - 2]
    # the ragged last row off by 2^-15 |xi'|
    b3 = base.copy()
    b3[r1 - 1, :, :] += 2.0 ** -15 * o.xi_norm
    for bad in (b1, b2, b3):
        with pytest.raises(AssertionError):
            gc.check_core_slabs(orc, Ut, xip, o.Z, bad, range(r3), prec)
