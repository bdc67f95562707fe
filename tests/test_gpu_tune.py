"""GPU tests of the core tile autotuner through the C-ABI: every tile candidate
gives a core within its precision of the oracle's exact core of Z; the tuned
choice is one of the candidates and reproduces that candidate's result bit for
bit, on the single path and in a batch (first run tuned, later runs replayed).
Every case takes eps >= 1e-5, where the BF16x3 core runs (checked through the
report's core_precision)."""
import numpy as np
import pytest

from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp32": 2e-6, "bf16x3": 2.0 ** -15}     # |beta - beta_exact(Z)| / |xi'|
CORE = {"fp64": 0, "fp32": 1, "bf16x3": 2}       # rhosvd_precision of the core


def to_dev(ci):
    import torch
    from paper_2201_12663_amd import rhosvd
    U = [rhosvd.to_device(u) for u in ci.U]
    return (U[0], U[1], U[2], torch.from_numpy(np.ascontiguousarray(ci.xi)).cuda(), ci.eps)


def run_single(ci, prec, tile, repeat=1):
    import torch
    from paper_2201_12663_amd import rhosvd
    red = rhosvd.Reducer(precision=prec, core_tile=tile)
    p = to_dev(ci)
    outs = []
    for _ in range(repeat):
        red.reduce(*p)
        res = red.get(sigma=False)
        torch.cuda.synchronize()
        assert res.report["core_precision"] == CORE[prec]
        outs.append((res.ranks, [z.cpu().numpy() for z in res.Z], res.beta.cpu().numpy(), red.last_core_tile()))
    red.close()
    return outs


def oracle_core_error(orc, ci, Z, beta, prec):
    """Every slab element by element (gpu_cases.check_core_slabs, which asserts)
    and the Frobenius distance from the exact core of Z relative to |xi'|."""
    import gpu_cases as gc
    Ut, xip, _, _ = orc.normalize(ci.U, ci.xi)
    gc.check_core_slabs(orc, Ut, xip, Z, beta, range(beta.shape[2]), prec, what=ci.name)
    be = orc.core([orc.project(Z[l], Ut[l]) for l in range(3)], xip)
    return float(np.linalg.norm((beta - be).ravel())) / float(np.linalg.norm(xip))


CASES = [("newton n160 R640", lambda: inputs.newton_centres(2, n=160, n_centres=20, eps=1e-5)),
         ("gauss n200 R700", lambda: inputs.small_gaussian_sum(4, n=200, R=700, eps=1e-5))]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_every_tile_matches_oracle(orc, prec, tile, name, make):
    ci = make()
    (ranks, Z, beta, used), = run_single(ci, prec, tile)
    assert used == tile
    e = oracle_core_error(orc, ci, Z, beta, prec)
    print(f"{name} {prec} tile {tile}: ranks {ranks} core error {e:.3e} |xi'|", flush=True)
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("tile", [64, 128])
def test_ragged_last_row_block_matches_oracle(orc, prec, tile):
    """r1 = 145: the last row block holds 17 rows (at 64 and at 128 rows per tile).
    With 81 tiles per row block the core stays one launch; the split of such a
    block into 32-row tiles, taken where the launch runs many rounds of workgroups,
    is checked at the full 1024 x 4096 size (test_gpu_parity).  Every slab against
    the oracle's core of the path's own Z."""
    ci = inputs.newton_centres(3, n=200, n_centres=24, eps=1e-4)
    (ranks, Z, beta, used), = run_single(ci, prec, tile)
    assert used == tile
    assert 128 < ranks[0] <= 160, ranks
    e = oracle_core_error(orc, ci, Z, beta, prec)
    print(f"ragged last row block {prec} tile {tile}: ranks {ranks} core error {e:.3e} |xi'|", flush=True)
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_tuned_tile_reproduces_the_candidate(prec):
    ci = CASES[0][1]()
    tuned = run_single(ci, prec, 0, repeat=2)
    t = tuned[0][3]
    assert t in (64, 128)
    assert tuned[1][3] == t                      # the shape class is cached
    (_, _, b_other, t_other), = run_single(ci, prec, 0)
    assert t_other == t                          # and shared with a later handle
    (ranks, Z, beta, used), = run_single(ci, prec, t)
    assert used == t
    for _, _, b, _ in tuned:
        assert np.array_equal(b, beta)
    assert np.array_equal(b_other, beta)


def test_fp64_core_has_one_tile():
    ci = CASES[0][1]()
    (_, _, _, used), = run_single(ci, "fp64", 0)
    assert used == 64
    from paper_2201_12663_amd import rhosvd
    with pytest.raises(rhosvd.RhosvdError):
        rhosvd.Reducer(precision="fp64", core_tile=128)
    with pytest.raises(rhosvd.RhosvdError):
        rhosvd.Reducer(precision="fp32", core_tile=96)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batched_tuning_then_replay(orc, prec):
    """The first batched call of a plan times both tiles on the persistent core
    and records the graph with the winner; the replay gives the same cores, and
    so does a plan with that tile fixed."""
    import torch
    from paper_2201_12663_amd import rhosvd
    cis = [inputs.small_gaussian_sum(seed=30 + i, n=n, R=R, eps=1e-5) for i, (n, R) in
           enumerate([(64, 300), (130, 500), (100, 90), (200, 1200)])]
    probs = [to_dev(ci) for ci in cis]
    red = rhosvd.Reducer(precision=prec)
    out1, desc, res, outs = red.reduce_batched(probs)
    t = red.last_core_tile()
    assert t in (64, 128)
    assert all(o["core_precision"] == CORE[prec] for o in out1)
    first = [o["beta"].clone() for o in out1]
    red.reduce_batched_raw(desc)
    torch.cuda.synchronize()
    assert red.batch_uses_graph()
    assert red.last_core_tile() == t
    for o, b in zip(out1, first):
        assert torch.equal(o["beta"], b)
    fixed = rhosvd.Reducer(precision=prec, core_tile=t)
    out2, _, _, _ = fixed.reduce_batched(probs)
    torch.cuda.synchronize()
    for ci, o, b in zip(cis, out2, first):
        assert torch.equal(o["beta"], b), ci.name
        Z = [z.cpu().numpy() for z in o["Z"]]
        assert oracle_core_error(orc, ci, Z, o["beta"].cpu().numpy(), prec) <= TOL[prec]
    red.close()
    fixed.close()
