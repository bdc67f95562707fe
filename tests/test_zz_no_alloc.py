"""GPU test of rhosvd_t2c_noalloc (include/rhosvd.h) through the C-ABI: the
one-call Tucker-to-canonical transform that allocates nothing (its workspace is
a static device array) gives the handle path's results (rhosvd_t2c +
rhosvd_t2c_get) bit for bit, on two calls in a row, the second with a smaller
core; the capacity status and the size limit."""
import numpy as np
import pytest

from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu


def fortran_dev(beta):
    import torch
    r1, r2, r3 = beta.shape
    flat = torch.from_numpy(np.asfortranarray(beta).ravel(order="F")).cuda()
    return flat.view(r3, r2, r1).permute(2, 1, 0)


def core(seed, shape, eps):
    """slices with singular values well above and well below the threshold"""
    from oracle import t2c as ot
    r1, r2, r3 = shape
    thr = ot.t2c_threshold(eps, r1, r2, r3)
    g = np.random.default_rng(seed)
    k = min(r1, r2)
    spectra = []
    for m in range(r3):
        q = int(g.integers(0, k + 1))
        spectra.append(np.concatenate([np.geomspace(2.0, 1e-5, q), np.geomspace(thr / 10, thr / 1e3, k - q)]))
    return inputs.core_with_slice_spectra(seed, r1, r2, r3, spectra)


def noalloc(beta_d, eps, cap, fill=0.0):
    import torch
    from paper_2201_12663_amd import rhosvd
    r1, r2, r3 = beta_d.shape
    w = torch.full((max(cap, 1),), fill, dtype=torch.float64, device="cuda")
    F1 = rhosvd.colmajor_empty(r1, max(cap, 1)).fill_(fill)
    F2 = rhosvd.colmajor_empty(r2, max(cap, 1)).fill_(fill)
    sl = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    R = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    bound = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    rc = rhosvd.t2c_noalloc(beta_d, eps, cap, w, F1, F2, sl, R, bound, status)
    torch.cuda.synchronize()
    return rc, dict(R=int(R.item()), bound=float(bound.item()), status=int(status.item()), weights=w, F1=F1, F2=F2,
                    slice=sl)


def test_noalloc_matches_the_handle_path_twice():
    import torch
    from paper_2201_12663_amd import rhosvd
    eps = 1e-6
    red = rhosvd.Reducer()
    for seed, shape in ((1, (48, 40, 30)), (2, (20, 13, 9))):      # the second call smaller
        beta_d = fortran_dev(core(seed, shape, eps))
        ref = red.t2c(beta_d, eps)
        torch.cuda.synchronize()
        cap = shape[2] * min(shape[0], shape[1])
        rc, got = noalloc(beta_d, eps, cap)
        print(shape, "R", got["R"], "handle path R", ref["R"], flush=True)
        assert rc == 0 and got["status"] == 0
        assert got["R"] == ref["R"] > 0
        assert got["bound"] == ref["bound"]
        R = ref["R"]
        assert torch.equal(got["weights"][:R], ref["weights"])
        assert torch.equal(got["F1"][:, :R], ref["F1"])
        assert torch.equal(got["F2"][:, :R], ref["F2"])
        assert torch.equal(got["slice"][:R], ref["slice"])
    red.close()


def test_noalloc_capacity_and_limits():
    import torch
    eps = 1e-6
    beta_d = fortran_dev(core(3, (16, 16, 8), eps))
    rc, full = noalloc(beta_d, eps, 8 * 16)
    assert rc == 0 and full["status"] == 0 and full["R"] > 4
    rc, got = noalloc(beta_d, eps, 4, fill=7.0)
    assert rc == 0 and got["status"] == -8 and got["R"] == full["R"]
    assert torch.all(got["weights"] == 7.0) and torch.all(got["F1"] == 7.0)
    # 128^3: the Jacobi fits one workgroup's LDS, but not the 8 MiB scratch
    rc, _ = noalloc(fortran_dev(np.zeros((128, 128, 128))), eps, 1)
    assert rc == -7
    rc, _ = noalloc(beta_d, -1.0, 8)
    assert rc == -1
