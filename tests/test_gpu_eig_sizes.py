"""The FP64 eigensolver at every rows-per-thread instance of the
tridiagonalization (m = min(n, R) from 700 to 2000: 3, 5, 6, 7 and 8 rows per
thread; m = 1300 on the R < n side).  The Gram route's singular values are
checked against LAPACK's SVD of the same normalized factor (a library routine
with the same definition, independent of the library under test; the oracle's
Jacobi SVD would take minutes at these sizes), and Z against orthonormality and
the captured energy.  Inputs: dense standard-normal side matrices, whose
spectra sit far above the FP64 Gram route's noise floor."""
import numpy as np
import pytest

from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("n,R", [(700, 760), (1100, 1150), (1300, 1400), (1400, 1300), (1700, 1780),
                                 (2000, 2048)])
def test_gram_eigensolver_at_every_rows_per_thread(orc, n, R):
    import torch
    from paper_2201_12663_amd import rhosvd
    _flush(f"eigensolver sizes: n={n} R={R}")
    ci = inputs.random_dense(5, n, R, eps=1e-3)
    U = [rhosvd.to_device(u) for u in ci.U]
    xd = torch.from_numpy(ci.xi).cuda()
    red = rhosvd.Reducer(precision="fp64", refine_tails="off")   # the eigensolver's own spectrum
    ranks = red.reduce(U[0], U[1], U[2], xd, ci.eps)
    res = red.get(beta=False, sigma=False)
    sig = [red.spectrum(l).cpu().numpy() for l in range(3)]
    Z = [z.cpu().numpy() for z in res.Z]
    torch.cuda.synchronize()
    red.close()
    m = min(n, R)
    Ut, _, _, _ = orc.normalize(ci.U, ci.xi)
    for l in range(3):
        assert sig[l].shape == (m,)
        r = ranks[l]
        orth = float(np.max(np.abs(Z[l].T @ Z[l] - np.eye(r))))
        _flush(f"  mode {l}: rank {r}, Z orthogonality {orth:.2e}")
        assert orth <= 1e-12
    # spectrum and subspace of the first mode (the three are drawn alike)
    ref = np.linalg.svd(Ut[0], compute_uv=False)
    # the Gram route's eigenvalues carry an absolute error of a few u |G|
    err = float(np.max(np.abs(sig[0] ** 2 - ref ** 2))) / ref[0] ** 2
    r = ranks[0]
    captured = float(np.linalg.norm(Z[0].T @ Ut[0]) ** 2)
    energy = float(np.sum(ref[:r] ** 2))
    _flush(f"  mode 0: eigenvalue error {err:.2e} |G|, captured energy rel. diff "
           f"{abs(captured - energy) / energy:.2e}")
    assert err <= 1e-12
    assert abs(captured - energy) <= 1e-12 * energy
