"""Host checks of the seeded input generators shared by the oracle and the HIP path."""
import numpy as np

from paper_2201_12663_amd import inputs


def test_batch_params_and_torch_sampler_reproduce_batch_problem():
    """The parameter-only draw and the torch sampler (used to build large batches
    on the device) give exactly the tensors of batch_problem."""
    for idx, (n, R) in enumerate([(64, 100), (40, 33), (128, 64)]):
        ci = inputs.batch_problem(0, idx, n, R)
        a, c, xi = inputs.batch_problem_params(0, idx, n, R)
        U = inputs.gaussian_side_matrices_torch(n, a, c, device="cpu")
        for l in range(3):
            assert U[l].shape == (n, R) and U[l].stride() == (1, n)
            assert np.array_equal(U[l].numpy(), ci.U[l])
        assert np.array_equal(xi, ci.xi)


def test_batch_shapes_follow_the_recipe():
    shapes = inputs.batch_shapes(seed=0, count=256)
    ns = {n for n, _ in shapes}
    Rs = np.array([R for _, R in shapes])
    assert ns <= {128, 256, 512, 1024, 2048} and len(ns) == 5
    assert Rs.min() >= 64 and Rs.max() <= 8192
    # log-uniform: about half of the R below the geometric midpoint 724
    assert 0.4 < np.mean(Rs < 724) < 0.6
