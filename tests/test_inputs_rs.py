"""CPU checks of the range-separated workload generators (Section 4): the
sinc-quadrature Gaussian sums approximate their radial functions on the grid,
the long-range split keeps exactly the terms with t_k <= 1 (eq. eqn:RS_repres),
the Hadamard cube's columns are the Gaussians with summed exponents (the
product identity of Lemma 4.3's proof), and the multi-Slater sum has N R_l terms
whose full tensor matches the direct sum of Slater functions at sample points."""
import math

import numpy as np

from paper_2201_12663_amd import inputs


def test_newton_sinc_sum_and_split():
    t, w, info = inputs.newton_sinc_terms(19, 257)
    assert len(t) == 19 and np.all(w > 0)
    assert int(np.sum(t <= 1.0)) == 10                 # R_l = 10 of R = 19, as in Section 5
    z = np.geomspace(0.2, 30.0, 50)
    approx = (w[None, :] * np.exp(-z[:, None] ** 2 * t[None, :] ** 2)).sum(axis=1)
    assert np.max(np.abs(approx * z - 1.0)) <= 0.02
    assert info["rel_err"] <= 0.02


def test_newton_cubed_is_the_pointwise_cube():
    ci = inputs.newton_cubed(n=33, R=7, b=5.0)
    V, w, _ = inputs.newton_kernel(33, 7, 5.0)
    t, _, _ = inputs.newton_sinc_terms(7, 33, 5.0)
    assert ci.R == 343
    x = inputs.collocation_grid(33, 5.0)
    a, b, c = 2, 5, 6
    col = ci.U[0][:, a * 49 + b * 7 + c]
    assert np.allclose(col, np.exp(-(t[a] ** 2 + t[b] ** 2 + t[c] ** 2) * x ** 2), rtol=1e-13, atol=1e-300)
    assert ci.xi[a * 49 + b * 7 + c] == w[a] * w[b] * w[c]
    # the full tensor is the cube of the kernel's, entry by entry
    P = np.einsum("k,ik,jk,lk->ijl", w, V, V, V)
    idx = (3, 17, 29)
    val = sum(ci.xi[k] * ci.U[0][idx[0], k] * ci.U[1][idx[1], k] * ci.U[2][idx[2], k] for k in range(ci.R))
    assert math.isclose(val, P[idx] ** 3, rel_tol=1e-12)
    lr = inputs.newton_cubed(n=33, R=7, b=5.0, long_range=True)
    assert lr.R == int(np.sum(t <= 1.0)) ** 3


def test_slater_sum_and_lattice():
    lam = 0.5
    tau, w, info = inputs.slater_sinc_terms(lam, 8, 3, 384)
    assert int(np.sum(tau <= 1.0)) == 3
    rho = np.geomspace(1e-2, 300.0, 60)
    approx = (w[None, :] * np.exp(-rho[:, None] * tau[None, :])).sum(axis=1)
    assert np.max(np.abs(approx - np.exp(-lam * np.sqrt(rho)))) <= 0.01
    ci = inputs.multi_slater((3, 2, 2), n=40, long_range=False)
    N = 12
    assert ci.R == N * 8
    nodes, c = ci.meta["nodes"], ci.meta["c"]
    assert nodes.shape == (N, 3) and np.all(np.abs(c) <= 5.0)
    x = inputs.collocation_grid(40, 10.0)
    for i, j, k in [(3, 20, 37), (19, 21, 18)]:
        val = float(np.sum(ci.xi * ci.U[0][i] * ci.U[1][j] * ci.U[2][k]))
        p = np.array([x[i], x[j], x[k]])
        direct = sum(c[q] * float((w * np.exp(-tau * np.sum((p - nodes[q]) ** 2))).sum()) for q in range(N))
        assert math.isclose(val, direct, rel_tol=1e-10, abs_tol=1e-12)
    f = inputs.multi_slater((4, 4, 4), n=32, amplitudes="function")
    assert f.R == 64 * 3
    assert np.allclose(f.meta["c"], inputs.slater_amplitude_function(f.meta["nodes"]))
