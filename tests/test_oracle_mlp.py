"""Pins of the FP64 oracle of the rank-proposal network: the back-propagated
gradient against central finite differences of the loss (the definition of the
derivative), closed forms of the loss and of the first Adam step, the features'
definition on a sketch with known singular values, and planted mistakes that
these pins catch."""
import numpy as np
import pytest

from oracle import mlp

SMALL = [(5, 4), (6, 5), (2, 6)]      # same structure as the network, small enough for differences


def fd_grad(p, X, T, idx, sizes, h=1e-6):
    out = []
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        out.append((mlp.loss(p + e, X, T, sizes) - mlp.loss(p - e, X, T, sizes)) / (2 * h))
    return np.array(out)


def test_param_count_matches_layout():
    assert mlp.N_PARAMS == 128 * 67 + 128 + 128 * 128 + 128 + 2 * 128 + 2 == 25474
    p = mlp.init_params(0)
    assert p.size == mlp.N_PARAMS
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(p)
    assert W1.shape == (128, 67) and W2.shape == (128, 128) and W3.shape == (2, 128)


def test_gradient_matches_finite_differences():
    g = np.random.default_rng(3)
    sizes = SMALL
    p = mlp.init_params(1, sizes) + 0.05 * g.standard_normal(sum(o * i + o for o, i in sizes))
    X = g.standard_normal((7, 4))
    T = g.standard_normal((7, 2))
    L, G = mlp.loss_and_grad(p, X, T, sizes)
    assert abs(L - mlp.loss(p, X, T, sizes)) <= 1e-15 * max(1.0, L)
    idx = np.arange(p.size)
    fd = fd_grad(p, X, T, idx, sizes)
    assert np.allclose(G, fd, rtol=1e-6, atol=1e-9)


def test_gradient_full_size_on_sampled_coordinates():
    g = np.random.default_rng(4)
    p = mlp.init_params(2)
    X = g.standard_normal((9, 67))
    T = g.standard_normal((9, 2))
    _, G = mlp.loss_and_grad(p, X, T)
    idx = g.choice(p.size, size=60, replace=False)
    assert np.allclose(G[idx], fd_grad(p, X, T, idx, mlp.SIZES), rtol=1e-5, atol=1e-8)


def test_zero_weights_closed_form():
    """With every weight zero the output is b3 for every sample: L = mean |b3 - t|^2 / 2
    and dL/db3 = mean(b3 - t); every other gradient entry is zero."""
    p = np.zeros(mlp.N_PARAMS)
    p[-2:] = [0.5, -1.5]
    X = np.random.default_rng(5).standard_normal((4, 67))
    T = np.array([[1.0, 0.0], [0.0, 1.0], [2.0, -2.0], [0.5, 0.5]])
    L, G = mlp.loss_and_grad(p, X, T)
    d = np.array([0.5, -1.5]) - T
    assert abs(L - 0.5 * np.sum(d ** 2) / 4) <= 1e-15
    assert np.allclose(G[-2:], d.mean(axis=0), rtol=0, atol=1e-15)
    assert np.all(G[:-2] == 0.0)


def test_first_adam_step_moves_by_lr_times_sign():
    """With bias correction the first Adam step is lr * g / (|g| + eps)."""
    g = np.array([3.0, -2.0, 1e-3, 0.0])
    p, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_sketch_features_of_known_spectrum():
    """Ut with orthonormal columns scaled by known singular values and Omega = I
    (R = 32): the features are log10(s_k / s_1) / 16 of those values."""
    n, R = 40, 32
    q, _ = np.linalg.qr(np.random.default_rng(6).standard_normal((n, R)))
    s = np.logspace(0, -20, R)
    U = q * s
    F = mlp.sketch_features([U, U, U], np.eye(R), n, R, 1e-5)
    want = np.maximum(np.log10(s / s[0]) / 16.0, -1.0)
    for l in range(3):
        assert np.allclose(F[l, :32], want, atol=1e-6)
        assert np.all(F[l, 32:64] == 0.0)
        assert np.allclose(F[l, 64:], [np.log(n) / 10, np.log(R) / 10, np.log(1e-5) / 10])


def test_planted_mistakes_are_caught(monkeypatch):
    """A backward pass without the ReLU mask, or with the weight gradient
    transposed in the batch sum, fails the finite-difference pin."""
    g = np.random.default_rng(7)
    sizes = SMALL
    p = mlp.init_params(3, sizes) + 0.1 * g.standard_normal(sum(o * i + o for o, i in sizes))
    X = g.standard_normal((6, 4))
    T = g.standard_normal((6, 2))
    fd = fd_grad(p, X, T, np.arange(p.size), sizes)

    def no_mask(p, X, T, sizes=mlp.SIZES):
        B = X.shape[0]
        layers = mlp.unpack(np.asarray(p, dtype=np.float64), sizes)
        Y, Zs, Hs = mlp.forward(p, X, sizes)
        grads = [None] * len(layers)
        dZ = (Y - T) / B
        for l in range(len(layers) - 1, -1, -1):
            W, _ = layers[l]
            grads[l] = (dZ.T @ Hs[l], dZ.sum(axis=0))
            if l > 0:
                dZ = dZ @ W                       # mistake: ReLU mask dropped
        return 0.0, np.concatenate([np.concatenate([a.ravel(), b]) for a, b in grads])

    _, Gbad = no_mask(p, X, T, sizes)
    assert not np.allclose(Gbad, fd, rtol=1e-6, atol=1e-9)
    _, G = mlp.loss_and_grad(p, X, T, sizes)
    Gbad2 = G.copy()
    Gbad2[:20] = G[:20].reshape(5, 4).T.ravel()[:20]      # W1 gradient transposed
    assert not np.allclose(Gbad2, fd, rtol=1e-6, atol=1e-9)
