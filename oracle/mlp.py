"""FP64 oracle of the rank-proposal network (test infrastructure only).

Plain numpy, written from the definitions: a multilayer perceptron
    x (67) -> relu(W1 x + b1) (128) -> relu(W2 h1 + b2) (128) -> W3 h2 + b3 (2),
the mean-squared-error loss L = 1/(2B) sum_b sum_o (y_bo - t_bo)^2, its gradient
by the chain rule (back-propagation), Adam (Kingma & Ba, 2015) with bias
correction, and the per-mode sketch features the network reads.

The network is not part of the paper's method: it proposes ranks and sketch
widths for a randomized range finder (Halko, Martinsson & Tropp, 2011) whose
result is certified a posteriori against the truncation threshold.

Parameter vector layout (shared with the library's C-ABI by specification):
W1 (128 x 67, row-major) | b1 | W2 (128 x 128) | b2 | W3 (2 x 128) | b3.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 67, 128, 2
SIZES = [(N_HID, N_IN), (N_HID, N_HID), (N_OUT, N_HID)]
N_PARAMS = sum(o * i + o for o, i in SIZES)
N_SKETCH = 32          # sketch columns; their singular values fill the first 32 features


def unpack(p: np.ndarray, sizes=SIZES):
    """Views (W_l, b_l) of a flat parameter vector."""
    out, k = [], 0
    for o, i in sizes:
        W = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((W, b))
    assert k == p.size
    return out


def init_params(seed: int, sizes=SIZES) -> np.ndarray:
    """He-uniform weights, zero biases (a reproducible starting point)."""
    g = np.random.Generator(np.random.Philox(key=[20, int(seed)]))
    parts = []
    for o, i in sizes:
        lim = np.sqrt(6.0 / i)
        parts.append(g.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def forward(p: np.ndarray, X: np.ndarray, sizes=SIZES):
    """Network output Y (B x out) and the pre-activations of the hidden layers."""
    layers = unpack(np.asarray(p, dtype=np.float64), sizes)
    H = np.asarray(X, dtype=np.float64)
    Zs, Hs = [], [H]
    for l, (W, b) in enumerate(layers):
        Z = H @ W.T + b
        if l + 1 < len(layers):
            Zs.append(Z)
            H = np.maximum(Z, 0.0)
            Hs.append(H)
        else:
            H = Z
    return H, Zs, Hs


def loss(p, X, T, sizes=SIZES) -> float:
    Y, _, _ = forward(p, X, sizes)
    return 0.5 * float(np.sum((Y - T) ** 2)) / X.shape[0]


def loss_and_grad(p, X, T, sizes=SIZES):
    """L and dL/dp by the chain rule, layer by layer from the output back."""
    B = X.shape[0]
    layers = unpack(np.asarray(p, dtype=np.float64), sizes)
    Y, Zs, Hs = forward(p, X, sizes)
    L = 0.5 * float(np.sum((Y - T) ** 2)) / B
    grads = [None] * len(layers)
    dZ = (Y - T) / B                                   # dL/d(output pre-activation)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        Hin = Hs[l]
        grads[l] = (dZ.T @ Hin, dZ.sum(axis=0))        # dL/dW_l, dL/db_l
        if l > 0:
            dH = dZ @ W                                # dL/dH_{l-1}
            dZ = dH * (Zs[l - 1] > 0.0)                # through the ReLU
    return L, np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t = 1, 2, ...): returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def sketch_features(Ut: list, omega: np.ndarray, n: int, R: int, eps: float) -> np.ndarray:
    """Per-mode features (3 x 67) from the Gaussian sketch Y_l = U~_l Omega[:, :32]:
    log10(sigma_k / sigma_1) / 16 for the 32 singular values of Y_l (clamped at
    -1, i.e. 16 decades), 32 zeros, then ln(n)/10, ln(R)/10, ln(eps)/10."""
    F = np.zeros((3, N_IN))
    for l in range(3):
        Y = Ut[l] @ omega[:, :N_SKETCH]
        s = np.linalg.svd(Y, compute_uv=False)
        s1 = s[0] if s.size and s[0] > 0 else 1.0
        with np.errstate(divide="ignore"):
            f = np.log10(np.maximum(s, 0.0) / s1) / 16.0
        F[l, :min(N_SKETCH, s.size)] = np.maximum(f[:N_SKETCH], -1.0)
        if s.size < N_SKETCH:
            F[l, s.size:N_SKETCH] = -1.0
        F[l, 64] = np.log(n) / 10.0
        F[l, 65] = np.log(R) / 10.0
        F[l, 66] = np.log(eps) / 10.0
    return F
