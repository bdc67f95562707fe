"""Training and evaluation of the rank-proposal network (learned rank proposal
for the randomized range finder of rhosvd_reduce_learned).

Everything numeric runs in the library: features (rhosvd_sketch_features),
labels (the plain method's ranks, rhosvd_reduce), the network's forward and
backward passes and Adam steps (rhosvd_net_*).  This module only draws the
problems, batches the samples and keeps the loop.

Targets per mode (both as fractions of m = min(n, R)): the plain method's rank
r (with the residual-refined cut, so that the labels are not inflated by the
Gram route's FP64 noise floor), and a sketch width p = min(m, ceil(1.1 r) + 16)
that leaves the range finder room to certify.

    python -m paper_2201_12663_amd.ranknet train --problems 768 --out PATH
    python -m paper_2201_12663_amd.ranknet evaluate --params PATH --problems 256
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "ranknet_params.npy")
SKETCH_W = 64          # test-matrix columns for the features


def device_problem(family: str, seed: int, index: int, n: int, R: int, eps: float):
    """One problem of the rank-proposal workloads sampled on the device:
    (U1, U2, U3, xi, eps).  family "newton": the uneven batch's construction;
    "smooth": inputs.smooth_problem_params."""
    import torch
    from . import inputs
    if family == "newton":
        a, c, xi = inputs.batch_problem_params(seed, index, n, R, eps)
    else:
        a, c, xi = inputs.smooth_problem_params(seed, index, n, R)
    U = inputs.gaussian_side_matrices_torch(n, a, c)
    return (U[0], U[1], U[2], torch.from_numpy(np.ascontiguousarray(xi)).cuda(), eps)


def omega_for(seed: int, R: int, w: int):
    import torch
    from . import inputs
    return torch.from_numpy(inputs.gaussian_test_matrix(seed, R, w)).cuda()


def targets(ranks, m: int) -> np.ndarray:
    t = np.zeros((3, 2), dtype=np.float32)
    for l, r in enumerate(ranks):
        p = min(m, math.ceil(1.1 * r) + 16)
        t[l] = (r / m, p / m)
    return t


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases, as float32 (the library's layout)."""
    g = np.random.Generator(np.random.Philox(key=[21, int(seed)]))
    parts = []
    for o, i in [(128, 67), (128, 128), (2, 128)]:
        lim = math.sqrt(6.0 / i)
        parts.append(g.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def dataset(red, shapes, seed: int, log=print):
    """Features and targets of the given problems (3 samples per problem)."""
    import torch
    X, T, meta = [], [], []
    t0 = time.perf_counter()
    for i, (fam, n, R, eps) in enumerate(shapes):
        p = device_problem(fam, seed, i, n, R, eps)
        om = omega_for(seed * 100003 + i, R, SKETCH_W)
        f = red.sketch_features(*p, om)
        r = red.reduce(*p)
        X.append(f.cpu().numpy())
        T.append(targets(r, min(n, R)))
        meta.append((fam, n, R, eps, tuple(r)))
        if (i + 1) % 64 == 0:
            log(f"  dataset: {i + 1}/{len(shapes)} problems, {time.perf_counter() - t0:.1f} s")
        del p, om
    torch.cuda.synchronize()
    return np.concatenate(X), np.concatenate(T), meta


def train(red, X: np.ndarray, T: np.ndarray, epochs: int = 300, lr: float = 1e-3, batch: int = 256, seed: int = 0,
          params: np.ndarray | None = None, log=print):
    """Mini-batch Adam on the library's kernels; returns (params, loss history)."""
    import torch
    red.net_set(torch.from_numpy(init_params(seed) if params is None else params).cuda())
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).cuda()
    g = np.random.Generator(np.random.Philox(key=[22, int(seed)]))
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(g.permutation(X.shape[0])).cuda()
        tot = 0.0
        nb = 0
        for b0 in range(0, X.shape[0], batch):
            idx = perm[b0:b0 + batch]
            xb = Xd.index_select(0, idx).contiguous()
            tb = Td.index_select(0, idx).contiguous()
            loss, _ = red.net_train_step(xb, tb, lr)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        if ep % 50 == 0 or ep == epochs - 1:
            log(f"  epoch {ep}: loss {hist[-1]:.3e}")
    return red.net_get().cpu().numpy(), hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "evaluate"])
    ap.add_argument("--problems", type=int, default=768)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_PARAMS)
    ap.add_argument("--params", default=DEFAULT_PARAMS)
    args = ap.parse_args()
    from . import inputs, rhosvd
    log = lambda m: print(m, file=sys.stderr, flush=True)
    # labels: the plain method with the residual-refined cut (refine_tails), whose
    # ranks are not inflated by the Gram route's FP64 noise floor
    red = rhosvd.Reducer(precision="fp64", refine_tails=True)
    if args.cmd == "train":
        shapes = inputs.ranknet_shapes(args.seed, args.problems)
        X, T, meta = dataset(red, shapes, args.seed, log)
        params, hist = train(red, X, T, epochs=args.epochs, seed=args.seed, log=log)
        np.save(args.out, params)
        print(json.dumps(dict(problems=len(shapes), samples=int(X.shape[0]), final_loss=hist[-1],
                              first_loss=hist[0], out=args.out)))
    else:
        import torch
        params = np.load(args.params)
        red.net_set(torch.from_numpy(params).cuda())
        shapes = inputs.ranknet_shapes(10_000 + args.seed, args.problems)
        X, T, meta = dataset(red, shapes, 10_000 + args.seed, log)
        Y = red.net_forward(torch.from_numpy(X).cuda()).cpu().numpy()
        err = np.abs(Y[:, 0] - T[:, 0])
        print(json.dumps(dict(problems=len(shapes), rank_frac_mae=float(err.mean()),
                              rank_frac_p95=float(np.percentile(err, 95)))))


if __name__ == "__main__":
    main()
