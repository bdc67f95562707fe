"""Write the stored expected values for the full-size parity tests.

Every value written here comes from the CPU oracle (oracle/) on inputs from the
seeded generators; nothing is read from the GPU path.

    python tests/golden/make_golden.py newton1024 [seed]
    python tests/golden/make_golden.py hadamard512 [seed]
    python tests/golden/make_golden.py batch [seed]

newton1024: n=1024 grid on [-10,10]^3, R=4096 = 128 random +-1 charges x a
32-term Gaussian sum for 1/|x| (exponents log-spaced in [1e-2, 1e4]), eps=1e-5.
Stores ranks, all singular values per mode, |A|, |xi'|, tau, tails at the cut,
the Theorem 2.3 bound, the exact error (Gram identity) and sampled core entries
at indices whose singular vectors are well separated.

hadamard512: n=512 grid on [-10,10]^3, the pointwise product of two 300-term
Gaussian sums (R = 90000), eps in {1e-4, 1e-6}.  |A| from the product formed on
the grid; per eps the ranks, tau, tails at the cut, the Theorem 2.3 bound, the
exact error of the oracle's reduction against the materialized A, and (eps =
1e-4) sampled core entries.

batch: two problems of the uneven batch (seed 0 of the batch shapes) at their
real sizes, the largest n <= R one (index 58: n=2048, R=7115) and the largest
R < n one (index 179: n=2048, R=2041), each the first R terms of ceil(R/32)
charges x 32 Gaussian terms, eps=1e-5.  Stores what newton1024 stores.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2201_12663_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def separated(sigma, r, rel_gap=1e-4):
    """Indices k < r whose squared singular value is apart from its neighbours
    by more than rel_gap * sigma_1^2 (their singular vectors are well defined)."""
    s2 = sigma ** 2
    out = []
    for k in range(r):
        lo = s2[k - 1] - s2[k] if k > 0 else np.inf
        hi = s2[k] - s2[k + 1] if k + 1 < len(s2) else np.inf
        if min(lo, hi) > rel_gap * s2[0]:
            out.append(k)
    return out


def reduction_record(ci, res, err, sample_seed, per_mode=12):
    """Stored values of one oracle reduction: ranks, norms, tau, tails at the cut,
    the bound, the exact error, every singular value and sampled core entries at
    indices whose singular vectors are well separated."""
    g = np.random.default_rng(sample_seed)
    sep = [separated(res.sigma[l], res.ranks[l]) for l in range(3)]
    picks = [np.sort(g.choice(sep[l], size=min(per_mode, len(sep[l])), replace=False)) for l in range(3)]
    sub = oracle.core([res.V[l][picks[l], :] for l in range(3)], res.xip)
    samples = []
    for a, j1 in enumerate(picks[0]):
        for b, j2 in enumerate(picks[1]):
            for c, j3 in enumerate(picks[2]):
                if (a + b + c) % 7 == 0:
                    samples.append([int(j1), int(j2), int(j3), float(sub[a, b, c])])
    return dict(
        n=ci.n, R=ci.R, eps=ci.eps,
        ranks=list(res.ranks), a_norm=res.a_norm, xi_norm=res.xi_norm, tau=res.tau,
        tail_at_rank=[float(res.tails[l][res.ranks[l]]) for l in range(3)],
        tail_below_rank=[float(res.tails[l][res.ranks[l] - 1]) for l in range(3)],
        bound=res.bound, error=err, sweeps=res.sweeps,
        sigma=[[float(x) for x in res.sigma[l]] for l in range(3)],
        beta_samples=samples,
        z_sign_rule="largest-magnitude entry of each column positive")


def batch(seed=0):
    shapes = inputs.batch_shapes(seed=seed, count=256)
    out = dict(workload="uneven batch, seed %d: the largest n <= R and the largest R < n problem" % seed,
               problems=[])
    for idx in (58, 179):
        n, R = shapes[idx]
        t0 = time.time()
        ci = inputs.batch_problem(seed, idx, n, R)
        res = oracle.rhosvd(ci.U, ci.xi, ci.eps, with_core=False)
        Ut, xip, _, _ = oracle.normalize(ci.U, ci.xi)
        t1 = time.time()
        err = oracle.error_gram(Ut, xip, res.Z)
        t2 = time.time()
        rec = reduction_record(ci, res, err, 1000 + idx)
        rec.update(index=idx, seconds=dict(reduce=t1 - t0, error=t2 - t1))
        out["problems"].append(rec)
        print(idx, (n, R), rec["ranks"], "err/|A|", err / res.a_norm, "secs", rec["seconds"], flush=True)
    path = os.path.join(HERE, f"batch_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


def newton1024(seed=0):
    t0 = time.time()
    ci = inputs.newton_centres(seed)
    res = oracle.rhosvd(ci.U, ci.xi, ci.eps, with_core=False)
    Ut, xip, _, _ = oracle.normalize(ci.U, ci.xi)
    t1 = time.time()
    err = oracle.error_gram(Ut, xip, res.Z)
    t2 = time.time()
    g = np.random.default_rng(1234)
    sep = [separated(res.sigma[l], res.ranks[l]) for l in range(3)]
    picks = [np.sort(g.choice(sep[l], size=min(12, len(sep[l])), replace=False)) for l in range(3)]
    sub = oracle.core([res.V[l][picks[l], :] for l in range(3)], res.xip)
    samples = []
    for a, j1 in enumerate(picks[0]):
        for b, j2 in enumerate(picks[1]):
            for c, j3 in enumerate(picks[2]):
                if (a + b + c) % 7 == 0:
                    samples.append([int(j1), int(j2), int(j3), float(sub[a, b, c])])
    out = dict(
        workload="newton-n1024-R4096", seed=seed, eps=ci.eps,
        ranks=list(res.ranks), a_norm=res.a_norm, xi_norm=res.xi_norm, tau=res.tau,
        tail_at_rank=[float(res.tails[l][res.ranks[l]]) for l in range(3)],
        tail_below_rank=[float(res.tails[l][res.ranks[l] - 1]) for l in range(3)],
        bound=res.bound, error=err, sweeps=res.sweeps,
        sigma=[[float(x) for x in res.sigma[l]] for l in range(3)],
        beta_samples=samples,
        z_sign_rule="largest-magnitude entry of each column positive",
        seconds=dict(reduce=t1 - t0, error=t2 - t1),
    )
    path = os.path.join(HERE, f"newton1024_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["ranks"], "err/|A|", err / res.a_norm, "secs", out["seconds"])


def hadamard512(seed=0):
    t0 = time.time()
    ci = inputs.hadamard_product(seed)
    Ut, xip, _, _ = oracle.normalize(ci.U, ci.xi)
    xi_norm = float(np.linalg.norm(xip))
    a_norm = oracle.anorm_hadamard(ci.meta["factors"])
    svd = [oracle.svd_left(Ut[l]) for l in range(3)]
    sigma = [s for s, _, _ in svd]
    tl = [oracle.tails(s) for s in sigma]
    A = oracle.hadamard_full(ci.meta["factors"])
    t1 = time.time()
    per_eps = []
    for eps in (1e-4, 1e-6):
        tau = oracle.truncation_threshold(eps, a_norm, xi_norm)
        ranks = [oracle.choose_rank(tl[l], tau) for l in range(3)]
        Z = [oracle.sign_normalize(svd[l][1][:, :ranks[l]]) for l in range(3)]
        V = [oracle.project(Z[l], Ut[l]) for l in range(3)]
        beta = oracle.core(V, xip)
        err = oracle.error_dense(A, beta, Z)
        bound = oracle.theorem23_bound(xi_norm, [tl[l][ranks[l]] for l in range(3)])
        entry = dict(eps=eps, tau=tau, ranks=ranks, bound=bound, error=err,
                     beta_norm=float(np.linalg.norm(beta.ravel())),
                     tail_at_rank=[float(tl[l][ranks[l]]) for l in range(3)],
                     tail_below_rank=[float(tl[l][ranks[l] - 1]) for l in range(3)])
        if eps == 1e-4:
            g = np.random.default_rng(4321)
            sep = [separated(sigma[l], ranks[l]) for l in range(3)]
            picks = [np.sort(g.choice(sep[l], size=min(10, len(sep[l])), replace=False)) for l in range(3)]
            samples = []
            for a, j1 in enumerate(picks[0]):
                for b, j2 in enumerate(picks[1]):
                    for c, j3 in enumerate(picks[2]):
                        if (a + 2 * b + c) % 5 == 0:
                            samples.append([int(j1), int(j2), int(j3), float(beta[j1, j2, j3])])
            entry["beta_samples"] = samples
        per_eps.append(entry)
        print(eps, ranks, "err/|A|", err / a_norm, "bound/|A|", bound / a_norm, flush=True)
    t2 = time.time()
    out = dict(
        workload="hadamard-n512-R90000", seed=seed, a_norm=a_norm, xi_norm=xi_norm,
        dropped=int(np.sum(xip == 0.0)), sweeps=[sw for _, _, sw in svd],
        sigma=[[float(x) for x in s] for s in sigma], cases=per_eps,
        z_sign_rule="largest-magnitude entry of each column positive",
        seconds=dict(svd_and_norm=t1 - t0, reductions=t2 - t1),
    )
    path = os.path.join(HERE, f"hadamard512_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["seconds"])


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "newton1024"
    seed = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    {"newton1024": newton1024, "hadamard512": hadamard512, "batch": batch}[which](seed)
