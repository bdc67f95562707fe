"""Reductions in flight at once: handles are independent, so host threads and
streams may run them side by side (the benchmark's in-flight modes).  Two host
threads with two handles each, every handle on its own stream, reduce the same
input eight times; every result must equal the one-at-a-time reduction bit for
bit (ranks, Z, beta), for the FP64 and the BF16x3 cores."""
import threading

import numpy as np
import pytest

from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_threads_and_streams_reproduce_the_sequential_reduction(prec):
    import torch
    from paper_2201_12663_amd import rhosvd
    ci = inputs.newton_centres(3, n=384, n_centres=40, eps=1e-5)
    print(f"concurrency {prec}: n={ci.n} R={ci.R}", flush=True)
    U = [rhosvd.to_device(u) for u in ci.U]
    xi = torch.from_numpy(np.ascontiguousarray(ci.xi)).cuda()
    ref = rhosvd.Reducer(precision=prec)
    r0 = ref.reduce(U[0], U[1], U[2], xi, ci.eps)
    res0 = ref.get()
    torch.cuda.synchronize()
    Z0 = [z.cpu().numpy() for z in res0.Z]
    b0 = res0.beta.cpu().numpy()
    ref.close()
    T, H, N = 2, 2, 4
    reds = [[rhosvd.Reducer(precision=prec, stream=torch.cuda.Stream()) for _ in range(H)] for _ in range(T)]
    out, errors = [], []

    def worker(ti):
        try:
            for i in range(N):
                red = reds[ti][i % H]
                r = red.reduce(U[0], U[1], U[2], xi, ci.eps)
                res = red.get()
                red.stream.synchronize()
                out.append((tuple(r), [z.cpu().numpy() for z in res.Z], res.beta.cpu().numpy()))
        except Exception as e:
            errors.append(e)

    ths = [threading.Thread(target=worker, args=(ti,)) for ti in range(T)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    for row in reds:
        for red in row:
            red.close()
    assert not errors, errors
    assert len(out) == T * N
    for r, Z, b in out:
        assert r == tuple(r0)
        for l in range(3):
            assert np.array_equal(Z[l], Z0[l])
        assert np.array_equal(b, b0)


def test_batched_pass_beside_single_reductions():
    """A batched pass (its eigensolver launched without the cooperative guarantee,
    inside a recorded graph) while another host thread runs single reductions on
    another stream: every batched result equals the batch run alone, bit for bit.
    Its workgroups may wait for CUs the other work holds; they wait, they do not
    fail."""
    import torch
    from paper_2201_12663_amd import rhosvd
    shapes = [(160, 640), (72, 40), (200, 257), (256, 1024), (129, 64), (300, 900)]
    cis = [inputs.batch_problem(seed=11, index=i, n=n, R=R, eps=1e-5) for i, (n, R) in enumerate(shapes)]
    probs = []
    for ci in cis:
        U = [rhosvd.to_device(u) for u in ci.U]
        probs.append((U[0], U[1], U[2], torch.from_numpy(np.ascontiguousarray(ci.xi)).cuda(), ci.eps))
    print("batched beside single reductions", flush=True)

    def batch_once(red):
        out, _, _, _ = red.reduce_batched(probs)
        red.stream.synchronize()
        return [(o["status"], tuple(o["ranks"]), [z.cpu().numpy() for z in o["Z"]],
                 None if o["beta"] is None else o["beta"].cpu().numpy()) for o in out]

    alone = rhosvd.Reducer(precision="fp64", stream=torch.cuda.Stream())
    ref = batch_once(alone)
    alone.close()
    ci = inputs.newton_centres(4, n=512, n_centres=40, eps=1e-5)
    U = [rhosvd.to_device(u) for u in ci.U]
    xi = torch.from_numpy(np.ascontiguousarray(ci.xi)).cuda()
    single = rhosvd.Reducer(precision="bf16x3", stream=torch.cuda.Stream())
    batched = rhosvd.Reducer(precision="fp64", stream=torch.cuda.Stream())
    stop, errors, got = threading.Event(), [], []

    def singles():
        try:
            while not stop.is_set():
                r = single.reduce(U[0], U[1], U[2], xi, ci.eps)
                single.get(Z=False, sigma=False)
                single.stream.synchronize()
        except Exception as e:
            errors.append(e)

    def batches():
        try:
            for _ in range(3):
                got.append(batch_once(batched))
        except Exception as e:
            errors.append(e)
        finally:
            stop.set()

    ths = [threading.Thread(target=singles), threading.Thread(target=batches)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    single.close()
    batched.close()
    assert not errors, errors
    for run in got:
        for (s0, r0, Z0, b0), (s1, r1, Z1, b1) in zip(ref, run):
            assert s0 == s1 and r0 == r1
            for l in range(3):
                assert np.array_equal(Z0[l], Z1[l])
            assert (b0 is None and b1 is None) or np.array_equal(b0, b1)
