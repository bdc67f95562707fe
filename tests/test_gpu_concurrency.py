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
