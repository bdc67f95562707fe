"""The caller's allocator (rhosvd_create_with_allocator) through the C-ABI: with
PyTorch's caching allocator the handle's workspace (single path and batch plan)
is counted by torch.cuda.memory_allocated and returned on close, and the results
equal those of a handle on hipMalloc bit for bit."""
import numpy as np
import pytest

from paper_2201_12663_amd import inputs

pytestmark = pytest.mark.gpu


def test_workspace_comes_from_the_torch_allocator():
    import torch
    from paper_2201_12663_amd import rhosvd
    ci = inputs.newton_centres(2, n=160, n_centres=20, eps=1e-5)
    U = [rhosvd.to_device(u) for u in ci.U]
    xi = torch.from_numpy(ci.xi).cuda()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    a = rhosvd.Reducer(precision="fp32", torch_allocator=True)
    ra = a.reduce(U[0], U[1], U[2], xi, ci.eps)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - base
    n_pad, R_pad = 192, 640
    print("workspace through torch:", grown, "bytes", flush=True)
    assert grown >= 3 * n_pad * R_pad * 8           # at least the normalized side matrices
    res_a = a.get()
    b = rhosvd.Reducer(precision="fp32", torch_allocator=False)
    rb = b.reduce(U[0], U[1], U[2], xi, ci.eps)
    res_b = b.get()
    torch.cuda.synchronize()
    assert ra == rb
    assert torch.equal(res_a.beta, res_b.beta)
    for l in range(3):
        assert torch.equal(res_a.Z[l], res_b.Z[l])
    # the batch plan's workspace too
    before = torch.cuda.memory_allocated()
    out, desc, res, outs = a.reduce_batched([(U[0], U[1], U[2], xi, ci.eps)])
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before > 3 * n_pad * R_pad * 8
    assert out[0]["ranks"] == tuple(ra)
    del out, desc, res, outs, res_a, res_b
    a.close()
    b.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= base + 4096
