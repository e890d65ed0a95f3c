"""GPU: the allocation-free projection adjoint (phx_project_adjoint_dev_noalloc) against the
allocating one (phx_project_adjoint_dev), through the C ABI.

Two calls in a row, the second with a smaller design (the scratch array keeps the first
call's contents), each bit-identical to the allocating call (the same kernels on the same
inputs); the library holds no workspace after the allocation-free calls on a fresh context
and torch's allocator is untouched by them; sizes beyond the scratch are rejected.
"""
import numpy as np
import pytest

from paper_1603_06855_amd import phx

pytestmark = pytest.mark.gpu


def test_noalloc_projection_adjoint_matches_the_allocating_call():
    import torch
    dev = torch.device("cuda:0")
    cases = [(64, 2, 2.8, 4.0, False), (32, 2, 2.8, 16.0, True), (18, 1, 1.6, 1.0, False)]
    rng = np.random.default_rng(17)
    inputs = []
    for nv, sp, r, beta, oct_ in cases:
        p = phx.projection(nv, sp, r, beta, oct_)
        nx = phx.projection_size(p)
        x = torch.from_numpy(rng.random(nx)).to(dev)
        g = torch.from_numpy(rng.standard_normal(nv ** 3)).to(dev)
        out = torch.full((nx,), float("nan"), dtype=torch.float64, device=dev)
        inputs.append((p, x, g, out))
    torch.cuda.synchronize()
    with phx.Context(0) as ctx:
        before = torch.cuda.memory_allocated(dev)
        for p, x, g, out in inputs:  # largest first, then smaller ones
            ctx.project_adjoint_dev_noalloc(p, x, g, out)
        torch.cuda.synchronize()
        assert ctx.stat("mem_bytes") == 0
        assert torch.cuda.memory_allocated(dev) == before
        for p, x, g, out in inputs:
            ref = ctx.project_adjoint_dev(p, x, g)
            assert torch.isfinite(out).all()
            assert torch.equal(out, ref), (p.nv, p.spacing, p.octant)
        # again, in the other order, into the same outputs
        for p, x, g, out in reversed(inputs):
            out.fill_(float("nan"))
            ctx.project_adjoint_dev_noalloc(p, x, g, out)
            torch.cuda.synchronize()
            assert torch.equal(out, ctx.project_adjoint_dev(p, x, g))
        # beyond the scratch: rejected before any device work
        p = phx.projection(66, 2, 2.8, 1.0, False)
        x = torch.zeros(phx.projection_size(p), dtype=torch.float64, device=dev)
        g = torch.zeros(66 ** 3, dtype=torch.float64, device=dev)
        with pytest.raises(phx.PhxError) as e:
            ctx.project_adjoint_dev_noalloc(p, x, g, torch.empty_like(x))
        assert e.value.code == phx.EINVAL and "64" in e.value.msg
