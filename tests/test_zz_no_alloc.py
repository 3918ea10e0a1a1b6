"""The allocation-free forward pass of the proposal network
(vp_proposal_forward_noalloc) against vp_proposal_forward through the C ABI:
the same kernels on the static device scratch must give the same logits bit
for bit, on two calls in a row (the second with fewer configurations, so that
stale activations of the first call would show), and a batch beyond the
scratch is rejected on the host before anything is launched."""
import numpy as np
import pytest

from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_forward_matches_the_allocating_one():
    import torch
    from paper_1908_09359_amd import binding as B
    Ly, Lx, n_max = 16, 16, 168          # 168 * 256 * 97 floats fit the 4 Mi-float scratch
    print("no-alloc proposal forward 16x16: n = 168, then n = 37", flush=True)
    dev = torch.device("cuda")
    ctx = B.Context(B.lattice(Ly, Lx, 2, 4, 1.0, 0.0, B.VP_FP32, n_max + 1), seed=3)
    w = torch.tensor(W.random_proposal_weights(seed=11, scale=0.2, bias=0.3), device=dev)
    ctx.vp_proposal_set_weights(0, w)
    for n, seed in ((n_max, 5), (37, 6)):
        sp = torch.tensor(W.random_configs(Ly, Lx, n, seed=seed), dtype=torch.int8, device=dev)
        ref = torch.full((n, Ly, Lx), float("nan"), dtype=torch.float32, device=dev)
        got = torch.full((n, Ly, Lx), float("nan"), dtype=torch.float32, device=dev)
        ctx.vp_proposal_forward(0, sp, n, ref)
        ctx.vp_proposal_forward_noalloc(0, sp, n, got)
        torch.cuda.synchronize()
        assert torch.isfinite(ref).all()
        assert torch.equal(got, ref), (n, float((got - ref).abs().max()))
        # the logits depend on the configuration (not a constant map)
        assert float(ref.std()) > 1e-3
    too_many = torch.zeros((n_max + 1, Ly * Lx), dtype=torch.int8, device=dev)
    out = torch.empty((n_max + 1, Ly, Lx), dtype=torch.float32, device=dev)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_proposal_forward_noalloc(0, too_many, n_max + 1, out)
    assert ei.value.status == B.VP_ERR_ARG
    ctx.close()
