"""The uneven batch at its own shape: J1-J2 (J2 = 0.5) lattices of 8x8, 12x12 and
16x16 at D=8, Dc=16 in one persistent launch per sweep (vp_sample_batch).

* float64, one chain per lattice: every decision, E_loc and log|Psi| of the
  batched sweep against the oracle's chain of the 8x8 lattice (the larger two
  are checked against themselves run alone, below, and their fixed
  configurations against the oracle in tests/test_gpu_fullsize.py);
* VP_BF16 with 1024 chains per lattice (the workload's size): the batched
  sweeps produce, lattice by lattice, the same chains bit for bit as each
  lattice sampled alone with the same persistent kernel, and finite outputs.
"""
import numpy as np
import pytest

from oracle import lattice as olat
from oracle import vmc
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = (8, 12, 16)
D, DC, J2 = 8, 16, 0.5


def _B():
    from paper_1908_09359_amd import binding
    return binding


def _bufs(torch, n, nm, N, np_half, dt):
    dev = torch.device("cuda")
    return dict(log_abs_psi=torch.empty(n * nm, dtype=torch.float64, device=dev),
                sign=torch.empty(n * nm, dtype=torch.int8, device=dev),
                e_loc=torch.empty(n * nm, dtype=torch.float64, device=dev),
                dlnpsi=torch.empty((n * nm, np_half), dtype=dt, device=dev) if np_half else None,
                spins_out=torch.empty((n * nm, N), dtype=torch.int8, device=dev))


def _context(B, torch, prec, n, seed):
    ctx = B.Context([B.lattice(L, L, D, DC, 1.0, J2, prec, n) for L in SIZES], seed=seed)
    dev = torch.device("cuda")
    Ts = []
    for i, L in enumerate(SIZES):
        T = W.random_tensors(L, L, D, seed=400 + L)
        Ts.append(T)
        ctx.vp_set_tensors(i, torch.tensor(T, dtype=torch.float64, device=dev))
        ctx.vp_init_chains(i, None)
        ctx.vp_set_schedule(i, B.VP_SCHED_PERSISTENT)
    return ctx, Ts


def test_batch_fp64_matches_oracle_chain():
    import torch
    B = _B()
    seed, nm = 31, 1
    print("uneven batch 8x8 + 12x12 + 16x16 J2=0.5 D=8 Dc=16 fp64, 1 chain each", flush=True)
    ctx, Ts = _context(B, torch, B.VP_FP64, 1, seed)
    outs = [_bufs(torch, 1, nm, L * L, 0, torch.float64) for L in SIZES]
    ctx.vp_sample_batch([0, 1, 2], 0, nm, outs)
    ctx.vp_sync()
    L = SIZES[0]
    lat = olat.Lattice(L, L, D, DC, J2=J2)
    ch = vmc.Chain(lat, olat.neel_shuffled(lat, seed, 0, 0), seed, 0, 0)
    o = vmc.run_chain(Ts[0], lat, ch, 0, nm)[0]
    assert np.array_equal(outs[0]["spins_out"][0].cpu().numpy(), o["spins"])
    assert abs(outs[0]["e_loc"][0].item() - o["e_loc"]) / (L * L) <= 1e-10
    assert abs(outs[0]["log_abs_psi"][0].item() - o["log_abs_psi"]) <= 1e-10 * max(1.0, abs(o["log_abs_psi"]))
    for b in outs[1:]:
        assert np.isfinite(b["e_loc"].cpu().numpy()).all()
    ctx.close()


def test_batch_bf16_1024_chains_equals_each_lattice_alone():
    import torch
    B = _B()
    seed, n, nm = 32, 1024, 2
    print("uneven batch 8x8 + 12x12 + 16x16 J2=0.5 D=8 Dc=16 bf16, 1024 chains each, 2 sweeps", flush=True)
    ctx, _ = _context(B, torch, B.VP_BF16, n, seed)
    outs = [_bufs(torch, n, nm, L * L, 0, torch.float64) for L in SIZES]
    ctx.vp_sample_batch([0, 1, 2], 0, nm, outs)
    ctx.vp_sync()
    batched = [{k: v.cpu().numpy() for k, v in b.items() if v is not None} for b in outs]
    ctx.close()
    del outs
    torch.cuda.empty_cache()
    for i, L in enumerate(SIZES):
        print(f"  {L}x{L} alone", flush=True)
        ctx, _ = _context(B, torch, B.VP_BF16, n, seed)
        b = _bufs(torch, n, nm, L * L, 0, torch.float64)
        ctx.vp_sample(i, 0, nm, b["log_abs_psi"], b["sign"], b["e_loc"], None, b["spins_out"])
        ctx.vp_sync()
        assert np.array_equal(b["spins_out"].cpu().numpy(), batched[i]["spins_out"]), L
        assert np.array_equal(b["e_loc"].cpu().numpy(), batched[i]["e_loc"]), L
        assert np.array_equal(b["log_abs_psi"].cpu().numpy(), batched[i]["log_abs_psi"]), L
        assert np.isfinite(batched[i]["e_loc"]).all()
        ctx.close()
        del b
        torch.cuda.empty_cache()
