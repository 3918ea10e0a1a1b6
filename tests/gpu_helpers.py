"""Helpers for the GPU parity tests: run the HIP library through its C ABI on
torch-allocated device buffers, and the oracle on the same inputs."""
import numpy as np

from oracle import lattice as olat
from oracle import vmc


def n_pairs(Ly, Lx, J2, geometry=0):
    diag = J2 != 0.0 or geometry == 1
    n = Ly * (Lx - 1) + (Ly - 1) * Lx + (2 * (Ly - 1) * (Lx - 1) if diag else 0)
    if geometry == 1 and J2 != 0.0:
        n += (Ly - 1) * max(Lx - 2, 0) + max(Ly - 2, 0) * (Lx - 1)
    return n


def gpu_eval(Ly, Lx, D, Dc, J2, prec, T, cfgs, n_chains=None, compress=0, fit_sweeps=0, geometry=0):
    import torch
    from paper_1908_09359_amd import binding as B
    n = len(cfgs)
    lat = B.lattice(Ly, Lx, D, Dc, 1.0, J2, prec, n_chains or n, compress, fit_sweeps, geometry)
    ctx = B.Context(lat, seed=1)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    sp = torch.tensor(np.asarray(cfgs), dtype=torch.int8, device=dev)
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    dt = torch.float32 if prec == B.VP_FP32 else torch.float64
    dl = torch.empty((n, ctx.num_params() // 2), dtype=dt, device=dev)
    ra = torch.empty((n, n_pairs(Ly, Lx, J2, geometry)), dtype=torch.float64, device=dev)
    ctx.vp_eval(0, sp, n, lp, sg, el, dl, ra)
    torch.cuda.synchronize()
    out = dict(log_abs_psi=lp.cpu().numpy(), sign=sg.cpu().numpy(), e_loc=el.cpu().numpy(),
               dlnpsi=dl.double().cpu().numpy(), ratios=ra.cpu().numpy())
    ctx.close()
    return out


def oracle_eval(Ly, Lx, D, Dc, J2, T, cfgs, compress_mode="canonical", fit_sweeps=2, geometry=0):
    lat = olat.Lattice(Ly, Lx, D, Dc, J2=J2, compress_mode=compress_mode, fit_sweeps=fit_sweeps,
                       geometry=("square", "triangular")[geometry])
    outs = [vmc.eval_config(T, lat, c) for c in cfgs]
    return dict(log_abs_psi=np.array([o["log_abs_psi"] for o in outs]),
                sign=np.array([o["sign"] for o in outs]),
                e_loc=np.array([o["e_loc"] for o in outs]),
                dlnpsi=np.stack([o["dlnpsi"] for o in outs]),
                ratios=np.stack([o["ratios"] for o in outs]))
