"""GPU parity of the variational boundary fit (VP_COMPRESS_VARIATIONAL, App. B)
against the oracle's fit (``oracle.peps.compress_variational``) through the C ABI.

The fitted state depends on the start and the sweep count, which both sides fix
identically, but not on the QR gauge (pinned in tests/test_oracle_variational.py),
so the GPU's own Householder QR and the oracle's LAPACK QR give the same state
to rounding.  A fixed number of sweeps is a smooth function of the inputs (no
truncation at a nearly degenerate cut decides it), so the small-lattice float64
bounds apply: |dE/site| <= 1e-10, log|Psi| 1e-10, ratios and log-derivatives
1e-9 relative.  float32 (the fit in the working precision): |dE/site| <= 1e-4.
A float64 chain sampled with the fit makes the oracle's decisions bit for bit.
"""
import numpy as np
import pytest

import gpu_helpers as H
from oracle import lattice as olat
from oracle import vmc
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu


def _B():
    from paper_1908_09359_amd import binding
    return binding


def _compare(g, o, N, tol_e, tol_lp, tol_rel):
    assert np.array_equal(g["sign"], o["sign"])
    assert np.max(np.abs(g["log_abs_psi"] - o["log_abs_psi"])) <= tol_lp
    assert np.max(np.abs(g["e_loc"] - o["e_loc"])) / N <= tol_e
    scale = np.maximum(1.0, np.abs(o["ratios"]))
    assert np.max(np.abs(g["ratios"] - o["ratios"]) / scale) <= tol_rel
    for gd, od in zip(g["dlnpsi"], o["dlnpsi"]):
        assert np.max(np.abs(gd - od)) <= tol_rel * max(1.0, np.max(np.abs(od)))


@pytest.mark.parametrize("Ly,Lx,D,Dc,J2,sweeps", [
    (4, 4, 2, 4, 0.0, 1),     # full rank: the fit is exact
    (4, 4, 3, 3, 0.5, 0),     # the start's projection alone
    (4, 4, 3, 3, 0.5, 2),
    (6, 6, 3, 7, 0.5, 1),     # ragged generic shapes
    (1, 4, 3, 2, 0.0, 2),     # a single row
    (4, 1, 3, 2, 0.0, 1),     # a single column
    (6, 6, 4, 8, 0.5, 2),     # fused 3-line steps, D=4 Dc=8
    (6, 6, 8, 16, 0.0, 2),    # fused 3-line steps, D=8 Dc=16, truncated rows
    (4, 6, 6, 12, 0.5, 3),
    (4, 6, 8, 24, 0.5, 2),    # Dc = 3D at D=8: generic steps, the work-group QR (up to 192 x 24)
])
def test_fit_fp64_parity(Ly, Lx, D, Dc, J2, sweeps):
    B = _B()
    print(f"fit fp64 {Ly}x{Lx} D={D} Dc={Dc} J2={J2} sweeps={sweeps}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=300 + Ly * Lx + D)
    cfgs = W.random_configs(Ly, Lx, 2, seed=17)
    g = H.gpu_eval(Ly, Lx, D, Dc, J2, B.VP_FP64, T, cfgs, compress=B.VP_COMPRESS_VARIATIONAL, fit_sweeps=sweeps)
    o = H.oracle_eval(Ly, Lx, D, Dc, J2, T, cfgs, compress_mode="variational", fit_sweeps=sweeps)
    _compare(g, o, Ly * Lx, 1e-10, 1e-10, 1e-9)


def test_fit_at_full_rank_equals_canonical():
    """Dc at the exact rank: both truncations are the exact contraction."""
    B = _B()
    print("fit vs canonical at full rank 4x4 D=2 Dc=4", flush=True)
    T = W.random_tensors(4, 4, 2, seed=41)
    cfgs = W.random_configs(4, 4, 4, seed=42)
    g = H.gpu_eval(4, 4, 2, 4, 0.0, B.VP_FP64, T, cfgs, compress=B.VP_COMPRESS_VARIATIONAL, fit_sweeps=1)
    c = H.gpu_eval(4, 4, 2, 4, 0.0, B.VP_FP64, T, cfgs)
    assert np.max(np.abs(g["e_loc"] - c["e_loc"])) / 16 <= 1e-12
    assert np.max(np.abs(g["log_abs_psi"] - c["log_abs_psi"])) <= 1e-12


@pytest.mark.parametrize("Ly,Lx,D,Dc", [(6, 6, 4, 8), (4, 6, 8, 16), (4, 6, 8, 24)])
def test_fit_fp32_parity(Ly, Lx, D, Dc):
    B = _B()
    print(f"fit fp32 {Ly}x{Lx} D={D} Dc={Dc}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=51)
    cfgs = W.random_configs(Ly, Lx, 3, seed=52)
    g = H.gpu_eval(Ly, Lx, D, Dc, 0.0, B.VP_FP32, T, cfgs, compress=B.VP_COMPRESS_VARIATIONAL, fit_sweeps=2)
    o = H.oracle_eval(Ly, Lx, D, Dc, 0.0, T, cfgs, compress_mode="variational", fit_sweeps=2)
    assert np.array_equal(g["sign"], o["sign"])
    assert np.max(np.abs(g["e_loc"] - o["e_loc"])) / (Ly * Lx) <= 1e-4
    assert np.max(np.abs(g["log_abs_psi"] - o["log_abs_psi"])) <= 1e-4


@pytest.mark.parametrize("Ly,Lx,D,Dc", [(4, 6, 3, 4), (6, 6, 8, 16)])
def test_fit_chain_fp64_bit_exact(Ly, Lx, D, Dc):
    """Sampling with the fit: two chains, one burn-in and two measured sweeps;
    every decision and every measured output against the oracle's chains."""
    import torch
    B = _B()
    print(f"fit chains fp64 {Ly}x{Lx} D={D} Dc={Dc}", flush=True)
    seed, n, nb, nm = 61, 2, 1, 2
    T = W.random_tensors(Ly, Lx, D, seed=62)
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, B.VP_FP64, n, B.VP_COMPRESS_VARIATIONAL, 2), seed=seed)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None)
    lp = torch.empty(n * nm, dtype=torch.float64, device=dev)
    sg = torch.empty(n * nm, dtype=torch.int8, device=dev)
    el = torch.empty(n * nm, dtype=torch.float64, device=dev)
    so = torch.empty((n * nm, Ly * Lx), dtype=torch.int8, device=dev)
    ctx.vp_sample(0, nb, nm, lp, sg, el, None, so)
    ctx.vp_sync()
    lp, el, so = lp.cpu().numpy(), el.cpu().numpy(), so.cpu().numpy()
    ctx.close()
    lat = olat.Lattice(Ly, Lx, D, Dc, compress_mode="variational", fit_sweeps=2)
    for c in range(n):
        ch = vmc.Chain(lat, olat.neel_shuffled(lat, seed, 0, c), seed, 0, c)
        outs = vmc.run_chain(T, lat, ch, nb, nm)
        for m, o in enumerate(outs):
            row = c * nm + m
            assert np.array_equal(so[row], o["spins"]), (c, m)
            assert abs(el[row] - o["e_loc"]) / (Ly * Lx) <= 1e-10
            assert abs(lp[row] - o["log_abs_psi"]) <= 1e-10 * max(1.0, abs(o["log_abs_psi"]))
