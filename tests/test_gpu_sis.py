"""GPU parity of the spin-inversion symmetrised evaluation (Sec. III,
Phi(S) = Psi(S) + Psi(Sbar)) through the C ABI (``vp_eval_sis``).

* Against the oracle (``oracle.sis``, which forms every Phi(S')/Phi(S) from the
  pair ratios of S and Sbar) on exact and truncated networks, the fused D=8,
  Dc=16 shape and float32.  The bounds follow from those of the plain
  evaluation (log|Psi| within t_l, E_loc within t_e per site: 1e-10 and 1e-10 in
  float64, 1e-3 and 1e-4 in float32) through the condition number of the sum,
  kappa = (|Psi(S)| + |Psi(Sbar)|) / |Phi(S)| >= 1: log|Phi| within kappa t_l,
  log w within 2 (kappa + 1) t_l, E_Phi within kappa (t_e N + t_l |E_Phi|), and
  the sign exact wherever kappa t_l < 1/2.  Random tensors do give
  configurations with Psi(Sbar) close to -Psi(S) (kappa ~ 10^3).
* At 16x16, D=8, Dc=16 (properties that hold at any size): Phi(Sbar) = Phi(S),
  so S and Sbar in one batch give the same sign, log|Phi| and E_Phi; the
  difference of their log-weights is twice the difference of vp_eval's
  log|Psi|; spin-independent tensors give Phi = 2 Psi (log w = log 4, E_Phi = E_loc).
"""
import math

import numpy as np
import pytest

from oracle import sis
from oracle.lattice import Lattice
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(Ly, Lx, D, Dc, J2, prec, T, cfgs, also_eval=False):
    import torch
    from paper_1908_09359_amd import binding as B
    n = len(cfgs)
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, J2, prec, n), seed=1)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    sp = torch.tensor(np.asarray(cfgs), dtype=torch.int8, device=dev)
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    lw = torch.empty(n, dtype=torch.float64, device=dev)
    ctx.vp_eval_sis(0, sp, n, lp, sg, el, lw)
    torch.cuda.synchronize()
    out = dict(log_abs_phi=lp.cpu().numpy(), sign=sg.cpu().numpy(), e_loc=el.cpu().numpy(),
               log_w=lw.cpu().numpy())
    if also_eval:
        ctx.vp_eval(0, sp, n, lp, sg, el)
        torch.cuda.synchronize()
        out["psi"] = dict(log_abs_psi=lp.cpu().numpy(), sign=sg.cpu().numpy(), e_loc=el.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("Ly,Lx,D,Dc,J2,ncfg,prec", [
    (4, 4, 2, 4, 0.0, 6, "VP_FP64"),    # exact contraction
    (4, 4, 3, 3, 0.5, 4, "VP_FP64"),    # truncated, diagonal J2 pairs
    (4, 4, 8, 16, 0.5, 2, "VP_FP64"),   # fused MFMA 2-row and 3-line steps, D=8 Dc=16
    (6, 6, 4, 8, 0.5, 3, "VP_FP32"),    # float32 contractions (one configuration with kappa ~ 600)
])
def test_sis_matches_oracle(Ly, Lx, D, Dc, J2, ncfg, prec):
    from paper_1908_09359_amd import binding as B
    print(f"sis {prec} {Ly}x{Lx} D={D} Dc={Dc} J2={J2}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=300 + Ly * Lx + D)
    cfgs = W.random_configs(Ly, Lx, ncfg, seed=11)
    g = _run(Ly, Lx, D, Dc, J2, getattr(B, prec), T, cfgs)
    lat = Lattice(Ly, Lx, D, Dc, J2=J2)
    o = [sis.eval_config(T, lat, c) for c in cfgs]
    N = Ly * Lx
    t_l, t_e = (1e-10, 1e-10) if prec == "VP_FP64" else (1e-3, 1e-4)
    kappa = np.array([math.exp(x["log_abs_psi"] - x["log_abs_phi"]) + math.exp(x["log_abs_psi_rev"] - x["log_abs_phi"])
                      for x in o])
    print("kappa", kappa, flush=True)
    e_o = np.array([x["e_loc"] for x in o])
    sure = kappa * t_l < 0.5
    assert np.array_equal(g["sign"][sure], np.array([x["sign"] for x in o])[sure])
    assert np.all(np.abs(g["log_abs_phi"] - np.array([x["log_abs_phi"] for x in o])) <= kappa * t_l)
    assert np.all(np.abs(g["log_w"] - np.array([x["log_w"] for x in o])) <= 2 * (kappa + 1) * t_l)
    assert np.all(np.abs(g["e_loc"] - e_o) <= kappa * (t_e * N + t_l * np.abs(e_o)))


def test_sis_reversal_invariance_full_size():
    from paper_1908_09359_amd import binding as B
    Ly, Lx, D, Dc, J2 = 16, 16, 8, 16, 0.5
    print(f"sis invariance {Ly}x{Lx} D={D} Dc={Dc}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=2024)
    c = W.random_configs(Ly, Lx, 2, seed=5)
    cfgs = np.concatenate([c, 1 - c]).astype(np.int8)
    g = _run(Ly, Lx, D, Dc, J2, B.VP_FP64, T, cfgs, also_eval=True)
    N = Ly * Lx
    for i in range(2):
        j = i + 2
        assert g["sign"][i] == g["sign"][j] != 0
        assert abs(g["log_abs_phi"][i] - g["log_abs_phi"][j]) <= 1e-12 * max(1.0, abs(g["log_abs_phi"][i]))
        assert abs(g["e_loc"][i] - g["e_loc"][j]) / N <= 1e-12
        lpsi = g["psi"]["log_abs_psi"]
        assert abs((g["log_w"][i] - g["log_w"][j]) - 2.0 * (lpsi[j] - lpsi[i])) <= 1e-9
        # E_Phi lies between the two local energies it mixes when Psi(S), Psi(Sbar) share a sign
        e = g["psi"]["e_loc"]
        if g["psi"]["sign"][i] == g["psi"]["sign"][j]:
            assert min(e[i], e[j]) - 1e-9 <= g["e_loc"][i] <= max(e[i], e[j]) + 1e-9


def test_sis_spin_independent_tensors_give_twice_psi():
    from paper_1908_09359_amd import binding as B
    Ly, Lx, D, Dc, J2 = 8, 8, 4, 8, 0.5
    print(f"sis spin-independent {Ly}x{Lx} D={D} Dc={Dc}", flush=True)
    lat = Lattice(Ly, Lx, D, Dc, J2=J2)
    T = W.random_tensors(Ly, Lx, D, seed=8)
    for y in range(Ly):
        for x in range(Lx):
            n = int(np.prod(lat.dims(y, x)))
            o = lat.offsets[lat.site(y, x)]
            T[o + n:o + 2 * n] = T[o:o + n]
    g = _run(Ly, Lx, D, Dc, J2, B.VP_FP64, T, W.random_configs(Ly, Lx, 3, seed=1), also_eval=True)
    assert np.array_equal(g["sign"], g["psi"]["sign"])
    assert np.max(np.abs(g["log_w"] - math.log(4.0))) <= 1e-12
    assert np.max(np.abs(g["log_abs_phi"] - (g["psi"]["log_abs_psi"] + math.log(2.0)))) <= 1e-12 * Ly * Lx
    assert np.max(np.abs(g["e_loc"] - g["psi"]["e_loc"])) <= 1e-12 * Ly * Lx


def test_sis_errors_are_reported():
    import torch
    from paper_1908_09359_amd import binding as B
    print("sis errors", flush=True)
    Ly, Lx, D, Dc = 4, 4, 2, 4
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, B.VP_FP64, 2), seed=1)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(W.random_tensors(Ly, Lx, D, seed=1), dtype=torch.float64, device=dev))
    lp = torch.empty(3, dtype=torch.float64, device=dev)
    sg = torch.empty(3, dtype=torch.int8, device=dev)
    el = torch.empty(3, dtype=torch.float64, device=dev)
    lw = torch.empty(3, dtype=torch.float64, device=dev)
    cfgs = torch.tensor(W.random_configs(Ly, Lx, 3, seed=2), dtype=torch.int8, device=dev)
    with pytest.raises(B.VPError):
        ctx.vp_eval_sis(0, cfgs, 3, lp, sg, el, lw)      # more configurations than chains
    with pytest.raises(B.VPError):
        ctx.vp_eval_sis(0, cfgs, 0, lp, sg, el, lw)      # empty batch
    bad = cfgs.clone()
    bad[0, 0] = 1 - bad[0, 0]
    with pytest.raises(B.VPError):
        ctx.vp_eval_sis(0, bad, 1, lp, sg, el, lw)       # outside S^z_tot = 0
    ctx.vp_eval_sis(0, cfgs, 2, lp, sg, el, lw)          # still usable afterwards
    torch.cuda.synchronize()
    assert np.all(np.isfinite(lw[:2].cpu().numpy()))
    ctx.close()
