"""GPU parity of the spin-inversion symmetrised evaluation (Sec. II.B,
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


def test_sis_reweighted_samples_give_energy_of_phi():
    """The whole workflow on an enumerable lattice (2x4, exact contraction): 8192 independent
    chains of the GPU sampler (|Psi|^2, one sample each after 24 sweeps) and their log-weights
    from vp_eval_sis.  Tensors: a reversal-symmetric PEPS (T_k[1] = T_k[0] with bond index 0 <-> 1
    on every leg of dimension 2, so Psi(Sbar) = Psi(S)) plus 0.1 times a random one, a state near
    a symmetric one, as after an optimisation.  Checked within 5 standard errors: the mean weight
    against <Phi|Phi>/<Psi|Psi> and sum w E_Phi / sum w against <Phi|H|Phi>/<Phi|Phi>, both from
    the dense Phi = Psi + P Psi."""
    import torch
    import bruteforce as bf
    from paper_1908_09359_amd import binding as B
    Ly, Lx, D, Dc, J2, n = 2, 4, 2, 8, 0.3, 8192
    print(f"sis reweighted sampling {Ly}x{Lx} D={D} {n} chains", flush=True)
    lat = Lattice(Ly, Lx, D, Dc, J2=J2)
    T = W.random_tensors(Ly, Lx, D, seed=31)
    for y in range(Ly):
        for x in range(Lx):
            dims = lat.dims(y, x)
            m = int(np.prod(dims))
            o = lat.offsets[lat.site(y, x)]
            a = T[o:o + m].reshape(dims)
            for ax, d in enumerate(dims):
                if d == 2:
                    a = np.flip(a, axis=ax)
            T[o + m:o + 2 * m] = a.reshape(-1)
    T = T + 0.1 * W.random_tensors(Ly, Lx, D, seed=32)
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, J2, B.VP_FP64, n), seed=77)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None)
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    lw = torch.empty(n, dtype=torch.float64, device=dev)
    so = torch.empty((n, Ly * Lx), dtype=torch.int8, device=dev)
    ctx.vp_sample(0, 23, 1, lp, sg, el, None, so)
    ctx.vp_eval_sis(0, so, n, lp, sg, el, lw)
    ctx.vp_sync()
    e_phi, w = el.cpu().numpy(), np.exp(lw.cpu().numpy())
    ctx.close()
    configs = bf.sz0_configs(Ly * Lx)
    index = {c.tobytes(): i for i, c in enumerate(configs)}
    psi = bf.amplitudes(T, Ly, Lx, D, configs)
    phi = psi + psi[[index[(1 - c).astype(np.int8).tobytes()] for c in configs]]
    Hm = np.zeros((len(configs), len(configs)))
    for k, s in enumerate(configs):
        for i, j, J in bf.bonds(Ly, Lx, 1.0, J2):
            if s[i] == s[j]:
                Hm[k, k] += 0.25 * J
            else:
                Hm[k, k] -= 0.25 * J
                t = s.copy()
                t[i], t[j] = s[j], s[i]
                Hm[index[t.tobytes()], k] += 0.5 * J
    norm_ratio = float(phi @ phi / (psi @ psi))
    exact_phi = float(phi @ Hm @ phi / (phi @ phi))
    exact_psi = float(psi @ Hm @ psi / (psi @ psi))
    w_mean, w_err = float(np.mean(w)), float(np.std(w) / np.sqrt(n))
    est = float(np.sum(w * e_phi) / np.sum(w))
    sigma = float(np.sqrt(np.sum(w ** 2 * (e_phi - est) ** 2)) / np.sum(w))
    ess = float(np.sum(w) ** 2 / np.sum(w ** 2))
    print(f"mean weight {w_mean:.5f} +- {w_err:.5f} (exact {norm_ratio:.5f}); reweighted E {est:.5f} +- "
          f"{sigma:.5f} (exact Phi {exact_phi:.5f}, Psi {exact_psi:.5f}); effective samples {ess:.0f}",
          flush=True)
    assert abs(w_mean - norm_ratio) <= 5.0 * w_err
    assert abs(est - exact_phi) <= 5.0 * sigma
