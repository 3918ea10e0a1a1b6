"""Chains of |Phi|^2 on the GPU (VP_SAMPLER_SIS_PAIR; Sec. II.B's weight of the
spin-inversion symmetrised amplitude Phi(S) = Psi(S) + Psi(Sbar)), through the
C ABI, against the oracle's pair chains (``oracle.sis.run_pair_chain``).

* float64: every sampled configuration and both accept counts equal the
  oracle's (each decision compares the same Philox uniform with |Phi(S')/Phi(S)|^2
  formed from ratios that agree to rounding), log|Phi| within 1e-10 and E_Phi
  within 1e-10 per site, at exact, truncated (J1-J2) and fused-step shapes;
* float32: the visited configurations evaluated by the oracle (``sis.eval_config``)
  give the same E_Phi to 1e-4 per site;
* the stationary distribution: 256 GPU pairs on a 2x3 lattice visit the
  S^z = 0 configurations with the dense |Phi|^2 / Z (chi-square; consecutive
  sweeps are correlated, so the p-value is a coarse gate), and their mean E_Phi
  agrees with <Phi|H|Phi>/<Phi|Phi> of the dense state within 5 standard errors;
* the rules: an odd chain count, log-derivative outputs, another schedule, the
  batched and the split sampler are rejected.
"""
import numpy as np
import pytest

import bruteforce as bf
from oracle import lattice as olat
from oracle import sis, vmc
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu


def _B():
    from paper_1908_09359_amd import binding
    return binding


def _gpu_pair_sample(Ly, Lx, D, Dc, J2, prec, T, n_pairs, n_burn, n_meas, seed):
    import torch
    B = _B()
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, J2, prec, 2 * n_pairs), seed=seed)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None)
    ctx.vp_set_sampler(0, B.VP_SAMPLER_SIS_PAIR)
    n, N = n_pairs * n_meas, Ly * Lx
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    so = torch.empty((n, N), dtype=torch.int8, device=dev)
    acc = torch.zeros((n_pairs, 2), dtype=torch.int64, device=dev)
    ctx.vp_sample(0, n_burn, n_meas, lp, sg, el, None, so, acc)
    ctx.vp_sync()
    out = dict(log_abs_phi=lp.cpu().numpy().reshape(n_pairs, n_meas), sign=sg.cpu().numpy().reshape(n_pairs, n_meas),
               e_loc=el.cpu().numpy().reshape(n_pairs, n_meas), spins=so.cpu().numpy().reshape(n_pairs, n_meas, N),
               accept=acc.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("Ly,Lx,D,Dc,J2,pairs,burn,meas", [
    (4, 4, 2, 4, 0.0, 2, 3, 5),    # exact contraction
    (4, 4, 3, 3, 0.5, 3, 2, 3),    # truncated, J1-J2 (diagonal terms in E_Phi)
    (4, 4, 4, 8, 0.0, 1, 1, 2),    # fused MFMA steps, D=4 Dc=8
    (4, 4, 8, 16, 0.5, 1, 1, 1),   # fused MFMA steps, D=8 Dc=16, J1-J2
])
def test_pair_chains_match_oracle_fp64(Ly, Lx, D, Dc, J2, pairs, burn, meas):
    B = _B()
    print(f"|Phi|^2 pair chains fp64 {Ly}x{Lx} D={D} Dc={Dc} J2={J2} pairs={pairs} {burn}+{meas}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=900 + D)
    seed = 61
    g = _gpu_pair_sample(Ly, Lx, D, Dc, J2, B.VP_FP64, T, pairs, burn, meas, seed)
    lat = olat.Lattice(Ly, Lx, D, Dc, J2=J2)
    N = Ly * Lx
    for c in range(pairs):
        ch = vmc.Chain(lat, olat.neel_shuffled(lat, seed, 0, c), seed, 0, c)
        o = sis.run_pair_chain(T, lat, ch, burn, meas)
        assert np.array_equal(g["spins"][c], np.stack([x["spins"] for x in o])), c
        assert tuple(g["accept"][c]) == (ch.accepted, ch.proposed)
        assert np.array_equal(g["sign"][c], np.array([x["sign"] for x in o]))
        assert np.max(np.abs(g["log_abs_phi"][c] - np.array([x["log_abs_phi"] for x in o]))) <= 1e-10
        assert np.max(np.abs(g["e_loc"][c] - np.array([x["e_loc"] for x in o]))) / N <= 1e-10
    assert g["accept"][:, 0].sum() > 0


def test_pair_chains_fp32_measure_phi():
    B = _B()
    Ly, Lx, D, Dc = 6, 6, 3, 6
    print(f"|Phi|^2 pair chains fp32 {Ly}x{Lx} D={D} Dc={Dc} 4 pairs 1+2", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=5)
    g = _gpu_pair_sample(Ly, Lx, D, Dc, 0.0, B.VP_FP32, T, 4, 1, 2, seed=9)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    cfgs = g["spins"].reshape(-1, Ly * Lx)
    assert np.all(cfgs.sum(1) == Ly * Lx // 2)
    for c, e, s in zip(cfgs, g["e_loc"].reshape(-1), g["sign"].reshape(-1)):
        ref = sis.eval_config(T, lat, c)
        assert s == ref["sign"]
        assert abs(e - ref["e_loc"]) / (Ly * Lx) <= 1e-4


def test_pair_chains_sample_phi_squared_on_the_gpu():
    B = _B()
    Ly, Lx, D, Dc = 2, 3, 2, 8
    pairs, burn, meas = 256, 10, 40
    print(f"|Phi|^2 stationary distribution 2x3 D=2 {pairs} pairs {burn}+{meas}", flush=True)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    T = np.random.default_rng(3).standard_normal(lat.Np) / D ** 2
    g = _gpu_pair_sample(Ly, Lx, D, Dc, 0.0, B.VP_FP64, T, pairs, burn, meas, seed=11)
    configs = bf.sz0_configs(6)
    psi = bf.amplitudes(T, Ly, Lx, D, configs)
    psi_rev = bf.amplitudes(T, Ly, Lx, D, 1 - np.asarray(configs))
    phi = psi + psi_rev
    p = phi ** 2 / np.sum(phi ** 2)
    index = {c.tobytes(): i for i, c in enumerate(configs)}
    counts = np.zeros(len(configs))
    for s in g["spins"].reshape(-1, 6):
        counts[index[s.astype(np.int8).tobytes()]] += 1
    import scipy.stats
    n = counts.sum()
    keep = p * n >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(p[keep] * n, p[~keep].sum() * n)
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    pval = scipy.stats.chisquare(obs, exp)[1]
    # <Phi|H|Phi>/<Phi|Phi> of the dense state (the sector is closed under H and under the reversal)
    e_exact = bf.sector_energy(phi, np.asarray(configs), Ly, Lx)
    e = g["e_loc"]
    per_pair = e.mean(axis=1)
    err = per_pair.std(ddof=1) / np.sqrt(pairs)
    print(f"chi-square p {pval:.3g}; mean E_Phi {e.mean():.6f} +- {err:.6f}, exact {e_exact:.6f}", flush=True)
    assert pval > 1e-4
    assert abs(e.mean() - e_exact) <= 5 * err


def test_pair_sampler_rules():
    import torch
    B = _B()
    dev = torch.device("cuda")
    T = torch.tensor(W.random_tensors(4, 4, 2, seed=1), dtype=torch.float64, device=dev)
    ctx = B.Context(B.lattice(4, 4, 2, 4, 1.0, 0.0, B.VP_FP64, 3), seed=1)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_set_sampler(0, B.VP_SAMPLER_SIS_PAIR)
    assert ei.value.status == B.VP_ERR_SHAPE
    ctx.close()
    ctx = B.Context([B.lattice(4, 4, 2, 4, 1.0, 0.0, B.VP_FP64, 4), B.lattice(4, 4, 2, 6, 1.0, 0.0, B.VP_FP64, 4)],
                    seed=1)
    for k in (0, 1):
        ctx.vp_set_tensors(k, T)
        ctx.vp_init_chains(k, None)
    ctx.vp_set_sampler(0, B.VP_SAMPLER_SIS_PAIR)
    lp = torch.empty(2, dtype=torch.float64, device=dev)
    sg = torch.empty(2, dtype=torch.int8, device=dev)
    el = torch.empty(2, dtype=torch.float64, device=dev)
    dl = torch.empty((2, ctx.num_params() // 2), dtype=torch.float64, device=dev)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_sample(0, 0, 1, lp, sg, el, dl)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    ctx.vp_set_schedule(0, B.VP_SCHED_GRAPH)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_sample(0, 0, 1, lp, sg, el)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    ctx.vp_set_schedule(0, B.VP_SCHED_PHASES)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_sample_batch([0], 1, 0)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    with pytest.raises(B.VPError) as ei:
        ctx.vp_sample_split(0, 1, 1, 0, None, None, None)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    ctx.vp_sample(0, 1, 1, lp, sg, el)  # the per-phase schedule without log-derivatives runs
    ctx.vp_sync()
    assert np.all(np.isfinite(el.cpu().numpy()))
    sched, ms = ctx.vp_autotune(0, 1)  # times the per-phase schedule alone
    assert sched == B.VP_SCHED_PHASES and ms[0] > 0 and ms[1] == -1.0 and ms[2] == -1.0
    ctx.close()


def test_pair_chains_bf16_sampling_measure_in_float64():
    """VP_BF16: the pair decisions use bf16-operand ratios, the measurement runs in
    float64, so every measured sample equals the oracle's evaluation of its
    configuration at the float64 bounds."""
    B = _B()
    Ly, Lx, D, Dc = 6, 6, 4, 8
    print("|Phi|^2 pair chains bf16 6x6 D=4 Dc=8 3 pairs 1+2", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=13)
    g = _gpu_pair_sample(Ly, Lx, D, Dc, 0.0, B.VP_BF16, T, 3, 1, 2, seed=17)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    cfgs = g["spins"].reshape(-1, Ly * Lx)
    assert np.all(cfgs.sum(1) == Ly * Lx // 2)
    for c, e, la, s in zip(cfgs, g["e_loc"].reshape(-1), g["log_abs_phi"].reshape(-1), g["sign"].reshape(-1)):
        ref = sis.eval_config(T, lat, c)
        assert s == ref["sign"]
        assert abs(la - ref["log_abs_phi"]) <= 1e-9
        assert abs(e - ref["e_loc"]) / (Ly * Lx) <= 1e-9
    assert g["accept"][:, 0].sum() > 0
