"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances: float64 contractions agree with the oracle to |dE/site| <= 1e-10
(and log|Psi|, every ratio and every log-derivative to ~1e-9 relative);
float32 contractions to |dE/site| <= 1e-4.  Metropolis decisions and Philox
streams of the float64 path are bit-exact.
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


@pytest.mark.parametrize("Ly,Lx,D,Dc,J2,ncfg", [
    (4, 4, 2, 4, 0.0, 8),     # exact contraction (Dc = exact rank)
    (4, 4, 3, 3, 0.5, 4),     # truncated, diagonal J2 pairs
    (6, 6, 3, 7, 0.5, 3),     # ragged GEMM tiles (D*Dc = 21, Dc^2*D = 147)
    (2, 6, 2, 3, 0.0, 3),     # two rows: no bulk row
    (1, 4, 3, 2, 0.0, 2),     # a single row: no vertical pairs
    (4, 1, 3, 2, 0.0, 2),     # a single column: no horizontal pairs
    (6, 6, 4, 8, 0.5, 2),     # fused MFMA 2-row step, D=4 Dc=8
    (4, 4, 6, 12, 0.0, 2),    # fused MFMA 2-row step, D=6 Dc=12 (padded 16x16 tiles)
    (4, 4, 8, 16, 0.5, 2),    # fused MFMA 2-row step, D=8 Dc=16
    (2, 4, 8, 16, 0.0, 2),
    (4, 4, 5, 18, 0.0, 2),    # more than 16 kept vectors in the eigensolver (Dc = 18 at bonds of dim 25)
])
def test_eval_fp64_parity(Ly, Lx, D, Dc, J2, ncfg):
    B = _B()
    print(f"eval fp64 {Ly}x{Lx} D={D} Dc={Dc} J2={J2}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=100 + Ly * Lx + D)
    cfgs = W.random_configs(Ly, Lx, ncfg, seed=7)
    g = H.gpu_eval(Ly, Lx, D, Dc, J2, B.VP_FP64, T, cfgs)
    o = H.oracle_eval(Ly, Lx, D, Dc, J2, T, cfgs)
    _compare(g, o, Ly * Lx, 1e-10, 1e-10, 1e-9)


def test_eval_fp32_parity_8x8():
    B = _B()
    print("eval fp32 8x8 D=4 Dc=8", flush=True)
    T = W.random_tensors(8, 8, 4, seed=11)
    cfgs = W.random_configs(8, 8, 4, seed=12)
    g = H.gpu_eval(8, 8, 4, 8, 0.0, B.VP_FP32, T, cfgs)
    o = H.oracle_eval(8, 8, 4, 8, 0.0, T, cfgs)
    assert np.array_equal(g["sign"], o["sign"])
    assert np.max(np.abs(g["e_loc"] - o["e_loc"])) / 64 <= 1e-4
    assert np.max(np.abs(g["log_abs_psi"] - o["log_abs_psi"])) <= 1e-3


@pytest.mark.parametrize("Ly,Lx,D,Dc,J2", [(4, 4, 8, 16, 0.5), (6, 6, 4, 8, 0.0), (4, 6, 6, 12, 0.5)])
def test_eval_fp32_parity_fused_shapes(Ly, Lx, D, Dc, J2):
    B = _B()
    print(f"eval fp32 {Ly}x{Lx} D={D} Dc={Dc} J2={J2}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=21)
    cfgs = W.random_configs(Ly, Lx, 3, seed=22)
    g = H.gpu_eval(Ly, Lx, D, Dc, J2, B.VP_FP32, T, cfgs)
    o = H.oracle_eval(Ly, Lx, D, Dc, J2, T, cfgs)
    assert np.array_equal(g["sign"], o["sign"])
    assert np.max(np.abs(g["e_loc"] - o["e_loc"])) / (Ly * Lx) <= 1e-4
    assert np.max(np.abs(g["log_abs_psi"] - o["log_abs_psi"])) <= 1e-3


def test_sampler_fp64_bit_exact_fused_shape():
    """Chains on the fused 2-row path (D=4, Dc=8): decisions bit-exact against the oracle."""
    B = _B()
    print("sample fp64 6x6 D=4 Dc=8 3 chains 1+2", flush=True)
    T = W.random_tensors(6, 6, 4, seed=88)
    lat = olat.Lattice(6, 6, 4, 8)
    g = _gpu_sample(6, 6, 4, 8, 0.0, B.VP_FP64, T, 3, 1, 2, seed=41)
    for c in range(3):
        ch = vmc.Chain(lat, olat.neel_shuffled(lat, 41, 0, c), 41, 0, c)
        o = vmc.run_chain(T, lat, ch, 1, 2)
        assert np.array_equal(g["spins"][c], np.stack([x["spins"] for x in o])), c
        assert np.max(np.abs(g["e_loc"][c] - np.array([x["e_loc"] for x in o]))) / 36 <= 1e-10
        assert tuple(g["accept"][c]) == (ch.accepted, ch.proposed)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sampler_bit_exact_d8_dc16(prec):
    """The benchmark's bond dimensions (fused 3-line and 2-row steps, defects) on a 4x6 lattice:
    float64 decisions bit-exact against the oracle; float32 measurements of the visited states."""
    B = _B()
    print(f"sample {prec} 4x6 D=8 Dc=16 3 chains 1+2", flush=True)
    T = W.random_tensors(4, 6, 8, seed=89)
    lat = olat.Lattice(4, 6, 8, 16)
    if prec == "fp64":
        g = _gpu_sample(4, 6, 8, 16, 0.0, B.VP_FP64, T, 3, 1, 2, seed=43)
        for c in range(3):
            ch = vmc.Chain(lat, olat.neel_shuffled(lat, 43, 0, c), 43, 0, c)
            o = vmc.run_chain(T, lat, ch, 1, 2)
            assert np.array_equal(g["spins"][c], np.stack([x["spins"] for x in o])), c
            assert np.max(np.abs(g["e_loc"][c] - np.array([x["e_loc"] for x in o]))) / 24 <= 1e-10
            assert np.max(np.abs(g["log_abs_psi"][c] - np.array([x["log_abs_psi"] for x in o]))) <= 1e-10
            for m in range(2):
                od = np.asarray(o[m]["dlnpsi"]).ravel()
                assert np.max(np.abs(g["dlnpsi"][c, m] - od)) <= 1e-9 * max(1.0, np.max(np.abs(od)))
            assert tuple(g["accept"][c]) == (ch.accepted, ch.proposed)
    else:
        g = _gpu_sample(4, 6, 8, 16, 0.0, B.VP_FP32, T, 3, 1, 2, seed=43)
        cfgs = g["spins"].reshape(6, 24)
        o = H.oracle_eval(4, 6, 8, 16, 0.0, T, cfgs)
        assert np.max(np.abs(g["e_loc"].ravel() - o["e_loc"])) / 24 <= 1e-4
        assert np.max(np.abs(g["log_abs_psi"].ravel() - o["log_abs_psi"])) <= 1e-3


def test_eval_more_chains_than_configs():
    """n_cfg below the context's chain count (a ragged last batch)."""
    B = _B()
    T = W.random_tensors(4, 4, 2, seed=5)
    cfgs = W.random_configs(4, 4, 3, seed=6)
    g = H.gpu_eval(4, 4, 2, 4, 0.0, B.VP_FP64, T, cfgs, n_chains=8)
    o = H.oracle_eval(4, 4, 2, 4, 0.0, T, cfgs)
    _compare(g, o, 16, 1e-10, 1e-10, 1e-9)


def _gpu_sample(Ly, Lx, D, Dc, J2, prec, T, n_chains, n_burn, n_meas, seed, spins=None):
    import torch
    B = _B()
    lat = B.lattice(Ly, Lx, D, Dc, 1.0, J2, prec, n_chains)
    ctx = B.Context(lat, seed=seed)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None if spins is None else torch.tensor(spins, dtype=torch.int8, device=dev))
    n = n_chains * n_meas
    N = Ly * Lx
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    dt = torch.float32 if prec == B.VP_FP32 else torch.float64
    dl = torch.empty((n, ctx.num_params() // 2), dtype=dt, device=dev)
    so = torch.empty((n, N), dtype=torch.int8, device=dev)
    acc = torch.zeros((n_chains, 2), dtype=torch.int64, device=dev)
    ctx.vp_sample(0, n_burn, n_meas, lp, sg, el, dl, so, acc)
    ctx.vp_sync()
    out = dict(log_abs_psi=lp.cpu().numpy().reshape(n_chains, n_meas), sign=sg.cpu().numpy().reshape(n_chains, n_meas),
               e_loc=el.cpu().numpy().reshape(n_chains, n_meas),
               dlnpsi=dl.double().cpu().numpy().reshape(n_chains, n_meas, -1),
               spins=so.cpu().numpy().reshape(n_chains, n_meas, N), accept=acc.cpu().numpy())
    ctx.close()
    return out


def test_sampler_fp64_bit_exact_single_chain():
    """4x4, D=2, Dc=4, one chain from the Neel state, 16 burn-in + 256 measured sweeps."""
    B = _B()
    print("sample fp64 4x4 D=2 Dc=4 1 chain 16+256", flush=True)
    T = W.random_tensors(4, 4, 2, seed=1908)
    lat = olat.Lattice(4, 4, 2, 4)
    neel = olat.neel(lat)
    g = _gpu_sample(4, 4, 2, 4, 0.0, B.VP_FP64, T, 1, 16, 256, seed=9359, spins=neel[None])
    ch = vmc.Chain(lat, neel, 9359, 0, 0)
    o = vmc.run_chain(T, lat, ch, 16, 256)
    assert np.array_equal(g["spins"][0], np.stack([x["spins"] for x in o]))
    assert np.max(np.abs(g["e_loc"][0] - np.array([x["e_loc"] for x in o]))) / 16 <= 1e-10
    assert np.max(np.abs(g["log_abs_psi"][0] - np.array([x["log_abs_psi"] for x in o]))) <= 1e-10
    assert np.array_equal(g["sign"][0], np.array([x["sign"] for x in o]))
    assert np.max(np.abs(g["dlnpsi"][0] - np.stack([x["dlnpsi"] for x in o]))) <= 1e-9 * max(
        1.0, np.max(np.abs(np.stack([x["dlnpsi"] for x in o]))))
    assert tuple(g["accept"][0]) == (ch.accepted, ch.proposed)


def test_sampler_fp64_bit_exact_shuffled_chains_truncated():
    """Several chains from Philox-shuffled Neel starts on a truncated 4x4 J1-J2 network."""
    B = _B()
    print("sample fp64 4x4 D=3 Dc=3 J2=0.5 5 chains 2+3", flush=True)
    T = W.random_tensors(4, 4, 3, seed=77)
    lat = olat.Lattice(4, 4, 3, 3, J2=0.5)
    g = _gpu_sample(4, 4, 3, 3, 0.5, B.VP_FP64, T, 5, 2, 3, seed=31)
    for c in range(5):
        start = olat.neel_shuffled(lat, 31, 0, c)
        ch = vmc.Chain(lat, start, 31, 0, c)
        o = vmc.run_chain(T, lat, ch, 2, 3)
        assert np.array_equal(g["spins"][c], np.stack([x["spins"] for x in o])), c
        assert np.max(np.abs(g["e_loc"][c] - np.array([x["e_loc"] for x in o]))) / 16 <= 1e-10
        assert tuple(g["accept"][c]) == (ch.accepted, ch.proposed)


def test_sampler_fp32_measurements_match_oracle_on_visited_configs():
    B = _B()
    print("sample fp32 6x6 D=3 Dc=6 8 chains 1+2", flush=True)
    T = W.random_tensors(6, 6, 3, seed=3)
    g = _gpu_sample(6, 6, 3, 6, 0.0, B.VP_FP32, T, 8, 1, 2, seed=5)
    cfgs = g["spins"].reshape(-1, 36)
    o = H.oracle_eval(6, 6, 3, 6, 0.0, T, cfgs)
    assert np.all(cfgs.sum(1) == 18)
    assert np.max(np.abs(g["e_loc"].reshape(-1) - o["e_loc"])) / 36 <= 1e-4
    assert np.array_equal(g["sign"].reshape(-1), o["sign"])


def test_init_tensors_match_oracle():
    import torch
    B = _B()
    lat = B.lattice(4, 6, 2, 4, 1.0, 0.0, B.VP_FP64, 6)
    ctx = B.Context(lat, seed=42)
    ctx.vp_init_tensors(0, seed=1234, scale=0.0, perturb=1e-2)
    Td = torch.empty(ctx.num_params(), dtype=torch.float64, device="cuda")
    ctx.vp_get_tensors(0, Td)
    ref = olat.init_tensors(olat.Lattice(4, 6, 2, 4), 1234, 0, perturb=1e-2)
    assert np.max(np.abs(Td.cpu().numpy() - ref)) <= 1e-14
    # the Philox-shuffled chain starts are checked bit-exactly through the sampler test above
    ctx.close()


def test_gradient_matches_oracle():
    import torch
    B = _B()
    Ly, Lx, D = 4, 4, 2
    T = W.random_tensors(Ly, Lx, D, seed=8)
    cfgs = W.random_configs(Ly, Lx, 16, seed=9)
    o = H.oracle_eval(Ly, Lx, D, 4, 0.0, T, cfgs)
    lat = B.lattice(Ly, Lx, D, 4, 1.0, 0.0, B.VP_FP64, 16)
    ctx = B.Context(lat, seed=1)
    dev = torch.device("cuda")
    g = torch.empty(ctx.num_params(), dtype=torch.float64, device=dev)
    em = torch.empty(1, dtype=torch.float64, device=dev)
    ctx.vp_gradient(0, torch.tensor(o["e_loc"], device=dev), torch.tensor(o["dlnpsi"], device=dev),
                    torch.tensor(cfgs, dtype=torch.int8, device=dev), 16, g, em)
    torch.cuda.synchronize()
    gref, eref = vmc.gradient(olat.Lattice(Ly, Lx, D, 4), o["e_loc"], o["dlnpsi"], cfgs)
    assert abs(em.item() - eref) <= 1e-12 * max(1.0, abs(eref))
    assert np.max(np.abs(g.cpu().numpy() - gref)) <= 1e-11 * max(1.0, np.max(np.abs(gref)))
    # sign-gradient step (Eq. (10)) on the device vs the oracle
    ctx.vp_set_tensors(0, torch.tensor(T, device=dev))
    ctx.vp_sign_sgd_update(0, g, 0.005, 3)
    Tn = torch.empty_like(g)
    ctx.vp_get_tensors(0, Tn)
    ref = vmc.sign_sgd(T, g.cpu().numpy(), 0.005, 1, 0, 3)
    assert np.max(np.abs(Tn.cpu().numpy() - ref)) <= 1e-15
    ctx.close()


def test_errors_are_reported():
    import torch
    B = _B()
    dev = torch.device("cuda")
    lat = B.lattice(4, 4, 1, 2, 1.0, 0.0, B.VP_FP64, 2)
    ctx = B.Context(lat, seed=1)
    # D=1 Neel product state: every other configuration has Psi = 0
    Np = ctx.num_params()
    T = np.zeros(Np)
    neel = olat.neel(olat.Lattice(4, 4, 1, 2))
    for k in range(16):
        T[2 * k + int(neel[k])] = 1.0
    ctx.vp_set_tensors(0, torch.tensor(T, device=dev))
    cfgs = np.stack([neel, W.random_configs(4, 4, 1, seed=3)[0]])
    lp = torch.empty(2, dtype=torch.float64, device=dev)
    sg = torch.empty(2, dtype=torch.int8, device=dev)
    el = torch.empty(2, dtype=torch.float64, device=dev)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_eval(0, torch.tensor(cfgs, dtype=torch.int8, device=dev), 2, lp, sg, el)
    assert ei.value.status == B.VP_ERR_ZERO_AMPLITUDE
    # the Neel configuration alone evaluates to the closed form -0.375 per site
    ctx.vp_eval(0, torch.tensor(neel[None], dtype=torch.int8, device=dev), 1, lp, sg, el)
    torch.cuda.synchronize()
    assert abs(el[0].item() / 16 + 0.375) < 1e-14
    bad = np.zeros((1, 16), dtype=np.int8)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_eval(0, torch.tensor(bad, device=dev), 1, lp, sg, el)
    assert ei.value.status == B.VP_ERR_SHAPE
    ctx.close()
