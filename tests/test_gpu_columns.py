"""Column-wise vertical bonds on the GPU (VP_VERT_COLUMN) against the oracle's
column-wise reading (``oracle.columns``), through the C ABI.

* Evaluation, float64: sign, log|Psi|, E_loc, every pair ratio and the
  log-derivatives at the square-lattice parity bounds, on square and
  rectangular lattices, exact and truncated, generic and fused steps (the
  transposed lattice of a 4x6 one is 6x4).
* Sampling, float64: every sampled configuration, E_loc and the summed move
  counts equal the oracle's chain (horizontal bonds with row boundaries, then
  vertical bonds with column boundaries, the column pass keyed by lattice
  index + 65536).
* Sampling, float32: the visited configurations' E_loc against the oracle to
  1e-4 per site.
* The rules: J2, the triangular geometry, the learned sampler, another
  schedule, the ratio trace and the batched and split samplers are rejected.
"""
import numpy as np
import pytest

from oracle import columns as cols
from oracle import lattice as olat
from oracle import vmc
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu

COL = 1  # VP_VERT_COLUMN


def _B():
    from paper_1908_09359_amd import binding
    return binding


def _gpu_eval(Ly, Lx, D, Dc, prec, T, cfgs):
    import torch
    B = _B()
    n, N = len(cfgs), Ly * Lx
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, prec, n, vertical=COL), seed=1)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    sp = torch.tensor(np.asarray(cfgs), dtype=torch.int8, device=dev)
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    dt = torch.float32 if prec == B.VP_FP32 else torch.float64
    dl = torch.empty((n, ctx.num_params() // 2), dtype=dt, device=dev)
    ra = torch.empty((n, Ly * (Lx - 1) + (Ly - 1) * Lx), dtype=torch.float64, device=dev)
    ctx.vp_eval(0, sp, n, lp, sg, el, dl, ra)
    torch.cuda.synchronize()
    out = dict(log_abs_psi=lp.cpu().numpy(), sign=sg.cpu().numpy(), e_loc=el.cpu().numpy(),
               dlnpsi=dl.double().cpu().numpy(), ratios=ra.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("Ly,Lx,D,Dc,ncfg", [
    (4, 4, 2, 4, 6),     # exact contraction
    (4, 4, 3, 3, 4),     # truncated
    (3, 4, 3, 4, 4),     # rectangular: the transposed lattice is 4x3
    (4, 6, 4, 8, 2),     # fused steps, D=4 Dc=8 (transposed 6x4)
    (4, 4, 8, 16, 2),    # fused steps, D=8 Dc=16
])
def test_column_eval_fp64_parity(Ly, Lx, D, Dc, ncfg):
    B = _B()
    print(f"column-wise eval fp64 {Ly}x{Lx} D={D} Dc={Dc}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=800 + Ly * Lx + D)
    cfgs = W.random_configs(Ly, Lx, ncfg, seed=19)
    g = _gpu_eval(Ly, Lx, D, Dc, B.VP_FP64, T, cfgs)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    N = Ly * Lx
    for i, c in enumerate(cfgs):
        o = cols.eval_config(T, lat, c)
        assert g["sign"][i] == o["sign"]
        assert abs(g["log_abs_psi"][i] - o["log_abs_psi"]) <= 1e-10
        assert abs(g["e_loc"][i] - o["e_loc"]) / N <= 1e-10
        scale = np.maximum(1.0, np.abs(o["ratios"]))
        assert np.max(np.abs(g["ratios"][i] - o["ratios"]) / scale) <= 1e-9
        assert np.max(np.abs(g["dlnpsi"][i] - o["dlnpsi"])) <= 1e-9 * max(1.0, np.max(np.abs(o["dlnpsi"])))


def _gpu_sample(Ly, Lx, D, Dc, prec, T, n_chains, n_burn, n_meas, seed):
    import torch
    B = _B()
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, prec, n_chains, vertical=COL), seed=seed)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None)
    n, N = n_chains * n_meas, Ly * Lx
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    dt = torch.float32 if prec == B.VP_FP32 else torch.float64
    dl = torch.empty((n, ctx.num_params() // 2), dtype=dt, device=dev)
    so = torch.empty((n, N), dtype=torch.int8, device=dev)
    acc = torch.zeros((n_chains, 2), dtype=torch.int64, device=dev)
    ctx.vp_sample(0, n_burn, n_meas, lp, sg, el, dl, so, acc)
    mc = torch.zeros((n_chains, 4), dtype=torch.int64, device=dev)
    ctx.vp_move_counts(0, mc)
    ctx.vp_sync()
    out = dict(moves=mc.cpu().numpy(), log_abs_psi=lp.cpu().numpy().reshape(n_chains, n_meas), sign=sg.cpu().numpy().reshape(n_chains, n_meas),
               e_loc=el.cpu().numpy().reshape(n_chains, n_meas), dlnpsi=dl.double().cpu().numpy().reshape(n_chains, n_meas, -1),
               spins=so.cpu().numpy().reshape(n_chains, n_meas, N), accept=acc.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("Ly,Lx,D,Dc,chains,burn,meas", [(4, 4, 2, 4, 2, 2, 3), (4, 6, 3, 3, 2, 1, 2)])
def test_column_sampler_fp64_matches_oracle(Ly, Lx, D, Dc, chains, burn, meas):
    B = _B()
    print(f"column-wise sampler fp64 {Ly}x{Lx} D={D} Dc={Dc} {chains} chains {burn}+{meas}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=71)
    seed = 23
    g = _gpu_sample(Ly, Lx, D, Dc, B.VP_FP64, T, chains, burn, meas, seed)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    N = Ly * Lx
    for c in range(chains):
        ch = vmc.Chain(lat, olat.neel_shuffled(lat, seed, 0, c), seed, 0, c)
        o = cols.run_chain(T, lat, ch, burn, meas)
        assert np.array_equal(g["spins"][c], np.stack([x["spins"] for x in o])), c
        assert tuple(g["accept"][c]) == (ch.accepted, ch.proposed)
        assert tuple(g["moves"][c]) == (ch.accepted, ch.proposed, 0, 0)
        assert np.array_equal(g["sign"][c], np.array([x["sign"] for x in o]))
        assert np.max(np.abs(g["log_abs_psi"][c] - np.array([x["log_abs_psi"] for x in o]))) <= 1e-10
        assert np.max(np.abs(g["e_loc"][c] - np.array([x["e_loc"] for x in o]))) / N <= 1e-10
        for gd, od in zip(g["dlnpsi"][c], [x["dlnpsi"] for x in o]):
            assert np.max(np.abs(gd - od)) <= 1e-9 * max(1.0, np.max(np.abs(od)))
    assert g["accept"][:, 0].sum() > 0


def test_column_sampler_fp32_measures_the_visited_configurations():
    B = _B()
    Ly, Lx, D, Dc = 6, 6, 3, 6
    print("column-wise sampler fp32 6x6 D=3 Dc=6 4 chains 1+2", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=3)
    g = _gpu_sample(Ly, Lx, D, Dc, B.VP_FP32, T, 4, 1, 2, seed=5)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    cfgs = g["spins"].reshape(-1, Ly * Lx)
    assert np.all(cfgs.sum(1) == Ly * Lx // 2)
    for c, e, s in zip(cfgs, g["e_loc"].reshape(-1), g["sign"].reshape(-1)):
        o = cols.eval_config(T, lat, c)
        assert s == o["sign"]
        assert abs(e - o["e_loc"]) / (Ly * Lx) <= 1e-4


def test_column_mode_rules():
    import torch
    B = _B()
    for kw, status in ((dict(J2=0.5), B.VP_ERR_UNSUPPORTED), (dict(geometry=1), B.VP_ERR_UNSUPPORTED)):
        J2 = kw.get("J2", 0.0)
        with pytest.raises(B.VPError) as ei:
            B.Context(B.lattice(4, 4, 2, 4, 1.0, J2, B.VP_FP64, 2, geometry=kw.get("geometry", 0), vertical=COL))
        assert ei.value.status == status
    dev = torch.device("cuda")
    T = torch.tensor(W.random_tensors(4, 4, 2, seed=1), dtype=torch.float64, device=dev)
    ctx = B.Context([B.lattice(4, 4, 2, 4, 1.0, 0.0, B.VP_FP64, 2, vertical=COL),
                     B.lattice(4, 4, 2, 4, 1.0, 0.0, B.VP_FP64, 2)], seed=1)
    for k in (0, 1):
        ctx.vp_set_tensors(k, T)
        ctx.vp_init_chains(k, None)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_set_sampler(0, B.VP_SAMPLER_SIS_PAIR)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    tr = torch.zeros((2, 24, 2), dtype=torch.float64, device=dev)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_trace_ratios(0, tr)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    ctx.vp_set_schedule(0, B.VP_SCHED_PERSISTENT)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_sample(0, 1, 0, None, None, None)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    ctx.vp_set_schedule(0, B.VP_SCHED_PHASES)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_sample_batch([0], 1, 0)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    with pytest.raises(B.VPError) as ei:
        ctx.vp_sample_split(1, 0, 1, 0, None, None, None)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
    # the lattice index space holds the caller's two lattices only
    with pytest.raises(B.VPError) as ei:
        ctx.vp_init_chains(2, None)
    assert ei.value.status == B.VP_ERR_ARG
    ctx.close()


def test_column_sampler_bf16_measures_in_float64():
    """VP_BF16 with column-wise vertical bonds: bf16-operand ratios decide the moves
    of both passes, the measurement runs in float64 and equals the oracle's
    column-wise evaluation of every visited configuration."""
    B = _B()
    Ly, Lx, D, Dc = 6, 6, 4, 8
    print("column-wise sampler bf16 6x6 D=4 Dc=8 3 chains 1+2", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=29)
    g = _gpu_sample(Ly, Lx, D, Dc, B.VP_BF16, T, 3, 1, 2, seed=31)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    cfgs = g["spins"].reshape(-1, Ly * Lx)
    assert np.all(cfgs.sum(1) == Ly * Lx // 2)
    for c, e, lp, s in zip(cfgs, g["e_loc"].reshape(-1), g["log_abs_psi"].reshape(-1), g["sign"].reshape(-1)):
        o = cols.eval_config(T, lat, c)
        assert s == o["sign"]
        assert abs(lp - o["log_abs_psi"]) <= 1e-9
        assert abs(e - o["e_loc"]) / (Ly * Lx) <= 1e-9
    assert g["accept"][:, 0].sum() > 0


def test_autotune_keeps_the_per_phase_schedule():
    import torch
    B = _B()
    dev = torch.device("cuda")
    ctx = B.Context(B.lattice(4, 4, 2, 4, 1.0, 0.0, B.VP_FP64, 4, vertical=COL), seed=3)
    ctx.vp_set_tensors(0, torch.tensor(W.random_tensors(4, 4, 2, seed=5), dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None)
    sched, ms = ctx.vp_autotune(0, 2)
    assert sched == B.VP_SCHED_PHASES and ms[0] > 0 and ms[1] == -1.0 and ms[2] == -1.0
    ctx.close()
