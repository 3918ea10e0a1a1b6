"""Reduced-precision sampling (bf16 operands, f32 accumulation) against the oracle.

The bf16 mode changes only the ratios that decide Metropolis moves; Psi, E_loc
and the log-derivatives are measured in float64 (tensors and boundaries are
stored in float64; the sampling kernels round their operands to bf16).  So:

* the sampler's own ratios are traced (vp_trace_ratios) and the oracle replays
  the same sweep with the same decisions, recomputing every ratio in float64;
  every decision must also agree with the sampler's own ratio and the shared
  Philox uniform (bit-exact decision logic);
* the fixed-configuration gate (64 configurations of the 16x16, D=6, Dc=12
  workload, stored by tests/golden/make_c3_gate.py from the oracle): float64
  (the bf16 mode's measurement) within 3x each configuration's float64 floor,
  float32 within 3x its float32-level floor (tests/golden/c3_gate_floors.json),
  and the bf16 operand path's sampling decisions on that workload;
* chains sampled with bf16 ratios and with float32 ratios give the same energy
  within their statistical error.
"""
import json
import os

import numpy as np
import pytest

from oracle import lattice as olat
from oracle import philox
from oracle import vmc
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_gate_16x16_D6_Dc12.json")


def _B():
    from paper_1908_09359_amd import binding as B
    return B


def n_bonds(Ly, Lx):
    return Ly * (Lx - 1) + (Ly - 1) * Lx


def _traced_sweep(Ly, Lx, D, Dc, prec, T, starts, seed):
    """One measured sweep of len(starts) chains with the ratio trace on."""
    import torch
    B = _B()
    n = len(starts)
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, prec, n), seed=seed)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, torch.tensor(np.asarray(starts), dtype=torch.int8, device=dev))
    tr = torch.full((n, n_bonds(Ly, Lx), 2), -7.0, dtype=torch.float64, device=dev)
    ctx.vp_trace_ratios(0, tr)
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    so = torch.empty((n, Ly * Lx), dtype=torch.int8, device=dev)
    ctx.vp_sample(0, 0, 1, lp, sg, el, None, so, None)
    ctx.vp_sync()
    out = dict(trace=tr.cpu().numpy(), spins=so.cpu().numpy(), e_loc=el.cpu().numpy(),
               log_abs_psi=lp.cpu().numpy())
    ctx.vp_trace_ratios(0, None)
    ctx.close()
    return out


def _replay(T, lat, start, seed, chain, trace):
    """The oracle's float64 ratios along the sampler's own decisions."""
    ch = vmc.Chain(lat, start, seed, 0, chain)
    ch.trace = {}
    ch.forced = {b: bool(trace[b, 1] == 1.0) for b in range(trace.shape[0])}
    vmc.run_chain(T, lat, ch, 1, 0)
    return ch.trace, ch.spins


def _check_sweep(Ly, Lx, D, Dc, prec, n, seed):
    T = W.random_tensors(Ly, Lx, D, seed=seed)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    starts = [olat.neel_shuffled(lat, seed, 0, c) for c in range(n)]
    g = _traced_sweep(Ly, Lx, D, Dc, prec, T, starts, seed)
    rel = []
    for c in range(n):
        tr = g["trace"][c]
        assert np.all(tr[:, 1] >= 0.0), "every bond must be written"
        ref, spins = _replay(T, lat, starts[c], seed, c, tr)
        # the sampler's final state is the oracle's under the same decisions
        assert np.array_equal(g["spins"][c], spins), c
        for b in range(tr.shape[0]):
            if b not in ref:
                assert tr[b, 0] == 0.0 and tr[b, 1] == 0.0, (c, b)
                continue
            # decision logic: bit-exact from the sampler's own ratio and the shared uniform
            u = philox.metropolis_uniform(seed, 0, c, 0, b)
            assert (u < tr[b, 0] ** 2) == (tr[b, 1] == 1.0), (c, b)
            rel.append(abs(tr[b, 0] - ref[b]) / max(abs(ref[b]), 1e-300))
    return np.array(rel)


def test_trace_fp64_matches_oracle():
    """The trace itself: float64 ratios equal the oracle's to rounding."""
    print("trace fp64 4x4 D=2 Dc=4 4 chains", flush=True)
    rel = _check_sweep(4, 4, 2, 4, _B().VP_FP64, 4, seed=12)
    assert len(rel) > 0 and rel.max() <= 1e-10


@pytest.mark.parametrize("Ly,Lx,D,Dc", [(6, 6, 4, 8), (6, 6, 3, 6), (8, 8, 6, 12), (6, 6, 8, 16)])
def test_sampling_ratios_bf16(Ly, Lx, D, Dc):
    """bf16-operand ratios against the float64 oracle along the same sweep.

    bf16 keeps 8 significant bits: each operand rounding is a relative
    perturbation of at most u = 2^-9, and a ratio is a quotient of two networks
    of ~Lx column steps, each step rounding its three operands once.  A
    network value then carries about sqrt(3 Lx) independent u-sized relative
    errors, amplified by its cancellation (sum |terms| / |sum|, O(1)-O(10) for
    these Gaussian tensors).  Bounds: median relative error <= 8 u sqrt(3 Lx),
    and 95% of ratios within 64 u sqrt(3 Lx); App. D's estimate for the
    sampler's tolerance (|dR/R| of a few per cent changes acceptance rates by
    as much) is the scale these protect.
    """
    print(f"trace bf16 {Ly}x{Lx} D={D} Dc={Dc}", flush=True)
    rel = _check_sweep(Ly, Lx, D, Dc, _B().VP_BF16, 3, seed=20 + D)
    u = 2.0 ** -9
    scale = u * np.sqrt(3 * Lx)
    print(f"bf16 ratio rel err: median {np.median(rel):.3e} p95 {np.quantile(rel, 0.95):.3e} "
          f"max {rel.max():.3e} (n={len(rel)}, u sqrt(3Lx) = {scale:.3e})", flush=True)
    assert np.median(rel) <= 8 * scale
    assert np.quantile(rel, 0.95) <= 64 * scale


def test_sampling_ratios_fp32():
    """The same replay in float32: ratios to float32 rounding (u = 2^-24, same growth model)."""
    print("trace fp32 6x6 D=4 Dc=8", flush=True)
    rel = _check_sweep(6, 6, 4, 8, _B().VP_FP32, 3, seed=31)
    scale = 2.0 ** -24 * np.sqrt(3 * 6)
    print(f"fp32 ratio rel err: median {np.median(rel):.3e} max {rel.max():.3e}", flush=True)
    assert np.median(rel) <= 64 * scale
    assert np.quantile(rel, 0.95) <= 1024 * scale


FLOORS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_gate_floors.json")


def _gate():
    with open(GOLDEN) as f:
        doc = json.load(f)
    with open(FLOORS) as f:
        fl = json.load(f)
    w = doc["workload"]
    T = W.random_tensors(w["Ly"], w["Lx"], w["D"], seed=w["tensor_seed"], perturb=w["perturb"])
    cfgs = np.array([[int(ch) for ch in r["spins"]] for r in doc["configs"]], dtype=np.int8)
    assert [r["index"] for r in fl["configs"]] == list(range(len(cfgs)))
    return doc, fl, w, T, cfgs


def _gate_eval(prec, w, T, cfgs):
    import torch
    B = _B()
    n = len(cfgs)
    ctx = B.Context(B.lattice(w["Ly"], w["Lx"], w["D"], w["Dc"], w["J1"], w["J2"], prec, n), seed=1)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    dt = torch.float32 if prec == B.VP_FP32 else torch.float64
    dl = torch.empty((n, ctx.num_params() // 2), dtype=dt, device=dev)
    ctx.vp_eval(0, torch.tensor(cfgs, device=dev), n, lp, sg, el, dl, None)
    ctx.vp_sync()
    out = dict(e_loc=el.cpu().numpy(), log_abs_psi=lp.cpu().numpy(), sign=sg.cpu().numpy(),
               dlnpsi=dl.double().cpu().numpy())
    ctx.close()
    return out


def _gate_errors(doc, g):
    w = doc["workload"]
    N = w["Ly"] * w["Lx"]
    e_ref = np.array([r["e_loc"] for r in doc["configs"]])
    lp_ref = np.array([r["log_abs_psi"] for r in doc["configs"]])
    idx = np.array(doc["dlnpsi_index"])
    dl_ref = np.array([r["dlnpsi_sample"] for r in doc["configs"]])
    dl_norm = np.array([r["dlnpsi_norm"] for r in doc["configs"]])
    e_err = np.abs(g["e_loc"] - e_ref) / N
    lp_err = np.abs(g["log_abs_psi"] - lp_ref)
    dl_err = np.linalg.norm(g["dlnpsi"][:, idx] - dl_ref, axis=1) / (dl_norm * np.sqrt(len(idx) / g["dlnpsi"].shape[1]))
    return e_err, lp_err, dl_err


def test_c3_gate_fp64_within_floors():
    """The 64 fixed configurations of the 16x16, D=6, Dc=12 workload in float64:
    every configuration's |dE_loc|/N within max(1e-10, 3 x its float64 floor)
    (tests/golden/c3_gate_floors.json: the oracle against itself under 2^-52
    perturbations of every compression input, six seeds).  The bf16 mode
    measures in float64 (bf16 operands only decide Metropolis moves), so its
    evaluation is bit-identical to this one."""
    B = _B()
    doc, fl, w, T, cfgs = _gate()
    print(f"fp64 gate {w['Ly']}x{w['Lx']} D={w['D']} Dc={w['Dc']} {len(cfgs)} configs", flush=True)
    g = _gate_eval(B.VP_FP64, w, T, cfgs)
    e_err, lp_err, dl_err = _gate_errors(doc, g)
    floor = np.array([r["floor"]["f64"]["e_site"] for r in fl["configs"]])
    bound = np.maximum(1e-10, 3.0 * floor)
    ratio = e_err / np.maximum(floor, 1e-300)
    print(f"fp64 |dE|/N: median {np.median(e_err):.2e}, max {e_err.max():.2e}; deviation / floor: median "
          f"{np.median(ratio):.2f}, max {ratio.max():.2f}; within 1e-10: {(e_err <= 1e-10).sum()}/{len(e_err)}; "
          f"max |dlog|psi|| {lp_err.max():.2e}", flush=True)
    assert np.array_equal(g["sign"], np.array([r["sign"] for r in doc["configs"]]))
    assert np.all(e_err <= bound), np.flatnonzero(e_err > bound)
    assert lp_err.max() <= 1e-8
    assert dl_err.max() <= 1e-6
    gb = _gate_eval(B.VP_BF16, w, T, cfgs)
    for key in ("e_loc", "log_abs_psi", "sign", "dlnpsi"):
        assert np.array_equal(gb[key], g[key]), key


def test_c3_gate_fp32_within_floors():
    """The same 64 configurations in float32 (the plain path's precision):
    each |dE_loc|/N within max(1e-4, 3 x its float32-level floor) (the oracle
    with float32 storage modelled: site tensors, compression inputs and the
    compressed boundaries multiplied by (1 + 2^-24 xi), eight seeds); the
    configurations meeting 1e-4 itself are counted and printed."""
    B = _B()
    doc, fl, w, T, cfgs = _gate()
    print(f"fp32 gate {w['Ly']}x{w['Lx']} D={w['D']} Dc={w['Dc']} {len(cfgs)} configs", flush=True)
    g = _gate_eval(B.VP_FP32, w, T, cfgs)
    e_err, lp_err, _ = _gate_errors(doc, g)
    floor = np.array([r["floor"]["f32"]["e_site"] for r in fl["configs"]])
    bound = np.maximum(1e-4, 3.0 * floor)
    print(f"fp32 |dE|/N: median {np.median(e_err):.2e}, p90 {np.quantile(e_err, 0.9):.2e}, max {e_err.max():.2e}; "
          f"deviation / floor max {np.max(e_err / floor):.2f}; within 1e-4: {(e_err <= 1e-4).sum()}/{len(e_err)}; "
          f"float32 floors: median {np.median(floor):.2e}, max {floor.max():.2e}", flush=True)
    assert np.all(np.isfinite(g["e_loc"]))
    assert np.all(e_err <= bound), np.flatnonzero(e_err > bound)


def test_c3_gate_bf16_sampling_decisions():
    """The bf16 operand path on the gate's workload: one traced bf16 sweep from
    four of the gate's equilibrated configurations (oracle chain states),
    replayed by the oracle in float64 along the same decisions.  The sampler
    tolerance this protects: with the shared Philox uniforms, at most 2% of the
    Metropolis decisions may differ from the decisions the float64 ratios would
    take, and the median relative ratio error stays within 8 u sqrt(3 Lx)."""
    B = _B()
    doc, fl, w, T, cfgs = _gate()
    Ly, Lx, D, Dc = w["Ly"], w["Lx"], w["D"], w["Dc"]
    starts = [cfgs[i] for i in (32, 41, 50, 63)]
    print(f"bf16 traced sweep on the gate workload, {len(starts)} chains", flush=True)
    seed = 77
    g = _traced_sweep(Ly, Lx, D, Dc, B.VP_BF16, T, starts, seed)
    lat = olat.Lattice(Ly, Lx, D, Dc, J1=w["J1"], J2=w["J2"])
    rel, flips, visited = [], 0, 0
    for c in range(len(starts)):
        tr = g["trace"][c]
        ref, spins = _replay(T, lat, starts[c], seed, c, tr)
        assert np.array_equal(g["spins"][c], spins), c
        for b, r64 in ref.items():
            u = philox.metropolis_uniform(seed, 0, c, 0, b)
            visited += 1
            flips += (u < tr[b, 0] ** 2) != (u < r64 ** 2)
            rel.append(abs(tr[b, 0] - r64) / max(abs(r64), 1e-300))
    rel = np.array(rel)
    scale = 2.0 ** -9 * np.sqrt(3 * Lx)
    print(f"bf16 on the gate workload: median rel ratio error {np.median(rel):.3e} (8 u sqrt(3Lx) = {8 * scale:.3e}), "
          f"p95 {np.quantile(rel, 0.95):.3e}; decisions differing from float64: {flips}/{visited}", flush=True)
    assert visited > 100
    assert flips <= 0.02 * visited
    assert np.median(rel) <= 8 * scale


def test_bf16_chains_energy_matches_fp32():
    """Chains driven by bf16 ratios sample the same distribution as float32 chains.

    6x6, D=4, Dc=8, 256 chains, 4 burn-in + 12 measured sweeps each; the chain
    means are independent, so the standard error of the mean is their spread
    over sqrt(chains); the two estimates must agree within 4 combined standard
    errors.
    """
    import torch
    B = _B()
    Ly = Lx = 6
    T = W.random_tensors(Ly, Lx, 4, seed=606)
    means = {}
    for prec in (B.VP_FP32, B.VP_BF16):
        print(f"chains prec={prec} 6x6 D=4 Dc=8 256 x (4+12)", flush=True)
        n, nm = 256, 12
        ctx = B.Context(B.lattice(Ly, Lx, 4, 8, 1.0, 0.0, prec, n), seed=4242)
        dev = torch.device("cuda")
        ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
        ctx.vp_init_chains(0, None)
        lp = torch.empty(n * nm, dtype=torch.float64, device=dev)
        sg = torch.empty(n * nm, dtype=torch.int8, device=dev)
        el = torch.empty(n * nm, dtype=torch.float64, device=dev)
        ctx.vp_sample(0, 4, nm, lp, sg, el)
        ctx.vp_sync()
        cm = el.cpu().numpy().reshape(n, nm).mean(axis=1) / (Ly * Lx)
        means[prec] = (cm.mean(), cm.std(ddof=1) / np.sqrt(n))
        ctx.close()
    (m1, s1), (m2, s2) = means[B.VP_FP32], means[B.VP_BF16]
    print(f"E/N fp32 {m1:.5f} +- {s1:.5f}   bf16 {m2:.5f} +- {s2:.5f}", flush=True)
    assert abs(m1 - m2) <= 4 * np.hypot(s1, s2)


def test_bf16_learned_chains_energy_matches_fp32_pairs():
    """Learned plaquette moves with bf16 inference of the network keep |Psi|^2
    stationary: their chains' energy agrees with float32 pair sweeps within 4
    combined standard errors (6x6, D=4, Dc=8, 256 chains, 4 + 12 sweeps; network
    with random weights and output bias 0.5, so moves are proposed often)."""
    import torch
    B = _B()
    Ly = Lx = 6
    T = W.random_tensors(Ly, Lx, 4, seed=606)
    th = W.random_proposal_weights(seed=61, scale=0.2, bias=0.5)
    means, prop = {}, 0
    for prec, learned in ((B.VP_FP32, False), (B.VP_BF16, True)):
        print(f"chains prec={prec} learned={learned} 6x6 D=4 Dc=8 256 x (4+12)", flush=True)
        n, nm = 256, 12
        ctx = B.Context(B.lattice(Ly, Lx, 4, 8, 1.0, 0.0, prec, n), seed=4343)
        dev = torch.device("cuda")
        ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
        ctx.vp_init_chains(0, None)
        if learned:
            ctx.vp_proposal_set_weights(0, torch.tensor(th, device=dev))
            ctx.vp_set_sampler(0, B.VP_SAMPLER_LEARNED_PLAQ)
        lp = torch.empty(n * nm, dtype=torch.float64, device=dev)
        sg = torch.empty(n * nm, dtype=torch.int8, device=dev)
        el = torch.empty(n * nm, dtype=torch.float64, device=dev)
        ctx.vp_sample(0, 4, nm, lp, sg, el)
        ctx.vp_sync()
        if learned:
            cnt = torch.empty((n, 4), dtype=torch.int64, device=dev)
            ctx.vp_move_counts(0, cnt)
            c = cnt.cpu().numpy().sum(axis=0)
            prop, acc = c[3], c[2]
        cm = el.cpu().numpy().reshape(n, nm).mean(axis=1) / (Ly * Lx)
        means[learned] = (cm.mean(), cm.std(ddof=1) / np.sqrt(n))
        ctx.close()
    (m1, s1), (m2, s2) = means[False], means[True]
    print(f"E/N fp32 pairs {m1:.5f} +- {s1:.5f}   bf16 learned {m2:.5f} +- {s2:.5f}; plaquette moves "
          f"{acc} of {prop}", flush=True)
    assert prop > 0 and acc > 0
    assert abs(m1 - m2) <= 4 * np.hypot(s1, s2)

