"""What the trained plaquette proposal gains over pair sweeps alone, on a
correlated state (the random i.i.d. workloads decorrelate within one sweep, so
no proposal can gain there).

The state: the simple-update state (App. A, vp_simple_update) of the 8x8
Heisenberg lattice at D=4, 200 steps of dt 0.05 from seeded random tensors
(about -0.613 per site).  Both samplers run in float64 from the same
Neel-shuffled starts, 256 chains, 30 burn-in and 60 measured sweeps: pair sweeps alone, and pair sweeps
plus learned plaquette moves (network trained on the pair sampler's
configurations and their plaquette ratios).  Printed per sampler: tau_int of
E_loc/N and of M_z^2 (a function of the configuration alone), the acceptance
rates and the effective samples per second (samples/s / 2 tau_int).  Asserted:
both sample |Psi|^2 of the same state, so their energies agree within 4
combined standard errors (tau-corrected), and the learned moves are proposed
and accepted.
"""
import numpy as np
import pytest

from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu

L, D, DC, NCH, NB, NM = 8, 4, 8, 256, 30, 60


def _B():
    from paper_1908_09359_amd import binding
    return binding


def _state(B, torch):
    """The simple-update state (App. A) of the L x L Heisenberg lattice at bond
    dimension D: 200 steps of dt 0.05 from seeded random tensors."""
    dev = torch.device("cuda")
    ctx = B.Context(B.lattice(L, L, D, 4, 1.0, 0.0, B.VP_FP64, 1), seed=7)
    ctx.vp_init_tensors(0, seed=7, scale=0.0, perturb=0.0)
    ch = torch.zeros(200, dtype=torch.float64, device=dev)
    ctx.vp_simple_update(0, 0.05, 200, ch)
    T = torch.empty(ctx.num_params(), dtype=torch.float64, device=dev)
    ctx.vp_get_tensors(0, T)
    ctx.vp_sync()
    c = ch.cpu().numpy()
    ctx.close()
    print(f"simple update: lambda change {c[0]:.2e} -> {c[-1]:.2e}", flush=True)
    return T.cpu().numpy()


def _run(B, torch, T, learned):
    import time
    dev = torch.device("cuda")
    ctx = B.Context(B.lattice(L, L, D, DC, 1.0, 0.0, B.VP_FP64, NCH), seed=9)
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None)
    N = L * L
    if learned:
        # training data: configurations of the pair sampler and their plaquette-flip ratios
        so = torch.empty((4 * NCH, N), dtype=torch.int8, device=dev)
        lp = torch.empty(4 * NCH, dtype=torch.float64, device=dev)
        sg = torch.empty(4 * NCH, dtype=torch.int8, device=dev)
        el = torch.empty(4 * NCH, dtype=torch.float64, device=dev)
        ctx.vp_sample(0, NB, 4, lp, sg, el, None, so)
        last = so.view(NCH, 4, N)[:, -1].contiguous()
        rho = torch.empty((4 * NCH, (L - 1) * (L - 1)), dtype=torch.float64, device=dev)
        for k in range(4):
            ctx.vp_plaquette_ratios(0, so[k * NCH:(k + 1) * NCH].contiguous(), NCH, rho[k * NCH:(k + 1) * NCH])
        ctx.vp_proposal_set_weights(0, torch.tensor(W.random_proposal_weights(seed=4), device=dev))
        ctx.vp_proposal_train(0, so, rho, so.shape[0], 6, 256, 3e-3, 11)
        ctx.vp_init_chains(0, last)
        ctx.vp_set_sampler(0, B.VP_SAMPLER_LEARNED_PLAQ)
    lp = torch.empty(NCH * NM, dtype=torch.float64, device=dev)
    sg = torch.empty(NCH * NM, dtype=torch.int8, device=dev)
    el = torch.empty(NCH * NM, dtype=torch.float64, device=dev)
    so = torch.empty((NCH * NM, N), dtype=torch.int8, device=dev)
    ctx.vp_sample(0, NB, 0, lp, sg, el)
    ctx.vp_sync()
    c0 = torch.empty((NCH, 4), dtype=torch.int64, device=dev)
    ctx.vp_move_counts(0, c0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.vp_sample(0, 0, NM, lp, sg, el, None, so)
    ctx.vp_sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c1 = torch.empty((NCH, 4), dtype=torch.int64, device=dev)
    ctx.vp_move_counts(0, c1)
    cnt = (c1 - c0).sum(dim=0).cpu().numpy()
    e = el.cpu().numpy().reshape(NCH, NM) / N
    g = so.cpu().numpy().reshape(NCH, NM, L, L).astype(np.float64)
    stag = (-1.0) ** np.add.outer(np.arange(L), np.arange(L))
    m2 = (((0.5 - g) * stag).sum(axis=(2, 3)) / N) ** 2
    ctx.close()
    out = {"rate": NCH * NM / dt, "pair_accept": cnt[0] / max(cnt[1], 1),
           "plaq_accept": cnt[2] / max(cnt[3], 1), "plaq_per_sweep": cnt[3] / NCH / NM}
    for name, x in (("e", e), ("m2", m2)):
        tau, mean, err = B.vp_stats_tau(x, 5.0)
        out[name] = (float(np.mean(tau)), mean, err)
    return out


def test_learned_moves_on_a_correlated_state():
    import torch
    B = _B()
    print(f"learned-move gain: {L}x{L} D={D} Dc={DC} (simple-update state), {NCH} chains", flush=True)
    T = _state(B, torch)
    res = {}
    for learned in (False, True):
        r = _run(B, torch, T, learned)
        name = "learned" if learned else "pairs"
        res[name] = r
        print(f"{name:8s}: tau_int(E) {r['e'][0]:.3f}, tau_int(Mz^2) {r['m2'][0]:.3f}, E/N {r['e'][1]:.5f} +- "
              f"{r['e'][2]:.5f}, pair acc {r['pair_accept']:.3f}, plaquette acc {r['plaq_accept']:.3f} "
              f"({r['plaq_per_sweep']:.1f}/sweep), {r['rate']:.0f} samples/s, effective (E) "
              f"{r['rate'] / (2 * r['e'][0]):.0f}/s, effective (Mz^2) {r['rate'] / (2 * r['m2'][0]):.0f}/s", flush=True)
    p, q = res["pairs"], res["learned"]
    gain_e = (q["rate"] / q["e"][0]) / (p["rate"] / p["e"][0])
    gain_m = (q["rate"] / q["m2"][0]) / (p["rate"] / p["m2"][0])
    print(f"learned / pairs at equal error: {gain_e:.3f} (E_loc), {gain_m:.3f} (Mz^2); "
          f"tau ratio (E) {p['e'][0] / q['e'][0]:.3f}, (Mz^2) {p['m2'][0] / q['m2'][0]:.3f}", flush=True)
    assert abs(p["e"][1] - q["e"][1]) <= 4.0 * np.hypot(p["e"][2], q["e"][2])
    assert q["plaq_per_sweep"] > 0 and q["plaq_accept"] > 0
