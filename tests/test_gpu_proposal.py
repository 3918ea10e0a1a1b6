"""Learned plaquette proposal on the GPU against the oracle.

* plaquette-flip ratios (vp_plaquette_ratios) against ``vmc.plaquette_ratios``;
* the batched network forward and the loss gradient against ``oracle.proposal``;
* the learned sampler's chains bit-exact against the oracle's in float64;
* |Psi|^2 stationary under the learned sampler (exact distribution, chi-square);
* training lowers the loss on sampler-generated configurations.
"""
import numpy as np
import pytest
import scipy.stats

import bruteforce as bf
from oracle import lattice as olat
from oracle import proposal as P
from oracle import vmc
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu


def _B():
    from paper_1908_09359_amd import binding as B
    return B


def _theta(seed, bias4=0.0, scale=0.3):
    th = (np.random.default_rng(seed).standard_normal(P.n_params()) * scale).astype(np.float32)
    th[-1] = bias4
    return th


def _ctx(Ly, Lx, D, Dc, prec, n, seed=1, T=None, theta=None):
    import torch
    B = _B()
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, prec, n), seed=seed)
    dev = torch.device("cuda")
    if T is not None:
        ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    if theta is not None:
        ctx.vp_proposal_set_weights(0, torch.tensor(theta, dtype=torch.float32, device=dev))
    return ctx


@pytest.mark.parametrize("Ly,Lx,D,Dc,prec,tol", [(4, 4, 2, 4, 0, 1e-10), (6, 6, 4, 8, 0, 1e-10),
                                                  (4, 6, 3, 5, 0, 1e-10), (6, 6, 4, 8, 1, 1e-3),
                                                  (4, 6, 8, 16, 0, 1e-10)])
def test_plaquette_ratios_match_oracle(Ly, Lx, D, Dc, prec, tol):
    import torch
    print(f"plaquette ratios {Ly}x{Lx} D={D} Dc={Dc} prec={prec}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=50 + D)
    cfgs = W.random_configs(Ly, Lx, 3, seed=51)
    lat = olat.Lattice(Ly, Lx, D, Dc)
    ctx = _ctx(Ly, Lx, D, Dc, prec, 3, T=T)
    dev = torch.device("cuda")
    out = torch.full((3, (Ly - 1) * (Lx - 1)), 7.0, dtype=torch.float64, device=dev)
    ctx.vp_plaquette_ratios(0, torch.tensor(cfgs, device=dev), 3, out)
    g = out.cpu().numpy()
    ctx.close()
    for c in range(3):
        ref = vmc.plaquette_ratios(T, lat, cfgs[c]).ravel()
        mov = P.movable(cfgs[c], Ly, Lx).ravel()
        assert np.all(g[c][~mov] == 0.0)
        err = np.abs(g[c] - ref) / np.maximum(np.abs(ref), 1.0)
        assert err.max() <= tol, (c, err.max())


def test_forward_matches_oracle():
    import torch
    Ly, Lx = 5, 6
    print("proposal forward 5x6", flush=True)
    th = _theta(1)
    cfgs = W.random_configs(Ly, Lx, 4, seed=2)
    ctx = _ctx(Ly, Lx, 2, 4, 1, 4, theta=th)
    dev = torch.device("cuda")
    z = torch.empty((4, Ly, Lx), dtype=torch.float32, device=dev)
    ctx.vp_proposal_forward(0, torch.tensor(cfgs, device=dev), 4, z)
    g = z.cpu().numpy()
    ctx.close()
    for c in range(4):
        ref, _ = P.forward(th.astype(np.float64), cfgs[c], Ly, Lx)
        # float32 sums of <= 289 terms of size ~0.3 x activations: relative 1e-5 of the map's scale
        assert np.max(np.abs(g[c] - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref))), c


def test_loss_gradient_matches_oracle():
    import torch
    Ly, Lx, n = 4, 6, 5
    print("proposal loss/grad 4x6", flush=True)
    th = _theta(3)
    cfgs = W.random_configs(Ly, Lx, n, seed=4)
    rho = np.random.default_rng(5).normal(0, 1.2, size=(n, Ly - 1, Lx - 1))
    targets = np.minimum(1.0, rho ** 2)
    ref_l = P.loss(th.astype(np.float64), cfgs, targets, Ly, Lx)
    ref_g = P.backward(th.astype(np.float64), cfgs, targets, Ly, Lx)
    ctx = _ctx(Ly, Lx, 2, 4, 1, n, theta=th)
    dev = torch.device("cuda")
    grad = torch.empty(P.n_params(), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    ctx.vp_proposal_loss_grad(0, torch.tensor(cfgs, device=dev),
                              torch.tensor(rho.reshape(n, -1), dtype=torch.float64, device=dev), n, grad, loss)
    g = grad.double().cpu().numpy()
    ctx.close()
    assert abs(loss.item() - ref_l) <= 1e-5 * max(1.0, abs(ref_l))
    # float32 forward and backward: 1e-4 of the gradient's scale per layer block
    bounds = np.cumsum([0] + [co * ci * 9 + co for ci, co in P.LAYERS])
    for i in range(4):
        a, b = bounds[i], bounds[i + 1]
        assert np.max(np.abs(g[a:b] - ref_g[a:b])) <= 1e-4 * max(1e-3, np.max(np.abs(ref_g[a:b]))), i


@pytest.mark.parametrize("Ly,Lx,D,Dc,n,sweeps", [(4, 4, 2, 4, 3, 6), (6, 6, 4, 8, 2, 3), (4, 5, 3, 4, 2, 3),
                                                 (4, 6, 8, 16, 2, 2)])
def test_learned_sampler_bit_exact_fp64(Ly, Lx, D, Dc, n, sweeps):
    """Learned chains in float64: every configuration and move count equals the oracle's."""
    import torch
    B = _B()
    print(f"learned sampler fp64 {Ly}x{Lx} D={D} Dc={Dc} {n} chains x {sweeps}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=60 + Ly)
    th = _theta(61, bias4=0.5)
    seed = 77
    ctx = _ctx(Ly, Lx, D, Dc, B.VP_FP64, n, seed=seed, T=T, theta=th)
    dev = torch.device("cuda")
    ctx.vp_init_chains(0, None)
    ctx.vp_set_sampler(0, B.VP_SAMPLER_LEARNED_PLAQ)
    N = Ly * Lx
    lp = torch.empty(n * sweeps, dtype=torch.float64, device=dev)
    sg = torch.empty(n * sweeps, dtype=torch.int8, device=dev)
    el = torch.empty(n * sweeps, dtype=torch.float64, device=dev)
    so = torch.empty((n * sweeps, N), dtype=torch.int8, device=dev)
    cnt = torch.empty((n, 4), dtype=torch.int64, device=dev)
    ctx.vp_sample(0, 0, sweeps, lp, sg, el, None, so, None)
    ctx.vp_move_counts(0, cnt)
    ctx.vp_sync()
    spins = so.cpu().numpy().reshape(n, sweeps, N)
    e = el.cpu().numpy().reshape(n, sweeps)
    counts = cnt.cpu().numpy()
    ctx.close()
    lat = olat.Lattice(Ly, Lx, D, Dc)
    for c in range(n):
        ch = vmc.Chain(lat, olat.neel_shuffled(lat, seed, 0, c), seed, 0, c)
        o = vmc.run_chain(T, lat, ch, 0, sweeps, proposal=th.astype(np.float64))
        assert np.array_equal(spins[c], np.stack([x["spins"] for x in o])), c
        assert np.max(np.abs(e[c] - np.array([x["e_loc"] for x in o]))) / N <= 1e-10
        assert tuple(counts[c]) == (ch.accepted, ch.proposed, ch.plaq_accepted, ch.plaq_proposed), c
    assert counts[:, 3].sum() > 0 and counts[:, 2].sum() > 0


def test_learned_sampler_samples_psi2():
    """2x4, exact contraction: 2048 independent chains, one sample each after 24 sweeps."""
    import torch
    B = _B()
    Ly, Lx, D = 2, 4, 2
    n = 2048
    print("learned sampler chi2 2x4 2048 chains", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=13)
    th = _theta(14, bias4=1.0)
    ctx = _ctx(Ly, Lx, D, 8, B.VP_FP64, n, seed=99, T=T, theta=th)
    dev = torch.device("cuda")
    ctx.vp_init_chains(0, None)
    ctx.vp_set_sampler(0, B.VP_SAMPLER_LEARNED_PLAQ)
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    so = torch.empty((n, Ly * Lx), dtype=torch.int8, device=dev)
    cnt = torch.empty((n, 4), dtype=torch.int64, device=dev)
    ctx.vp_sample(0, 23, 1, lp, sg, el, None, so, None)
    ctx.vp_move_counts(0, cnt)
    ctx.vp_sync()
    samples = so.cpu().numpy()
    counts = cnt.cpu().numpy().sum(axis=0)
    ctx.close()
    assert counts[3] > 0 and 0 < counts[2] < counts[3]
    configs = bf.sz0_configs(Ly * Lx)
    psi = bf.amplitudes(T, Ly, Lx, D, configs)
    p = psi ** 2 / np.sum(psi ** 2)
    index = {c.tobytes(): i for i, c in enumerate(configs)}
    obs = np.zeros(len(configs))
    for s in samples:
        obs[index[s.tobytes()]] += 1
    keep = p * n >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(p[keep] * n, p[~keep].sum() * n)
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    stat, pval = scipy.stats.chisquare(o, e)
    assert pval > 1e-3, (stat, pval)


def test_training_lowers_the_loss():
    """Sampler configurations -> plaquette ratios -> Adam: the epoch loss falls and the
    trained propensity tracks the acceptance probability better than the untrained one."""
    import torch
    B = _B()
    Ly, Lx, D, Dc, n = 6, 6, 4, 8, 256
    print("proposal training 6x6 D=4 Dc=8 256 configs", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=70)
    th = _theta(71, scale=0.05)
    ctx = _ctx(Ly, Lx, D, Dc, B.VP_FP32, n, seed=72, T=T, theta=th)
    dev = torch.device("cuda")
    ctx.vp_init_chains(0, None)
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    so = torch.empty((n, Ly * Lx), dtype=torch.int8, device=dev)
    ctx.vp_sample(0, 3, 1, lp, sg, el, None, so, None)
    rho = torch.empty((n, (Ly - 1) * (Lx - 1)), dtype=torch.float64, device=dev)
    ctx.vp_plaquette_ratios(0, so, n, rho)
    grad = torch.empty(P.n_params(), dtype=torch.float32, device=dev)
    l0 = torch.empty(1, dtype=torch.float64, device=dev)
    ctx.vp_proposal_loss_grad(0, so, rho, n, grad, l0)
    losses = torch.empty(8, dtype=torch.float64, device=dev)
    ctx.vp_proposal_train(0, so, rho, n, 8, 32, 3e-3, 5, losses)
    l1 = torch.empty(1, dtype=torch.float64, device=dev)
    ctx.vp_proposal_loss_grad(0, so, rho, n, grad, l1)
    ctx.vp_sync()
    ls = losses.cpu().numpy()
    print(f"loss before {l0.item():.4f} epochs {np.round(ls, 4)} after {l1.item():.4f}", flush=True)
    ctx.close()
    assert np.all(np.isfinite(ls))
    assert l1.item() < l0.item() and ls[-1] < ls[0]


@pytest.mark.parametrize("prec", ["VP_FP64", "VP_FP32", "VP_BF16"])
def test_sweep_logits_match_oracle(prec):
    """The network as the learned sweep evaluates it (vp_proposal_logits_sweep: the
    local 9x9 window of every plaquette, both directions of the move) against the
    oracle's full-lattice forward pass at the plaquette's top-left site.  float64:
    1e-12; float32: 1e-5 relative to the largest |logit|; bf16 inference against
    the oracle's bf16 inference (forward_bf16): median 1e-5 and at most 2e-2 of the
    largest |logit| (an activation that sits at a bf16 rounding boundary can round
    the other way under a different float32 summation order), and measurably away
    from the float64 network (the rounding is really there)."""
    import torch
    from oracle import proposal as Pn
    B = _B()
    Ly, Lx, n = 6, 8, 6
    print(f"sweep logits {prec} {Ly}x{Lx}, {n} configurations", flush=True)
    th = np.random.default_rng(12).normal(scale=0.2, size=Pn.n_params()).astype(np.float32)
    cfgs = W.random_configs(Ly, Lx, n, seed=13)
    dev = torch.device("cuda")
    ctx = B.Context(B.lattice(Ly, Lx, 2, 4, 1.0, 0.0, getattr(B, prec), 1), seed=1)
    ctx.vp_proposal_set_weights(0, torch.tensor(th, device=dev))
    sp = torch.tensor(cfgs, dtype=torch.int8, device=dev)
    P = (Ly - 1) * (Lx - 1)
    got = {}
    for flip in (0, 1):
        out = torch.empty((n, P), dtype=torch.float64, device=dev)
        ctx.vp_proposal_logits_sweep(0, sp, n, flip, out)
        torch.cuda.synchronize()
        got[flip] = out.cpu().numpy()
    ctx.close()
    theta = th.astype(np.float64)
    ref = {0: np.zeros((n, P)), 1: np.zeros((n, P))}
    ref64 = {0: np.zeros((n, P)), 1: np.zeros((n, P))}
    fwd = Pn.forward_bf16 if prec == "VP_BF16" else (lambda t, s, a, b: Pn.forward(t, s, a, b)[0])
    for i in range(n):
        for q in range(P):
            y, x = divmod(q, Lx - 1)
            for flip in (0, 1):
                s = cfgs[i].reshape(Ly, Lx).copy()
                if flip:
                    s[y:y + 2, x:x + 2] ^= 1
                ref[flip][i, q] = fwd(theta, s.ravel(), Ly, Lx)[y, x]
                ref64[flip][i, q] = Pn.forward(theta, s.ravel(), Ly, Lx)[0][y, x]
    scale = max(np.abs(ref[0]).max(), np.abs(ref[1]).max())
    d = np.concatenate([np.abs(got[f] - ref[f]).ravel() for f in (0, 1)])
    print(f"{prec}: max |dz| {d.max():.2e}, median {np.median(d):.2e}, largest |z| {scale:.2f}", flush=True)
    if prec == "VP_FP64":
        assert d.max() <= 1e-12 * max(1.0, scale)
    elif prec == "VP_FP32":
        assert d.max() <= 1e-5 * max(1.0, scale)
    else:
        d64 = np.concatenate([np.abs(got[f] - ref64[f]).ravel() for f in (0, 1)])
        print(f"bf16 against the float64 network: median {np.median(d64):.2e}", flush=True)
        assert np.median(d) <= 1e-5 * max(1.0, scale)
        assert d.max() <= 2e-2 * max(1.0, scale)
        assert np.median(d64) >= 20 * max(np.median(d), 1e-7)

