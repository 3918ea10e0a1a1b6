"""Algorithm 1 on the GPU (vp_optimize): sampling, the Eq. (5) gradient and the
Eq. (10) sign-gradient update, step after step.

* one float64 step against the oracle: the oracle's chains (the sampler is
  bit-exact), its gradient and its sign-gradient update give the same tensors;
* a short optimisation of the 4x4 Heisenberg antiferromagnet at D=2 from
  random tensors lowers the energy towards the exact ground state
  (-0.5743/site by exact diagonalisation in the S^z = 0 sector), with staged
  step lengths as the paper uses;
* the paper's order (Sec. II.B): the simple-update state (App. A) as the
  start of Algorithm 1.  At 4x4, D=4 (exact contraction, Dc=16) the same 40
  optimisation steps started from the simple-update state reach the exact
  energy to about 1e-4 per site, from random tensors 0.017 above it.
"""
import numpy as np
import pytest

from oracle import lattice as olat
from oracle import vmc
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu


def _B():
    from paper_1908_09359_amd import binding as B
    return B


def test_one_step_matches_oracle():
    import torch
    B = _B()
    Ly, Lx, D, Dc, n, nb, nm, seed, delta = 4, 4, 2, 4, 4, 1, 2, 19, 0.01
    print("optimize one step 4x4 D=2 Dc=4", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=81)
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, B.VP_FP64, n), seed=seed)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None)
    e = ctx.vp_optimize(0, [delta], nb, nm, step0=0)
    Tg = torch.empty(len(T), dtype=torch.float64, device=dev)
    ctx.vp_get_tensors(0, Tg)
    ctx.vp_sync()
    Tg = Tg.cpu().numpy()
    ctx.close()
    lat = olat.Lattice(Ly, Lx, D, Dc)
    el, dl, sp = [], [], []
    for c in range(n):
        ch = vmc.Chain(lat, olat.neel_shuffled(lat, seed, 0, c), seed, 0, c)
        for x in vmc.run_chain(T, lat, ch, nb, nm):
            el.append(x["e_loc"])
            dl.append(np.asarray(x["dlnpsi"]).ravel())
            sp.append(x["spins"])
    g, E = vmc.gradient(lat, el, dl, sp)
    To = vmc.sign_sgd(T, g, delta, seed, 0, 0)
    assert abs(e[0] - E) <= 1e-10 * max(1.0, abs(E))
    # an element whose gradient is at rounding level may take either sign
    clear = np.abs(g) > 1e-9 * np.max(np.abs(g))
    assert np.max(np.abs(Tg - To)[clear]) <= 1e-12
    assert np.all(np.abs(Tg - T) <= delta + 1e-15)
    assert np.count_nonzero(Tg != T) > len(T) // 2


def test_optimisation_lowers_the_energy():
    import torch
    B = _B()
    Ly, Lx, D, Dc, n = 4, 4, 2, 4, 128
    print("optimize 4x4 D=2 Dc=4 Heisenberg, 128 chains", flush=True)
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, B.VP_FP64, n), seed=5)
    ctx.vp_init_tensors(0, seed=6, scale=0.0, perturb=0.0)
    ctx.vp_init_chains(0, None)
    deltas = [0.05] * 30 + [0.02] * 30 + [0.01] * 20
    e = np.array(ctx.vp_optimize(0, deltas, 2, 8)) / (Ly * Lx)
    ctx.close()
    print("E/site first", e[:3], "last", e[-3:], flush=True)
    assert np.all(np.isfinite(e))
    assert e[-10:].mean() < e[:3].mean() - 0.1
    # D=2 reaches about -0.556 here (3% above the exact -0.5743)
    assert e[-10:].mean() < -0.53


def test_simple_update_start_then_optimisation():
    import torch
    B = _B()
    Ly, Lx, D, Dc, n = 4, 4, 4, 16, 128
    print("simple update + optimize 4x4 D=4 Dc=16 Heisenberg, 128 chains", flush=True)
    deltas = [0.005] * 20 + [0.002] * 20
    out = {}
    for start in ("random", "simple update"):
        ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, B.VP_FP64, n), seed=5)
        ctx.vp_init_tensors(0, seed=6, scale=0.0, perturb=0.0)
        if start == "simple update":
            ctx.vp_simple_update(0, 0.05, 100)
        ctx.vp_init_chains(0, None)
        e = np.array(ctx.vp_optimize(0, deltas, 4, 8)) / (Ly * Lx)
        ctx.close()
        assert np.all(np.isfinite(e))
        out[start] = e
        print(f"{start}: E/site first {e[:3]}, last 10 {e[-10:].mean():.5f}", flush=True)
    su, rnd = out["simple update"], out["random"]
    # the simple-update state alone is at -0.5627 per site; measured after 40 steps:
    # -0.57426 from it against -0.5578 from random tensors (exact -0.57433)
    assert su[-10:].mean() < rnd[-10:].mean() - 0.005
    assert su[-10:].mean() < -0.570


def test_zero_amplitude_stops_before_the_update():
    """A chain whose configuration has Psi = 0 is flagged by the sampler and left
    unmeasured; vp_optimize must report it before its gradient or update can
    touch the tensors."""
    import torch
    B = _B()
    Ly, Lx, D, Dc = 4, 4, 2, 4
    print("optimize with a zero-amplitude chain 4x4 D=2 Dc=4", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=83)
    n0 = 1 * 1 * D * D          # site (0, 0): dims (l, u, r, d) = (1, 1, D, D)
    T[n0:2 * n0] = 0.0          # T_0[s = 1] = 0: every configuration with s_0 = 1 has Psi = 0
    lat = olat.Lattice(Ly, Lx, D, Dc)
    good = olat.neel(lat)       # s_0 = 0
    bad = 1 - good              # s_0 = 1
    assert good[0] == 0 and bad[0] == 1
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, B.VP_FP64, 2), seed=7)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, torch.tensor(np.stack([good, bad]), dtype=torch.int8, device=dev))
    with pytest.raises(B.VPError) as ei:
        ctx.vp_optimize(0, [0.01, 0.01], 0, 2)
    assert ei.value.status == B.VP_ERR_ZERO_AMPLITUDE
    Tg = torch.empty(len(T), dtype=torch.float64, device=dev)
    ctx.vp_get_tensors(0, Tg)
    torch.cuda.synchronize()
    assert np.array_equal(Tg.cpu().numpy(), T)
    ctx.close()
