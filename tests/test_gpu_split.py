"""Two truncation cutoffs on the GPU (Sec. II.A, App. D): chains moved at Dc1,
their states measured at Dc2.

The oracle side composes two pinned oracle functions: its chain at Dc1 (the
decisions, hence the configurations, are the sampler's) and its fixed-
configuration evaluation at Dc2.  float64: configurations bit-exact, E_loc,
log|Psi| and dlnPsi to rounding.  The paper's production shape (D=8,
Dc1 = 2D = 16, Dc2 = 3D = 24) is measured with the variational fit (App. B),
the compression the paper itself uses; the canonical one stops at D*Dc = 128.
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


@pytest.mark.parametrize("Ly,Lx,D,Dc1,Dc2,J2,fit2", [(4, 4, 3, 4, 9, 0.0, 0), (4, 6, 4, 8, 12, 0.5, 0),
                                                     (4, 6, 8, 16, 24, 0.5, 2)])
def test_split_cutoffs_match_oracle(Ly, Lx, D, Dc1, Dc2, J2, fit2):
    import torch
    B = _B()
    print(f"split {Ly}x{Lx} D={D} Dc1={Dc1} Dc2={Dc2} J2={J2} "
          f"{'fit ' + str(fit2) + ' sweeps' if fit2 else 'canonical'} at Dc2", flush=True)
    n, nb, nm, seed = 3, 1, 2, 31
    N = Ly * Lx
    T = W.random_tensors(Ly, Lx, D, seed=70 + D)
    ctx = B.Context([B.lattice(Ly, Lx, D, Dc1, 1.0, J2, B.VP_FP64, n),
                     B.lattice(Ly, Lx, D, Dc2, 1.0, J2, B.VP_FP64, n,
                               B.VP_COMPRESS_VARIATIONAL if fit2 else B.VP_COMPRESS_CANONICAL, fit2)], seed=seed)
    dev = torch.device("cuda")
    tt = torch.tensor(T, dtype=torch.float64, device=dev)
    ctx.vp_set_tensors(0, tt)
    ctx.vp_set_tensors(1, tt)
    ctx.vp_init_chains(0, None)
    lp = torch.empty(n * nm, dtype=torch.float64, device=dev)
    sg = torch.empty(n * nm, dtype=torch.int8, device=dev)
    el = torch.empty(n * nm, dtype=torch.float64, device=dev)
    dl = torch.empty((n * nm, ctx.num_params(1) // 2), dtype=torch.float64, device=dev)
    so = torch.empty((n * nm, N), dtype=torch.int8, device=dev)
    ctx.vp_sample_split(0, 1, nb, nm, lp, sg, el, dl, so)
    ctx.vp_sync()
    g = dict(lp=lp.cpu().numpy().reshape(n, nm), sg=sg.cpu().numpy().reshape(n, nm),
             el=el.cpu().numpy().reshape(n, nm), dl=dl.cpu().numpy().reshape(n, nm, -1),
             so=so.cpu().numpy().reshape(n, nm, N))
    ctx.close()
    lat1 = olat.Lattice(Ly, Lx, D, Dc1, J2=J2)
    lat2 = (olat.Lattice(Ly, Lx, D, Dc2, J2=J2, compress_mode="variational", fit_sweeps=fit2) if fit2
            else olat.Lattice(Ly, Lx, D, Dc2, J2=J2))
    differs = 0.0
    for c in range(n):
        ch = vmc.Chain(lat1, olat.neel_shuffled(lat1, seed, 0, c), seed, 0, c)
        o1 = vmc.run_chain(T, lat1, ch, nb, nm)
        for m in range(nm):
            s = o1[m]["spins"]
            assert np.array_equal(g["so"][c, m], s), (c, m)
            o2 = vmc.eval_config(T, lat2, s)
            assert g["sg"][c, m] == o2["sign"]
            assert abs(g["lp"][c, m] - o2["log_abs_psi"]) <= 1e-10
            assert abs(g["el"][c, m] - o2["e_loc"]) / N <= 1e-10
            od = np.asarray(o2["dlnpsi"]).ravel()
            assert np.max(np.abs(g["dl"][c, m] - od)) <= 1e-9 * max(1.0, np.max(np.abs(od)))
            differs = max(differs, abs(o2["e_loc"] - o1[m]["e_loc"]))
    # the measuring cutoff is really used: the truncated Dc1 energy differs
    assert differs > 1e-8


def test_split_rejects_mismatched_lattices():
    import torch
    B = _B()
    ctx = B.Context([B.lattice(4, 4, 2, 2, 1.0, 0.0, B.VP_FP64, 2),
                     B.lattice(4, 4, 3, 4, 1.0, 0.0, B.VP_FP64, 2)], seed=3)
    dev = torch.device("cuda")
    lp = torch.empty(2, dtype=torch.float64, device=dev)
    sg = torch.empty(2, dtype=torch.int8, device=dev)
    el = torch.empty(2, dtype=torch.float64, device=dev)
    with pytest.raises(Exception):
        ctx.vp_sample_split(0, 1, 0, 1, lp, sg, el)
    ctx.close()
