"""GPU simple update (vp_simple_update, App. A) against the oracle
(oracle/simple_update.py), through the C ABI.

The two sides take the SVD differently (the GPU from the eigenproblem of
Theta Theta^T, the oracle from LAPACK), so their site tensors may differ by a
sign on each link (a gauge that cancels in the state).  Compared: every
link's lambda (unique), App. A's convergence measure per step, and every
amplitude of the absorbed state in the S^z = 0 sector by exact contraction
(tests/bruteforce.py).  Bounds: 1e-12 on the lambdas, 1e-11 relative on the
amplitudes and 1e-10 relative on the changes (measured: 5e-15 and 2e-14; a few
steps from random tensors, so no nearly degenerate truncation decides the
result, and the Gram route's squared conditioning stays far below them).

The J1-J2 cases add the next-nearest-neighbour (three-site) update of Fig. 8.

Also: two calls of 2 and 3 steps give the 5-step call bit for bit; zero steps
leave the tensors unchanged; a negative step count is rejected; with J1 = 0
the two diagonals of a 2x2 plaquette converge to two singlets (E = -3/2); and
on the 4x4 Heisenberg lattice at D = 4, 100 steps of dt = 0.05 bring the
energy of the absorbed state within 5% of the exact ground energy and not
below it.
"""
import numpy as np
import pytest

import bruteforce as bf
from oracle import lattice as olat
from oracle import simple_update as su
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu


def _B():
    from paper_1908_09359_amd import binding
    return binding


def _n_links(Ly, Lx):
    return Ly * (Lx - 1) + (Ly - 1) * Lx


def _gpu_su(Ly, Lx, D, T, calls, J2=0.0):
    """Run vp_simple_update once per (dt, steps) in calls; returns T, lambdas, changes."""
    import torch
    B = _B()
    ctx = B.Context(B.lattice(Ly, Lx, D, 4, 1.0, J2, B.VP_FP64, 1), seed=1)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    changes = []
    for dt, steps in calls:
        ch = torch.zeros(max(steps, 1), dtype=torch.float64, device=dev)
        ctx.vp_simple_update(0, dt, steps, ch)
        changes += ch.cpu().numpy()[:steps].tolist()
    Tg = torch.empty(ctx.num_params(), dtype=torch.float64, device=dev)
    ctx.vp_get_tensors(0, Tg)
    lam = torch.empty((_n_links(Ly, Lx), D), dtype=torch.float64, device=dev)
    ctx.vp_simple_update_lambdas(0, lam)
    torch.cuda.synchronize()
    out = Tg.cpu().numpy(), lam.cpu().numpy(), np.array(changes)
    ctx.close()
    return out


@pytest.mark.parametrize("Ly,Lx,D,J2,dt,steps", [
    (1, 4, 4, 0.0, 0.1, 2),     # open chain, no truncation (exact Trotter product on the oracle side)
    (4, 1, 4, 0.0, 0.1, 2),     # the same along the vertical links
    (3, 4, 3, 0.0, 0.05, 3),    # truncated, ragged rows of links
    (4, 4, 2, 0.0, 0.1, 4),
    (2, 6, 4, 0.0, 0.05, 3),    # QR-reduced sites (outer extent 16 > 2D = 8)
    (3, 4, 3, 0.5, 0.05, 3),    # J1-J2: three-site updates, every plaquette class
    (4, 4, 2, 0.5, 0.1, 3),
    (3, 4, 4, 0.3, 0.05, 2),    # QR-reduced end sites of the diagonals (interior sites: 64 > 2D rows)
])
def test_simple_update_matches_oracle(Ly, Lx, D, J2, dt, steps):
    print(f"simple update {Ly}x{Lx} D={D} J2={J2} dt={dt} steps={steps}", flush=True)
    lat = olat.Lattice(Ly, Lx, D, 4, J2=J2)
    T = W.random_tensors(Ly, Lx, D, seed=400 + Ly * Lx + D)
    Tg, lam_g, ch_g = _gpu_su(Ly, Lx, D, T, [(dt, steps)], J2=J2)
    To, ch_o, _, lam_o = su.simple_update(T, lat, dt, steps)
    assert np.max(np.abs(lam_g - np.array(lam_o))) <= 1e-12
    assert np.max(np.abs(ch_g - np.array(ch_o)) / np.maximum(np.abs(ch_o), 1e-300)) <= 1e-10
    cfgs = np.array(bf.sz0_configs(Ly * Lx))
    pg = bf.amplitudes(Tg, Ly, Lx, D, cfgs)
    po = bf.amplitudes(To, Ly, Lx, D, cfgs)
    dev = np.max(np.abs(pg - po)) / np.max(np.abs(po))
    print(f"max |dlambda| {np.max(np.abs(lam_g - np.array(lam_o))):.2e}, amplitudes {dev:.2e}", flush=True)
    assert dev <= 1e-11


def test_continuation_and_zero_steps_are_exact():
    Ly, Lx, D = 3, 4, 3
    T = W.random_tensors(Ly, Lx, D, seed=77)
    T5, lam5, ch5 = _gpu_su(Ly, Lx, D, T, [(0.05, 5)])
    T23, lam23, ch23 = _gpu_su(Ly, Lx, D, T, [(0.05, 2), (0.05, 3)])
    assert np.array_equal(T5, T23) and np.array_equal(lam5, lam23) and np.array_equal(ch5, ch23)
    T0, lam0, _ = _gpu_su(Ly, Lx, D, T, [(0.05, 0)])
    assert np.array_equal(T0, T) and np.all(lam0 == 1.0)


def test_state_rules():
    import torch
    B = _B()
    dev = torch.device("cuda")
    ctx = B.Context(B.lattice(4, 4, 2, 4, 1.0, 0.0, B.VP_FP64, 1), seed=1)
    ctx.vp_init_tensors(0, seed=3, scale=0.0, perturb=0.0)
    with pytest.raises(B.VPError) as ei:
        ctx.vp_simple_update(0, 0.05, -1)
    assert ei.value.status == B.VP_ERR_ARG
    ctx.vp_init_tensors(0, seed=3, scale=0.0, perturb=0.0)
    ctx.vp_simple_update(0, 0.05, 2)
    lam = torch.empty((_n_links(4, 4), 2), dtype=torch.float64, device=dev)
    ctx.vp_simple_update_lambdas(0, lam)
    ctx.vp_init_tensors(0, seed=4, scale=0.0, perturb=0.0)  # new tensors: the evolution is gone
    with pytest.raises(B.VPError) as ei:
        ctx.vp_simple_update_lambdas(0, lam)
    assert ei.value.status == B.VP_ERR_ARG
    ctx.close()


def test_decoupled_diagonals_converge_to_two_singlets():
    """J1 = 0, J2 = 1 on 2x2: the diagonals are independent pairs; the evolution
    (three-site updates only) reaches the product of their singlets, E = -3/2."""
    import itertools
    T = W.random_tensors(2, 2, 4, seed=8)
    B = _B()
    import torch
    dev = torch.device("cuda")
    ctx = B.Context(B.lattice(2, 2, 4, 4, 0.0, 1.0, B.VP_FP64, 1), seed=1)
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ch = torch.zeros(150, dtype=torch.float64, device=dev)
    ctx.vp_simple_update(0, 0.2, 150, ch)
    Tg = torch.empty(ctx.num_params(), dtype=torch.float64, device=dev)
    ctx.vp_get_tensors(0, Tg)
    torch.cuda.synchronize()
    Tg = Tg.cpu().numpy()
    ctx.close()
    cfgs = np.array(list(itertools.product([0, 1], repeat=4)), dtype=np.int8)
    psi = bf.amplitudes(Tg, 2, 2, 4, cfgs)
    sz = np.array([[0.5, 0.0], [0.0, -0.5]])
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    h = np.kron(sz, sz) + 0.5 * (np.kron(sp, sp.T) + np.kron(sp.T, sp))

    def apply(v, i, j):
        t = np.moveaxis(v.reshape([2] * 4), [i, j], [0, 1])
        sh = t.shape
        return np.moveaxis((h @ t.reshape(4, -1)).reshape(sh), [0, 1], [i, j]).ravel()
    e = psi @ (apply(psi, 0, 3) + apply(psi, 1, 2)) / (psi @ psi)
    print(f"decoupled diagonals: E {e:.12f}, last change {ch[-1].item():.2e}", flush=True)
    assert abs(e + 1.5) <= 1e-10


def _exact_ground_energy_4x4():
    import scipy.sparse
    import scipy.sparse.linalg
    Ly = Lx = 4
    N = 16
    cfgs = np.array(bf.sz0_configs(N))
    codes = (cfgs.astype(np.int64) << np.arange(N, dtype=np.int64)[::-1]).sum(axis=1)
    order = np.argsort(codes)
    rows, cols, vals = [], [], []
    diag = np.zeros(len(cfgs))
    for y in range(Ly):
        for x in range(Lx):
            k = y * Lx + x
            for k2 in ([k + 1] if x < Lx - 1 else []) + ([k + Lx] if y < Ly - 1 else []):
                par = cfgs[:, k] == cfgs[:, k2]
                diag += np.where(par, 0.25, -0.25)
                idx = np.nonzero(~par)[0]
                partner = codes[idx] ^ ((1 << (N - 1 - k)) | (1 << (N - 1 - k2)))
                j = order[np.searchsorted(codes[order], partner)]
                rows += idx.tolist(); cols += j.tolist(); vals += [0.5] * len(idx)
    n = len(cfgs)
    H = scipy.sparse.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr() + scipy.sparse.diags(diag)
    return float(scipy.sparse.linalg.eigsh(H, k=1, which="SA")[0][0])


def test_simple_update_approaches_the_ground_state_4x4():
    Ly = Lx = 4
    D = 4
    print("simple update 4x4 D=4, 100 steps of dt 0.05", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=5)
    Tg, _, ch = _gpu_su(Ly, Lx, D, T, [(0.05, 100)])
    cfgs = np.array(bf.sz0_configs(16))
    e0 = bf.sector_energy(bf.amplitudes(T, Ly, Lx, D, cfgs), cfgs, Ly, Lx)
    e = bf.sector_energy(bf.amplitudes(Tg, Ly, Lx, D, cfgs), cfgs, Ly, Lx)
    ex = _exact_ground_energy_4x4()
    print(f"E/site: start {e0 / 16:.5f}, after {e / 16:.5f}, exact {ex / 16:.5f}; last change {ch[-1]:.2e}",
          flush=True)
    assert e >= ex - 1e-9
    assert e <= 0.95 * ex
    assert ch[-1] < 0.1 * ch[0]
