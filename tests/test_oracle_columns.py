"""Pins of the oracle's column-wise vertical bonds (``oracle.columns``; App. C's
"similarly computed" read as 3-line networks between column boundary MPS).

* The transposed PEPS is the same state: every amplitude of the transposed
  configuration equals the original's (brute force, independent of
  ``oracle.peps``), on lattices with Ly != Lx.
* Exact regime (Dc at the exact rank): the column-wise evaluation equals brute
  force in E_loc and in every ratio, horizontal and vertical.
* The chain samples |Psi|^2 (chi-square on a 2x3 lattice) and moves the
  magnetisation between the rows (the vertical bonds are visited).
* The nearest-neighbour square lattice only: J2 != 0 and the triangular
  geometry are rejected.
"""
import itertools

import numpy as np
import pytest
import scipy.stats

import bruteforce as bf
from oracle import columns as cols
from oracle import vmc
from oracle.lattice import Lattice, neel_shuffled


def _T(lat, seed):
    return np.random.default_rng(seed).standard_normal(lat.Np) / lat.D ** 2


@pytest.mark.parametrize("Ly,Lx,D", [(2, 3, 2), (3, 4, 2), (4, 2, 3)])
def test_transposed_peps_is_the_same_state(Ly, Lx, D):
    lat = Lattice(Ly, Lx, D, 16)
    T = _T(lat, 7)
    lt, Tt = cols.transposed(lat), cols.transpose_tensors(T, lat)
    cfgs = np.array(list(itertools.product([0, 1], repeat=Ly * Lx)), dtype=np.int8)
    psi = bf.amplitudes(T, Ly, Lx, D, cfgs)
    psi_t = bf.amplitudes(Tt, Lx, Ly, D, np.stack([cols.transpose_spins(c, lat) for c in cfgs]))
    assert np.max(np.abs(psi - psi_t)) <= 1e-13 * np.max(np.abs(psi))
    for c in cfgs[:5]:
        assert np.array_equal(cols.untranspose_spins(cols.transpose_spins(c, lat), lat), c)


@pytest.mark.parametrize("Ly,Lx", [(4, 4), (3, 4), (4, 3)])
def test_exact_regime_equals_brute_force(Ly, Lx):
    lat = Lattice(Ly, Lx, 2, 16)
    T = _T(lat, 11)
    cfgs = bf.sz0_configs(Ly * Lx)[::97][:6]
    e_ref, psi = bf.local_energies(T, Ly, Lx, 2, 1.0, 0.0, cfgs)
    bl = bf.bonds(Ly, Lx, 1.0, 0.0)
    for c, er, pr in zip(cfgs, e_ref, psi):
        o = cols.eval_config(T, lat, c)
        assert abs(o["e_loc"] - er) <= 1e-10 * max(1.0, abs(er))
        assert abs(o["log_abs_psi"] - np.log(abs(pr))) <= 1e-11 and o["sign"] == np.sign(pr)
        for b, (i, j, _) in enumerate(bl):
            if c[i] != c[j]:
                f = c.copy()
                f[i], f[j] = c[j], c[i]
                rho = bf.amplitudes(T, Ly, Lx, 2, f[None])[0] / pr
                assert abs(o["ratios"][b] - rho) <= 1e-9 * max(1.0, abs(rho))
            else:
                assert o["ratios"][b] == 0.0


def test_chain_samples_psi_squared_and_visits_vertical_bonds():
    lat = Lattice(2, 3, 2, 8)
    T = _T(lat, 1)
    configs = bf.sz0_configs(6)
    psi = bf.amplitudes(T, 2, 3, 2, configs)
    p = psi ** 2 / np.sum(psi ** 2)
    index = {c.tobytes(): i for i, c in enumerate(configs)}
    counts = np.zeros(len(configs))
    for chain in range(4):
        ch = vmc.Chain(lat, neel_shuffled(lat, 9359, 0, chain), 1234, 0, chain)
        for smp in cols.run_chain(T, lat, ch, 10, 500):
            counts[index[smp["spins"].tobytes()]] += 1
    n = counts.sum()
    keep = p * n >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(p[keep] * n, p[~keep].sum() * n)
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    assert scipy.stats.chisquare(obs, exp)[1] > 1e-4
    top = {int(c[:3].sum()) for c, k in zip(configs, counts) if k > 0}
    assert len(top) > 1


def test_rejects_diagonal_terms():
    with pytest.raises(ValueError):
        cols.transposed(Lattice(4, 4, 2, 4, J2=0.5))
    with pytest.raises(ValueError):
        cols.transposed(Lattice(4, 4, 2, 4, geometry="triangular"))
