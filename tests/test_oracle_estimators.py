"""Pins of the oracle's estimators and updates (Eqs. (2), (5), (10); Alg. 1; SR).

* Eq. (5) with exact weights |Psi|^2/Z, fed by the oracle's E_loc and G, equals
  one half of the finite-difference derivative of the exactly summed energy
  (the factor 2 of a real wave function is left out of Eq. (5)).
* ``gradient`` on explicit samples: hand-computed two-sample value, invariance
  under a constant shift of E_loc.
* SR: Cholesky solve, a general dense solve and the sample-space
  (push-through) form give the same update.
* Sign-gradient update: moves each element against the gradient sign by at
  most the step length, leaves zero-gradient elements untouched.
"""
import numpy as np
import scipy.linalg

import bruteforce as bf
from oracle import vmc
from oracle.lattice import Lattice, compact_size


def test_eq5_matches_finite_difference_of_exact_energy():
    Ly, Lx, D = 3, 4, 2
    lat = Lattice(Ly, Lx, D, 16, J2=0.3)
    T = np.random.default_rng(1).standard_normal(lat.Np) / 4
    cf = bf.sz0_configs(lat.N)

    def energy(Tv):
        e, psi = bf.local_energies(Tv, Ly, Lx, D, 1.0, 0.3, cf)
        w = psi ** 2
        return float(np.sum(w * e) / np.sum(w))

    outs = [vmc.eval_config(T, lat, c) for c in cf]
    w = np.exp(2 * np.array([o['log_abs_psi'] for o in outs]))
    w /= w.sum()
    e = np.array([o['e_loc'] for o in outs])
    O = np.stack([vmc.expand_dlnpsi(lat, o['dlnpsi'], c) for o, c in zip(outs, cf)])
    g = (w[:, None] * O * e[:, None]).sum(0) - (w[:, None] * O).sum(0) * (w * e).sum()
    assert abs((w * e).sum() - energy(T)) < 1e-11
    rng = np.random.default_rng(2)
    for p in rng.choice(lat.Np, size=6, replace=False):
        h = 1e-5
        Tp, Tm = T.copy(), T.copy()
        Tp[p] += h
        Tm[p] -= h
        fd = (energy(Tp) - energy(Tm)) / (2 * h)
        assert abs(2 * g[p] - fd) < 1e-6 * max(1.0, abs(fd)), (p, 2 * g[p], fd)


def test_gradient_two_samples_by_hand():
    lat = Lattice(1, 2, 1, 1)   # Np = 4, compact size 2
    dl = np.array([[1.0, 2.0], [3.0, 5.0]])
    spins = np.array([[0, 1], [1, 0]], dtype=np.int8)
    e = np.array([1.0, 3.0])
    g, E = vmc.gradient(lat, e, dl, spins)
    # full layout: sample 0 -> [1, 0, 0, 2], sample 1 -> [0, 3, 5, 0]
    # <O E> = ([1,0,0,2] + 3 [0,3,5,0]) / 2 ; <O> = ([1,3,5,2]) / 2 ; <E> = 2
    expect = (np.array([1, 9, 15, 2]) / 2) - (np.array([1, 3, 5, 2]) / 2) * 2
    assert E == 2.0
    assert np.allclose(g, expect)
    g2, _ = vmc.gradient(lat, e + 7.0, dl, spins)
    assert np.allclose(g2, g)


def test_sr_three_routes_agree():
    lat = Lattice(2, 2, 2, 4)
    rng = np.random.default_rng(3)
    Ns = 40
    dl = rng.standard_normal((Ns, compact_size(lat)))
    spins = np.array([rng.permutation([0, 0, 1, 1]) for _ in range(Ns)], dtype=np.int8)
    e = rng.standard_normal(Ns)
    shift = 1e-4
    delta, g = vmc.sr_step(lat, e, dl, spins, shift)
    O = np.stack([vmc.expand_dlnpsi(lat, dl[i], spins[i]) for i in range(Ns)])
    Ob = O - O.mean(0)
    S = Ob.T @ Ob / Ns + shift * np.eye(lat.Np)
    g_ref, _ = vmc.gradient(lat, e, dl, spins)
    assert np.allclose(g, g_ref, atol=1e-13)
    assert np.allclose(delta, scipy.linalg.solve(S, g_ref, assume_a='pos'), rtol=1e-8, atol=1e-10)
    Eb = e - e.mean()
    push = Ob.T @ np.linalg.solve(Ob @ Ob.T / Ns + shift * np.eye(Ns), Eb) / Ns
    assert np.allclose(delta, push, rtol=1e-7, atol=1e-9)


def test_sign_sgd_eq10():
    rng = np.random.default_rng(4)
    T = rng.standard_normal(200)
    g = rng.standard_normal(200)
    g[::7] = 0.0
    out = vmc.sign_sgd(T, g, 0.005, seed=1, lattice_id=0, step=3)
    d = out - T
    assert np.all(d[g == 0] == 0)
    nz = g != 0
    assert np.all(np.sign(d[nz]) == -np.sign(g[nz]))
    assert np.all(np.abs(d) <= 0.005)
    assert np.std(np.abs(d[nz])) > 0.0005   # r is drawn per element
    again = vmc.sign_sgd(T, g, 0.005, seed=1, lattice_id=0, step=3)
    assert np.array_equal(out, again)
