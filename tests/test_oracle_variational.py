"""Pins of the oracle's variational boundary fit (``oracle.peps.compress_variational``,
App. B): the iterative compression that minimises ||B - U||^2.

* exact at full rank: with Dc at or above every bond's rank one sweep
  reproduces B (a random MPS, and a PEPS row applied to a boundary);
* the distance ||B - U_s|| to the MPS it fits never increases from one sweep to
  the next, and after enough sweeps it is at most that of the canonical SVD
  compression (sequential truncation is not the optimum of the fit);
* on two sites (one bond) the fit converges to the Eckart-Young optimum, i.e.
  the canonical compression;
* the fitted state does not depend on the QR's sign and gauge conventions
  (a QR whose Q is rotated by a random orthogonal matrix gives the same state);
* the output is right-orthonormal on sites 1..n-1 with a unit-norm site 0;
* Psi, E_loc and the ratios of a lattice evaluated with the fit at full rank
  equal the brute-force contraction (``tests/bruteforce.py``).
All distances are computed from dense state vectors.
"""
import numpy as np
import pytest

import bruteforce as bf
from oracle import lattice as olat
from oracle import peps
from oracle import vmc
from paper_1908_09359_amd import workloads as W


def _dense(U, lognu=0.0):
    v = U[0]
    for s in U[1:]:
        v = np.tensordot(v, s, axes=(v.ndim - 1, 0))
    return v.reshape(-1) * np.exp(lognu)


def _random_mps(rng, n, chi, p, decay=0.0):
    B = []
    for j in range(n):
        a = 1 if j == 0 else chi
        b = 1 if j == n - 1 else chi
        t = rng.standard_normal((a, p, b))
        if decay and b > 1:
            t = t * np.exp(-decay * np.arange(b))
        B.append(t)
    return B


def test_exact_at_full_rank_random_mps():
    rng = np.random.default_rng(1)
    B = _random_mps(rng, 6, 12, 3)
    vB = _dense(B)
    U, ln = peps.compress_variational(B, 1000, 1)
    assert np.linalg.norm(_dense(U, ln) - vB) <= 1e-12 * np.linalg.norm(vB)


def test_exact_at_full_rank_peps_row():
    lat = olat.Lattice(3, 4, 2, 16)
    T = W.random_tensors(3, 4, 2, seed=5)
    s = W.random_configs(3, 4, 1, seed=6)[0]
    Uc, _ = peps.upper_boundaries(T, lat, s, upto=0)
    B = peps.absorb_down(Uc[1], peps.row_tensors(T, lat, s, 1))
    vB = _dense(B)
    U, ln = peps.compress_variational(B, 16, 1)
    assert np.linalg.norm(_dense(U, ln) - vB) <= 1e-12 * np.linalg.norm(vB)


def test_distance_never_increases_and_ends_below_canonical():
    rng = np.random.default_rng(2)
    B = _random_mps(rng, 6, 12, 3)
    vB = _dense(B)
    d = [np.linalg.norm(_dense(*peps.compress_variational(B, 4, s)) - vB) for s in range(9)]
    assert all(d[i + 1] <= d[i] * (1 + 1e-12) for i in range(len(d) - 1)), d
    assert d[-1] < d[0]
    dc = np.linalg.norm(_dense(*peps.compress(B, 4)) - vB)
    assert d[-1] <= dc * (1 + 1e-12), (d[-1], dc)


def test_two_sites_converge_to_eckart_young():
    rng = np.random.default_rng(3)
    B = [rng.standard_normal((1, 6, 10)), rng.standard_normal((10, 7, 1))]
    vc = _dense(*peps.compress(B, 3))
    errs = [np.linalg.norm(_dense(*peps.compress_variational(B, 3, s)) - vc) / np.linalg.norm(vc)
            for s in (1, 5, 60)]
    assert errs[0] > 1e-3 and errs[2] < 1e-12 and errs[2] < errs[1] < errs[0]


def test_state_independent_of_qr_gauge():
    rng = np.random.default_rng(4)
    B = _random_mps(rng, 5, 10, 3, decay=0.2)
    ref = _dense(*peps.compress_variational(B, 4, 3))
    g = np.random.default_rng(5)

    def rotated_qr(M):
        Q = np.linalg.qr(M, mode='reduced')[0]
        O = np.linalg.qr(g.standard_normal((Q.shape[1], Q.shape[1])))[0]
        return Q @ O

    other = _dense(*peps.compress_variational(B, 4, 3, qr=rotated_qr))
    assert np.linalg.norm(other - ref) <= 1e-12 * np.linalg.norm(ref)


def test_output_gauge():
    rng = np.random.default_rng(6)
    B = _random_mps(rng, 5, 9, 2)
    U, _ = peps.compress_variational(B, 4, 2)
    assert abs(np.linalg.norm(U[0]) - 1.0) < 1e-14
    for s in U[1:]:
        k = s.shape[0]
        m = s.reshape(k, -1)
        assert np.allclose(m @ m.T, np.eye(k), atol=1e-13)


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_eval_with_the_fit_at_full_rank_is_exact(J2):
    Ly, Lx, D = 4, 4, 2
    lat = olat.Lattice(Ly, Lx, D, 4, J2=J2, compress_mode="variational", fit_sweeps=1)
    T = W.random_tensors(Ly, Lx, D, seed=7)
    cfgs = W.random_configs(Ly, Lx, 3, seed=8)
    psi = bf.amplitudes(T, Ly, Lx, D, cfgs)
    for c, ps in zip(cfgs, psi):
        o = vmc.eval_config(T, lat, c)
        assert o["sign"] == np.sign(ps)
        assert abs(o["log_abs_psi"] - np.log(abs(ps))) < 1e-11
        ref = vmc.eval_config(T, olat.Lattice(Ly, Lx, D, 4, J2=J2), c)
        assert abs(o["e_loc"] - ref["e_loc"]) < 1e-10 * Ly * Lx
        assert np.allclose(o["ratios"], ref["ratios"], rtol=1e-9, atol=1e-12)
