"""Pins of the oracle's spin-inversion symmetrised amplitude, Phi(S) = Psi(S) + Psi(Sbar)
(Sec. II.B, symmetrised wave function; observables weighted by |Phi(S)|^2).

* Brute force: with exact contractions (Dc at the exact rank), E_Phi(S) equals
  sum_S' <S|H|S'> Phi(S')/Phi(S) written out with dense amplitudes of S' and of
  its reversal (``bruteforce``, independent of ``oracle.peps``), and
  log|Phi(S)| equals log|Psi(S) + Psi(Sbar)| of the dense amplitudes.
* Rayleigh quotient: over the whole S^z = 0 sector, the |Psi|^2 samples
  reweighted by w(S) give sum |Phi|^2 E_Phi / sum |Phi|^2 = <Phi|H|Phi>/<Phi|Phi>
  with the dense state vector Phi = Psi + P Psi (P the reversal) and the dense
  Hamiltonian.
* Reversal invariance on truncated networks: Phi(Sbar) = Phi(S), so the sign,
  log|Phi| and E_Phi of S and Sbar agree (a formula that used the ratios of S
  for both terms would break it).
* Spin-independent tensors (T_k[1] = T_k[0]): Psi(Sbar) = Psi(S), so Phi = 2 Psi,
  E_Phi = E_loc and w = 4.
* ``reweighted_mean`` against closed forms (equal weights, a zero weight, integer weights).
"""
import math

import numpy as np

import bruteforce as bf
from oracle import sis, vmc
from oracle.lattice import Lattice
from paper_1908_09359_amd import workloads as W


def _dense_index(configs):
    return {c.tobytes(): i for i, c in enumerate(configs)}


def test_flip_reverses_every_spin():
    s = np.array([0, 1, 1, 0, 1, 0], dtype=np.int8)
    assert np.array_equal(sis.flip(s), np.array([1, 0, 0, 1, 0, 1], dtype=np.int8))
    assert np.array_equal(sis.flip(sis.flip(s)), s)


def test_local_energy_matches_brute_force_definition():
    Ly, Lx, D, Dc, J2 = 4, 4, 2, 4, 0.5
    T = W.random_tensors(Ly, Lx, D, seed=41)
    lat = Lattice(Ly, Lx, D, Dc, J2=J2)
    cfgs = W.random_configs(Ly, Lx, 5, seed=3)
    for s in cfgs:
        o = sis.eval_config(T, lat, s)
        sb = sis.flip(s)
        phi = bf.amplitudes(T, Ly, Lx, D, np.stack([s]))[0] + bf.amplitudes(T, Ly, Lx, D, np.stack([sb]))[0]
        e = 0.0
        for i, j, J in bf.bonds(Ly, Lx, 1.0, J2):
            if s[i] == s[j]:
                e += 0.25 * J
                continue
            e -= 0.25 * J
            t = s.copy()
            t[i], t[j] = s[j], s[i]
            phit = (bf.amplitudes(T, Ly, Lx, D, np.stack([t]))[0]
                    + bf.amplitudes(T, Ly, Lx, D, np.stack([sis.flip(t)]))[0])
            e += 0.5 * J * phit / phi
        assert o["sign"] == (1 if phi > 0 else -1)
        assert abs(o["log_abs_phi"] - math.log(abs(phi))) < 1e-11
        assert abs(o["e_loc"] - e) < 1e-10 * Ly * Lx


def test_reweighted_energy_is_rayleigh_quotient_of_phi():
    Ly, Lx, D, Dc, J2 = 2, 4, 2, 4, 0.3
    N = Ly * Lx
    T = W.random_tensors(Ly, Lx, D, seed=5)
    lat = Lattice(Ly, Lx, D, Dc, J2=J2)
    configs = bf.sz0_configs(N)
    index = _dense_index(configs)
    psi = bf.amplitudes(T, Ly, Lx, D, configs)
    rev = np.array([index[sis.flip(c).tobytes()] for c in configs])
    phi = psi + psi[rev]
    Hm = np.zeros((len(configs), len(configs)))
    for k, s in enumerate(configs):
        for i, j, J in bf.bonds(Ly, Lx, 1.0, J2):
            if s[i] == s[j]:
                Hm[k, k] += 0.25 * J
            else:
                Hm[k, k] -= 0.25 * J
                t = s.copy()
                t[i], t[j] = s[j], s[i]
                Hm[index[t.tobytes()], k] += 0.5 * J
    exact = phi @ Hm @ phi / (phi @ phi)
    outs = [sis.eval_config(T, lat, c) for c in configs]
    e_phi = np.array([o["e_loc"] for o in outs])
    log_w = np.array([o["log_w"] for o in outs])
    # each configuration enters with its |Psi|^2 probability, then the weight w
    p = psi ** 2 / np.sum(psi ** 2)
    num = np.sum(p * np.exp(log_w) * e_phi)
    den = np.sum(p * np.exp(log_w))
    assert abs(num / den - exact) < 1e-11
    # reweighted_mean over an exact "sample" (each configuration repeated in proportion p is
    # replaced by folding p into the log-weights)
    assert abs(sis.reweighted_mean(e_phi, log_w + np.log(p)) - exact) < 1e-11
    # and without symmetrisation the same estimator gives the energy of Psi
    e_psi = np.array([vmc.eval_config(T, lat, c)["e_loc"] for c in configs])
    assert abs(np.sum(p * e_psi) - psi @ Hm @ psi / (psi @ psi)) < 1e-11


def test_reversal_invariance_on_truncated_networks():
    Ly, Lx, D, Dc, J2 = 4, 4, 3, 3, 0.5
    T = W.random_tensors(Ly, Lx, D, seed=77)
    lat = Lattice(Ly, Lx, D, Dc, J2=J2)
    for s in W.random_configs(Ly, Lx, 3, seed=9):
        a = sis.eval_config(T, lat, s)
        b = sis.eval_config(T, lat, sis.flip(s))
        assert a["sign"] == b["sign"]
        assert abs(a["log_abs_phi"] - b["log_abs_phi"]) < 1e-12
        assert abs(a["e_loc"] - b["e_loc"]) < 1e-11 * Ly * Lx
        # the two log-weights are taken against different denominators
        assert abs((a["log_w"] - b["log_w"]) - 2.0 * (vmc.eval_config(T, lat, sis.flip(s))["log_abs_psi"]
                                                      - vmc.eval_config(T, lat, s)["log_abs_psi"])) < 1e-11


def test_spin_independent_tensors_give_phi_twice_psi():
    Ly, Lx, D, Dc, J2 = 3, 4, 2, 4, 0.0
    lat = Lattice(Ly, Lx, D, Dc, J2=J2)
    T = W.random_tensors(Ly, Lx, D, seed=12)
    for y in range(Ly):
        for x in range(Lx):
            k = lat.site(y, x)
            n = int(np.prod(lat.dims(y, x)))
            o = lat.offsets[k]
            T[o + n:o + 2 * n] = T[o:o + n]
    for s in W.random_configs(Ly, Lx, 3, seed=2):
        a = vmc.eval_config(T, lat, s)
        o = sis.eval_config(T, lat, s)
        assert o["sign"] == a["sign"]
        assert abs(o["log_abs_phi"] - (a["log_abs_psi"] + math.log(2.0))) < 1e-12
        assert abs(o["e_loc"] - a["e_loc"]) < 1e-12 * Ly * Lx
        assert abs(o["log_w"] - math.log(4.0)) < 1e-12


def test_reweighted_mean_closed_forms():
    v = np.array([1.0, 2.0, 4.0, 8.0])
    # equal weights give the plain mean, whatever their common scale
    assert abs(sis.reweighted_mean(v, np.full(4, 700.0)) - 3.75) < 1e-15
    # a weight of zero (log w = -inf) drops its sample
    assert abs(sis.reweighted_mean(v, np.array([0.0, 0.0, 0.0, -np.inf])) - 7.0 / 3.0) < 1e-15
    # w = (1, 2, 3, 4): sum w v / sum w = (1 + 4 + 12 + 32) / 10
    assert abs(sis.reweighted_mean(v, np.log([1.0, 2.0, 3.0, 4.0])) - 4.9) < 1e-14


def _phi2_distribution(T, lat, configs):
    """|Phi(S)|^2 / Z over the S^z = 0 sector from dense amplitudes of S and its reversal."""
    psi = bf.amplitudes(T, lat.Ly, lat.Lx, lat.D, configs)
    psi_rev = bf.amplitudes(T, lat.Ly, lat.Lx, lat.D, 1 - np.asarray(configs))
    phi2 = (psi + psi_rev) ** 2
    return phi2 / phi2.sum()


def _chi2_pvalue(counts, p):
    import scipy.stats
    n = counts.sum()
    keep = p * n >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(p[keep] * n, p[~keep].sum() * n)
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    return scipy.stats.chisquare(obs, exp)[1]


def test_pair_chains_sample_phi_squared():
    """Chains of the pair (S, Sbar) visit the S^z = 0 configurations of a 2x3
    lattice with the frequencies |Phi|^2 / Z of the dense amplitudes (chi-square;
    consecutive sweeps are correlated, so the p-value is a coarse gate), while
    the plain chain on the same tensors does not (its weight is |Psi|^2): the
    check would catch an acceptance that left out the reversed chain."""
    from oracle.lattice import neel_shuffled
    lat = Lattice(2, 3, 2, 8)
    T = np.random.default_rng(3).standard_normal(lat.Np) / lat.D ** 2
    configs = bf.sz0_configs(6)
    p_phi = _phi2_distribution(T, lat, configs)
    index = _dense_index(configs)
    counts = np.zeros(len(configs))
    counts_plain = np.zeros(len(configs))
    for chain in range(4):
        start = neel_shuffled(lat, 9359, 0, chain)
        ch = vmc.Chain(lat, start, 1234, 0, chain)
        for smp in sis.run_pair_chain(T, lat, ch, 10, 600):
            counts[index[smp["spins"].tobytes()]] += 1
        ch = vmc.Chain(lat, start, 1234, 0, chain)
        for smp in vmc.run_chain(T, lat, ch, 10, 600):
            counts_plain[index[smp["spins"].tobytes()]] += 1
    assert _chi2_pvalue(counts, p_phi) > 1e-4
    assert _chi2_pvalue(counts_plain, p_phi) < 1e-8


def test_pair_chain_measurements_equal_the_fixed_configuration_evaluation():
    """Every measured sample of the pair chain (truncated 4x4, D=3, Dc=3, J2 = 0.5)
    equals ``eval_config`` of its configuration: sign, log|Phi| and E_Phi."""
    lat = Lattice(4, 4, 3, 3, J2=0.5)
    T = W.random_tensors(4, 4, 3, seed=41)
    from oracle.lattice import neel_shuffled
    ch = vmc.Chain(lat, neel_shuffled(lat, 5, 0, 1), 77, 0, 1)
    samples = sis.run_pair_chain(T, lat, ch, 1, 3)
    moved = False
    for smp in samples:
        ref = sis.eval_config(T, lat, smp["spins"])
        assert smp["sign"] == ref["sign"]
        assert abs(smp["log_abs_phi"] - ref["log_abs_phi"]) <= 1e-10
        assert abs(smp["e_loc"] - ref["e_loc"]) <= 1e-10 * max(1.0, abs(ref["e_loc"]))
        moved |= not np.array_equal(smp["spins"], neel_shuffled(lat, 5, 0, 1))
    assert moved and ch.accepted > 0
