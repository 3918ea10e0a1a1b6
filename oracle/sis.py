"""Spin-inversion symmetrised amplitude of the oracle (test infrastructure only).

Sec. II.B (symmetrised wave function): after the optimisation the amplitude
Psi(S) is replaced by Phi(S) = Psi(S) + Psi(Sbar), where Sbar reverses every
spin of S, and observables are taken with the weight |Phi(S)|^2.

* ``flip``          -- Sbar.
* ``eval_config``   -- (sign, log|Phi(S)|), the local energy of Phi,
                       E_Phi(S) = sum_S' <S|H|S'> Phi(S')/Phi(S), and
                       log w(S) = log(|Phi(S)|^2 / |Psi(S)|^2), the weight that
                       turns a sample drawn from |Psi|^2 into one of |Phi|^2.
                       Each Phi(S')/Phi(S) is formed from the method's own pair
                       ratios of S and of Sbar: S' exchanges one antiparallel
                       pair of S, and Sbar' (the reversal of S') exchanges the
                       same pair of Sbar, so
                       Phi(S')/Phi(S) = (Psi(S) r + Psi(Sbar) rbar) / (Psi(S) + Psi(Sbar))
                       with r = Psi(S')/Psi(S), rbar = Psi(Sbar')/Psi(Sbar).
                       The Heisenberg elements are invariant under the reversal
                       (<Sbar|H|Sbar'> = <S|H|S'>).  Also returned: log|Psi(S)|
                       and log|Psi(Sbar)|, which fix the conditioning of the sum.
* ``reweighted_mean`` -- <O>_Phi = sum_i w_i O_i / sum_i w_i over samples drawn
                       from |Psi|^2.
* ``run_pair_chain``  -- chains that sample |Phi|^2 itself: the chain of S and the
                       chain of Sbar visit the bonds together; a move exchanges
                       the same pair in both, and is accepted with
                       |Phi(S')/Phi(S)|^2, the ratio formed as above from the two
                       chains' pair ratios and their current amplitudes.

Pinned in the tests by brute force (dense state vectors and Hamiltonian on
small lattices), by the reversal invariance Phi(Sbar) = Phi(S) and by the case
of spin-independent tensors, where Phi = 2 Psi.
"""
import math

import numpy as np

from .lattice import bonds, local_energy
from .peps import (ZeroAmplitude, absorb_down, amplitude, compress_boundary, env3_left, env4_left,
                   row3_envs, row3_value, row4_envs, row_tensors, trivial_mps)
from . import philox
from . import vmc


def flip(spins):
    """Sbar: every spin reversed (s -> 1 - s)."""
    return (1 - np.asarray(spins, dtype=np.int8)).astype(np.int8)


def eval_config(T, lat, spins):
    """Phi(S) as (sign, log|Phi|), E_Phi(S) and log w(S) for a fixed configuration.

    Psi(S), Psi(Sbar) and the pair ratios of both come from ``vmc.eval_config``
    (the method's contraction at the lattice's Dc).  Raises ZeroAmplitude when
    Phi(S) = 0 (Psi(Sbar) = -Psi(S)).
    """
    a = vmc.eval_config(T, lat, spins)
    b = vmc.eval_config(T, lat, flip(spins))
    # Psi(S) = sa e^la, Psi(Sbar) = sb e^lb; work relative to e^m, m = max(la, lb)
    m = max(a["log_abs_psi"], b["log_abs_psi"])
    pa = a["sign"] * math.exp(a["log_abs_psi"] - m)
    pb = b["sign"] * math.exp(b["log_abs_psi"] - m)
    phi = pa + pb
    if phi == 0.0:
        raise ZeroAmplitude("Phi(S) = 0")
    index = {(p, q): i for i, (p, q, _) in enumerate(bonds(lat))}

    def phi_ratio(p, q):
        i = index[(p, q)]
        return (pa * a["ratios"][i] + pb * b["ratios"][i]) / phi

    e_phi = local_energy(lat, spins, phi_ratio)
    log_abs_phi = m + math.log(abs(phi))
    return dict(sign=1 if phi > 0 else -1, log_abs_phi=log_abs_phi, e_loc=e_phi,
                log_w=2.0 * (log_abs_phi - a["log_abs_psi"]),
                log_abs_psi=a["log_abs_psi"], log_abs_psi_rev=b["log_abs_psi"])


def reweighted_mean(values, log_w):
    """<O>_Phi from samples of |Psi|^2: sum w O / sum w, w = exp(log_w) (shifted by its maximum)."""
    log_w = np.asarray(log_w, dtype=np.float64)
    w = np.exp(log_w - np.max(log_w))
    return float(np.sum(w * np.asarray(values, dtype=np.float64)) / np.sum(w))


# --------------------------------------------------------------------------
# Chains of |Phi|^2 (Sec. II.B's weight, sampled directly)
# --------------------------------------------------------------------------

def _phi_ratio(amp, amp_rev, r, r_rev):
    """Phi(S')/Phi(S) from Psi(S) = amp, Psi(Sbar) = amp_rev (each (sign, log|.|)) and
    the pair ratios r = Psi(S')/Psi(S), r_rev = Psi(Sbar')/Psi(Sbar)."""
    m = max(amp[1], amp_rev[1])
    pa = amp[0] * math.exp(amp[1] - m)
    pb = amp_rev[0] * math.exp(amp_rev[1] - m)
    phi = pa + pb
    if phi == 0.0:
        raise ZeroAmplitude("Phi(S) = 0")
    return (pa * r + pb * r_rev) / phi


def _times(amp, r):
    """The amplitude (sign, log|.|) multiplied by the ratio r."""
    if r == 0.0:
        return (amp[0], -math.inf)
    return (amp[0] * (1 if r > 0 else -1), amp[1] + math.log(abs(r)))


def _pair_decide(ch, chb, amp, amp_rev, nums, dens, bond, pair):
    """The Metropolis test of one pair exchange for both chains (S and Sbar);
    returns the updated amplitudes."""
    for num, den in zip(nums, dens):
        if den == 0.0:
            raise ZeroAmplitude("Metropolis denominator is zero")
        if not (math.isfinite(num) and math.isfinite(den)):
            raise FloatingPointError("non-finite amplitude ratio")
    r, r_rev = nums[0] / dens[0], nums[1] / dens[1]
    q = _phi_ratio(amp, amp_rev, r, r_rev)
    take = philox.metropolis_uniform(ch.seed, ch.lattice_id, ch.chain_id, ch.sweep, bond) < q * q
    (y1, x1), (y2, x2) = pair
    for c in (ch, chb):
        c.proposed += 1
        if take:
            s = c.spins.reshape(c.lat.Ly, c.lat.Lx)
            s[y1, x1], s[y2, x2] = s[y2, x2], s[y1, x1]
            c.accepted += 1
    if take:
        return _times(amp, r), _times(amp_rev, r_rev)
    return amp, amp_rev


def _pair_pass(T, lat, chains, Dls, amps):
    """One top-down pass of the chain pair (S, Sbar) in the bond order of the
    plain sampler (``vmc._top_down_pass``): every ratio of each chain from its
    own environments, one decision per bond for both.  Returns each chain's
    upper boundaries and the freshly contracted amplitudes of the final pair."""
    ch, chb = chains
    U = [[trivial_mps(lat.Lx)], [trivial_mps(lat.Lx)]]
    lam = [[0.0], [0.0]]
    last = [None, None]
    bond = 0
    for y in range(lat.Ly):
        Uy1 = [U[c][-1] for c in (0, 1)]
        Dn = [Dls[c][y + 1] for c in (0, 1)]
        Renv = [row3_envs(Uy1[c], row_tensors(T, lat, chains[c].spins, y), Dn[c])[1] for c in (0, 1)]
        L = [np.ones((1, 1, 1)), np.ones((1, 1, 1))]
        for x in range(lat.Lx - 1):
            s = ch.spins.reshape(lat.Ly, lat.Lx)
            if s[y, x] != s[y, x + 1]:
                nums, dens = [], []
                for c in (0, 1):
                    sp = chains[c].spins
                    row = row_tensors(T, lat, sp, y)
                    fl = row_tensors(T, lat, sp, y, flips=((y, x), (y, x + 1)))
                    num = env3_left(env3_left(L[c], Uy1[c][x], fl[x], Dn[c][x]), Uy1[c][x + 1], fl[x + 1],
                                    Dn[c][x + 1])
                    den = env3_left(env3_left(L[c], Uy1[c][x], row[x], Dn[c][x]), Uy1[c][x + 1], row[x + 1],
                                    Dn[c][x + 1])
                    nums.append(vmc._dot(num, Renv[c][x + 2]))
                    dens.append(vmc._dot(den, Renv[c][x + 2]))
                amps = _pair_decide(ch, chb, amps[0], amps[1], nums, dens, bond, ((y, x), (y, x + 1)))
            for c in (0, 1):
                row = row_tensors(T, lat, chains[c].spins, y)
                L[c] = env3_left(L[c], Uy1[c][x], row[x], Dn[c][x])
            bond += 1
        if y == lat.Ly - 1:
            for c in (0, 1):
                last[c] = row3_value(Uy1[c], row_tensors(T, lat, chains[c].spins, y), Dn[c])
            break
        D2 = [Dls[c][y + 2] for c in (0, 1)]
        R4 = [row4_envs(Uy1[c], row_tensors(T, lat, chains[c].spins, y),
                        row_tensors(T, lat, chains[c].spins, y + 1), D2[c])[1] for c in (0, 1)]
        L4 = [np.ones((1, 1, 1, 1)), np.ones((1, 1, 1, 1))]
        for x in range(lat.Lx):
            s = ch.spins.reshape(lat.Ly, lat.Lx)
            if s[y, x] != s[y + 1, x]:
                nums, dens = [], []
                for c in (0, 1):
                    sp = chains[c].spins
                    r1, r2 = row_tensors(T, lat, sp, y), row_tensors(T, lat, sp, y + 1)
                    f1 = row_tensors(T, lat, sp, y, flips=((y, x),))
                    f2 = row_tensors(T, lat, sp, y + 1, flips=((y + 1, x),))
                    num = env4_left(L4[c], Uy1[c][x], f1[x], f2[x], D2[c][x])
                    den = env4_left(L4[c], Uy1[c][x], r1[x], r2[x], D2[c][x])
                    nums.append(vmc._dot(num, R4[c][x + 1]))
                    dens.append(vmc._dot(den, R4[c][x + 1]))
                amps = _pair_decide(ch, chb, amps[0], amps[1], nums, dens, bond, ((y, x), (y + 1, x)))
            for c in (0, 1):
                sp = chains[c].spins
                r1, r2 = row_tensors(T, lat, sp, y), row_tensors(T, lat, sp, y + 1)
                L4[c] = env4_left(L4[c], Uy1[c][x], r1[x], r2[x], D2[c][x])
            bond += 1
        for c in (0, 1):
            Uy, lognu = compress_boundary(absorb_down(Uy1[c], row_tensors(T, lat, chains[c].spins, y)), lat)
            U[c].append(Uy)
            lam[c].append(lam[c][-1] + lognu)
    fresh = []
    for c in (0, 1):
        if last[c] == 0.0:
            raise ZeroAmplitude("Psi = 0")
        fresh.append((1 if last[c] > 0 else -1, lam[c][lat.Ly - 1] + math.log(abs(last[c]))))
    return U, fresh


def run_pair_chain(T, lat, ch, n_burn, n_meas):
    """n_burn + n_meas sweeps of the chain pair (S, Sbar) that samples |Phi(S)|^2.

    ``ch`` is the chain of S (its Philox stream decides every move); the chain
    of Sbar starts at the reversal of ``ch.spins`` and stays its reversal.  The
    amplitudes the decisions use start as the top-down contractions of both
    configurations, are multiplied by the accepted ratios during a pass and
    are replaced by the pass's final contractions at its end.  Each measured
    sweep gives (sign, log|Phi|, E_Phi, spins of S): both chains are measured
    as in ``vmc.run_chain`` and combined as in ``eval_config``.
    """
    chb = vmc.Chain(lat, flip(ch.spins), ch.seed, ch.lattice_id, ch.chain_id, ch.sweep)
    chains = (ch, chb)
    Dls = [vmc._lower_boundaries(T, lat, c.spins) for c in chains]
    amps = [amplitude(T, lat, c.spins) for c in chains]
    out = []
    for i in range(n_burn + n_meas):
        U, amps = _pair_pass(T, lat, chains, Dls, amps)
        meas = []
        for c in (0, 1):
            e_loc, _, ratios, Dls[c] = vmc._measure(T, lat, chains[c].spins, U[c])
            meas.append((e_loc, ratios))
        if i >= n_burn:
            index = {(p, q): j for j, (p, q, _) in enumerate(bonds(lat))}
            m = max(amps[0][1], amps[1][1])
            pa = amps[0][0] * math.exp(amps[0][1] - m)
            pb = amps[1][0] * math.exp(amps[1][1] - m)
            phi = pa + pb
            if phi == 0.0:
                raise ZeroAmplitude("Phi(S) = 0")

            def phi_ratio(p, q):
                j = index[(p, q)]
                return (pa * meas[0][1][j] + pb * meas[1][1][j]) / phi

            out.append(dict(sign=1 if phi > 0 else -1, log_abs_phi=m + math.log(abs(phi)),
                            e_loc=local_energy(lat, ch.spins, phi_ratio), spins=ch.spins.copy()))
        ch.sweep += 1
        chb.sweep += 1
    return out
