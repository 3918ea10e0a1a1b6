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

Pinned in the tests by brute force (dense state vectors and Hamiltonian on
small lattices), by the reversal invariance Phi(Sbar) = Phi(S) and by the case
of spin-independent tensors, where Phi = 2 Psi.
"""
import math

import numpy as np

from .lattice import bonds, local_energy
from .peps import ZeroAmplitude
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
