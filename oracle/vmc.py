"""Variational Monte Carlo layer of the oracle (test infrastructure only).

* ``eval_config``  -- Psi(S), E_loc(S), the log-derivatives G(S) and every pair
                      ratio for one fixed configuration.
* ``Chain`` / ``run_chain`` -- the sequential bond-visiting Metropolis sampler
                      of Sec. II.A Eq. (9): one sweep = a top-down pass that
                      visits every horizontal bond of row y (left to right),
                      then every vertical bond between rows y and y+1, then
                      forms U_y; followed by a bottom-up pass that measures and
                      rebuilds the lower boundaries for the next sweep.
* ``gradient``     -- Eq. (5): <G E_loc> - <G><E_loc> (Alg. 1, gradient step).
* ``sr_step``      -- stochastic reconfiguration: (S + shift I) delta = g with
                      S the covariance of G, solved by Cholesky.
* ``sign_sgd``     -- Eq. (10): A <- A - r * delta * sgn(dE/dA), r ~ U[0,1)
                      per element.

Ratios Psi(S')/Psi(S) use the auxiliary tensors of App. C: every ratio is the
value of the same row (or row-pair) network with the exchanged tensors, divided
by that network with the current tensors.

Parity: at Dc >= exact rank everything here is pinned by brute force in the
tests; on truncated networks the pins are the invariants listed in ``peps``.
"""
import math

import numpy as np

from . import philox
from .lattice import (bonds, bond_elements, compact_offsets, compact_size, site_tensor, transpose_lattice,
                      transpose_spins, transpose_tensors)
from .peps import (ZeroAmplitude, absorb_down, compress, compress_boundary, defect3, env3_left, env4_left,
                   lower_boundary, row3_envs, row4_envs, row_tensors, trivial_mps,
                   upper_boundaries, row3_value)


def _dot(L, R):
    return float(np.tensordot(L, R, axes=L.ndim))


def _lower_boundaries(T, lat, spins):
    """D_y for y = Ly..1 (D[Ly] trivial) for the configuration ``spins``."""
    Dl = {lat.Ly: trivial_mps(lat.Lx)}
    for y in range(lat.Ly - 1, 0, -1):
        Dl[y], _ = lower_boundary(Dl[y + 1], T, lat, spins, y)
    return Dl


def _measure(T, lat, spins, U, collect_ratios=True):
    """Bottom-up measurement pass (App. C): E_loc, compact G, ratios, new lower boundaries.

    ``U[y+1]`` must hold U_y for the configuration ``spins``.
    """
    s = np.asarray(spins).reshape(lat.Ly, lat.Lx)
    coffs = compact_offsets(lat)
    G = np.zeros(compact_size(lat))
    ratio = {}
    Dl = {lat.Ly: trivial_mps(lat.Lx)}
    for y in range(lat.Ly - 1, -1, -1):
        Dn = Dl[y + 1]
        row = row_tensors(T, lat, spins, y)
        Lenv, Renv = row3_envs(U[y], row, Dn)
        Ny = _dot(Lenv[1], Renv[1])
        if Ny == 0.0:
            raise ZeroAmplitude("row network value is zero")
        # Log-derivatives of the sites of row y (Eqs. (6)-(7)), normalised by N_y.
        for x in range(lat.Lx):
            Delta = defect3(Lenv[x], U[y][x], Dn[x], Renv[x + 1])
            k = lat.site(y, x)
            G[coffs[k]:coffs[k] + Delta.size] = (Delta / Ny).ravel()
        # Horizontal pairs of row y.
        for x in range(lat.Lx - 1):
            if s[y, x] != s[y, x + 1]:
                fl = row_tensors(T, lat, spins, y, flips=((y, x), (y, x + 1)))
                Lm = env3_left(Lenv[x], U[y][x], fl[x], Dn[x])
                Lm = env3_left(Lm, U[y][x + 1], fl[x + 1], Dn[x + 1])
                ratio[((y, x), (y, x + 1))] = _dot(Lm, Renv[x + 2]) / Ny
        # Vertical and diagonal pairs between rows y and y+1.
        if y < lat.Ly - 1:
            D2 = Dl[y + 2]
            row2 = row_tensors(T, lat, spins, y + 1)
            L4, R4 = row4_envs(U[y], row, row2, D2)
            N4 = _dot(L4[1], R4[1])
            if N4 == 0.0:
                raise ZeroAmplitude("row-pair network value is zero")
            for x in range(lat.Lx):
                if s[y, x] != s[y + 1, x]:
                    f1 = row_tensors(T, lat, spins, y, flips=((y, x),))
                    f2 = row_tensors(T, lat, spins, y + 1, flips=((y + 1, x),))
                    Lm = env4_left(L4[x], U[y][x], f1[x], f2[x], D2[x])
                    ratio[((y, x), (y + 1, x))] = _dot(Lm, R4[x + 1]) / N4
            if lat.diagonals:
                for x in range(lat.Lx - 1):
                    for p, q in (((y, x), (y + 1, x + 1)), ((y, x + 1), (y + 1, x))):
                        if s[p] != s[q]:
                            f1 = row_tensors(T, lat, spins, y, flips=(p, q))
                            f2 = row_tensors(T, lat, spins, y + 1, flips=(p, q))
                            Lm = env4_left(L4[x], U[y][x], f1[x], f2[x], D2[x])
                            Lm = env4_left(Lm, U[y][x + 1], f1[x + 1], f2[x + 1], D2[x + 1])
                            ratio[(p, q)] = _dot(Lm, R4[x + 2]) / N4
            if lat.knights:
                ratio.update(_knight_ratios(T, lat, spins, y, U[y], row, row2, D2, L4, R4, N4))
        if y >= 1:
            Dl[y], _ = lower_boundary(Dn, T, lat, spins, y)
    if lat.knights and lat.Ly > 2:
        ratio.update(_long_knight_ratios(T, lat, spins))
    e_loc = 0.0
    ratio_vec = np.zeros(len(bonds(lat)))
    for i, (p, q, J) in enumerate(bonds(lat)):
        diag, off = bond_elements(s[p], s[q], J)
        e_loc += diag
        if off != 0.0:
            e_loc += off * ratio[(p, q)]
            ratio_vec[i] = ratio[(p, q)]
    return e_loc, G, ratio_vec, Dl


def _knight_ratios(T, lat, spins, y, Uy, row, row2, D2, L4, R4, N4):
    """Ratios of the knight bonds (y,x)-(y+1,x+2) of row pair y: the 2-row network
    with site (y,x) flipped in column x, column x+1 unchanged and site (y+1,x+2)
    flipped in column x+2, divided by the same network with the current tensors."""
    s = np.asarray(spins).reshape(lat.Ly, lat.Lx)
    out = {}
    for x in range(lat.Lx - 2):
        p, q = (y, x), (y + 1, x + 2)
        if s[p] != s[q]:
            f1 = row_tensors(T, lat, spins, y, flips=(p,))
            f2 = row_tensors(T, lat, spins, y + 1, flips=(q,))
            Lm = L4[x]
            for c in (x, x + 1, x + 2):
                Lm = env4_left(Lm, Uy[c], f1[c], f2[c], D2[c])
            out[(p, q)] = _dot(Lm, R4[x + 3]) / N4
    return out


def _long_knight_ratios(T, lat, spins):
    """Ratios of the knight bonds (y,x)-(y+2,x+1), which span three rows: each is the
    knight bond (x,y)-(x+1,y+2) of the transposed lattice (the same state), taken
    there by ``_knight_ratios`` with that lattice's boundaries for its configuration."""
    lt, Tt, st = transpose_lattice(lat), transpose_tensors(T, lat), transpose_spins(spins, lat)
    U, _ = upper_boundaries(Tt, lt, st)
    Dl = _lower_boundaries(Tt, lt, st)
    out = {}
    for yt in range(lt.Ly - 1):
        r1, r2, D2 = row_tensors(Tt, lt, st, yt), row_tensors(Tt, lt, st, yt + 1), Dl[yt + 2]
        L4, R4 = row4_envs(U[yt], r1, r2, D2)
        N4 = _dot(L4[1], R4[1])
        if N4 == 0.0:
            raise ZeroAmplitude("row-pair network value is zero")
        for (p, q), rho in _knight_ratios(Tt, lt, st, yt, U[yt], r1, r2, D2, L4, R4, N4).items():
            # (x, y)-(x+1, y+2) of the transposed lattice is (y, x)-(y+2, x+1)
            out[((p[1], p[0]), (q[1], q[0]))] = rho
    return out


def plaquette_ratios(T, lat, spins):
    """Psi(S')/Psi(S) for the flip of every movable plaquette, [Ly-1][Lx-1] (0 elsewhere).

    Each is the two-row network of rows y, y+1 (between U_{y-1} and D_{y+2})
    with both columns x, x+1 exchanged, divided by the same network with the
    current tensors -- the vertical-pair construction of App. C with two
    columns modified.
    """
    from . import proposal as P
    s = np.asarray(spins)
    U, _ = upper_boundaries(T, lat, s)
    Dl = _lower_boundaries(T, lat, s)
    mov = P.movable(s, lat.Ly, lat.Lx)
    out = np.zeros((lat.Ly - 1, lat.Lx - 1))
    for y in range(lat.Ly - 1):
        r1, r2, D2 = row_tensors(T, lat, s, y), row_tensors(T, lat, s, y + 1), Dl[y + 2]
        L4, R4 = row4_envs(U[y], r1, r2, D2)
        N4 = _dot(L4[1], R4[1])
        if N4 == 0.0:
            raise ZeroAmplitude("row-pair network value is zero")
        for x in range(lat.Lx - 1):
            if mov[y, x]:
                sites = ((y, x), (y, x + 1), (y + 1, x), (y + 1, x + 1))
                f1 = row_tensors(T, lat, s, y, flips=sites)
                f2 = row_tensors(T, lat, s, y + 1, flips=sites)
                Lm = env4_left(env4_left(L4[x], U[y][x], f1[x], f2[x], D2[x]), U[y][x + 1], f1[x + 1], f2[x + 1],
                               D2[x + 1])
                out[y, x] = _dot(Lm, R4[x + 2]) / N4
    return out


def eval_config(T, lat, spins):
    """Psi, E_loc, G and pair ratios for a fixed configuration.

    Returns dict(sign, log_abs_psi, e_loc, dlnpsi (compact: occupied slot of
    every site, in parameter-layout order), ratios (one per entry of
    ``lattice.bonds``; 0 for parallel pairs)).
    """
    U, lam = upper_boundaries(T, lat, spins)
    last = row3_value(U[lat.Ly - 1], row_tensors(T, lat, spins, lat.Ly - 1), trivial_mps(lat.Lx))
    if last == 0.0:
        raise ZeroAmplitude("Psi(S) = 0")
    e_loc, G, ratios, _ = _measure(T, lat, spins, U)
    return dict(sign=1 if last > 0 else -1, log_abs_psi=lam[lat.Ly - 1] + math.log(abs(last)),
                e_loc=e_loc, dlnpsi=G, ratios=ratios)


# --------------------------------------------------------------------------
# Sequential bond-visiting Metropolis (Sec. II.A Eq. (9))
# --------------------------------------------------------------------------

class Chain:
    """State of one Markov chain: spins, the sweep counter and its Philox stream ids.

    Test hooks, neither of which changes the arithmetic: ``trace`` (a dict, or
    None) receives bond -> Psi(S')/Psi(S) for every proposal; ``forced`` (a
    dict bond -> bool, or None) replaces the Metropolis test by a given
    decision, so that another sampler's sweep can be replayed and its ratios
    recomputed here.
    """

    def __init__(self, lat, spins, seed, lattice_id, chain_id, sweep=0):
        self.lat = lat
        self.spins = np.array(spins, dtype=np.int8).copy()
        self.seed, self.lattice_id, self.chain_id = seed, lattice_id, chain_id
        self.sweep = sweep
        self.accepted = 0
        self.proposed = 0
        self.trace = None
        self.forced = None
        self.plaq_accepted = 0
        self.plaq_proposed = 0


def _top_down_pass(T, lat, ch, Dl, proposal=None, vertical=True):
    """Visit every bond once in the pinned order, accepting with r < |Psi(S_b)/Psi(S_a)|^2.

    With ``proposal`` (flat network parameters, see ``oracle.proposal``) the
    row-pair step also visits plaquette (y, x) right after the vertical bond
    (y, x)-(y+1, x), for x = 0..Lx-2 (``_plaquette_step``).  With
    ``vertical=False`` only the horizontal bonds are visited (each keeps its
    bond index y(2Lx-1)+x); the vertical ones are left to another pass.

    Returns the upper boundaries of the final configuration and (sign, log|Psi|).
    """
    s = ch.spins.reshape(lat.Ly, lat.Lx)
    U = [trivial_mps(lat.Lx)]
    lam = [0.0]
    bond = 0
    last = None
    for y in range(lat.Ly):
        Uy1, Dn = U[-1], Dl[y + 1]
        # Horizontal bonds of row y.
        row = row_tensors(T, lat, ch.spins, y)
        _, Renv = row3_envs(Uy1, row, Dn)
        L = np.ones((1, 1, 1))
        for x in range(lat.Lx - 1):
            if s[y, x] != s[y, x + 1]:
                row = row_tensors(T, lat, ch.spins, y)
                fl = row_tensors(T, lat, ch.spins, y, flips=((y, x), (y, x + 1)))
                num = env3_left(env3_left(L, Uy1[x], fl[x], Dn[x]), Uy1[x + 1], fl[x + 1], Dn[x + 1])
                den = env3_left(env3_left(L, Uy1[x], row[x], Dn[x]), Uy1[x + 1], row[x + 1], Dn[x + 1])
                _accept(ch, _dot(num, Renv[x + 2]), _dot(den, Renv[x + 2]), bond,
                        ((y, x), (y, x + 1)))
            row = row_tensors(T, lat, ch.spins, y)
            L = env3_left(L, Uy1[x], row[x], Dn[x])
            bond += 1
        if y == lat.Ly - 1:
            row = row_tensors(T, lat, ch.spins, y)
            last = row3_value(Uy1, row, Dn)
            break
        if not vertical:
            bond += lat.Lx
            Uy, lognu = compress_boundary(absorb_down(Uy1, row_tensors(T, lat, ch.spins, y)), lat)
            U.append(Uy)
            lam.append(lam[-1] + lognu)
            continue
        # Vertical bonds between rows y and y+1.
        D2 = Dl[y + 2]
        r1 = row_tensors(T, lat, ch.spins, y)
        r2 = row_tensors(T, lat, ch.spins, y + 1)
        _, R4 = row4_envs(Uy1, r1, r2, D2)
        L4 = np.ones((1, 1, 1, 1))
        for x in range(lat.Lx):
            r1 = row_tensors(T, lat, ch.spins, y)
            r2 = row_tensors(T, lat, ch.spins, y + 1)
            if s[y, x] != s[y + 1, x]:
                f1 = row_tensors(T, lat, ch.spins, y, flips=((y, x),))
                f2 = row_tensors(T, lat, ch.spins, y + 1, flips=((y + 1, x),))
                num = env4_left(L4, Uy1[x], f1[x], f2[x], D2[x])
                den = env4_left(L4, Uy1[x], r1[x], r2[x], D2[x])
                _accept(ch, _dot(num, R4[x + 1]), _dot(den, R4[x + 1]), bond,
                        ((y, x), (y + 1, x)))
                r1 = row_tensors(T, lat, ch.spins, y)
                r2 = row_tensors(T, lat, ch.spins, y + 1)
            if proposal is not None and x < lat.Lx - 1:
                _plaquette_step(T, lat, ch, proposal, y, x, L4, Uy1, D2, R4)
                r1 = row_tensors(T, lat, ch.spins, y)
                r2 = row_tensors(T, lat, ch.spins, y + 1)
            L4 = env4_left(L4, Uy1[x], r1[x], r2[x], D2[x])
            bond += 1
        # Row y is final for this sweep: form U_y.
        Uy, lognu = compress_boundary(absorb_down(Uy1, row_tensors(T, lat, ch.spins, y)), lat)
        U.append(Uy)
        lam.append(lam[-1] + lognu)
    if last == 0.0:
        raise ZeroAmplitude("Psi(S) = 0")
    return U, (1 if last > 0 else -1, lam[lat.Ly - 1] + math.log(abs(last)))


def _plaquette_step(T, lat, ch, theta, y, x, L4, Uy1, D2, R4):
    """Propose-or-stay Metropolis-Hastings move of plaquette (y, x) (learned sampler).

    Propose the flip of its four spins with probability pi(S) = sigmoid(f_x(S))
    when it holds two up and two down spins; accept with
    min[1, R pi(S')/pi(S)], R = (Psi(S')/Psi(S))^2 from the two-row network
    with both columns exchanged, divided by the same network with the current
    tensors.  Uniforms: words 0 (propose) and 1 (accept) of Philox counter
    (chain, sweep, y(Lx-1)+x, TAG_PLAQ).
    """
    from . import proposal as P
    s = ch.spins.reshape(lat.Ly, lat.Lx)
    if not P.movable(ch.spins, lat.Ly, lat.Lx)[y, x]:
        return
    q = y * (lat.Lx - 1) + x
    u_prop, u_acc = philox.plaquette_uniforms(ch.seed, ch.lattice_id, ch.chain_id, ch.sweep, q)
    pi = P.propensity(theta, ch.spins, lat.Ly, lat.Lx, y, x)
    if not u_prop < pi:
        return
    sites = ((y, x), (y, x + 1), (y + 1, x), (y + 1, x + 1))
    r1 = row_tensors(T, lat, ch.spins, y)
    r2 = row_tensors(T, lat, ch.spins, y + 1)
    f1 = row_tensors(T, lat, ch.spins, y, flips=sites)
    f2 = row_tensors(T, lat, ch.spins, y + 1, flips=sites)
    num = env4_left(env4_left(L4, Uy1[x], f1[x], f2[x], D2[x]), Uy1[x + 1], f1[x + 1], f2[x + 1], D2[x + 1])
    den = env4_left(env4_left(L4, Uy1[x], r1[x], r2[x], D2[x]), Uy1[x + 1], r1[x + 1], r2[x + 1], D2[x + 1])
    num, den = _dot(num, R4[x + 2]), _dot(den, R4[x + 2])
    if den == 0.0:
        raise ZeroAmplitude("Metropolis denominator is zero")
    if not (math.isfinite(num) and math.isfinite(den)):
        raise FloatingPointError("non-finite amplitude ratio")
    flipped = ch.spins.copy().reshape(lat.Ly, lat.Lx)
    for p in sites:
        flipped[p] = 1 - flipped[p]
    pi_back = P.propensity(theta, flipped.ravel(), lat.Ly, lat.Lx, y, x)
    if ch.trace is not None:
        ch.trace[("p", q)] = num / den
    ch.plaq_proposed += 1
    take = ch.forced[("p", q)] if ch.forced is not None else u_acc < (num / den) ** 2 * pi_back / pi
    if take:
        for p in sites:
            s[p] = 1 - s[p]
        ch.plaq_accepted += 1


def _accept(ch, num, den, bond, pair):
    if den == 0.0:
        raise ZeroAmplitude("Metropolis denominator is zero")
    if not (math.isfinite(num) and math.isfinite(den)):
        raise FloatingPointError("non-finite amplitude ratio")
    R = (num / den) ** 2
    if ch.trace is not None:
        ch.trace[bond] = num / den
    if ch.forced is not None:
        take = ch.forced[bond]
    else:
        take = philox.metropolis_uniform(ch.seed, ch.lattice_id, ch.chain_id, ch.sweep, bond) < R
    ch.proposed += 1
    if take:
        s = ch.spins.reshape(ch.lat.Ly, ch.lat.Lx)
        (y1, x1), (y2, x2) = pair
        s[y1, x1], s[y2, x2] = s[y2, x2], s[y1, x1]
        ch.accepted += 1


def run_chain(T, lat, ch, n_burn, n_meas, proposal=None):
    """Run n_burn + n_meas sweeps; measure after each of the last n_meas (Sec. II.A).

    ``proposal``: network parameters of the learned plaquette moves, or None
    for the plain sequential sweep.  Returns a list of per-sample dicts (sign,
    log_abs_psi, e_loc, dlnpsi, spins) and leaves the final state in ``ch``.
    """
    Dl = _lower_boundaries(T, lat, ch.spins)
    out = []
    for i in range(n_burn + n_meas):
        U, (sg, lp) = _top_down_pass(T, lat, ch, Dl, proposal)
        e_loc, G, _, Dl = _measure(T, lat, ch.spins, U)
        if i >= n_burn:
            out.append(dict(sign=sg, log_abs_psi=lp, e_loc=e_loc, dlnpsi=G,
                            spins=ch.spins.copy()))
        ch.sweep += 1
    return out


# --------------------------------------------------------------------------
# Estimators and updates (Eqs. (2), (5), (10); Alg. 1)
# --------------------------------------------------------------------------

def expand_dlnpsi(lat, compact, spins):
    """Scatter a compact log-derivative vector into the full parameter layout (slot s of every site)."""
    full = np.zeros(lat.Np)
    coffs = compact_offsets(lat)
    s = np.asarray(spins).reshape(-1)
    for k in range(lat.N):
        n = coffs[k + 1] - coffs[k] if k + 1 < lat.N else compact_size(lat) - coffs[k]
        o = lat.offsets[k] + int(s[k]) * n
        full[o:o + n] = compact[coffs[k]:coffs[k] + n]
    return full


def gradient(lat, e_loc, dlnpsi, spins):
    """dE/dA = <G E_loc> - <G><E_loc> over all samples (Eq. (5)); returns (g, <E_loc>)."""
    e = np.asarray(e_loc, dtype=np.float64)
    O = np.stack([expand_dlnpsi(lat, dlnpsi[i], spins[i]) for i in range(len(e))])
    E = e.mean()
    g = (O * e[:, None]).mean(axis=0) - O.mean(axis=0) * E
    return g, E


def sr_step(lat, e_loc, dlnpsi, spins, shift):
    """Solve (S + shift I) delta = g, S = Obar^T Obar / Ns, g = Obar^T Ebar / Ns, by Cholesky."""
    import scipy.linalg
    e = np.asarray(e_loc, dtype=np.float64)
    O = np.stack([expand_dlnpsi(lat, dlnpsi[i], spins[i]) for i in range(len(e))])
    Ob = O - O.mean(axis=0)
    Eb = e - e.mean()
    Ns = len(e)
    S = Ob.T @ Ob / Ns
    g = Ob.T @ Eb / Ns
    S[np.diag_indices_from(S)] += shift
    c = np.linalg.cholesky(S)
    z = scipy.linalg.solve_triangular(c, g, lower=True)
    return scipy.linalg.solve_triangular(c.T, z, lower=False), g


def sign_sgd(T, g, step_len, seed, lattice_id, step):
    """Eq. (10): A <- A - r delta sgn(g), r from counter (p, step, 0, TAG_SGD) per element."""
    out = np.array(T, dtype=np.float64, copy=True)
    for p in range(len(out)):
        if g[p] != 0.0:
            w = philox.philox4x64_10((p, step, 0, philox.TAG_SGD), (seed, lattice_id))
            out[p] -= philox.uniform53(w[0]) * step_len * (1.0 if g[p] > 0 else -1.0)
    return out
