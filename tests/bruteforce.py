"""Exact (untruncated) amplitudes by dense row-by-row contraction, batched over configurations.

Independent of ``oracle.peps``: the parameter layout is re-derived here from its
definition (site-major, T_k[s][l][u][r][d], boundary legs of dimension 1) and
the network is contracted without any boundary-MPS compression, keeping the
full state over the open vertical legs (dimension D^Lx).  Only for small
lattices.
"""
import numpy as np


def layout(Ly, Lx, D):
    dims, offs, o = [], [], 0
    for y in range(Ly):
        for x in range(Lx):
            d = (D if x > 0 else 1, D if y > 0 else 1, D if x < Lx - 1 else 1, D if y < Ly - 1 else 1)
            dims.append(d)
            offs.append(o)
            o += 2 * int(np.prod(d))
    return dims, offs, o


def site_batch(T, Ly, Lx, D, k, s):
    """Tensors T_k[s_n] for every configuration n: shape (n, l, u, r, d)."""
    dims, offs, _ = layout(Ly, Lx, D)
    n = int(np.prod(dims[k]))
    blocks = np.stack([T[offs[k]:offs[k] + n].reshape(dims[k]),
                       T[offs[k] + n:offs[k] + 2 * n].reshape(dims[k])])
    return blocks[np.asarray(s, dtype=np.int64)]


def amplitudes(T, Ly, Lx, D, configs):
    """Psi(S) for every row of ``configs`` (shape (n, Ly*Lx), entries 0/1)."""
    configs = np.asarray(configs).reshape(len(configs), Ly * Lx)
    n = len(configs)
    v = np.ones((n, 1))
    for y in range(Ly):
        acc = None
        for x in range(Lx):
            t = site_batch(T, Ly, Lx, D, y * Lx + x, configs[:, y * Lx + x])  # n,l,u,r,d
            if acc is None:
                acc = t[:, 0].transpose(0, 1, 3, 2)  # n, u, d, r
            else:
                # acc: n, U, Dd, r ; t: n, r(=l), u, r', d
                nn, U, Dd, r = acc.shape
                _, l, u, r2, d = t.shape
                a = np.einsum('nUDk,nkuqd->nUuDdq', acc, t)
                acc = a.reshape(nn, U * u, Dd * d, r2)
        acc = acc[..., 0]
        v = np.einsum('nu,nud->nd', v, acc)
    return v[:, 0]


def sz0_configs(N):
    import itertools
    out = []
    for c in itertools.combinations(range(N), N // 2):
        s = np.zeros(N, dtype=np.int8)
        s[list(c)] = 1
        out.append(s)
    return np.array(out)


def bonds(Ly, Lx, J1, J2, triangular=False):
    """Bond list in the same order as the method's: horizontal, vertical, two diagonals per plaquette.
    triangular: J1 on the diagonal (y,x)-(y+1,x+1), J2 on the anti-diagonal, then (J2 != 0) the knight
    bonds (y,x)-(y+1,x+2) and (y,x)-(y+2,x+1)."""
    out = []
    for y in range(Ly):
        for x in range(Lx - 1):
            out.append((y * Lx + x, y * Lx + x + 1, J1))
    for y in range(Ly - 1):
        for x in range(Lx):
            out.append((y * Lx + x, (y + 1) * Lx + x, J1))
    if J2 != 0.0 or triangular:
        for y in range(Ly - 1):
            for x in range(Lx - 1):
                out.append((y * Lx + x, (y + 1) * Lx + x + 1, J1 if triangular else J2))
                out.append((y * Lx + x + 1, (y + 1) * Lx + x, J2))
    if triangular and J2 != 0.0:
        for y in range(Ly - 1):
            for x in range(Lx - 2):
                out.append((y * Lx + x, (y + 1) * Lx + x + 2, J2))
        for y in range(Ly - 2):
            for x in range(Lx - 1):
                out.append((y * Lx + x, (y + 2) * Lx + x + 1, J2))
    return out


def local_energies(T, Ly, Lx, D, J1, J2, configs, triangular=False):
    """E_loc(S) = sum_S' <S'|H|S> Psi(S')/Psi(S), with H = sum J S_i.S_j written out directly."""
    configs = np.asarray(configs)
    psi = amplitudes(T, Ly, Lx, D, configs)
    e = np.zeros(len(configs))
    for i, j, J in bonds(Ly, Lx, J1, J2, triangular):
        if J == 0.0:
            continue
        par = configs[:, i] == configs[:, j]
        e += np.where(par, 0.25 * J, -0.25 * J)
        flipped = configs.copy()
        flipped[:, i], flipped[:, j] = configs[:, j], configs[:, i]
        anti = ~par
        if anti.any():
            pf = amplitudes(T, Ly, Lx, D, flipped[anti])
            e[anti] += 0.5 * J * pf / psi[anti]
    return e, psi


def sector_energy_bonds(psi, configs, N, bond_list):
    """<psi|H|psi> / <psi|psi> over the S^z = 0 amplitudes psi (rows of ``configs``) for
    H = sum over (i, j, J) of J S_i.S_j (the configurations' exchanged partners found by bit code)."""
    configs = np.asarray(configs)
    codes = (configs.astype(np.int64) << np.arange(N, dtype=np.int64)[::-1]).sum(axis=1)
    order = np.argsort(codes)
    sorted_codes = codes[order]
    num = 0.0
    for k, k2, J in bond_list:
        if J == 0.0:
            continue
        par = configs[:, k] == configs[:, k2]
        num += J * np.sum(np.where(par, 0.25, -0.25) * psi * psi)
        anti = ~par
        partner = codes[anti] ^ ((1 << (N - 1 - k)) | (1 << (N - 1 - k2)))
        j = order[np.searchsorted(sorted_codes, partner)]
        num += 0.5 * J * np.sum(psi[anti] * psi[j])
    return float(num / (psi @ psi))


def sector_energy(psi, configs, Ly, Lx, J1=1.0, triangular=False):
    """<psi|H|psi> / <psi|psi> for amplitudes psi of every S^z = 0 configuration
    (rows of ``configs``), H the nearest-neighbour Heisenberg lattice (triangular:
    with the diagonal (y,x)-(y+1,x+1) as a further nearest-neighbour bond):
    parallel pairs give J1/4, antiparallel pairs -J1/4 plus J1/2 times the
    amplitude of the exchanged configuration (found by its bit code)."""
    configs = np.asarray(configs)
    N = Ly * Lx
    codes = (configs.astype(np.int64) << np.arange(N, dtype=np.int64)[::-1]).sum(axis=1)
    order = np.argsort(codes)
    sorted_codes = codes[order]
    num = 0.0
    for y in range(Ly):
        for x in range(Lx):
            k = y * Lx + x
            nb = ([k + 1] if x < Lx - 1 else []) + ([k + Lx] if y < Ly - 1 else [])
            if triangular and x < Lx - 1 and y < Ly - 1:
                nb.append(k + Lx + 1)
            for k2 in nb:
                par = configs[:, k] == configs[:, k2]
                num += J1 * np.sum(np.where(par, 0.25, -0.25) * psi * psi)
                anti = ~par
                partner = codes[anti] ^ ((1 << (N - 1 - k)) | (1 << (N - 1 - k2)))
                j = order[np.searchsorted(sorted_codes, partner)]
                num += 0.5 * J1 * np.sum(psi[anti] * psi[j])
    return float(num / (psi @ psi))

