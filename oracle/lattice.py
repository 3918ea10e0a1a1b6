"""Lattice geometry, tensor layout and Hamiltonian of the oracle (test infrastructure only).

Conventions (the paper leaves these open; readings are listed in the design notes):

* Sites (y, x), y = 0 the top row, x = 0 the left column, k = y*Lx + x.
* Physical index s in {0, 1}; s = 0 is S^z = +1/2.
* Site tensor T_k[s][l, u, r, d]: the rank-5 tensor A_k(s, l, r, u, d) of
  Sec. II.A Eq. (1) with the virtual legs stored in (l, u, r, d) order.  Legs on
  the open boundary have dimension 1, bulk legs dimension D.
* The parameter vector is the concatenation over k of T_k[s][l][u][r][d].
  For 32x32, D=8 it holds 7,496,192 numbers, the "about 7.5 x 10^6 variables"
  quoted in Sec. II.B.
* H = J1 sum_NN S_i.S_j + J2 sum_diag S_i.S_j with S = sigma/2 and open
  boundaries (Sec. III.A; the Hamiltonian elements of App. C Eq. (Elocal)).
  Pinned by reproducing exact-diagonalisation energies printed in Table III.
* The triangular lattice on the square grid (Sec. III.B, Fig. 7(a)): one
  diagonal of every plaquette, here (y,x)-(y+1,x+1), is a nearest-neighbour
  bond of coupling J1.  Its next-nearest neighbours (distance sqrt(3), coupling
  J2) are the other diagonal (y,x+1)-(y+1,x) and the two knight bonds
  (y,x)-(y+1,x+2) and (y,x)-(y+2,x+1).  On the open 4x4 lattice the choice of
  diagonal does not change the spectrum (a mirror image).
"""
import numpy as np

from . import philox


class Lattice:
    """An Ly x Lx open-boundary square lattice carrying a PEPS of bond dimension D."""

    def __init__(self, Ly, Lx, D, Dc, J1=1.0, J2=0.0, compress_mode="canonical", fit_sweeps=2,
                 geometry="square"):
        """compress_mode: the boundary truncation, "canonical" (SVD compression)
        or "variational" (the fit of App. B with fit_sweeps sweeps).  geometry:
        "square" (J2 on both diagonals) or "triangular" (J1 on the diagonal
        (y,x)-(y+1,x+1), J2 on the other diagonal and the knight bonds)."""
        if Ly < 1 or Lx < 1 or D < 1 or Dc < 1:
            raise ValueError("lattice sizes, D and Dc must be >= 1")
        if compress_mode not in ("canonical", "variational") or fit_sweeps < 0:
            raise ValueError("compress_mode is canonical or variational, fit_sweeps >= 0")
        if geometry not in ("square", "triangular"):
            raise ValueError("geometry is square or triangular")
        self.Ly, self.Lx, self.D, self.Dc = int(Ly), int(Lx), int(D), int(Dc)
        self.J1, self.J2 = float(J1), float(J2)
        self.geometry = geometry
        # couplings of the diagonal (y,x)-(y+1,x+1) and anti-diagonal (y,x+1)-(y+1,x) of a plaquette
        self.Jd = self.J1 if geometry == "triangular" else self.J2
        self.Ja = self.J2
        self.diagonals = self.Jd != 0.0 or self.Ja != 0.0
        # knight bonds (y,x)-(y+1,x+2) and (y,x)-(y+2,x+1) of the triangular lattice
        self.Jk = self.J2 if geometry == "triangular" else 0.0
        self.knights = self.Jk != 0.0
        self.compress_mode, self.fit_sweeps = compress_mode, int(fit_sweeps)
        self.N = self.Ly * self.Lx
        self.offsets = []
        off = 0
        for y in range(self.Ly):
            for x in range(self.Lx):
                self.offsets.append(off)
                off += 2 * int(np.prod(self.dims(y, x)))
        self.Np = off

    def dims(self, y, x):
        """(l, u, r, d) leg dimensions of site (y, x); open-boundary legs have dimension 1."""
        D = self.D
        return (D if x > 0 else 1, D if y > 0 else 1,
                D if x < self.Lx - 1 else 1, D if y < self.Ly - 1 else 1)

    def site(self, y, x):
        return y * self.Lx + x


def site_tensor(T, lat, y, x, s):
    """View of T_{y,x}[s] with shape (l, u, r, d)."""
    dl, du, dr, dd = lat.dims(y, x)
    n = dl * du * dr * dd
    o = lat.offsets[lat.site(y, x)] + int(s) * n
    return T[o:o + n].reshape(dl, du, dr, dd)


def compact_size(lat):
    """Length of one per-sample log-derivative vector: the occupied slot of every site."""
    return lat.Np // 2


def compact_offsets(lat):
    offs, o = [], 0
    for y in range(lat.Ly):
        for x in range(lat.Lx):
            offs.append(o)
            o += int(np.prod(lat.dims(y, x)))
    return offs


# --------------------------------------------------------------------------
# Hamiltonian (Sec. II.A Eq. (3); App. C Eq. (Elocal))
# --------------------------------------------------------------------------

def bonds(lat):
    """All interacting pairs ((y1,x1), (y2,x2), J): NN horizontal, NN vertical, when a
    diagonal is coupled both diagonals of every plaquette (an uncoupled one with J = 0),
    and on the triangular lattice with J2 != 0 the knight bonds (y,x)-(y+1,x+2), then
    (y,x)-(y+2,x+1)."""
    out = []
    for y in range(lat.Ly):
        for x in range(lat.Lx - 1):
            out.append(((y, x), (y, x + 1), lat.J1))
    for y in range(lat.Ly - 1):
        for x in range(lat.Lx):
            out.append(((y, x), (y + 1, x), lat.J1))
    if lat.diagonals:
        for y in range(lat.Ly - 1):
            for x in range(lat.Lx - 1):
                out.append(((y, x), (y + 1, x + 1), lat.Jd))
                out.append(((y, x + 1), (y + 1, x), lat.Ja))
    if lat.knights:
        for y in range(lat.Ly - 1):
            for x in range(lat.Lx - 2):
                out.append(((y, x), (y + 1, x + 2), lat.Jk))
        for y in range(lat.Ly - 2):
            for x in range(lat.Lx - 1):
                out.append(((y, x), (y + 2, x + 1), lat.Jk))
    return out


def bond_elements(si, sj, J):
    """Matrix elements of J S_i.S_j (S = sigma/2) acting on the pair (si, sj).

    Returns (diagonal, offdiagonal): <si sj|H_ij|si sj> = J/4 for parallel and
    -J/4 for antiparallel spins; <sj si|H_ij|si sj> = J/2 connects an
    antiparallel pair to its exchanged partner and is 0 otherwise.
    """
    if si == sj:
        return 0.25 * J, 0.0
    return -0.25 * J, 0.5 * J


def local_energy(lat, spins, ratio_of_pair):
    """E_loc(S) = sum over bonds of H_ij elements times Psi(S')/Psi(S) (App. C Eq. (Elocal)).

    ``ratio_of_pair((y1,x1),(y2,x2))`` returns Psi(S')/Psi(S) for S' = S with the
    two spins exchanged; it is called only for antiparallel pairs.
    """
    s = np.asarray(spins).reshape(lat.Ly, lat.Lx)
    e = 0.0
    for p, q, J in bonds(lat):
        diag, off = bond_elements(s[p], s[q], J)
        e += diag
        if off != 0.0:
            e += off * ratio_of_pair(p, q)
    return e


# --------------------------------------------------------------------------
# Inputs drawn by the method (tensor initialisation, chain starts)
# --------------------------------------------------------------------------

def init_tensors(lat, seed, lattice_id=0, scale=None, perturb=0.0):
    """T = scale * xi (+ perturb * xi'), xi, xi' ~ N(0,1) from Philox + Box-Muller.

    Element p of the parameter vector uses counter (p, 0, 0, TAG_INIT) (and
    TAG_PERTURB for xi') under key (seed, lattice_id).  The default scale is
    1/sqrt(D^4) for every site, boundary sites included.
    """
    if scale is None:
        scale = 1.0 / lat.D ** 2
    key = (seed, lattice_id)
    T = np.empty(lat.Np)
    for p in range(lat.Np):
        T[p] = scale * philox.gaussian((p, 0, 0, philox.TAG_INIT), key)
        if perturb != 0.0:
            T[p] += perturb * philox.gaussian((p, 0, 0, philox.TAG_PERTURB), key)
    return T


def neel(lat):
    """Neel configuration s(y,x) = (x + y) mod 2 (S^z_tot = 0 when N is even)."""
    return np.array([(x + y) % 2 for y in range(lat.Ly) for x in range(lat.Lx)], dtype=np.int8)


def neel_shuffled(lat, seed, lattice_id, chain):
    """Durstenfeld / Fisher-Yates shuffle of the Neel list with Philox indices.

    For i = N-1 down to 1: j = floor(u_i (i+1)), swap entries i and j, where
    u_i comes from counter (chain, 0, i, TAG_SHUFFLE) under key (seed, lattice_id).
    """
    s = neel(lat)
    for i in range(lat.N - 1, 0, -1):
        w = philox.philox4x64_10((chain, 0, i, philox.TAG_SHUFFLE), (seed, lattice_id))
        j = philox.bounded_index(w[0], i + 1)
        s[i], s[j] = s[j], s[i]
    return s


# --------------------------------------------------------------------------
# The transposed lattice: site (y, x) -> (x, y), legs (l, u, r, d) -> (u, l, d, r)
# --------------------------------------------------------------------------

def transpose_lattice(lat):
    """The Lx x Ly lattice of the transposed PEPS (same D, Dc, couplings, geometry and truncation;
    the diagonal (y,x)-(y+1,x+1) maps onto itself)."""
    return Lattice(lat.Lx, lat.Ly, lat.D, lat.Dc, J1=lat.J1, J2=lat.J2, compress_mode=lat.compress_mode,
                   fit_sweeps=lat.fit_sweeps, geometry=lat.geometry)


def transpose_tensors(T, lat):
    """T' with T'_(x,y)[s][u][l][d][r] = T_(y,x)[s][l][u][r][d], in the transposed lattice's layout."""
    lt = transpose_lattice(lat)
    out = np.zeros(lt.Np)
    for y in range(lat.Ly):
        for x in range(lat.Lx):
            for s in (0, 1):
                t = np.transpose(site_tensor(T, lat, y, x, s), (1, 0, 3, 2))
                dims = lt.dims(x, y)
                assert t.shape == dims
                n = int(np.prod(dims))
                o = lt.offsets[lt.site(x, y)] + s * n
                out[o:o + n] = t.ravel()
    return out


def transpose_spins(spins, lat):
    """s'(x, y) = s(y, x), in the transposed lattice's site order."""
    return np.asarray(spins, dtype=np.int8).reshape(lat.Ly, lat.Lx).T.ravel().copy()


def untranspose_spins(spins_t, lat):
    return np.asarray(spins_t, dtype=np.int8).reshape(lat.Lx, lat.Ly).T.ravel().copy()
