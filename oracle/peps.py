"""Single-layer PEPS contraction of the oracle (test infrastructure only).

At a fixed configuration S every site carries the 4-leg tensor t = T[s]
(Sec. II.A Eq. (4)); Psi(S) is the value of that single-layer network.

Boundary MPS (App. B, Fig. "boundaryMPS"): the first row is an MPS, every
other row an MPO.  Applying row y to the upper boundary U_{y-1} multiplies the
bond dimension by D; the result is brought back to Dc.  The paper does this by
a variational fit; the oracle uses the unique canonical SVD compression
instead (``compress``): left-to-right Householder QR with no truncation, then
right-to-left SVD keeping the Dc largest singular values.  Its output state
does not depend on QR/SVD sign or gauge choices, so an independent
implementation of the same compression can agree with it to rounding.

Row networks (App. C, Fig. "contraction"): with U_{y-1} above and D_{y+1}
below, N_y = <D_{y+1}|M_y|U_{y-1}>.  The left auxiliary tensor L(x) contracts
columns 0..x and the right one R(x) columns x..Lx-1, so N_y = L(x-1).R(x) for
every x.  Two-row ("4-line") networks <D_{y+2}|M_{y+1} M_y|U_{y-1}> serve the
vertical and diagonal pairs, which the paper says are computed "similarly".

Index conventions (true dimensions, no padding):

    upper boundary site  A[a, u, b]   a/b left/right bond, u = physical leg
                                      joined to the u leg of the next row
    lower boundary site  B[c, d, e]   d joined to the d leg of the row above
    PEPS site            t[l, u, r, d]
    3-line env           L[a, l, c]   (open legs of the contracted part)
    4-line env           L[a, l1, l2, c]

Parity: exact (Dc at or above the exact rank) results are pinned by brute-force
contraction in the tests; truncated results have no external truth and are
pinned only by invariants (gauge independence, Psi = L.R at every cut,
exactness as Dc grows, direct recontraction of every ratio).
"""
import math

import numpy as np

from .lattice import site_tensor


class ZeroAmplitude(ArithmeticError):
    """A network that must be non-zero (an amplitude or a ratio denominator) is exactly zero."""


def row_tensors(T, lat, spins, y, flips=()):
    """The tensors t_{y,x} = T_{y,x}[s_{y,x}] of row y; sites in ``flips`` use 1 - s."""
    s = np.asarray(spins).reshape(lat.Ly, lat.Lx)
    out = []
    for x in range(lat.Lx):
        sv = int(s[y, x])
        if (y, x) in flips:
            sv = 1 - sv
        out.append(site_tensor(T, lat, y, x, sv))
    return out


def trivial_mps(Lx):
    """The boundary above row 0 (below the last row): every leg of dimension 1."""
    return [np.ones((1, 1, 1)) for _ in range(Lx)]


# --------------------------------------------------------------------------
# Boundary MPS and its compression (App. B)
# --------------------------------------------------------------------------

def absorb_down(U, row):
    """M_y|U_{y-1}>: site x becomes B[(a,l), d, (b,r)] = sum_u A[a,u,b] t[l,u,r,d]."""
    out = []
    for A, t in zip(U, row):
        a, _, b = A.shape
        l, _, r, d = t.shape
        out.append(np.einsum('aub,lurd->aldbr', A, t).reshape(a * l, d, b * r))
    return out


def absorb_up(Dm, row):
    """<D_{y+1}|M_y: site x becomes B[(c,l), u, (e,r)] = sum_d B[c,d,e] t[l,u,r,d]."""
    out = []
    for B, t in zip(Dm, row):
        c, _, e = B.shape
        l, u, r, _ = t.shape
        out.append(np.einsum('cde,lurd->cluer', B, t).reshape(c * l, u, e * r))
    return out


def compress(B, Dc):
    """Canonical SVD compression of an open MPS to bond dimension Dc.

    1. For j = 0..n-2: thin QR of B_j reshaped (a_j p_j) x a_{j+1}; B_j <- Q,
       B_{j+1} <- R B_{j+1}.  Nothing is truncated.
    2. For j = n-1..1: SVD of B_j reshaped a_j x (p_j a_{j+1}) = U S V^T; keep
       k = min(Dc, a_j, p_j a_{j+1}) singular values (zeros included);
       B_j <- V^T[:k], B_{j-1} <- B_{j-1} (U[:, :k] S[:k]).
    3. The centre B_0 carries the norm nu; B_0 <- B_0 / nu.

    Returns (list of site tensors (k_j, p_j, k_{j+1}), log nu).  Raises
    ZeroAmplitude if the state is exactly zero.
    """
    B = [np.array(b, dtype=np.float64, copy=True) for b in B]
    n = len(B)
    for j in range(n - 1):
        a, p, b = B[j].shape
        Q, R = np.linalg.qr(B[j].reshape(a * p, b), mode='reduced')
        B[j] = Q.reshape(a, p, Q.shape[1])
        B[j + 1] = np.tensordot(R, B[j + 1], axes=(1, 0))
    for j in range(n - 1, 0, -1):
        a, p, b = B[j].shape
        U, S, Vt = np.linalg.svd(B[j].reshape(a, p * b), full_matrices=False)
        k = min(Dc, a, p * b)
        B[j] = Vt[:k].reshape(k, p, b)
        B[j - 1] = np.tensordot(B[j - 1], U[:, :k] * S[:k], axes=(2, 0))
    nu = float(np.linalg.norm(B[0]))
    if nu == 0.0:
        raise ZeroAmplitude("boundary MPS compressed to the zero state")
    B[0] = B[0] / nu
    return B, math.log(nu)


def variational_bond_dims(B, Dc):
    """Bond dimensions k_0..k_n of the fitted MPS: those of the canonical
    compression of B (left-to-right rank bounds, then k_j = min(Dc, bound_j,
    p_j k_{j+1}) from the right), so that both modes produce the same shapes."""
    n = len(B)
    bound = [1] * (n + 1)
    for j in range(n):
        a, p, b = B[j].shape
        bound[j + 1] = min(bound[j] * p, b)
    k = [1] * (n + 1)
    for j in range(n - 1, 0, -1):
        k[j] = min(Dc, bound[j], B[j].shape[1] * k[j + 1])
    return k


def _qr_q(M):
    """Q of the thin Householder QR of a tall matrix (LAPACK through numpy)."""
    return np.linalg.qr(M, mode='reduced')[0]


def _fit_env_left(L, Bj, Uj):
    """L_{j+1}[k', b] = sum L_j[k, a] U_j[k, p, k'] B_j[a, p, b]."""
    return np.einsum('ka,kpl,apb->lb', L, Uj, Bj, optimize=True)


def _fit_env_right(R, Bj, Uj):
    """R_j[k, a] = sum U_j[k, p, k'] B_j[a, p, b] R_{j+1}[k', b]."""
    return np.einsum('kpl,apb,lb->ka', Uj, Bj, R, optimize=True)


def _fit_center(L, Bj, R):
    """The site tensor that maximises the overlap with B given orthonormal
    neighbours: M[k, p, k'] = sum L[k, a] B_j[a, p, b] R[k', b]."""
    return np.einsum('ka,apb,lb->kpl', L, Bj, R, optimize=True)


def compress_variational(B, Dc, sweeps, qr=_qr_q):
    """Variational boundary-MPS fit (App. B): minimise ||B - U||^2 over MPS U of
    bond dimension Dc by alternating single-site updates (the iterative
    compression sweep the paper cites).  The paper fixes neither the start nor
    the number of sweeps; here they are:

    * start: the MPS of the leading k_j x k_{j+1} blocks of the sites of B
      (their first combined bond indices; k from ``variational_bond_dims``),
      brought to right-orthonormal form without changing its state: from the
      right, each site j >= 1 becomes the orthonormal rows Q of its LQ
      factorisation and the factor L = M Q^T moves into site j - 1;
    * right environments R_j = <U_j..U_{n-1}|B_j..B_{n-1}> of that start;
    * each sweep: left to right, j = 0..n-2, the optimal site given orthonormal
      neighbours, M = L_j B_j R_{j+1}, replaced by the Q of its QR
      ((k_j p) x k_{j+1}) and L_{j+1} updated; then right to left, j = n-1..1,
      the same M replaced by the orthonormal rows of its LQ (k_j x (p k_{j+1}))
      and R_j updated;
    * finally the optimal site 0, M_0 = B_0 R_1, carries the norm nu:
      U_0 = M_0 / nu.

    With orthonormal neighbours the fitted state is M_j in the basis they span,
    so the result does not depend on the sign or gauge conventions of the QR
    (``qr`` may be any thin QR).  Returns (sites (k_j, p_j, k_{j+1}), log nu);
    raises ZeroAmplitude if the fitted state is zero.  Parity: pinned by
    exactness at full rank, a monotonically decreasing distance over sweeps,
    the Eckart-Young optimum on two sites, and independence of the QR gauge
    (tests/test_oracle_variational.py); a rank-deficient centre (whose Q is
    completed arbitrarily) is parity unpinned.
    """
    B = [np.asarray(b, dtype=np.float64) for b in B]
    n = len(B)
    k = variational_bond_dims(B, Dc)
    U = [B[j][:k[j], :, :k[j + 1]].copy() for j in range(n)]

    def lq_rows(M):
        kj, p, kr = M.shape
        return qr(M.reshape(kj, p * kr).T).T.reshape(kj, p, kr)

    # right-orthonormal form of the start, state unchanged: U_j = L Q with Q's
    # rows orthonormal; L moves into site j - 1
    for j in range(n - 1, 0, -1):
        kj, p, kr = U[j].shape
        M = U[j].reshape(kj, p * kr)
        Q = lq_rows(U[j]).reshape(kj, p * kr)
        U[j] = Q.reshape(kj, p, kr)
        U[j - 1] = np.tensordot(U[j - 1], M @ Q.T, axes=(2, 0))
    R = [None] * (n + 1)
    R[n] = np.ones((1, 1))
    for j in range(n - 1, 0, -1):
        R[j] = _fit_env_right(R[j + 1], B[j], U[j])
    L = [None] * (n + 1)
    L[0] = np.ones((1, 1))
    for _ in range(sweeps):
        for j in range(n - 1):
            M = _fit_center(L[j], B[j], R[j + 1])
            kj, p, kr = M.shape
            U[j] = qr(M.reshape(kj * p, kr)).reshape(kj, p, kr)
            L[j + 1] = _fit_env_left(L[j], B[j], U[j])
        for j in range(n - 1, 0, -1):
            U[j] = lq_rows(_fit_center(L[j], B[j], R[j + 1]))
            R[j] = _fit_env_right(R[j + 1], B[j], U[j])
    M0 = _fit_center(L[0], B[0], R[1])
    nu = float(np.linalg.norm(M0))
    if nu == 0.0:
        raise ZeroAmplitude("boundary MPS fitted to the zero state")
    U[0] = M0 / nu
    return U, math.log(nu)


def compress_boundary(B, lat):
    """The lattice's truncation: the canonical SVD compression (default) or the
    variational fit with ``lat.fit_sweeps`` sweeps (``lat.compress_mode``)."""
    if getattr(lat, "compress_mode", "canonical") == "variational":
        return compress_variational(B, lat.Dc, lat.fit_sweeps)
    return compress(B, lat.Dc)


def upper_boundaries(T, lat, spins, upto=None):
    """U_{-1}, U_0, ..., U_{upto} (default Ly-2) and their cumulative log-scales.

    Returned lists are indexed by y+1: U[y+1] is U_y, lam[y+1] = sum of log nu.
    """
    if upto is None:
        upto = lat.Ly - 2
    U = [trivial_mps(lat.Lx)]
    lam = [0.0]
    for y in range(upto + 1):
        Uy, lognu = compress_boundary(absorb_down(U[-1], row_tensors(T, lat, spins, y)), lat)
        U.append(Uy)
        lam.append(lam[-1] + lognu)
    return U, lam


def lower_boundary(Dn, T, lat, spins, y):
    """D_y = C(<D_{y+1}|M_y) and its log-scale."""
    return compress_boundary(absorb_up(Dn, row_tensors(T, lat, spins, y)), lat)


# --------------------------------------------------------------------------
# Row networks and auxiliary tensors (App. C)
# --------------------------------------------------------------------------

def env3_left(L, A, t, B):
    """L(x)[b,r,e] = sum L(x-1)[a,l,c] A[a,u,b] t[l,u,r,d] B[c,d,e]."""
    X = np.einsum('alc,aub->lcub', L, A)
    X = np.einsum('lcub,lurd->cbrd', X, t)
    return np.einsum('cbrd,cde->bre', X, B)


def env3_right(R, A, t, B):
    """R(x)[a,l,c] = sum A[a,u,b] t[l,u,r,d] B[c,d,e] R(x+1)[b,r,e]."""
    X = np.einsum('aub,bre->aure', A, R)
    X = np.einsum('aure,lurd->aled', X, t)
    return np.einsum('aled,cde->alc', X, B)


def row3_envs(U, row, Dn):
    """Left and right auxiliary tensors of the 3-line network <Dn|row|U>.

    Lenv[x+1] = L(x) (Lenv[0] = ones), Renv[x] = R(x) (Renv[Lx] = ones).
    """
    n = len(row)
    Lenv = [np.ones((1, 1, 1))]
    for x in range(n):
        Lenv.append(env3_left(Lenv[-1], U[x], row[x], Dn[x]))
    Renv = [None] * (n + 1)
    Renv[n] = np.ones((1, 1, 1))
    for x in range(n - 1, -1, -1):
        Renv[x] = env3_right(Renv[x + 1], U[x], row[x], Dn[x])
    return Lenv, Renv


def row3_value(U, row, Dn):
    """N = <Dn|row|U> by a single left-to-right contraction."""
    L = np.ones((1, 1, 1))
    for x in range(len(row)):
        L = env3_left(L, U[x], row[x], Dn[x])
    return float(L.reshape(()))


def env4_left(L, A, t1, t2, B):
    """L(x)[b,r1,r2,e] = sum L(x-1)[a,l1,l2,c] A[a,u,b] t1[l1,u,r1,m] t2[l2,m,r2,d] B[c,d,e]."""
    X = np.einsum('awzc,aub->wzcub', L, A)
    X = np.einsum('wzcub,wurm->zcbrm', X, t1)
    X = np.einsum('zcbrm,zmsd->cbrsd', X, t2)
    return np.einsum('cbrsd,cde->brse', X, B)


def env4_right(R, A, t1, t2, B):
    """R(x)[a,l1,l2,c] = sum A[a,u,b] t1[l1,u,r1,m] t2[l2,m,r2,d] B[c,d,e] R(x+1)[b,r1,r2,e]."""
    X = np.einsum('aub,bwze->auwze', A, R)
    X = np.einsum('auwze,luwm->alzem', X, t1)
    X = np.einsum('alzem,kmzd->alked', X, t2)
    return np.einsum('alked,cde->alkc', X, B)


def row4_envs(U, row1, row2, Dn):
    n = len(row1)
    Lenv = [np.ones((1, 1, 1, 1))]
    for x in range(n):
        Lenv.append(env4_left(Lenv[-1], U[x], row1[x], row2[x], Dn[x]))
    Renv = [None] * (n + 1)
    Renv[n] = np.ones((1, 1, 1, 1))
    for x in range(n - 1, -1, -1):
        Renv[x] = env4_right(Renv[x + 1], U[x], row1[x], row2[x], Dn[x])
    return Lenv, Renv


def row4_value(U, row1, row2, Dn):
    L = np.ones((1, 1, 1, 1))
    for x in range(len(row1)):
        L = env4_left(L, U[x], row1[x], row2[x], Dn[x])
    return float(L.reshape(()))


def defect3(Lprev, A, B, Rnext):
    """Defect tensor of one site in a 3-line network (Sec. II.A Eq. (7)).

    Delta[l,u,r,d] = sum L(x-1)[a,l,c] A[a,u,b] R(x+1)[b,r,e] B[c,d,e]: the
    network with the site removed, so N = sum t * Delta.
    """
    X = np.einsum('alc,aub->lcub', Lprev, A)
    X = np.einsum('lcub,bre->lcure', X, Rnext)
    return np.einsum('lcure,cde->lurd', X, B)


# --------------------------------------------------------------------------
# Amplitude (Sec. II.A Eq. (4); App. B)
# --------------------------------------------------------------------------

def amplitude(T, lat, spins):
    """(sign, log|Psi(S)|) from the full top-down boundary contraction.

    log|Psi| = sum of the log-scales of U_0..U_{Ly-2} + log|<row_{Ly-1}|U_{Ly-2}>|.
    """
    U, lam = upper_boundaries(T, lat, spins)
    last = row3_value(U[lat.Ly - 1], row_tensors(T, lat, spins, lat.Ly - 1), trivial_mps(lat.Lx))
    if last == 0.0:
        raise ZeroAmplitude("Psi(S) = 0")
    return (1 if last > 0 else -1), lam[lat.Ly - 1] + math.log(abs(last))
