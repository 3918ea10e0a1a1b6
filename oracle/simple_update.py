"""Simple-update imaginary-time evolution (App. A), nearest- and
next-nearest-neighbour terms: test infrastructure only (tests/, never the
product path).

The PEPS is held as site tensors B_k (same layout as the parameter vector:
B_k[s][l, u, r, d]) and a diagonal matrix lambda on every link between
nearest neighbours (App. A: the environment of a tensor approximated by these
diagonal matrices).  A step applies exp(-dt J S_i.S_j) once to every
nearest-neighbour link; each application (App. A, Fig. 8 (b)-(h), here with
two sites instead of three):

1. the lambdas of the outer links are contracted into both site tensors;
2. QR of the first (outer legs x (s, bond)) and of the second tensor gives
   Q_A R_A and Q_B R_B (the reduced tensors R carry the physical and bond legs);
3. Theta = R_A lambda_bond R_B^T with the gate applied to the two physical legs;
4. SVD of Theta (rows (a, s_A), columns (s_B, b)), truncated to the link's
   dimension: the kept singular values, normalised, are the new lambda;
5. the new tensors are Q_A U and Q_B V with the outer lambdas divided out.

Readings (the paper is silent on these): the gate is the exact exponential of
the bond term; a step visits the links in four classes - horizontal links with
x even, horizontal with x odd, vertical with y even, vertical with y odd - and
links of one class share no site, so their updates commute exactly; the new
lambda is normalised to unit 2-norm; singular values below 1e-6 times the
largest are dropped (lambda 0, their vectors 0), and dividing by a lambda
means multiplying by 1/lambda where lambda > 0 and by 0 elsewhere; the start
is the given tensors with every lambda 1; the result absorbs lambda^(1/2)
into each of the two tensors of every link (App. A's last step).  The
convergence measure is App. A's: the mean over links of
||lambda(t+dt) - lambda(t)|| / ||lambda(t)|| over one step.

Diagonal terms (J2 on both diagonals of every plaquette; on the triangular
lattice J1 on the diagonal (y,x)-(y+1,x+1) and J2 on the other; its knight
bonds are left to the optimisation that follows) follow Fig. 8: the pair (B_1, B_3) is joined through a corner site B_2 (reading: the
diagonal (y,x)-(y+1,x+1) through (y,x+1), the anti-diagonal (y,x+1)-(y+1,x)
through (y,x)); B_1 and B_3 with their outer lambdas are QR-reduced to R_1
and R_3; the gate acts on the physical legs of B_1 and B_3 of
T_a = R_1 lambda_4 B_2 lambda_7 R_3^T (B_2 with its outer lambdas); a
truncated SVD splits T_a into R~_1, lambda~_4 and T_b; a second one splits
lambda~_4 T_b into T_c, lambda~_7 and R~_3; the new B_1 = Q_1 R~_1,
B_2 = T_c / lambda~_4 and B_3 = Q_3 R~_3, each with its outer lambdas divided
out.  A step visits the nearest-neighbour classes, then the plaquettes in four
classes (y mod 2, x mod 2), each class's diagonals and then its
anti-diagonals; plaquettes of one class share no site.

Pinned (tests/test_oracle_simple_update.py): the QR-reduced update equals the
update written out on the full two-site tensor (step 2 left out); without
truncation on open chains the result is the dense Trotter product of the same
gates applied to the start; one link converges to the singlet (-3/4); the gate
is the matrix exponential of the bond term.
"""
import numpy as np

DROP = 1e-6  # relative singular-value floor of step 4


def heisenberg_gate(dt, J):
    """exp(-dt J S_A.S_B) as G[t_A, t_B, s_A, s_B] (s = 0 is S^z = +1/2).

    S_A.S_B is 1/4 on the triplet and -3/4 on the singlet (ud - du)/sqrt(2)."""
    a = np.exp(-0.25 * dt * J)
    b = np.exp(0.75 * dt * J)
    G = np.zeros((2, 2, 2, 2))
    G[0, 0, 0, 0] = G[1, 1, 1, 1] = a
    G[0, 1, 0, 1] = G[1, 0, 1, 0] = 0.5 * (a + b)
    G[0, 1, 1, 0] = G[1, 0, 0, 1] = 0.5 * (a - b)
    return G


def link_index(lat, y, x, horizontal):
    """Horizontal links (y,x)-(y,x+1) first, row-major; then vertical (y,x)-(y+1,x)."""
    if horizontal:
        return y * (lat.Lx - 1) + x
    return lat.Ly * (lat.Lx - 1) + y * lat.Lx + x


def n_links(lat):
    return lat.Ly * (lat.Lx - 1) + (lat.Ly - 1) * lat.Lx


def leg_links(lat, y, x):
    """Link index of legs (l, u, r, d) of site (y, x); None on the open boundary."""
    return (link_index(lat, y, x - 1, True) if x > 0 else None,
            link_index(lat, y - 1, x, False) if y > 0 else None,
            link_index(lat, y, x, True) if x < lat.Lx - 1 else None,
            link_index(lat, y, x, False) if y < lat.Ly - 1 else None)


def link_classes(lat):
    """The four classes of links, each a list of ((y, x), (y2, x2), leg of A, leg of B)."""
    out = [[], [], [], []]
    for y in range(lat.Ly):
        for x in range(lat.Lx - 1):
            out[x % 2].append(((y, x), (y, x + 1), 2, 0))
    for y in range(lat.Ly - 1):
        for x in range(lat.Lx):
            out[2 + y % 2].append(((y, x), (y + 1, x), 3, 1))
    return out


def su_init(T, lat):
    """Site tensors (arrays (2, l, u, r, d)) of the flat parameter vector T and unit lambdas."""
    B = []
    for y in range(lat.Ly):
        for x in range(lat.Lx):
            dims = lat.dims(y, x)
            o = lat.offsets[lat.site(y, x)]
            B.append(np.array(T[o:o + 2 * int(np.prod(dims))], dtype=np.float64).reshape((2,) + dims))
    lam = [np.ones(lat.D) for _ in range(n_links(lat))]
    return B, lam


def _pinv(v):
    out = np.zeros_like(v)
    nz = v > 0.0
    out[nz] = 1.0 / v[nz]
    return out


def _scale_legs(A, vecs):
    """A[s, l, u, r, d] times vecs[q] on leg q (None: leave the leg)."""
    A = A.copy()
    for q, v in enumerate(vecs):
        if v is not None:
            shape = [1] * 5
            shape[1 + q] = v.shape[0]
            A = A * v.reshape(shape)
    return A


def _outer_lambdas(lat, lam, y, x, bond_leg, inverse=False):
    links = leg_links(lat, y, x)
    return [None if (q == bond_leg or links[q] is None) else (_pinv(lam[links[q]]) if inverse else lam[links[q]])
            for q in range(4)]


def _to_matrix(M, bond_leg):
    """(outer legs in (l, u, r, d) order) x (s, bond) of M[s, l, u, r, d]."""
    others = [q for q in range(4) if q != bond_leg]
    P = np.transpose(M, [1 + q for q in others] + [0, 1 + bond_leg])
    return P.reshape(-1, 2 * M.shape[1 + bond_leg]), P.shape[:3]


def _from_matrix(X, outer_shape, bond_leg, kdim):
    """Inverse of _to_matrix for X[(outer), (s, k)] with a bond leg of kdim."""
    others = [q for q in range(4) if q != bond_leg]
    P = X.reshape(tuple(outer_shape) + (2, kdim))
    order = [0] * 5
    # axes of P: others[0], others[1], others[2], s, bond -> target (s, l, u, r, d)
    src = {1 + others[0]: 0, 1 + others[1]: 1, 1 + others[2]: 2, 0: 3, 1 + bond_leg: 4}
    for t in range(5):
        order[t] = src[t]
    return np.transpose(P, order)


def _truncated_svd(Theta, kdim):
    U, S, Vt = np.linalg.svd(Theta, full_matrices=False)
    k = int(min(kdim, np.sum(S > DROP * S[0]))) if S[0] > 0 else 0
    lam_new = np.zeros(kdim)
    lam_new[:k] = S[:k] / np.linalg.norm(S[:k]) if k else 0.0
    Uk = np.zeros((U.shape[0], kdim))
    Vk = np.zeros((kdim, Vt.shape[1]))
    Uk[:, :k] = U[:, :k]
    Vk[:k] = Vt[:k]
    return Uk, lam_new, Vk


def su_bond(B, lam, lat, a, b, leg_a, leg_b, G, reduced=True):
    """Apply the gate G to the link between sites a and b (App. A, Fig. 8), in place.

    reduced=False writes the same update out on the full two-site tensor (no QR),
    the plain definition the reduced one is checked against."""
    (ya, xa), (yb, xb) = a, b
    ka, kb = lat.site(ya, xa), lat.site(yb, xb)
    link = leg_links(lat, ya, xa)[leg_a]
    kdim = lam[link].shape[0]
    MA = _scale_legs(B[ka], _outer_lambdas(lat, lam, ya, xa, leg_a))
    MB = _scale_legs(B[kb], _outer_lambdas(lat, lam, yb, xb, leg_b))
    XA, shape_a = _to_matrix(MA, leg_a)
    XB, shape_b = _to_matrix(MB, leg_b)
    if reduced:
        QA, RA = np.linalg.qr(XA, mode='reduced')
        QB, RB = np.linalg.qr(XB, mode='reduced')
    else:
        QA, RA = np.eye(XA.shape[0]), XA
        QB, RB = np.eye(XB.shape[0]), XB
    ra, rb = RA.shape[0], RB.shape[0]
    RA3 = RA.reshape(ra, 2, kdim)
    RB3 = RB.reshape(rb, 2, kdim)
    theta = np.einsum('ask,k,btk->asbt', RA3, lam[link], RB3)          # [a, s_A, b, s_B]
    theta = np.einsum('uvst,asbt->aubv', G, theta)                     # gate on (s_A, s_B)
    Theta = np.transpose(theta, (0, 1, 3, 2)).reshape(2 * ra, 2 * rb)   # rows (a, t_A), cols (t_B, b)
    U, lam_new, Vt = _truncated_svd(Theta, kdim)
    XA_new = (QA @ U.reshape(ra, 2 * kdim)).reshape(-1, 2 * kdim)       # [(outer), (t_A, i)]
    Vb = np.transpose(Vt.reshape(kdim, 2, rb), (2, 1, 0)).reshape(rb, 2 * kdim)
    XB_new = QB @ Vb                                                   # [(outer), (t_B, i)]
    A_new = _from_matrix(XA_new, shape_a, leg_a, kdim)
    B_new = _from_matrix(XB_new, shape_b, leg_b, kdim)
    B[ka] = _scale_legs(A_new, _outer_lambdas(lat, lam, ya, xa, leg_a, inverse=True))
    B[kb] = _scale_legs(B_new, _outer_lambdas(lat, lam, yb, xb, leg_b, inverse=True))
    lam[link] = lam_new


def nnn_paths(lat, y, x, anti):
    """(B_1, B_2, B_3) sites and the legs joining them for a diagonal of plaquette (y, x):
    ((y1, x1), leg of B_1 to B_2, (y2, x2), leg of B_2 to B_1, leg of B_2 to B_3, (y3, x3), leg of B_3 to B_2)."""
    if not anti:   # (y, x) - (y+1, x+1) through (y, x+1)
        return (y, x), 2, (y, x + 1), 0, 3, (y + 1, x + 1), 1
    return (y, x + 1), 0, (y, x), 2, 3, (y + 1, x), 1   # (y, x+1) - (y+1, x) through (y, x)


def plaquette_classes(lat):
    """Plaquettes (y, x) in four classes by (y mod 2, x mod 2); a class's plaquettes share no site."""
    out = [[], [], [], []]
    for y in range(lat.Ly - 1):
        for x in range(lat.Lx - 1):
            out[2 * (y % 2) + x % 2].append((y, x))
    return out


def su_nnn(B, lam, lat, y, x, anti, G, reduced=True):
    """Apply the gate G to the next-nearest-neighbour pair of plaquette (y, x) (App. A, Fig. 8), in place.

    reduced=False leaves out the QR reductions of B_1 and B_3 (the plain definition)."""
    (y1, x1), l1, (y2, x2), l21, l23, (y3, x3), l3 = nnn_paths(lat, y, x, anti)
    k1, k2, k3 = lat.site(y1, x1), lat.site(y2, x2), lat.site(y3, x3)
    link4 = leg_links(lat, y1, x1)[l1]
    link7 = leg_links(lat, y3, x3)[l3]
    D4, D7 = lam[link4].shape[0], lam[link7].shape[0]
    # (b) B_1, B_3 with their outer lambdas, QR-reduced
    X1, shape1 = _to_matrix(_scale_legs(B[k1], _outer_lambdas(lat, lam, y1, x1, l1)), l1)
    X3, shape3 = _to_matrix(_scale_legs(B[k3], _outer_lambdas(lat, lam, y3, x3, l3)), l3)
    if reduced:
        Q1, R1 = np.linalg.qr(X1, mode='reduced')
        Q3, R3 = np.linalg.qr(X3, mode='reduced')
    else:
        Q1, R1 = np.eye(X1.shape[0]), X1
        Q3, R3 = np.eye(X3.shape[0]), X3
    r1, r3 = R1.shape[0], R3.shape[0]
    R1 = R1.reshape(r1, 2, D4)
    R3 = R3.reshape(r3, 2, D7)
    # B_2 with its two outer lambdas as M2[k4, k7, o2, s2]
    links2 = leg_links(lat, y2, x2)
    outer2 = [q for q in range(4) if q not in (l21, l23)]
    M2 = _scale_legs(B[k2], [None if (q in (l21, l23) or links2[q] is None) else lam[links2[q]] for q in range(4)])
    M2 = np.transpose(M2, [1 + l21, 1 + l23] + [1 + q for q in outer2] + [0])
    o2_shape = M2.shape[2:4]
    M2 = M2.reshape(D4, D7, -1, 2)
    # (c) T_a[a1, s1, s2, o2, s3, a3] with lambda_4, lambda_7 and the gate on (s1, s3)
    Ta = np.einsum('aip,p,pqos,q,cjq->aisojc', R1, lam[link4], M2, lam[link7], R3, optimize=True)
    Ta = np.einsum('uvij,aisojc->ausovc', G, Ta, optimize=True)   # [a1, t1, s2, o2, t3, a3]
    n2 = Ta.shape[3]
    # (d) SVD rows (a1, t1): R~_1, lambda~_4, T_b
    U1, lam4, Tb = _truncated_svd(Ta.reshape(2 * r1, 2 * n2 * 2 * r3), D4)
    # (e) lambda~_4 T_b, rows (i4, s2, o2), columns (t3, a3): T_c, lambda~_7, R~_3
    Tb = (lam4[:, None] * Tb).reshape(D4 * 2 * n2, 2 * r3)
    Tc, lam7, V3 = _truncated_svd(Tb, D7)
    # (f) B~_1 = Q_1 R~_1 with the outer lambdas divided out
    X1n = (Q1 @ U1.reshape(r1, 2 * D4)).reshape(-1, 2 * D4)
    B[k1] = _scale_legs(_from_matrix(X1n, shape1, l1, D4), _outer_lambdas(lat, lam, y1, x1, l1, inverse=True))
    # (g) B~_2 = T_c / lambda~_4 with its outer lambdas divided out
    C = (Tc.reshape(D4, 2, n2, D7) * _pinv(lam4)[:, None, None, None])        # [i4, s2, o2, i7]
    C = C.reshape((D4, 2) + tuple(o2_shape) + (D7,))
    order = [0] * 5
    src = {1 + l21: 0, 0: 1, 1 + outer2[0]: 2, 1 + outer2[1]: 3, 1 + l23: 4}
    for t in range(5):
        order[t] = src[t]
    inv2 = [None if (q in (l21, l23) or links2[q] is None) else _pinv(lam[links2[q]]) for q in range(4)]
    B[k2] = _scale_legs(np.transpose(C, order), inv2)
    # (h) B~_3 = Q_3 R~_3 with the outer lambdas divided out
    Vb = np.transpose(V3.reshape(D7, 2, r3), (2, 1, 0)).reshape(r3, 2 * D7)
    B[k3] = _scale_legs(_from_matrix(Q3 @ Vb, shape3, l3, D7), _outer_lambdas(lat, lam, y3, x3, l3, inverse=True))
    lam[link4] = lam4
    lam[link7] = lam7


def su_step(B, lam, lat, dt, reduced=True):
    """One step over every nearest-neighbour link, class by class, then every coupled
    diagonal pair, plaquette class by class (a class's diagonals, then its
    anti-diagonals; an uncoupled diagonal is skipped); returns the mean relative
    change of the lambdas (App. A's convergence measure)."""
    G = heisenberg_gate(dt, lat.J1)
    old = [l.copy() for l in lam]
    for cls in link_classes(lat):
        for a, b, la, lb in cls:
            su_bond(B, lam, lat, a, b, la, lb, G, reduced)
    if lat.diagonals:
        gates = {False: heisenberg_gate(dt, lat.Jd), True: heisenberg_gate(dt, lat.Ja)}
        coupled = {False: lat.Jd != 0.0, True: lat.Ja != 0.0}
        for cls in plaquette_classes(lat):
            for anti in (False, True):
                if not coupled[anti]:
                    continue
                for (y, x) in cls:
                    su_nnn(B, lam, lat, y, x, anti, gates[anti], reduced)
    if not lam:
        return 0.0
    return float(np.mean([np.linalg.norm(n - o) / np.linalg.norm(o) for n, o in zip(lam, old)]))


def su_absorb(B, lam, lat):
    """The flat parameter vector with lambda^(1/2) absorbed into both tensors of every link."""
    out = []
    for y in range(lat.Ly):
        for x in range(lat.Lx):
            links = leg_links(lat, y, x)
            vecs = [None if l is None else np.sqrt(lam[l]) for l in links]
            out.append(_scale_legs(B[lat.site(y, x)], vecs).ravel())
    return np.concatenate(out)


def simple_update(T, lat, dt, steps):
    """`steps` steps from T (unit lambdas); returns (absorbed T, per-step changes, B, lambdas)."""
    B, lam = su_init(T, lat)
    changes = [su_step(B, lam, lat, dt) for _ in range(steps)]
    return su_absorb(B, lam, lat), changes, B, lam
