"""Pins of the oracle's simple update (App. A; oracle/simple_update.py), CPU only.

* The gate is the matrix exponential of J S_A.S_B (scipy's expm of the
  Pauli-matrix form).
* The QR-reduced bond update equals the same update written out on the full
  two-site tensor (no QR), in the lambdas and in every amplitude of the
  absorbed state (the bond gauges of the two may differ).
* Without truncation on open chains (1 x 4 and 4 x 1, D = 4: every cut has rank
  at most 4) a step is exact: the absorbed state is the dense product of the
  same gates, in the same order, applied to the start, up to normalisation.
* On one link the evolution converges to the singlet, E = -3/4.
* On a 2 x 4 lattice (D = 2, truncated): the energy of the absorbed state falls
  well below the start's and stays above the exact ground energy (variational),
  and the convergence measure decreases; the same with J2 = 0.5.
* Next-nearest-neighbour terms (Fig. 8's three-site update): the QR-reduced
  update equals the full one; from a product state where no truncation
  occurs, a step is the dense product of the same gates in the same order;
  with J1 = 0 the two diagonals of a 2 x 2 plaquette decouple and the
  evolution converges to two singlets, E = -3/2.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import bruteforce as bf
from oracle import lattice as olat
from oracle import simple_update as su
from paper_1908_09359_amd import workloads as W


def _bond_hamiltonian():
    sx = np.array([[0.0, 1.0], [1.0, 0.0]]) / 2
    sy = np.array([[0.0, -1.0j], [1.0j, 0.0]]) / 2
    sz = np.array([[1.0, 0.0], [0.0, -1.0]]) / 2
    return np.real(np.kron(sx, sx) + np.kron(sy, sy) + np.kron(sz, sz))


def _dense_state(T, Ly, Lx, D):
    """All 2^N amplitudes, configuration index = sum s_k 2^(N-1-k)."""
    N = Ly * Lx
    cfgs = np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.int8)
    return bf.amplitudes(T, Ly, Lx, D, cfgs)


def _apply_gate(psi, N, i, j, G4):
    """The 4 x 4 gate on sites i < j of the dense state."""
    t = psi.reshape([2] * N)
    t = np.moveaxis(t, [i, j], [0, 1])
    shp = t.shape
    t = (G4 @ t.reshape(4, -1)).reshape(shp)
    return np.moveaxis(t, [0, 1], [i, j]).ravel()


def _hpsi(psi, Ly, Lx, J2=0.0, J1=1.0, tri=False):
    """H psi: J1 on nearest-neighbour pairs, J2 on both diagonals of every plaquette
    (tri: the triangular lattice, J1 on the diagonal (y,x)-(y+1,x+1) alone)."""
    N = Ly * Lx
    h = _bond_hamiltonian()
    out = np.zeros_like(psi)
    for y in range(Ly):
        for x in range(Lx):
            k = y * Lx + x
            if x < Lx - 1 and J1:
                out += J1 * _apply_gate(psi, N, k, k + 1, h)
            if y < Ly - 1 and J1:
                out += J1 * _apply_gate(psi, N, k, k + Lx, h)
            if tri and x < Lx - 1 and y < Ly - 1:
                out += J1 * _apply_gate(psi, N, k, k + Lx + 1, h)
            if J2 and x < Lx - 1 and y < Ly - 1:
                out += J2 * _apply_gate(psi, N, k, k + Lx + 1, h)
                out += J2 * _apply_gate(psi, N, k + 1, k + Lx, h)
    return out


def _energy(psi, Ly, Lx, J2=0.0, J1=1.0, tri=False):
    return float(psi @ _hpsi(psi, Ly, Lx, J2, J1, tri) / (psi @ psi))


@pytest.mark.parametrize("dt,J", [(0.01, 1.0), (0.3, 1.0), (0.2, 0.5)])
def test_gate_is_the_exponential_of_the_bond_term(dt, J):
    G = su.heisenberg_gate(dt, J).reshape(4, 4)
    assert np.allclose(G, scipy.linalg.expm(-dt * J * _bond_hamiltonian()), atol=1e-15, rtol=1e-14)


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_reduced_update_equals_full_two_site_update(J2):
    Ly, Lx, D = 3, 4, 3
    lat = olat.Lattice(Ly, Lx, D, 16, J2=J2)
    T = W.random_tensors(Ly, Lx, D, seed=91)
    Br, lr = su.su_init(T, lat)
    Bf, lf = su.su_init(T, lat)
    for _ in range(3):
        cr = su.su_step(Br, lr, lat, 0.05, reduced=True)
        cf = su.su_step(Bf, lf, lat, 0.05, reduced=False)
        assert abs(cr - cf) <= 1e-10 * max(1.0, abs(cf))
    for a, b in zip(lr, lf):
        assert np.allclose(a, b, atol=1e-11)
    cfgs = np.array(bf.sz0_configs(Ly * Lx))
    pr = bf.amplitudes(su.su_absorb(Br, lr, lat), Ly, Lx, D, cfgs)
    pf = bf.amplitudes(su.su_absorb(Bf, lf, lat), Ly, Lx, D, cfgs)
    assert np.max(np.abs(pr - pf)) <= 1e-10 * np.max(np.abs(pf))


@pytest.mark.parametrize("Ly,Lx", [(1, 4), (4, 1)])
def test_untruncated_chain_is_the_dense_trotter_product(Ly, Lx):
    D, dt, steps = 4, 0.1, 2
    N = Ly * Lx
    lat = olat.Lattice(Ly, Lx, D, 16)
    T = W.random_tensors(Ly, Lx, D, seed=17)
    psi = _dense_state(T, Ly, Lx, D)
    G4 = su.heisenberg_gate(dt, 1.0).reshape(4, 4)
    for _ in range(steps):
        for cls in su.link_classes(lat):
            for (ya, xa), (yb, xb), _, _ in cls:
                psi = _apply_gate(psi, N, ya * Lx + xa, yb * Lx + xb, G4)
    Tsu, changes, _, _ = su.simple_update(T, lat, dt, steps)
    phi = _dense_state(Tsu, Ly, Lx, D)
    cos = abs(phi @ psi) / (np.linalg.norm(phi) * np.linalg.norm(psi))
    assert cos >= 1.0 - 1e-12
    assert len(changes) == steps and all(c > 0 for c in changes)


def test_one_link_converges_to_the_singlet():
    lat = olat.Lattice(1, 2, 2, 4)
    T = W.random_tensors(1, 2, 2, seed=3)
    Tsu, changes, _, lam = su.simple_update(T, lat, 0.2, 120)
    psi = _dense_state(Tsu, 1, 2, 2)
    assert abs(_energy(psi, 1, 2) + 0.75) <= 1e-9
    # the singlet has Schmidt rank 2 with equal weights
    assert np.allclose(lam[0], [np.sqrt(0.5), np.sqrt(0.5)], atol=1e-9)
    assert changes[-1] <= 1e-9


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_truncated_evolution_lowers_the_energy_variationally(J2):
    Ly, Lx, D = 2, 4, 2
    lat = olat.Lattice(Ly, Lx, D, 16, J2=J2)
    T = W.random_tensors(Ly, Lx, D, seed=23)
    e0 = _energy(_dense_state(T, Ly, Lx, D), Ly, Lx, J2)
    Tsu, changes, _, _ = su.simple_update(T, lat, 0.1, 40)
    e1 = _energy(_dense_state(Tsu, Ly, Lx, D), Ly, Lx, J2)
    # exact ground energy of the 2 x 4 open lattice by dense diagonalisation
    N = Ly * Lx
    H = np.zeros((2 ** N, 2 ** N))
    for k in range(2 ** N):
        e = np.zeros(2 ** N)
        e[k] = 1.0
        H[:, k] = _hpsi(e, Ly, Lx, J2)
    e_exact = np.linalg.eigvalsh(H)[0]
    assert e1 >= e_exact - 1e-12
    assert e1 < e0 - 1.0 and e1 < 0.9 * e_exact
    assert changes[-1] < 0.1 * changes[0]


def test_sector_energy_of_the_brute_force_helper():
    """bruteforce.sector_energy (used by the GPU tests) against the dense energy of
    the same state projected onto S^z = 0 (H conserves S^z)."""
    Ly, Lx, D = 2, 4, 2
    T = W.random_tensors(Ly, Lx, D, seed=29)
    psi = _dense_state(T, Ly, Lx, D)
    cfgs = np.array(list(itertools.product([0, 1], repeat=Ly * Lx)), dtype=np.int8)
    keep = cfgs.sum(axis=1) == Ly * Lx // 2
    psi0 = np.where(keep, psi, 0.0)
    assert abs(bf.sector_energy(psi[keep], cfgs[keep], Ly, Lx) - _energy(psi0, Ly, Lx)) <= 1e-12


def _product_state(lat, seed):
    """A random product state written into the bond-D layout (every virtual index 0)."""
    rng = np.random.default_rng(seed)
    T = np.zeros(lat.Np)
    for y in range(lat.Ly):
        for x in range(lat.Lx):
            o = lat.offsets[lat.site(y, x)]
            n = int(np.prod(lat.dims(y, x)))
            T[o], T[o + n] = rng.normal(size=2)
    return T


@pytest.mark.parametrize("Ly,Lx,D,J1,J2,tol", [(2, 2, 4, 0.0, 1.0, 1e-13), (2, 3, 8, 1.0, 0.5, 1e-10)])
def test_untruncated_nnn_step_is_the_dense_gate_product(Ly, Lx, D, J1, J2, tol):
    """From a product state the ranks stay within D for one step (the residue at
    2x3 is the 1e-6 singular-value floor): the state is the dense product of the
    step's gates, nearest-neighbour classes first, then the plaquette classes'
    diagonals and anti-diagonals."""
    N = Ly * Lx
    dt = 0.1
    lat = olat.Lattice(Ly, Lx, D, 16, J1=J1, J2=J2)
    T = _product_state(lat, 3)
    psi = _dense_state(T, Ly, Lx, D)
    G1 = su.heisenberg_gate(dt, J1).reshape(4, 4)
    G2 = su.heisenberg_gate(dt, J2).reshape(4, 4)
    for cls in su.link_classes(lat):
        for (ya, xa), (yb, xb), _, _ in cls:
            psi = _apply_gate(psi, N, ya * Lx + xa, yb * Lx + xb, G1)
    for cls in su.plaquette_classes(lat):
        for anti in (False, True):
            for (y, x) in cls:
                (y1, x1), _, _, _, _, (y3, x3), _ = su.nnn_paths(lat, y, x, anti)
                i, j = sorted((y1 * Lx + x1, y3 * Lx + x3))
                psi = _apply_gate(psi, N, i, j, G2)
    Tsu, _, _, _ = su.simple_update(T, lat, dt, 1)
    phi = _dense_state(Tsu, Ly, Lx, D)
    assert abs(phi @ psi) / (np.linalg.norm(phi) * np.linalg.norm(psi)) >= 1.0 - tol


def test_decoupled_diagonals_converge_to_two_singlets():
    lat = olat.Lattice(2, 2, 4, 16, J1=0.0, J2=1.0)
    T = W.random_tensors(2, 2, 4, seed=8)
    Tsu, changes, _, _ = su.simple_update(T, lat, 0.2, 150)
    assert abs(_energy(_dense_state(Tsu, 2, 2, 4), 2, 2, J2=1.0, J1=0.0) + 1.5) <= 1e-10
    assert changes[-1] <= 1e-9



def test_triangular_untruncated_step_is_the_dense_gate_product():
    """The triangular lattice (J1 on the diagonal (y,x)-(y+1,x+1), Sec. III.B):
    from a product state on 2 x 2 at D = 8 (no truncation; the residue is the
    1e-6 singular-value floor) a step is the dense product of the
    nearest-neighbour gates and then the diagonal's gate (three-site update
    through the corner (y,x+1)); the anti-diagonal is not touched."""
    Ly = Lx = 2
    N, D, dt = 4, 8, 0.1
    lat = olat.Lattice(Ly, Lx, D, 16, geometry="triangular")
    T = _product_state(lat, 5)
    psi = _dense_state(T, Ly, Lx, D)
    G1 = su.heisenberg_gate(dt, 1.0).reshape(4, 4)
    for cls in su.link_classes(lat):
        for (ya, xa), (yb, xb), _, _ in cls:
            psi = _apply_gate(psi, N, ya * Lx + xa, yb * Lx + xb, G1)
    psi = _apply_gate(psi, N, 0, 3, G1)
    Tsu, _, _, _ = su.simple_update(T, lat, dt, 1)
    phi = _dense_state(Tsu, Ly, Lx, D)
    assert abs(phi @ psi) / (np.linalg.norm(phi) * np.linalg.norm(psi)) >= 1.0 - 1e-10


def test_triangular_evolution_is_variational():
    """2 x 4 triangular lattice, D = 2 (truncated): the absorbed state's energy
    falls well below the start's (to within 15% of the ground energy; the
    frustrated lattice is further from a D = 2 state than the square one) and
    stays above the exact ground energy."""
    Ly, Lx, D = 2, 4, 2
    lat = olat.Lattice(Ly, Lx, D, 16, geometry="triangular")
    T = W.random_tensors(Ly, Lx, D, seed=31)
    e0 = _energy(_dense_state(T, Ly, Lx, D), Ly, Lx, tri=True)
    Tsu, changes, _, _ = su.simple_update(T, lat, 0.1, 40)
    e1 = _energy(_dense_state(Tsu, Ly, Lx, D), Ly, Lx, tri=True)
    N = Ly * Lx
    H = np.zeros((2 ** N, 2 ** N))
    for k in range(2 ** N):
        e = np.zeros(2 ** N)
        e[k] = 1.0
        H[:, k] = _hpsi(e, Ly, Lx, tri=True)
    e_exact = np.linalg.eigvalsh(H)[0]
    assert e1 >= e_exact - 1e-12
    assert e1 < e0 - 1.0 and e1 < 0.85 * e_exact
    assert changes[-1] < 0.1 * changes[0]
