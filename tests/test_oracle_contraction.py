"""Pins of the oracle's contraction layer (``oracle.peps``, ``oracle.vmc.eval_config``).

* Exact regime (Dc at or above the exact boundary rank): amplitudes, every pair
  ratio, E_loc and every log-derivative against an independent dense
  contraction (``tests/bruteforce.py``).  Log-derivatives use the fact that
  Psi is linear in each tensor element, so Psi(T + e_p) - Psi(T) is exactly
  dPsi/dT_p.
* Compression: against the dense definition of the canonical SVD compression
  (successive Eckart-Young truncation across the cuts n-1, ..., 1 of the full
  state vector) and against exactness when Dc reaches the rank.
* Truncated regime (no external truth): gauge invariance, Psi_row = L.R at
  every cut, the Euler relation sum t*G = 1, and direct recontraction of
  every ratio network.
* Closed forms: D=1 product states and the two-site singlet.
"""
import numpy as np
import pytest

import bruteforce as bf
from oracle import peps, vmc
from oracle.lattice import Lattice, bonds, compact_offsets, site_tensor


def _rand_T(lat, seed, scale=None):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(lat.Np) * (scale if scale is not None else 1.0 / lat.D ** 2)


def _configs(lat, n, seed):
    rng = np.random.default_rng(seed)
    base = np.array([1] * (lat.N // 2) + [0] * (lat.N - lat.N // 2), dtype=np.int8)
    return np.array([rng.permutation(base) for _ in range(n)])


# ---------------------------------------------------------------- exact regime

def test_amplitudes_exact_4x4():
    lat = Lattice(4, 4, 2, 4)
    T = _rand_T(lat, 1)
    cf = _configs(lat, 30, 2)
    ref = bf.amplitudes(T, 4, 4, 2, cf)
    for c, r in zip(cf, ref):
        sg, lp = peps.amplitude(T, lat, c)
        assert sg == np.sign(r)
        assert abs(lp - np.log(abs(r))) < 1e-11


@pytest.mark.parametrize("shape,J2", [((4, 4), 0.0), ((3, 4), 0.5)])
def test_eval_exact_eloc_ratios(shape, J2):
    Ly, Lx = shape
    lat = Lattice(Ly, Lx, 2, 16, J2=J2)
    T = _rand_T(lat, 3)
    cf = _configs(lat, 12, 4)
    e_ref, psi = bf.local_energies(T, Ly, Lx, 2, 1.0, J2, cf)
    bl = bf.bonds(Ly, Lx, 1.0, J2)
    assert [(p[0] * Lx + p[1], q[0] * Lx + q[1], J) for p, q, J in bonds(lat)] == bl
    for c, er, pr in zip(cf, e_ref, psi):
        out = vmc.eval_config(T, lat, c)
        assert abs(out['e_loc'] - er) < 1e-10 * max(1.0, abs(er))
        assert out['sign'] == np.sign(pr)
        assert abs(out['log_abs_psi'] - np.log(abs(pr))) < 1e-11
        for b, (i, j, _) in enumerate(bl):
            if c[i] != c[j]:
                f = c.copy()
                f[i], f[j] = c[j], c[i]
                rho = bf.amplitudes(T, Ly, Lx, 2, f[None])[0] / pr
                assert abs(out['ratios'][b] - rho) < 1e-9 * max(1.0, abs(rho))
            else:
                assert out['ratios'][b] == 0.0


@pytest.mark.parametrize("shape", [(4, 4), (3, 4)])
def test_eval_exact_eloc_ratios_triangular(shape):
    """The triangular lattice (J1 on the diagonal (y,x)-(y+1,x+1)): E_loc and the
    coupled pairs' ratios against brute force; the uncoupled anti-diagonal's
    ratio slot holds 0."""
    Ly, Lx = shape
    lat = Lattice(Ly, Lx, 2, 16, geometry="triangular")
    T = _rand_T(lat, 5)
    cf = _configs(lat, 12, 6)
    e_ref, psi = bf.local_energies(T, Ly, Lx, 2, 1.0, 0.0, cf, triangular=True)
    bl = bf.bonds(Ly, Lx, 1.0, 0.0, triangular=True)
    assert [(p[0] * Lx + p[1], q[0] * Lx + q[1], J) for p, q, J in bonds(lat)] == bl
    for c, er, pr in zip(cf, e_ref, psi):
        out = vmc.eval_config(T, lat, c)
        assert abs(out['e_loc'] - er) < 1e-10 * max(1.0, abs(er))
        for b, (i, j, J) in enumerate(bl):
            if c[i] != c[j] and J != 0.0:
                f = c.copy()
                f[i], f[j] = c[j], c[i]
                rho = bf.amplitudes(T, Ly, Lx, 2, f[None])[0] / pr
                assert abs(out['ratios'][b] - rho) < 1e-9 * max(1.0, abs(rho))
            else:
                assert out['ratios'][b] == 0.0


@pytest.mark.parametrize("shape", [(4, 4), (3, 4), (4, 3)])
def test_eval_exact_triangular_j2(shape):
    """The triangular lattice with J2 (the other diagonal and the knight bonds; the
    three-row ones through the transposed lattice): E_loc and every ratio against
    brute force in the exact regime."""
    Ly, Lx = shape
    J2 = 0.3
    lat = Lattice(Ly, Lx, 2, 16, J2=J2, geometry="triangular")
    T = _rand_T(lat, 9)
    cf = _configs(lat, 10, 8)
    e_ref, psi = bf.local_energies(T, Ly, Lx, 2, 1.0, J2, cf, triangular=True)
    bl = bf.bonds(Ly, Lx, 1.0, J2, triangular=True)
    assert [(p[0] * Lx + p[1], q[0] * Lx + q[1], J) for p, q, J in bonds(lat)] == bl
    for c, er, pr in zip(cf, e_ref, psi):
        out = vmc.eval_config(T, lat, c)
        assert abs(out['e_loc'] - er) < 1e-10 * max(1.0, abs(er))
        for b, (i, j, J) in enumerate(bl):
            if c[i] != c[j] and J != 0.0:
                f = c.copy()
                f[i], f[j] = c[j], c[i]
                rho = bf.amplitudes(T, Ly, Lx, 2, f[None])[0] / pr
                assert abs(out['ratios'][b] - rho) < 1e-9 * max(1.0, abs(rho))
            else:
                assert out['ratios'][b] == 0.0


def test_dlnpsi_exact_linearity():
    lat = Lattice(3, 4, 2, 16)
    T = _rand_T(lat, 5)
    coffs = compact_offsets(lat)
    for c in _configs(lat, 3, 6):
        out = vmc.eval_config(T, lat, c)
        psi0 = bf.amplitudes(T, 3, 4, 2, c[None])[0]
        for k in range(lat.N):
            y, x = divmod(k, lat.Lx)
            n = int(np.prod(lat.dims(y, x)))
            base = lat.offsets[k] + int(c[k]) * n
            Ts = np.repeat(T[None], n, axis=0)
            Ts[np.arange(n), base + np.arange(n)] += 1.0
            psis = np.array([bf.amplitudes(Ts[i], 3, 4, 2, c[None])[0] for i in range(n)])
            G_ref = (psis - psi0) / psi0
            G = out['dlnpsi'][coffs[k]:coffs[k] + n]
            assert np.allclose(G, G_ref, rtol=1e-8, atol=1e-9 * np.max(np.abs(G_ref)))


# ---------------------------------------------------------------- compression

def _dense(mps):
    v = mps[0]
    for A in mps[1:]:
        v = np.tensordot(v, A, axes=(v.ndim - 1, 0))
    return v.reshape(-1)


def _dense_truncation(v, dims, Dc):
    """Successive best rank-Dc approximations across cuts n-1, ..., 1 (Eckart-Young)."""
    n = len(dims)
    for cut in range(n - 1, 0, -1):
        left = int(np.prod(dims[:cut]))
        M = v.reshape(left, -1)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        k = min(Dc, len(S))
        v = ((U[:, :k] * S[:k]) @ Vt[:k]).reshape(-1)
    return v


@pytest.mark.parametrize("seed,Dc", [(0, 1), (1, 2), (2, 3), (3, 5)])
def test_compress_matches_dense_definition(seed, Dc):
    rng = np.random.default_rng(seed)
    p = [2, 3, 2, 3, 2]
    bd = [1, 4, 6, 5, 3, 1]
    mps = [rng.standard_normal((bd[j], p[j], bd[j + 1])) for j in range(5)]
    v = _dense(mps)
    out, lognu = peps.compress(mps, Dc)
    assert all(o.shape[0] <= Dc and o.shape[2] <= Dc for o in out)
    ref = _dense_truncation(v, p, Dc)
    got = _dense(out) * np.exp(lognu)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.linalg.norm(ref))
    assert abs(np.linalg.norm(_dense(out)) - 1.0) < 1e-13


def test_compress_exact_at_full_rank():
    rng = np.random.default_rng(9)
    mps = [rng.standard_normal(s) for s in [(1, 2, 3), (3, 2, 4), (4, 2, 3), (3, 2, 1)]]
    out, lognu = peps.compress(mps, 64)
    assert np.allclose(_dense(out) * np.exp(lognu), _dense(mps), rtol=1e-12, atol=1e-14)


def test_compress_zero_state_raises():
    mps = [np.zeros((1, 2, 2)), np.ones((2, 2, 1))]
    with pytest.raises(peps.ZeroAmplitude):
        peps.compress(mps, 2)


def test_dc_convergence_to_exact():
    lat = Lattice(4, 4, 2, 1)
    T = _rand_T(lat, 11)
    c = _configs(lat, 1, 12)[0]
    ex = bf.amplitudes(T, 4, 4, 2, c[None])[0]
    errs = []
    for Dc in (1, 2, 3, 4):
        l2 = Lattice(4, 4, 2, Dc)
        sg, lp = peps.amplitude(T, l2, c)
        errs.append(abs(sg * np.exp(lp) - ex) / abs(ex))
    assert errs[-1] < 1e-12
    assert errs[0] > 1e-6


# ---------------------------------------------------------------- truncated regime

def _gauge_horizontal(T, lat, y, x, G):
    """t_{y,x}[.,.,r,.] <- t G ; t_{y,x+1}[l,...] <- G^-1 t (exact network invariance)."""
    T = T.copy()
    Gi = np.linalg.inv(G)
    for s in (0, 1):
        a = site_tensor(T, lat, y, x, s)
        a[...] = np.einsum('lurd,rk->lukd', a.copy(), G)
        b = site_tensor(T, lat, y, x + 1, s)
        b[...] = np.einsum('kl,lurd->kurd', Gi, b.copy())
    return T


def _gauge_vertical(T, lat, y, x, G):
    T = T.copy()
    Gi = np.linalg.inv(G)
    for s in (0, 1):
        a = site_tensor(T, lat, y, x, s)
        a[...] = np.einsum('lurd,dk->lurk', a.copy(), G)
        b = site_tensor(T, lat, y + 1, x, s)
        b[...] = np.einsum('ku,lurd->lkrd', Gi, b.copy())
    return T


def test_truncated_gauge_properties():
    lat = Lattice(4, 4, 2, 2)
    T = _rand_T(lat, 21)
    c = _configs(lat, 1, 22)[0]
    ref = peps.amplitude(T, lat, c)
    rng = np.random.default_rng(23)
    Gh = rng.standard_normal((2, 2)) + 2 * np.eye(2)
    Th = _gauge_horizontal(T, lat, 1, 1, Gh)
    got = peps.amplitude(Th, lat, c)
    assert got[0] == ref[0] and abs(got[1] - ref[1]) < 1e-12
    O, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    To = _gauge_vertical(T, lat, 1, 2, O)
    got = peps.amplitude(To, lat, c)
    assert got[0] == ref[0] and abs(got[1] - ref[1]) < 1e-12
    # A general (non-orthogonal) vertical gauge changes the truncated amplitude:
    # the test above is sensitive to the boundary truncation.
    Tg = _gauge_vertical(T, lat, 1, 2, Gh)
    got = peps.amplitude(Tg, lat, c)
    assert abs(got[1] - ref[1]) > 1e-6


def test_truncated_row_invariants_and_euler():
    lat = Lattice(4, 5, 3, 3)
    T = _rand_T(lat, 31)
    c = _configs(lat, 1, 32)[0]
    U, _ = peps.upper_boundaries(T, lat, c)
    Dn = {lat.Ly: peps.trivial_mps(lat.Lx)}
    for y in range(lat.Ly - 1, 0, -1):
        Dn[y], _ = peps.lower_boundary(Dn[y + 1], T, lat, c, y)
    for y in range(lat.Ly):
        row = peps.row_tensors(T, lat, c, y)
        Lenv, Renv = peps.row3_envs(U[y], row, Dn[y + 1])
        vals = [float(np.tensordot(Lenv[x], Renv[x], axes=3)) for x in range(lat.Lx + 1)]
        assert np.allclose(vals, vals[0], rtol=1e-12)
        assert abs(peps.row3_value(U[y], row, Dn[y + 1]) - vals[0]) < 1e-12 * abs(vals[0])
    out = vmc.eval_config(T, lat, c)
    coffs = compact_offsets(lat)
    for k in range(lat.N):
        y, x = divmod(k, lat.Lx)
        t = site_tensor(T, lat, y, x, c[k]).ravel()
        g = out['dlnpsi'][coffs[k]:coffs[k] + t.size]
        assert abs(float(t @ g) - 1.0) < 1e-11


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_truncated_ratios_by_direct_recontraction(J2):
    lat = Lattice(4, 4, 3, 3, J2=J2)
    T = _rand_T(lat, 41)
    c = _configs(lat, 1, 42)[0]
    out = vmc.eval_config(T, lat, c)
    U, _ = peps.upper_boundaries(T, lat, c)
    Dn = {lat.Ly: peps.trivial_mps(lat.Lx)}
    for y in range(lat.Ly - 1, 0, -1):
        Dn[y], _ = peps.lower_boundary(Dn[y + 1], T, lat, c, y)
    s = c.reshape(lat.Ly, lat.Lx)
    for b, (p, q, J) in enumerate(bonds(lat)):
        if s[p] == s[q]:
            continue
        y = min(p[0], q[0])
        if p[0] == q[0]:
            num = peps.row3_value(U[y], peps.row_tensors(T, lat, c, y, flips=(p, q)), Dn[y + 1])
            den = peps.row3_value(U[y], peps.row_tensors(T, lat, c, y), Dn[y + 1])
        else:
            num = peps.row4_value(U[y], peps.row_tensors(T, lat, c, y, flips=(p, q)),
                                  peps.row_tensors(T, lat, c, y + 1, flips=(p, q)), Dn[y + 2])
            den = peps.row4_value(U[y], peps.row_tensors(T, lat, c, y),
                                  peps.row_tensors(T, lat, c, y + 1), Dn[y + 2])
        assert abs(out['ratios'][b] - num / den) < 1e-11 * max(1.0, abs(num / den))


# ---------------------------------------------------------------- closed forms

def _product_T(lat, amp0, amp1):
    """D=1 product state: T_k[s] = amp_s(k) (scalars)."""
    T = np.zeros(lat.Np)
    for k in range(lat.N):
        T[lat.offsets[k]] = amp0(k)
        T[lat.offsets[k] + 1] = amp1(k)
    return T


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_closed_form_uniform_product(J2):
    lat = Lattice(4, 4, 1, 2, J2=J2)
    T = _product_T(lat, lambda k: 1.0, lambda k: 1.0)
    nb = len(bonds(lat))
    for c in _configs(lat, 5, 51):
        out = vmc.eval_config(T, lat, c)
        expect = 0.25 * (24 * 1.0 + (nb - 24) * J2)
        assert abs(out['e_loc'] - expect) < 1e-13
        assert abs(out['log_abs_psi']) < 1e-13


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_closed_form_neel_product(J2):
    lat = Lattice(4, 4, 1, 2, J2=J2)
    neel = lambda k: (k // 4 + k % 4) % 2
    T = _product_T(lat, lambda k: 1.0 if neel(k) == 0 else 0.0, lambda k: 1.0 if neel(k) == 1 else 0.0)
    c = np.array([neel(k) for k in range(16)], dtype=np.int8)
    out = vmc.eval_config(T, lat, c)
    nd = len(bonds(lat)) - 24
    assert abs(out['e_loc'] - (-0.25 * 24 + 0.25 * J2 * nd)) < 1e-13
    # per site: -0.375 (Heisenberg), -0.234375 (J2 = 0.5)
    assert abs(out['e_loc'] / 16 - (-0.375 if J2 == 0 else -0.234375)) < 1e-13


def test_closed_form_singlet():
    lat = Lattice(1, 2, 2, 2)
    T = np.zeros(lat.Np)
    # site 0: T0[s][l=0,u=0,r=k,d=0] = delta(k, s); site 1: T1[1][k=0] = 1, T1[0][k=1] = -1
    site_tensor(T, lat, 0, 0, 0)[0, 0, 0, 0] = 1.0
    site_tensor(T, lat, 0, 0, 1)[0, 0, 1, 0] = 1.0
    site_tensor(T, lat, 0, 1, 1)[0, 0, 0, 0] = 1.0
    site_tensor(T, lat, 0, 1, 0)[1, 0, 0, 0] = -1.0
    for c in ([0, 1], [1, 0]):
        out = vmc.eval_config(T, lat, np.array(c, dtype=np.int8))
        assert abs(out['e_loc'] - (-0.75)) < 1e-14
