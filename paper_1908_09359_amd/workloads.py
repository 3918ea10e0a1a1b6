"""Seeded synthetic inputs shared by tests, the benchmark and the smoke check.

Nothing here computes any part of the method: only random tensors of the
PEPS's shape and random spin configurations in the S^z_tot = 0 sector.

Stand-in for the paper's workloads (its optimised PEPS tensors are not
available): i.i.d. real Gaussian site tensors of standard deviation 1/D^2 on
an open-boundary square lattice, with boundary legs of dimension 1, and
configurations drawn uniformly from the S^z_tot = 0 sector.
"""
import numpy as np

# Named workloads: (Ly, Lx, D, Dc, J2, precision, chains)
WORKLOADS = {
    "4x4_D2_Dc4_fp64": dict(Ly=4, Lx=4, D=2, Dc=4, J2=0.0, prec="fp64", chains=1),
    "8x8_D4_Dc8_fp32": dict(Ly=8, Lx=8, D=4, Dc=8, J2=0.0, prec="fp32", chains=1024),
    "16x16_D6_Dc12": dict(Ly=16, Lx=16, D=6, Dc=12, J2=0.0, prec="fp32", chains=4096),
    "16x16_D8_Dc16": dict(Ly=16, Lx=16, D=8, Dc=16, J2=0.0, prec="fp32", chains=4096),
}


def num_params(Ly, Lx, D):
    n = 0
    for y in range(Ly):
        for x in range(Lx):
            n += 2 * (D if x > 0 else 1) * (D if y > 0 else 1) * (D if x < Lx - 1 else 1) * (D if y < Ly - 1 else 1)
    return n


def random_tensors(Ly, Lx, D, seed, scale=None, perturb=0.0):
    """Flat float64 parameter vector, i.i.d. N(0, scale^2), scale = 1/D^2 by default,
    plus perturb * xi' with xi' ~ N(0, 1) from a second seeded stream."""
    rng = np.random.default_rng(seed)
    if scale is None:
        scale = 1.0 / D ** 2
    n = num_params(Ly, Lx, D)
    T = rng.standard_normal(n) * scale
    if perturb:
        T = T + perturb * np.random.default_rng([seed, 1]).standard_normal(n)
    return T


def random_configs(Ly, Lx, n, seed):
    """n spin configurations (int8 0/1) with exactly half the spins 1."""
    N = Ly * Lx
    rng = np.random.default_rng(seed)
    base = np.zeros(N, dtype=np.int8)
    base[: N // 2] = 1
    return np.stack([rng.permutation(base) for _ in range(n)]) if n else np.zeros((0, N), np.int8)


def random_proposal_weights(seed, n=19105, scale=0.05, bias=-1.0):
    """float32 start of the plaquette proposal network: i.i.d. N(0, scale^2)
    parameters and output bias `bias` (a propensity near sigmoid(bias))."""
    w = (np.random.default_rng(seed).standard_normal(n) * scale).astype(np.float32)
    w[-1] = bias
    return w


def random_sr_inputs(Ly, Lx, D, n_samples, seed):
    """Seeded stand-ins for one stochastic-reconfiguration step's inputs: E_loc
    ~ N(-10, 3^2), compact log-derivatives ~ N(0, 1) rounded to float32 (the
    float32 path stores them so) and returned as float64 [n_samples][Np/2], and
    uniform S^z = 0 configurations."""
    rng = np.random.default_rng(seed)
    nh = num_params(Ly, Lx, D) // 2
    e = rng.standard_normal(n_samples) * 3.0 - 10.0
    dl = rng.standard_normal((n_samples, nh), dtype=np.float32).astype(np.float64)
    spins = random_configs(Ly, Lx, n_samples, seed=seed + 1)
    return e, dl, spins


def pad_tensors(T_small, Ly, Lx, D_small, D_big, noise=0.0, seed=0):
    """The flat parameters of a bond-D_small PEPS written into the layout of
    bond D_big (entries with a virtual index >= D_small are zero, so the state
    is the same), plus noise * N(0, 1) on every entry of the D_big layout."""
    def dims(D, y, x):
        return ((D if x > 0 else 1), (D if y > 0 else 1), (D if x < Lx - 1 else 1), (D if y < Ly - 1 else 1))
    out = []
    o = 0
    for y in range(Ly):
        for x in range(Lx):
            ds, db = dims(D_small, y, x), dims(D_big, y, x)
            n = int(np.prod(ds))
            blk = np.zeros((2,) + db)
            blk[:, :ds[0], :ds[1], :ds[2], :ds[3]] = np.asarray(T_small[o:o + 2 * n]).reshape((2,) + ds)
            o += 2 * n
            out.append(blk.ravel())
    T = np.concatenate(out)
    if noise:
        T = T + noise * np.random.default_rng(seed).standard_normal(T.shape)
    return T
