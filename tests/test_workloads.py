"""The seeded input generators (paper_1908_09359_amd/workloads.py) hold none of
the method's arithmetic; these checks pin what they promise."""
import numpy as np

import bruteforce as bf
from oracle import lattice as olat
from paper_1908_09359_amd import workloads as W


def test_random_configs_in_sector():
    c = W.random_configs(6, 4, 50, seed=3)
    assert c.shape == (50, 24) and np.all(c.sum(axis=1) == 12) and set(np.unique(c)) <= {0, 1}


def test_pad_tensors_keeps_the_state():
    """Zero-padding a bond-2 PEPS into the bond-3 layout leaves every amplitude
    unchanged (brute-force contraction); the noise is the only difference."""
    Ly, Lx = 3, 4
    T2 = W.random_tensors(Ly, Lx, 2, seed=5)
    T3 = W.pad_tensors(T2, Ly, Lx, 2, 3)
    assert len(T3) == olat.Lattice(Ly, Lx, 3, 9).Np
    cfgs = W.random_configs(Ly, Lx, 6, seed=6)
    assert np.allclose(bf.amplitudes(T3, Ly, Lx, 3, cfgs), bf.amplitudes(T2, Ly, Lx, 2, cfgs), rtol=1e-13, atol=0)
    Tn = W.pad_tensors(T2, Ly, Lx, 2, 3, noise=1e-3, seed=7)
    d = Tn - T3
    assert 0.5e-3 < d.std() < 2e-3


def test_sr_inputs_are_float32_representable():
    e, dl, spins = W.random_sr_inputs(2, 4, 2, 10, seed=8)
    assert dl.dtype == np.float64 and np.array_equal(dl, dl.astype(np.float32).astype(np.float64))
    assert e.shape == (10,) and spins.shape == (10, 8)
