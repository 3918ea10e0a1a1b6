"""Write the expected solution of one stochastic-reconfiguration step at the 8x8,
D=4 size (Np = 21632 parameters, 20480 samples: 1024 chains x 20 sweeps).

    python tests/golden/make_sr_c2.py

Inputs: paper_1908_09359_amd.workloads.random_sr_inputs(8, 8, 4, 20480, seed
2020) (float32-rounded log-derivatives, as the float32 path stores them).
Expected: oracle.vmc.sr_step with shift 1e-4 (float64 Cholesky of S + shift I),
stored as 512 sampled entries of delta and of the gradient g, with max |delta|,
|delta|_2 and |g|_2.  Only the oracle computes anything stored here.
Output: sr_c2_8x8_D4.json.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

Ly, Lx, D, NS, SEED, SHIFT = 8, 8, 4, 20480, 2020, 1e-4


def main():
    from oracle import lattice as olat
    from oracle import vmc
    from paper_1908_09359_amd import workloads as W
    lat = olat.Lattice(Ly, Lx, D, 8)
    e, dl, spins = W.random_sr_inputs(Ly, Lx, D, NS, SEED)
    delta, g = vmc.sr_step(lat, e, dl, spins, SHIFT)
    idx = np.sort(np.random.default_rng(21).choice(lat.Np, size=512, replace=False))
    doc = dict(workload=dict(Ly=Ly, Lx=Lx, D=D, Np=lat.Np, n_samples=NS, seed=SEED, shift=SHIFT),
               index=[int(i) for i in idx], delta=[float(delta[i]) for i in idx], g=[float(g[i]) for i in idx],
               delta_max_abs=float(np.max(np.abs(delta))), delta_norm=float(np.linalg.norm(delta)),
               g_norm=float(np.linalg.norm(g)), source="oracle float64 (tests/golden/make_sr_c2.py)")
    out = os.path.join(HERE, "sr_c2_8x8_D4.json")
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
