"""Conditioning of the full-size evaluation (CPU only, oracle only; not collected by pytest).

Multiplies every input tensor of every boundary compression of the oracle by
(1 + eps xi), xi ~ N(0, 1) i.i.d. from a seeded stream, and reports how far
E_loc, log|Psi| and the pair ratios of one configuration move.  With eps at the
float64 unit (2^-52) this is the floor below which no float64 implementation of
the truncation can be expected to agree; with eps at the float32 unit (2^-24)
the floor of a float32 one.

    python tests/conditioning_probe.py [eps] [seed] [gate index]

Defaults: the 16x16 Heisenberg lattice, D=8, Dc=16, tensors and configurations
drawn as in tests/test_gpu_fullsize.py, eps = 2^-52.  With a gate index, the
configuration of that index in tests/golden/c3_gate_16x16_D6_Dc12.json on its
workload (16x16, D=6, Dc=12) instead.
"""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import lattice as olat  # noqa: E402
from oracle import peps, vmc  # noqa: E402
from paper_1908_09359_amd import workloads as W  # noqa: E402


def main():
    eps = float(sys.argv[1]) if len(sys.argv) > 1 else 2.0 ** -52
    seed = int(sys.argv[2]) if len(sys.argv) > 2 else 1
    if len(sys.argv) > 3:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "c3_gate_16x16_D6_Dc12.json")) as f:
            doc = json.load(f)
        w = doc["workload"]
        LY, LX, D, DC = w["Ly"], w["Lx"], w["D"], w["Dc"]
        T = W.random_tensors(LY, LX, D, seed=w["tensor_seed"], perturb=w["perturb"])
        cfgs = np.array([[int(ch) for ch in r["spins"]] for r in doc["configs"]], dtype=np.int8)
        k = int(sys.argv[3])
        lat = olat.Lattice(LY, LX, D, DC, J1=w["J1"], J2=w["J2"])
    else:
        LY, LX, D, DC, NCH = 16, 16, 8, 16, 1024
        T = W.random_tensors(LY, LX, D, seed=1908)
        cfgs = W.random_configs(LY, LX, NCH, seed=9359)
        k = int(np.random.default_rng(59).integers(NCH))
        lat = olat.Lattice(LY, LX, D, DC)
    base = vmc.eval_config(T, lat, cfgs[k])
    exact = peps.compress
    rng = np.random.default_rng(seed)

    def perturbed(B, Dc):
        return exact([b * (1.0 + eps * rng.standard_normal(b.shape)) for b in B], Dc)

    peps.compress = perturbed
    vmc.compress = perturbed
    try:
        p = vmc.eval_config(T, lat, cfgs[k])
    finally:
        peps.compress = exact
        vmc.compress = exact
    N = LY * LX
    dr = np.max(np.abs(p["ratios"] - base["ratios"]) / np.maximum(1.0, np.abs(base["ratios"])))
    print(f"configuration {k}, eps {eps:.3e}: dE/site {abs(p['e_loc'] - base['e_loc']) / N:.3e}, "
          f"dlog|Psi| {abs(p['log_abs_psi'] - base['log_abs_psi']):.3e}, ratios {dr:.3e}")


if __name__ == "__main__":
    main()
