"""Write the fixed-configuration gate of the 16x16, D=6, Dc=12 workload.

    python tests/golden/make_c3_gate.py [--procs 7]

Inputs: tensors from the seeded generator (N(0,1)/D^2 plus a 1e-2 N(0,1)
perturbation, seed 1908); 64 configurations: 32 Neel-shuffled starts (Philox,
chains 0..31) and the states of 32 oracle float64 chains (chains 32..63,
seed 9359) after 16 sweeps.  Expected values: the oracle's log|Psi|, sign,
E_loc and 64 sampled entries of the compact log-derivative vector, per
configuration.  Only the oracle computes anything stored here.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

Ly, Lx, D, Dc = 16, 16, 6, 12
T_SEED, PERTURB, CH_SEED, BURN = 1908, 1e-2, 9359, 16
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_gate_16x16_D6_Dc12.json")


def _tensors():
    from paper_1908_09359_amd.workloads import random_tensors
    return random_tensors(Ly, Lx, D, seed=T_SEED, perturb=PERTURB)


def _burned(chain):
    from threadpoolctl import threadpool_limits
    from oracle import lattice as olat, vmc
    lat = olat.Lattice(Ly, Lx, D, Dc)
    ch = vmc.Chain(lat, olat.neel_shuffled(lat, CH_SEED, 0, chain), CH_SEED, 0, chain)
    with threadpool_limits(limits=1):
        vmc.run_chain(_tensors(), lat, ch, BURN, 0)
    return ch.spins.copy()


def _eval(cfg):
    from threadpoolctl import threadpool_limits
    from oracle import lattice as olat, vmc
    lat = olat.Lattice(Ly, Lx, D, Dc)
    with threadpool_limits(limits=1):
        return vmc.eval_config(_tensors(), lat, np.asarray(cfg, dtype=np.int8))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=7)
    args = ap.parse_args()
    from oracle import lattice as olat
    lat = olat.Lattice(Ly, Lx, D, Dc)
    cfgs = [olat.neel_shuffled(lat, CH_SEED, 0, c) for c in range(32)]
    with mp.get_context("spawn").Pool(args.procs) as pool:
        cfgs += pool.map(_burned, range(32, 64))
        res = pool.map(_eval, cfgs)
    nh = len(res[0]["dlnpsi"])
    idx = np.sort(np.random.default_rng(7).choice(nh, size=64, replace=False))
    rows = []
    for c, r in zip(cfgs, res):
        rows.append(dict(spins="".join(str(int(v)) for v in c), log_abs_psi=r["log_abs_psi"], sign=int(r["sign"]),
                         e_loc=r["e_loc"], dlnpsi_norm=float(np.linalg.norm(r["dlnpsi"])),
                         dlnpsi_sample=[float(r["dlnpsi"][i]) for i in idx]))
    doc = dict(workload=dict(Ly=Ly, Lx=Lx, D=D, Dc=Dc, J1=1.0, J2=0.0, tensor_seed=T_SEED, perturb=PERTURB,
                             chain_seed=CH_SEED, burn_in=BURN),
               dlnpsi_index=[int(i) for i in idx], configs=rows,
               source="oracle float64 (tests/golden/make_c3_gate.py)")
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
