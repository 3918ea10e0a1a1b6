"""Write the expected values and rounding floors of the full-size parity cases.

    python tests/golden/make_floors.py fullsize [--procs 8]
    python tests/golden/make_floors.py c3 [--procs 8]
    python tests/golden/make_floors.py c4_8 | c4_12 | c5 [--procs 8]

``fullsize``: the 16x16 Heisenberg workload at D=8, Dc=16 (tensors seed 1908,
1024 configurations uniform in the S^z = 0 sector, seed 9359 -- the batch of
the benchmark's measured sweep).  For 8 configurations drawn by seed the oracle's
log|Psi|, sign, E_loc, every pair ratio and 256 sampled log-derivatives, and
the floors of tests/floors.py at the float64 unit (16 seeds, compression
inputs perturbed) and at the float32 unit (8 seeds, the float32-storage model:
site tensors, compression inputs and outputs perturbed).  Output: fullsize_16x16_D8_Dc16.json.

``c3``: the same floors for the 64 configurations of the 16x16, D=6, Dc=12
fixed-configuration gate (c3_gate_16x16_D6_Dc12.json).  Output:
c3_gate_floors.json.

``c4_8``, ``c4_12``: the J1-J2 workloads of the uneven batch (J2 = 0.5, D=8,
Dc=16) at 8x8 and 12x12, four seeded configurations each (tensors seed 1908,
configurations seed 9359), stored like ``fullsize`` (fullsize_8x8_D8_Dc16_J2.json,
fullsize_12x12_D8_Dc16_J2.json).  ``c5``: the 32x32 Heisenberg lattice at D=8,
Dc=16, one seeded configuration, float64 floor over 6 seeds
(fullsize_32x32_D8_Dc16.json).  ``fit2``: the 16x16 benchmark workload with the
variational boundary fit (two sweeps) instead of the canonical compression,
four of the benchmark batch's configurations, float64 floor over 6 seeds
(fullsize_16x16_D8_Dc16_fit2.json).

Only the oracle computes anything stored here.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

F64_SEEDS = list(range(1, 17))
F32_SEEDS = list(range(1, 9))


# name: (Ly, Lx, D, Dc, J2, configurations generated, configurations stored, float64 seeds, float32 seeds, file)
STORED = {
    "fullsize": (16, 16, 8, 16, 0.0, 1024, 8, F64_SEEDS, F32_SEEDS, "fullsize_16x16_D8_Dc16.json"),
    "c4_8": (8, 8, 8, 16, 0.5, 4, 4, F64_SEEDS, F32_SEEDS, "fullsize_8x8_D8_Dc16_J2.json"),
    "c4_12": (12, 12, 8, 16, 0.5, 4, 4, F64_SEEDS, F32_SEEDS, "fullsize_12x12_D8_Dc16_J2.json"),
    "c5": (32, 32, 8, 16, 0.0, 1, 1, F64_SEEDS[:6], [], "fullsize_32x32_D8_Dc16.json"),
    "fit2": (16, 16, 8, 16, 0.0, 1024, 4, F64_SEEDS[:6], F32_SEEDS, "fullsize_16x16_D8_Dc16_fit2.json"),
}
# workloads evaluated with the variational fit (App. B) instead of the canonical compression: sweeps
FIT_SWEEPS = {"fit2": 2}


def _workload(name):
    from oracle import lattice as olat
    from paper_1908_09359_amd import workloads as W
    if name in STORED:
        Ly, Lx, D, Dc, J2, n = STORED[name][:6]
        T = W.random_tensors(Ly, Lx, D, seed=1908)
        cfgs = W.random_configs(Ly, Lx, n, seed=9359)
        if name in FIT_SWEEPS:
            return olat.Lattice(Ly, Lx, D, Dc, J2=J2, compress_mode="variational",
                                fit_sweeps=FIT_SWEEPS[name]), T, cfgs
        return olat.Lattice(Ly, Lx, D, Dc, J2=J2), T, cfgs
    with open(os.path.join(HERE, "c3_gate_16x16_D6_Dc12.json")) as f:
        doc = json.load(f)
    w = doc["workload"]
    T = W.random_tensors(w["Ly"], w["Lx"], w["D"], seed=w["tensor_seed"], perturb=w["perturb"])
    cfgs = np.array([[int(ch) for ch in r["spins"]] for r in doc["configs"]], dtype=np.int8)
    return olat.Lattice(w["Ly"], w["Lx"], w["D"], w["Dc"], J1=w["J1"], J2=w["J2"]), T, cfgs


def _job(args):
    name, k, eps, seed = args
    from threadpoolctl import threadpool_limits
    from oracle import vmc
    import floors
    lat, T, cfgs = _workload(name)
    with threadpool_limits(limits=1):
        if eps == 0.0:
            r = vmc.eval_config(T, lat, cfgs[k])
        else:
            # float64: compression inputs; float32: the float32-storage model
            r = floors.perturbed_eval(T, lat, cfgs[k], eps, seed, storage=eps == floors.F32_UNIT)
    return (k, eps, seed), dict(sign=r["sign"], log_abs_psi=r["log_abs_psi"], e_loc=r["e_loc"],
                                ratios=r["ratios"], dlnpsi=r["dlnpsi"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c3"] + list(STORED))
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--f32-only", action="store_true",
                    help="recompute only the float32 floors and replace them in the existing output")
    args = ap.parse_args()
    import floors
    lat, T, cfgs = _workload(args.which)
    stored = args.which in STORED
    f64_seeds, f32_seeds = (STORED[args.which][7], STORED[args.which][8]) if stored else (F64_SEEDS, F32_SEEDS)
    if stored and STORED[args.which][6] < len(cfgs):
        idx = sorted(int(i) for i in np.random.default_rng(59).choice(len(cfgs), size=STORED[args.which][6],
                                                                      replace=False))
    else:
        idx = list(range(len(cfgs)))
    jobs = [(args.which, k, 0.0, 0) for k in idx]
    if not args.f32_only:
        jobs += [(args.which, k, floors.F64_UNIT, s) for k in idx for s in f64_seeds]
    jobs += [(args.which, k, floors.F32_UNIT, s) for k in idx for s in f32_seeds]
    with mp.get_context("spawn").Pool(args.procs) as pool:
        res = dict(pool.imap_unordered(_job, jobs))
    n = lat.Ly * lat.Lx
    rows = []
    nh = len(res[(idx[0], 0.0, 0)]["dlnpsi"])
    sample = np.sort(np.random.default_rng(7).choice(nh, size=256, replace=False))
    for k in idx:
        base = res[(k, 0.0, 0)]
        fl = {}
        for tag, eps, seeds in (("f64", floors.F64_UNIT, f64_seeds), ("f32", floors.F32_UNIT, f32_seeds)):
            if not seeds or (args.f32_only and tag == "f64"):
                continue
            per = [floors.deviations(res[(k, eps, s)], base, n) for s in seeds]
            fl[tag] = {key: max(p[key] for p in per) for key in per[0]}
            fl[tag + "_per_seed"] = per
        row = dict(index=k, floor=fl)
        if stored:
            row.update(log_abs_psi=base["log_abs_psi"], sign=int(base["sign"]), e_loc=base["e_loc"],
                       ratios=[float(v) for v in base["ratios"]],
                       dlnpsi_max_abs=float(np.max(np.abs(base["dlnpsi"]))),
                       dlnpsi_sample=[float(base["dlnpsi"][i]) for i in sample])
        rows.append(row)
    doc = dict(workload=dict(Ly=lat.Ly, Lx=lat.Lx, D=lat.D, Dc=lat.Dc, J1=lat.J1, J2=lat.J2,
                             compress_mode=lat.compress_mode, fit_sweeps=lat.fit_sweeps),
               eps=dict(f64=floors.F64_UNIT, f32=floors.F32_UNIT), seeds=dict(f64=f64_seeds, f32=f32_seeds),
               configs=rows, source="oracle float64 (tests/golden/make_floors.py)")
    if stored:
        doc["workload"].update(tensor_seed=1908, config_seed=9359, n_configs=len(cfgs))
        doc["dlnpsi_index"] = [int(i) for i in sample]
        out = os.path.join(HERE, STORED[args.which][9])
    else:
        out = os.path.join(HERE, "c3_gate_floors.json")
    if args.f32_only:
        with open(out) as f:
            old = json.load(f)
        for o, r in zip(old["configs"], rows):
            assert o["index"] == r["index"]
            for key in ("f32", "f32_per_seed"):
                if key in r["floor"]:
                    o["floor"][key] = r["floor"][key]
        old["f32_model"] = "storage"
        doc = old
    else:
        doc["f32_model"] = "storage"
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
