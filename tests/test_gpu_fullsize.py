"""Parity at full size, evaluated by the GPU in one call through the C ABI and
compared output by output (sign, log|Psi|, E_loc, every pair ratio, 256 sampled
log-derivatives) with oracle values stored by tests/golden/make_floors.py:

* the benchmark's 16x16 Heisenberg lattice, D=8, Dc=16, 1024 configurations
  (the batch one timed sweep measures), eight of them stored; with the
  canonical compression and with the variational fit (two sweeps, four stored);
* the J1-J2 lattices of the uneven batch (J2 = 0.5, D=8, Dc=16) at 8x8 and
  12x12, four seeded configurations each;
* the 32x32 Heisenberg lattice, D=8, Dc=16, one seeded configuration.

Bounds.  These random networks truncate at nearly degenerate singular values
(sigma_17 / sigma_16 is 0.98 at the median cut), so every output depends on the
last bits of every compression input.  The golden file holds, per
configuration and output, the oracle's own floor (tests/floors.py): the largest
deviation of the oracle from itself over 16 evaluations with every
compression input multiplied by (1 + 2^-52 xi).  It spans 2.7e-10 to 3.9e-7 per
site in E_loc over the eight 16x16 configurations.  The float64 assertion is
deviation <= max(small-lattice bound, 3 x floor) for every output of every
configuration.  float32: the floor of float32 storage (site tensors,
compression inputs and compressed boundaries multiplied by (1 + 2^-24 xi),
eight seeds) reaches O(0.01-1) per site at 16x16, so no float32 contraction of
this workload has a meaningful per-configuration E_loc; the float32 run is
held to 3 x that floor and its deviations are printed.  At 32x32 the float64 floor
itself reaches 0.09 per site in E_loc and 1.6 in log|Psi| (the truncated
contraction of this random network is chaotic at that size): the comparison
there is held to 3 x that floor, and the sign is compared only where log|Psi|
stands clear of its floor.
"""
import json
import os

import numpy as np
import pytest

import gpu_helpers as H
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _case(name):
    with open(os.path.join(GOLDEN_DIR, name)) as f:
        doc = json.load(f)
    w = doc["workload"]
    T = W.random_tensors(w["Ly"], w["Lx"], w["D"], seed=w["tensor_seed"])
    cfgs = W.random_configs(w["Ly"], w["Lx"], w["n_configs"], seed=w["config_seed"])
    return doc, T, cfgs


def _gpu(prec_name, doc, T, cfgs):
    from paper_1908_09359_amd import binding as B
    w = doc["workload"]
    fit = w.get("compress_mode", "canonical") == "variational"
    print(f"{w['Ly']}x{w['Lx']} D={w['D']} Dc={w['Dc']} J2={w['J2']} "
          f"{'fit ' + str(w['fit_sweeps']) + ' sweeps' if fit else 'canonical'} {prec_name}: "
          f"{len(cfgs)} configurations in one vp_eval", flush=True)
    return H.gpu_eval(w["Ly"], w["Lx"], w["D"], w["Dc"], w["J2"], getattr(B, prec_name), T, cfgs,
                      compress=B.VP_COMPRESS_VARIATIONAL if fit else B.VP_COMPRESS_CANONICAL,
                      fit_sweeps=w.get("fit_sweeps", 0) if fit else 0)


def _deviations(g, k, row, idx, n_sites):
    ref_r = np.asarray(row["ratios"])
    dl = g["dlnpsi"][k][idx]
    return dict(
        e_site=abs(g["e_loc"][k] - row["e_loc"]) / n_sites,
        log_abs_psi=abs(g["log_abs_psi"][k] - row["log_abs_psi"]),
        ratio=float(np.max(np.abs(g["ratios"][k] - ref_r) / np.maximum(1.0, np.abs(ref_r)))),
        dlnpsi=float(np.max(np.abs(dl - np.asarray(row["dlnpsi_sample"])))) / max(1.0, row["dlnpsi_max_abs"]),
    )


F64_MIN = dict(e_site=1e-10, log_abs_psi=1e-10, ratio=1e-9, dlnpsi=1e-9)
F32_MIN = dict(e_site=1e-4, log_abs_psi=1e-4, ratio=1e-3, dlnpsi=1e-3)


def _check(prec_name, tag, minimum, name):
    doc, T, cfgs = _case(name)
    g = _gpu(prec_name, doc, T, cfgs)
    w = doc["workload"]
    n = w["Ly"] * w["Lx"]
    idx = np.asarray(doc["dlnpsi_index"])
    assert np.all(np.isfinite(g["e_loc"])) and np.all(np.isfinite(g["log_abs_psi"]))
    worst = 0.0
    for row in doc["configs"]:
        k = row["index"]
        dv = _deviations(g, k, row, idx, n)
        fl = row["floor"][tag]
        lim = {key: max(minimum[key] * (max(1.0, abs(row["log_abs_psi"])) if key == "log_abs_psi" else 1.0),
                        3.0 * fl[key]) for key in dv}
        ratio = {key: dv[key] / max(fl[key], 1e-300) for key in dv}
        worst = max(worst, max(dv[key] / lim[key] for key in dv))
        print(f"{tag} configuration {k}: " + ", ".join(
            f"{key} {dv[key]:.2e} (floor {fl[key]:.2e}, x{ratio[key]:.2f})" for key in dv), flush=True)
        # a sign is decided only where |Psi| stands clear of its own floor
        if tag == "f64" and fl["log_abs_psi"] < 1e-3:
            assert g["sign"][k] == row["sign"], k
        for key in dv:
            assert dv[key] <= lim[key], (k, key, dv[key], lim[key])
    print(f"{tag}: largest deviation / bound {worst:.3f}", flush=True)


@pytest.mark.parametrize("name", ["fullsize_16x16_D8_Dc16.json", "fullsize_16x16_D8_Dc16_fit2.json",
                                  "fullsize_8x8_D8_Dc16_J2.json", "fullsize_12x12_D8_Dc16_J2.json",
                                  "fullsize_32x32_D8_Dc16.json"])
def test_full_size_fp64_against_floors(name):
    _check("VP_FP64", "f64", F64_MIN, name)


@pytest.mark.parametrize("name", ["fullsize_16x16_D8_Dc16.json", "fullsize_16x16_D8_Dc16_fit2.json",
                                  "fullsize_8x8_D8_Dc16_J2.json", "fullsize_12x12_D8_Dc16_J2.json"])
def test_full_size_fp32_against_floors(name):
    _check("VP_FP32", "f32", F32_MIN, name)
