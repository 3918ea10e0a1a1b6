"""The rounding floor behind the full-size parity bounds (tests/floors.py; oracle
only, CPU).

* With eps = 0 the perturbed evaluation is the oracle's evaluation itself.
* Without truncation (Dc at the exact rank) the floor is at rounding level:
  the floor measures how strongly the truncation's nearly degenerate cuts
  amplify one-ulp changes, not a defect of the perturbation.
* With truncation on a benchmark-like network it is orders of magnitude above
  rounding, and it grows in proportion to eps (first order).
* The stored floors are reproducible: a configuration of the 16x16, D=6, Dc=12
  gate recomputed with seed 1 gives the stored per-seed value bit for bit.
"""
import json
import os

import numpy as np

import floors
from oracle import lattice as olat
from oracle import vmc
from paper_1908_09359_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_zero_perturbation_is_the_oracle():
    lat = olat.Lattice(4, 4, 2, 2)
    T = W.random_tensors(4, 4, 2, seed=5)
    s = W.random_configs(4, 4, 1, seed=6)[0]
    a = vmc.eval_config(T, lat, s)
    b = floors.perturbed_eval(T, lat, s, 0.0, 1)
    assert a["e_loc"] == b["e_loc"] and a["log_abs_psi"] == b["log_abs_psi"]
    assert np.array_equal(a["ratios"], b["ratios"]) and np.array_equal(a["dlnpsi"], b["dlnpsi"])


def test_floor_is_rounding_level_without_truncation():
    lat = olat.Lattice(4, 4, 2, 4)  # Dc = 4 keeps the exact rank of every 4x4 D=2 boundary
    T = W.random_tensors(4, 4, 2, seed=7)
    s = W.random_configs(4, 4, 1, seed=8)[0]
    f = floors.floor(T, lat, s, floors.F64_UNIT, [1, 2, 3])
    assert f["e_site"] < 1e-13 and f["ratio"] < 1e-12


def test_floor_of_a_truncated_network_is_first_order_in_eps():
    lat = olat.Lattice(6, 6, 4, 4)  # D^2 = 16 > Dc: every interior boundary is truncated
    T = W.random_tensors(6, 6, 4, seed=9)
    s = W.random_configs(6, 6, 1, seed=10)[0]
    base = vmc.eval_config(T, lat, s)
    small = floors.floor(T, lat, s, 1e-12, [1], base)["ratio"]
    large = floors.floor(T, lat, s, 1e-10, [1], base)["ratio"]
    assert small > 1e-13  # far above what rounding alone would give at this size
    assert 30.0 < large / small < 300.0


def test_stored_gate_floor_is_reproducible():
    with open(os.path.join(GOLDEN, "c3_gate_16x16_D6_Dc12.json")) as f:
        gate = json.load(f)
    with open(os.path.join(GOLDEN, "c3_gate_floors.json")) as f:
        fl = json.load(f)
    w = gate["workload"]
    T = W.random_tensors(w["Ly"], w["Lx"], w["D"], seed=w["tensor_seed"], perturb=w["perturb"])
    lat = olat.Lattice(w["Ly"], w["Lx"], w["D"], w["Dc"], J1=w["J1"], J2=w["J2"])
    k = 24
    s = np.array([int(ch) for ch in gate["configs"][k]["spins"]], dtype=np.int8)
    base = vmc.eval_config(T, lat, s)
    dv = floors.deviations(floors.perturbed_eval(T, lat, s, floors.F64_UNIT, fl["seeds"]["f64"][0]), base,
                           lat.Ly * lat.Lx)
    stored = fl["configs"][k]["floor"]["f64_per_seed"][0]
    assert dv == stored
