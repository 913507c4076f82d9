"""Values the paper prints (tests/golden/paper_parameters.json, each entry
citing its table or section) against the oracle's constants and the
workloads' materials (not GPU).

* The AT1/AT2 table fixes c_w (8/3, 2); the oracle's AT1 module and the AT2
  gate default Psi_crit = Gc / (c_w l) must use them.
* The penalty parameter's formula and tol_ir.
* The tension/shear material: E = 210 GPa, nu = 0.3 reproduce the printed
  mu; the printed lambda equals lambda + mu of those constants, a misprint
  (the benchmark's lambda is E nu / ((1 + nu)(1 - 2 nu))) that the test
  records rather than follows.
* The L-shape material: the workloads' E and nu reproduce the printed mu and
  lambda to the printed digits.
"""
import json
import os

import numpy as np

import workloads as W
from oracle import Oracle, at1

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "paper_parameters.json")))


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def test_at_constants():
    cw = GOLDEN["at_models"]
    assert np.isclose(at1.C_W, 8.0 / 3.0) and cw["AT1"]["c_w"] == "8/3"
    assert cw["AT2"]["c_w"] == "2"
    m = W.Material()
    # AT2 gate default: Gc / (2 l); AT1: Gc / ((8/3) l)
    o = Oracle(W.homogeneous_bar(), 1)
    assert np.isclose(o.psi_crit, m.Gc / (2.0 * m.l))
    assert np.isclose(at1.psi_crit(m.Gc, m.l), m.Gc / (8.0 / 3.0 * m.l))
    assert GOLDEN["gate"]["d_max"] == W.homogeneous_bar().d_gate


def test_penalty_parameter():
    pen = GOLDEN["penalty"]
    p = W.homogeneous_bar()
    assert p.tol_ir == pen["tol_ir"]
    Gc, l = 2.7, 0.01
    assert np.isclose(at1.penalty_gamma(Gc, l, pen["tol_ir"]), 27 * Gc / (64 * l * 0.01 ** 2))


def test_tension_shear_material():
    g = GOLDEN["tension_shear_material"]
    m = W.config_tension512().material
    lam, mu = lame(m.E, m.nu)
    assert np.isclose(mu, g["mu_MPa"], rtol=5e-4)
    assert np.isclose(lam + mu, g["lambda_MPa_printed"], rtol=5e-4)   # the misprint
    assert not np.isclose(lam, g["lambda_MPa_printed"], rtol=0.1)
    assert m.eta == g["eta"] and m.Gc == g["Gc_N_per_mm"]
    assert W.config_shear1024().material.Gc == g["Gc_N_per_mm"]


def test_lshape_material():
    g = GOLDEN["lshape_material"]
    m = W.config_lshape2048().material
    lam, mu = lame(m.E, m.nu)
    assert np.isclose(mu, g["mu_MPa"], rtol=1e-3)
    assert np.isclose(lam, g["lambda_MPa"], rtol=1e-3)
    assert m.eta == g["eta"] and m.Gc == g["Gc_N_per_mm"]
