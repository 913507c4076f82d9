"""Energy pins of the oracle on cracked panels (not GPU).

At a fixed phase field d the displacement solve minimises the stored energy
Pi(u; d) = sum_q w_q [g(d_q) Psi+(eps_q) + Psi-(eps_q)] (Section 2) over
the displacements that meet the Dirichlet data lambda * u_unit.  The
reaction of the loaded group is then the load derivative of the minimum,
F = dPi_min/dlambda, at any damage state: before the peak, while the crack
runs, and once the ligament is broken.  The test freezes the d of a
converged load step, re-minimises at lambda +- h and compares the central
difference with the step's reaction force.  This ties the assembled
internal force, the Newton solve and the reaction sum to the energy's
definition, with the split and the degradation in their cracked regime,
rather than to the oracle's own residual.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from oracle.constitutive import degradation


def stored_energy(orc, u, d):
    parts = orc.energies(u, d)
    g = degradation(orc.mesh.interp(d), orc.eta)
    return float(np.sum(orc.mesh.wdet * (g * parts["psi_plus"] + parts["psi_minus"])))


def min_energy(orc, d, lam, u0):
    u = u0.copy()
    u[orc.u_fixed] = lam * orc.u_unit[orc.u_fixed]
    R0 = np.linalg.norm(orc.residual_u(u, d)[orc.u_free])
    u, _, ok = orc.newton(u, d, R0 if R0 > 0 else 1.0)
    assert ok
    return stored_energy(orc, u, d)


def _check_history(p, scheme, check_steps, rtol):
    p = dataclasses.replace(p, tol_newton=1e-12)
    orc = Oracle(p, scheme)
    seen = 0
    for k, lam in enumerate(p.loads, start=1):
        st = orc.load_step(float(lam))
        assert st.converged
        if k not in check_steps:
            continue
        h = 1e-3 * float(lam)
        d, u = orc.d.copy(), orc.u.copy()
        dE = (min_energy(orc, d, lam + h, u) - min_energy(orc, d, lam - h, u)) / (2 * h)
        assert dE == pytest.approx(st.force, rel=rtol), (k, dE, st.force)
        seen += 1
    assert seen == len(check_steps)
    return orc


@pytest.mark.parametrize("scheme", [0, 1])
def test_reaction_is_energy_derivative_through_fracture(scheme):
    # 16^2 notched tension panel, l = 2h: peak near step 4, the ligament
    # breaks by step 7 (d ~ 0.97 across it, force down by ~20x)
    p = W.tension_panel(n=16, l=0.125, du=1e-3, steps=7)
    orc = _check_history(p, scheme, {2, 4, 6, 7}, rtol=1e-6)
    lig = orc.d[8 * 17 + 9:9 * 17]
    assert lig.min() > 0.9


def test_reaction_is_energy_derivative_spectral_shear():
    p = W.shear_panel(n=8, l=0.2, du=4e-3, steps=3)
    _check_history(p, 1, {1, 2, 3}, rtol=1e-6)
