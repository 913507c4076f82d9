"""Pins for the oracle's AT1 model with penalised irreversibility (not GPU).

Homogeneous bar on rollers: the strain is fixed by the displacement data
(eps_yy = lambda / ly, sigma_xx = 0, plane strain), so Psi+ = E' eps^2 / 2
with E' = E / (1 - nu^2), uniform.  A uniform d annihilates the Laplacian,
and F_d = 0 reduces to the scalar equation (Section 2, eq_evolution_equation
with w(d) = d, c_w = 8/3)

    -2 (1 - d) Psi+ + Gc / (c_w l) + gamma min(d - d_prev, 0) = 0,
    gamma = 27 Gc / (64 l tol_ir^2),

whose solution is the loading branch d = 1 - Gc / (2 c_w l Psi+) where that
is >= d_prev, and the penalised branch
d = (2 Psi+ - Gc/(c_w l) + gamma d_prev) / (2 Psi+ + gamma) otherwise.  The
reaction force is g(d) E' eps W.  The constants here come from the paper's
formulas, not from the oracle's module.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from oracle import at1


def bar_at1_history(p):
    """(d, F) per load step of the AT1 bar from the scalar equation."""
    m = p.material
    Ep = m.E / (1 - m.nu ** 2)
    cw = 8.0 / 3.0
    gamma = 27.0 * m.Gc / (64.0 * m.l * p.tol_ir ** 2)
    d_prev, out = 0.0, []
    for lam in p.loads:
        eps = lam / p.ly
        psi = 0.5 * Ep * eps ** 2
        d = 1.0 - m.Gc / (2.0 * cw * m.l * psi) if psi > 0 else -np.inf
        if d < d_prev:
            d = (2 * psi - m.Gc / (cw * m.l) + gamma * d_prev) / (2 * psi + gamma)
        F = ((1 - d) ** 2 + m.eta) * Ep * eps * p.lx
        out.append((d, F))
        d_prev = d
    return out


def at1_bar(loads, **kw):
    p = W.homogeneous_bar(nx=3, ny=4, lx=1.0, ly=1.0, du=5e-3, steps=len(loads))
    return dataclasses.replace(p, loads=np.asarray(loads, float), phase_model=1, **kw)


LOADING = [0.005, 0.01, 0.015, 0.02, 0.025, 0.03]
UNLOADING = [0.01, 0.02, 0.03, 0.025, 0.015, 0.005, 0.02, 0.035]


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
@pytest.mark.parametrize("loads", [LOADING, UNLOADING], ids=["loading", "unloading"])
def test_at1_bar_closed_form(scheme, loads):
    p = at1_bar(loads)
    ref = bar_at1_history(p)
    o = Oracle(p, scheme)
    for lam, (d_ref, F_ref) in zip(p.loads, ref):
        st = o.load_step(float(lam))
        assert st.converged, (scheme, lam, st)
        # the loop stops at ||F_d|| <= tol_stag ||sum 2 Psi+ N||
        np.testing.assert_allclose(o.d, d_ref, rtol=0, atol=1e-9 + 2 * p.tol_stag)
        assert np.isclose(st.force, F_ref, rtol=1e-4)
        if scheme == 0:
            assert st.n_stag == 2


def test_at1_bar_branches_are_exercised():
    """The pins above cover the elastic stage (d slightly below 0 by the
    penalty), the loading branch, and unloading held by the penalty, and
    the violation of irreversibility stays below tol_ir."""
    p = at1_bar(UNLOADING)
    ref = bar_at1_history(p)
    ds = [d for d, _ in ref]
    assert ds[0] < 0                                  # elastic: penalised branch
    assert ds[2] > ds[1] > 0.1                        # loading branch
    drops = [ds[k - 1] - ds[k] for k in range(1, len(ds)) if ds[k] < ds[k - 1]]
    assert drops and max(drops) < p.tol_ir            # unloading held by the penalty
    assert max(drops) > 0


def test_at1_constants():
    """gamma and Psi_crit of the oracle's module against the paper's formulas."""
    Gc, l = 2.7, 0.03
    assert np.isclose(at1.penalty_gamma(Gc, l, 0.01), 27 * Gc / (64 * l * 1e-4))
    assert np.isclose(at1.psi_crit(Gc, l), 3 * Gc / (8 * l))


@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_at1_notched_panel_fixed_point(scheme):
    """At acceptance F_d meets the staggered tolerance, and the semismooth
    solve for the final energy ends at F_d = 0 to rounding with the penalty
    acting on part of the panel (the notch's neighbourhood pulls d below its
    committed value where Psi+ is small).  The penalty bounds the decrease
    only through gamma; no nodal bound holds near the notch, where the
    consistent-mass profile undershoots."""
    p = dataclasses.replace(W.tension_panel(n=10, l=0.2, du=2e-3, steps=5), phase_model=1)
    o = Oracle(p, scheme)
    for lam in p.loads:
        d_before = o.d.copy()
        st = o.load_step(float(lam))
        assert st.converged
        assert st.r_stag <= p.tol_stag
    parts = o.energies(o.u, o.d)
    psi = parts["psi_plus"]
    d, it, ok = at1.solve(o.mesh, psi, o.d, d_before, o.Gc, o.l, o.gamma, o.d_free)
    assert ok
    R = at1.residual(o.mesh, psi, d, d_before, o.Gc, o.l, o.gamma)[o.d_free]
    assert np.linalg.norm(R) <= 1e-9 * at1.driving_scale(o.mesh, psi, o.d_free)
    chi = at1.active(o.mesh, d, d_before)
    assert 0 < chi.sum() < chi.size


def test_at1_optimal_profile():
    """With Psi+ = 0 and d = 1 held on one edge, F_d = 0 is
    (2 Gc l / c_w) d'' = Gc / (c_w l) where d > 0: the classical AT1 profile
    d = (1 - x / (2l))^2 on x <= 2l, and d held near 0 by the penalty beyond
    (d_{n-1} = 0 there).  This pins the factor between the Laplacian and the
    AT1 source, which a uniform field never sees.  Q1 on a 1-element strip,
    h = l / 20."""
    from oracle.fem import Mesh
    l, Gc = 0.1, 2.7
    nx, lx = 100, 0.5
    mesh = Mesh(nx, 1, lx, lx / nx)
    x = np.tile(np.linspace(0.0, lx, nx + 1), 2)
    free = x > 0
    d0 = np.where(free, 0.0, 1.0)
    psi = np.zeros((mesh.conn.shape[0], 4))
    gamma = at1.penalty_gamma(Gc, l, 0.01)
    d, it, ok = at1.solve(mesh, psi, d0, d0.copy(), Gc, l, gamma, free)
    assert ok
    inside = x <= 2 * l - 2 * lx / nx
    np.testing.assert_allclose(d[inside], (1 - x[inside] / (2 * l)) ** 2, atol=2e-3)
    beyond = x >= 2 * l + 2 * lx / nx
    assert np.abs(d[beyond]).max() < 1e-3
