"""Pins for the oracle's staggered loop (not GPU).

* Homogeneous bar on rollers (no notch): plane-strain uniaxial stress with
  E' = E/(1-nu^2); the strain is fixed by the Dirichlet data, so
  H = E' eps^2 / 2, d = l E' eps^2 / (Gc + l E' eps^2) and the reaction force
  is g(d) E' eps W exactly.  ST needs two u-solves per step; a gated S*
  predictor overshoots once and is switched off by a negative trial
  increment, so at most three.
* Per-step fixed point on a small notched panel (both residuals at their
  tolerances at acceptance), for every scheme.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle


def bar_closed_form(p, lam):
    m = p.material
    Ep = m.E / (1 - m.nu ** 2)
    eps = lam / p.ly
    d = m.l * Ep * eps ** 2 / (m.Gc + m.l * Ep * eps ** 2)
    F = ((1 - d) ** 2 + m.eta) * Ep * eps * p.lx
    return d, F


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_homogeneous_bar_history(scheme):
    # psi_crit = Gc/(2l) = 45 MPa is crossed at eps ~ 2e-2 with these values
    p = W.homogeneous_bar(nx=3, ny=4, lx=1.0, ly=1.0, du=5e-3, steps=6)
    o = Oracle(p, scheme)
    for lam in p.loads:
        st = o.load_step(float(lam))
        d_ref, F_ref = bar_closed_form(p, lam)
        np.testing.assert_allclose(o.d, d_ref, rtol=1e-9)
        assert np.isclose(st.force, F_ref, rtol=1e-9)
        psi = 0.5 * p.material.E / (1 - p.material.nu ** 2) * (lam / p.ly) ** 2
        gated = psi > p.material.Gc / (2 * p.material.l)
        if scheme == 0 or not gated:
            assert st.n_stag == 2, (scheme, lam, st)
        else:
            assert st.n_trial >= 1
            assert st.n_stag == 3, (scheme, lam, st)
        assert st.converged


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_fixed_point_at_acceptance(scheme):
    p = W.tension_panel(n=8, l=0.2, du=2e-3, steps=4)
    o = Oracle(p, scheme)
    for lam in p.loads:
        st = o.load_step(float(lam))
        assert st.converged
        assert st.r_stag <= p.tol_stag
        R = o.residual_u(o.u, o.d)[o.u_free]
        # Newton criterion relative to the lifted residual of the step
        assert np.linalg.norm(R) < 1e-6 * max(1.0, np.abs(o.residual_u(o.u, o.d)).max())
        # consistent-mass Q1 has no discrete maximum principle: allow a small
        # overshoot next to the Dirichlet d = 1 notch
        assert np.all(o.d[o.d_free] >= -1e-2) and np.all(o.d <= 1.01)


def test_state_roundtrip():
    p = W.tension_panel(n=6, l=0.2, du=2e-3, steps=2)
    o = Oracle(p, 1)
    o.run()
    u, d, H = o.get_state()
    o2 = Oracle(p, 1)
    o2.set_state(u, d, H)
    np.testing.assert_array_equal(o2.u, o.u)
    np.testing.assert_array_equal(o2.d, o.d)
    np.testing.assert_array_equal(o2.H, o.H)
