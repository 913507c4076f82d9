"""Pins for the literal readings of the trial solve in the oracle (not GPU).

Homogeneous bar on rollers (no notch, no phase Dirichlet data): the strain is
fixed by the displacement data, eps_yy = lambda / ly and eps_xx from
sigma_xx = 0 (plane strain), independent of a uniform d.  Every quadrature
point then carries the same H, and the phase residual of a uniform d is
R_d = (c d - 2H) M 1, since the Laplacian annihilates constants.  The trial
block K_dd + K~ acts on a uniform increment as (c - c_S(d)) M, so the trial
increment is the scalar step Dd = -(c d - 2H) / a(d) with
  c     = Gc / l + 2H                         (AT2 mass coefficient),
  c_S   = 8 (1 - d)^2 / g(d) * Psi_S          (Section 3.4, eq. dpsi: the
                                               coupling block is -4 N (1-d)^2/g
                                               times 2 Psi_S),
  a(d)  = c - c_S(d), or max(c - c_S, theta c) with the floor,
and Psi_S = Psi_vol (S1), Psi_dev (S2) or Psi+ (S3) of the volumetric-
deviatoric split.  With trial_update = 1 each gated staggered iteration is
d <- d + Dd, an ungated one the standard solve d <- 2H / c, and the
staggered residual is |c d - 2H| / (2H).  This scalar map fixes N_stag and
d of every load step; the energies below come from the split's definitions,
not from the oracle's constitutive module.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from oracle import assembly as asm


def bar_energies(p, lam):
    """(Psi_vol, Psi_dev) of the bar at load lam from the split's definitions."""
    m = p.material
    lam_l = m.E * m.nu / ((1 + m.nu) * (1 - 2 * m.nu))
    mu = m.E / (2 * (1 + m.nu))
    K = lam_l + 2 * mu / 3
    eyy = lam / p.ly
    exx = -m.nu / (1 - m.nu) * eyy        # sigma_xx = 0 in plane strain
    tr = exx + eyy
    dev = np.array([exx - tr / 3, eyy - tr / 3, -tr / 3])
    psi_vol = 0.5 * K * max(tr, 0.0) ** 2
    psi_dev = mu * float(dev @ dev)
    return psi_vol, psi_dev


def scalar_map_history(p, scheme, floor, trial_only=True, slopes=False):
    """(n_stag, d) per load step of the trial-only scheme on the bar; with
    slopes, also the factor by which the step's final d amplifies an error
    of d: the product of |1 - c/a| (the map's derivative) over the trial
    iterations since the last standard solve, which lands on 2H/c whatever
    d was before it."""
    m = p.material
    psi_crit = m.Gc / (2 * m.l)
    d, H_prev, out, amp = 0.0, 0.0, [], 1.0
    for lam in p.loads:
        pv, pd = bar_energies(p, float(lam))
        psi = pv + pd
        H = max(H_prev, psi)
        c = m.Gc / m.l + 2 * H
        psi_s = {1: pv, 2: pd, 3: psi}.get(scheme, 0.0)
        n, r = 1, abs(c * d - 2 * H) / (2 * H)
        while r > p.tol_stag and n < p.max_stag:
            gated = scheme != 0 and psi > psi_crit and psi > H_prev and d < p.d_gate
            if gated and trial_only:
                om2 = (1 - d) ** 2
                a = c - 8 * om2 / (om2 + m.eta) * psi_s
                if floor:
                    a = max(a, p.trial_floor * c)
                d = d - (c * d - 2 * H) / a
                amp *= abs(1 - c / a)
            else:
                d = 2 * H / c
                amp = 1.0
            n += 1
            r = abs(c * d - 2 * H) / (2 * H)
        out.append((n, d, amp) if slopes else (n, d))
        H_prev = H
    return out


def bar(max_stag=6, **kw):
    p = W.homogeneous_bar(nx=3, ny=4, lx=1.0, ly=1.0, du=5e-3, steps=6)
    return dataclasses.replace(p, max_stag=max_stag, **kw)


@pytest.mark.parametrize("operator", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_trial_only_bar_follows_scalar_map(scheme, operator):
    p = bar(trial_operator=operator, trial_update=1)
    ref = scalar_map_history(p, scheme, floor=(operator == 0))
    o = Oracle(p, scheme)
    gated_steps = 0
    for lam, (n_ref, d_ref) in zip(p.loads, ref):
        st = o.load_step(float(lam))
        assert st.n_stag == n_ref, (scheme, operator, lam, st.n_stag, n_ref)
        np.testing.assert_allclose(o.d, d_ref, rtol=1e-8, atol=1e-12)
        gated_steps += st.n_trial > 0
    assert gated_steps >= 2


def test_scalar_map_separates_the_readings():
    """The pins above are not vacuous: on the bar the floored S2 and S3 maps
    converge within the cap while the unfloored ones run away (their slope
    c - c_S is negative once gated); S1's slope stays above theta c, so its
    floor never acts and both readings coincide there."""
    p = bar(trial_operator=0, trial_update=1)
    for scheme in (2, 3):
        fl = scalar_map_history(p, scheme, floor=True)
        lit = scalar_map_history(p, scheme, floor=False)
        assert all(n < p.max_stag for n, _ in fl)
        assert lit[-1][0] == p.max_stag and lit[-1][1] < 0
    assert scalar_map_history(p, 1, True) == scalar_map_history(p, 1, False)


def test_trial_only_without_gating_is_st():
    """Below psi_crit nothing is gated: the trial-only scheme is ST."""
    p = dataclasses.replace(W.tension_panel(n=8, l=0.2, du=2e-4, steps=3), trial_update=1,
                            trial_operator=1)
    a, b = Oracle(p, 3), Oracle(p, 0)
    for lam in p.loads:
        sa, sb = a.load_step(float(lam)), b.load_step(float(lam))
        assert sa.gated_max == 0 and sa.n_stag == sb.n_stag
        np.testing.assert_allclose(a.d, b.d, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("scheme", [1, 3])
def test_predict_correct_with_literal_operator_reaches_bar_fixed_point(scheme):
    """Trial -> predict -> correct with the unfloored block still stops at the
    bar's closed-form fixed point d = 2H/c (up to the staggered tolerance)."""
    p = bar(max_stag=500, trial_operator=1, trial_update=0)
    o = Oracle(p, scheme)
    m = p.material
    for lam in p.loads:
        st = o.load_step(float(lam))
        assert st.converged
        pv, pd = bar_energies(p, float(lam))
        H = pv + pd
        d_ref = 2 * H / (m.Gc / m.l + 2 * H)
        np.testing.assert_allclose(o.d, d_ref, rtol=2 * p.tol_stag)


def test_unfloored_coefficient_is_indefinite_where_floor_acts():
    """On a gated notched panel the S3 trial coefficient goes negative where
    the floor would act, and the direct solve satisfies the indefinite system."""
    # the first four steps converge and already floor (step 4: 685 points)
    p = W.tension_panel(n=12, l=0.1, du=1e-3, steps=4)
    p = dataclasses.replace(p, trial_operator=1)
    o = Oracle(p, 3)
    seen = False
    for lam in p.loads:
        st = o.load_step(float(lam))
        seen |= st.floor_hits > 0
    assert seen
    parts = o.energies(o.u, o.d)
    H = o.H
    dq = o.mesh.interp(o.d)
    gate = dq < p.d_gate
    c = asm.at2_coefficient(H, o.Gc, o.l)
    from oracle.constitutive import coupling_coefficient, scheme_part
    cS = coupling_coefficient(dq, o.eta, scheme_part(parts, 3))
    ct, hits = asm.trial_coefficient(c, cS, gate, p.trial_floor, floor=False)
    cf, hits_f = asm.trial_coefficient(c, cS, gate, p.trial_floor, floor=True)
    assert hits == hits_f
    below = gate & (c - cS < p.trial_floor * c)
    np.testing.assert_array_equal(ct[below], (c - cS)[below])
    np.testing.assert_array_equal(cf[below], (p.trial_floor * c)[below])
    np.testing.assert_array_equal(ct[~below], cf[~below])
    dd, _ = o.trial_increment(o.d, H, gate, scheme_part(parts, 3))
    A = asm.phase_matrix(o.mesh, ct, o.Gc, o.l)
    K, b = o.phase_system(H)
    f = o.d_free
    res = (A @ dd + (K @ o.d - b))[f]
    assert np.linalg.norm(res) <= 1e-8 * max(np.linalg.norm((K @ o.d - b)[f]), 1e-300)


@pytest.mark.parametrize("theta", [0.1, 0.3])
@pytest.mark.parametrize("scheme", [2, 3])
def test_floored_trial_increment_on_gated_bar(scheme, theta):
    """The floor theta: at the bar's first gated step every point has
    c - c_S < theta c for S2/S3, so the floored block acts on the uniform
    increment as theta c M and the increment is -(c d - 2H) / (theta c),
    with every gated point counted as floored."""
    p = dataclasses.replace(W.homogeneous_bar(nx=3, ny=4, du=5e-3, steps=4), trial_floor=theta)
    o = Oracle(p, scheme)
    for lam in p.loads[:3]:
        st = o.load_step(float(lam))
        assert st.n_trial == 0
    lam = float(p.loads[3])
    u = o.u.copy()
    u[o.u_fixed] = lam * o.u_unit[o.u_fixed]
    u, _, ok = o.newton(u, o.d, 1.0)
    assert ok
    parts = o.energies(u, o.d)
    H = np.maximum(o.H, parts["psi_plus"])
    gate = np.ones_like(H, dtype=bool)
    from oracle.constitutive import scheme_part
    dd, hits = o.trial_increment(o.d, H, gate, scheme_part(parts, scheme))
    m = p.material
    pv, pd = bar_energies(p, lam)
    Hs = pv + pd
    c = m.Gc / m.l + 2 * Hs
    d0 = float(o.d.mean())
    om2 = (1 - d0) ** 2
    cS = 8 * om2 / (om2 + m.eta) * {2: pd, 3: pv + pd}[scheme]
    assert c - cS < theta * c                       # the floor acts everywhere
    assert hits == gate.size
    np.testing.assert_allclose(dd, -(c * d0 - 2 * Hs) / (theta * c), rtol=1e-9)
