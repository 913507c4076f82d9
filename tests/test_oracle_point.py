"""Pins for the oracle's quadrature-point functions (not GPU).

Each check is tied to something other than the oracle's own formulas:
the undegraded energy identity (linear elasticity), derivatives by central
finite differences, and hand-computed strain states.
"""
import numpy as np
import pytest

from oracle import constitutive as C

E, NU = 2.1e5, 0.3
LAM, MU, K = C.lame(E, NU)


def lin_energy(eps):
    """Linear-elastic plane-strain energy lam/2 tr^2 + mu eps:eps (textbook)."""
    exx, eyy, g = eps[..., 0], eps[..., 1], eps[..., 2]
    t = exx + eyy
    return 0.5 * LAM * t ** 2 + MU * (exx ** 2 + eyy ** 2 + 0.5 * g ** 2)


def rand_eps(n, seed=0, scale=1e-3):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 3)) * scale


@pytest.mark.parametrize("split", [0, 1])
def test_energy_split_sums_to_linear_energy(split):
    cons = C.Constitutive(E, NU, split)
    eps = rand_eps(500, 1)
    p = cons.parts(eps)
    np.testing.assert_allclose(p["psi_plus"] + p["psi_minus"], lin_energy(eps), rtol=1e-12)
    assert np.all(p["psi_plus"] >= 0) and np.all(p["psi_minus"] >= 0)
    np.testing.assert_allclose(p["psi_plus"], p["psi_vol"] + p["psi_dev"], rtol=1e-14)


def total_energy(cons, eps, g):
    p = cons.parts(eps)
    return g * p["psi_plus"] + p["psi_minus"]


@pytest.mark.parametrize("split", [0, 1])
def test_stress_is_energy_gradient(split):
    cons = C.Constitutive(E, NU, split)
    eps = rand_eps(200, 2)
    g = np.random.default_rng(3).uniform(0.05, 1.0, size=200)
    sig = cons.stress(eps, g)
    h = 1e-9
    for k in range(3):
        ep = eps.copy(); ep[:, k] += h
        em = eps.copy(); em[:, k] -= h
        fd = (total_energy(cons, ep, g) - total_energy(cons, em, g)) / (2 * h)
        np.testing.assert_allclose(sig[:, k], fd, rtol=2e-5, atol=1e-6)


@pytest.mark.parametrize("split", [0, 1])
def test_tangent_is_stress_derivative(split):
    cons = C.Constitutive(E, NU, split)
    eps = rand_eps(300, 4)
    g = np.random.default_rng(5).uniform(0.05, 1.0, size=300)
    Ct = cons.tangent(eps, g)
    h = 1e-10
    for k in range(3):
        ep = eps.copy(); ep[:, k] += h
        em = eps.copy(); em[:, k] -= h
        fd = (cons.stress(ep, g) - cons.stress(em, g)) / (2 * h)
        # skip points where the perturbation crosses a kink (t = 0 or e_i = 0)
        pp, pm = cons.parts(ep), cons.parts(em)
        ok = np.sign(pp["t"]) == np.sign(pm["t"])
        if split == 1:
            ok &= (np.sign(pp["e1"]) == np.sign(pm["e1"])) & (np.sign(pp["e2"]) == np.sign(pm["e2"]))
        np.testing.assert_allclose(Ct[ok, :, k], fd[ok], rtol=1e-5, atol=1e-2)


def test_vd_hand_values():
    cons = C.Constitutive(E, NU, 0)
    # hydrostatic compression (in-plane): t < 0 -> psi_plus = mu * devdev only
    e = 1e-3
    p = cons.parts(np.array([[-e, -e, 0.0]]))
    t = -2 * e
    devdev = 2 * (-e - t / 3) ** 2 + (t / 3) ** 2
    assert np.isclose(p["psi_vol"][0], 0.0)
    assert np.isclose(p["psi_dev"][0], MU * devdev, rtol=1e-14)
    assert np.isclose(p["psi_minus"][0], 0.5 * K * t * t, rtol=1e-14)
    # pure shear gxy = 2e: t = 0 (inactive by the strict tie rule)
    p = cons.parts(np.array([[0.0, 0.0, 2 * e]]))
    assert p["psi_vol"][0] == 0.0 and np.isclose(p["psi_dev"][0], MU * 2 * e * e)
    s = cons.stress(np.array([[0.0, 0.0, 2 * e]]), np.array([0.5]))
    assert np.isclose(s[0, 2], MU * 0.5 * 2 * e) and abs(s[0, 0]) < 1e-20
    # equibiaxial tension, fully degraded volumetric part
    g = np.array([0.25])
    s = cons.stress(np.array([[e, e, 0.0]]), g)
    # sxx = 2 mu g (e - 2e/3) + g K 2e
    assert np.isclose(s[0, 0], 2 * MU * 0.25 * (e / 3) + 0.25 * K * 2 * e, rtol=1e-14)
    # uniaxial strain eyy = e (tension)
    s = cons.stress(np.array([[0.0, e, 0.0]]), np.array([1.0]))
    assert np.isclose(s[0, 1], (LAM + 2 * MU) * e, rtol=1e-13)
    assert np.isclose(s[0, 0], LAM * e, rtol=1e-13)


def test_vd_tie_rule_trace_zero_is_inactive():
    cons = C.Constitutive(E, NU, 0)
    eps = np.array([[1e-3, -1e-3, 0.0]])
    Ct = cons.tangent(eps, np.array([0.5]))
    # kappa = K (undegraded) at t = 0
    assert np.isclose(Ct[0, 0, 1], -2 * MU * 0.5 / 3 + K)


def test_spectral_hand_values():
    cons = C.Constitutive(E, NU, 1)
    e = 1e-3
    # principal strains (e, -e) rotated by 30 degrees
    th = np.pi / 6
    c, s = np.cos(th), np.sin(th)
    R = np.array([[c, -s], [s, c]])
    T = R @ np.diag([e, -e]) @ R.T
    eps = np.array([[T[0, 0], T[1, 1], 2 * T[0, 1]]])
    p = cons.parts(eps)
    assert np.isclose(p["e1"][0], e) and np.isclose(p["e2"][0], -e)
    assert np.isclose(p["psi_plus"][0], MU * e * e, rtol=1e-12)   # t = 0
    # degraded stress: g * 2 mu e n1n1 + 2 mu (-e) n2n2
    g = np.array([0.3])
    S = cons.stress(eps, g)
    ref = R @ np.diag([0.3 * 2 * MU * e, -2 * MU * e]) @ R.T
    np.testing.assert_allclose(S[0], [ref[0, 0], ref[1, 1], ref[0, 1]], rtol=1e-10, atol=1e-8)


def test_spectral_equals_vd_free_case_for_isotropic_tension():
    # equibiaxial tension: both splits put the whole energy in psi_plus
    eps = np.array([[1e-3, 1e-3, 0.0]])
    for split in (0, 1):
        p = C.Constitutive(E, NU, split).parts(eps)
        assert np.isclose(p["psi_plus"][0], lin_energy(eps)[0], rtol=1e-12)
        assert p["psi_minus"][0] == 0.0


def test_degradation():
    assert C.degradation(0.0, 1e-6) == 1.0 + 1e-6
    assert C.degradation(1.0, 1e-6) == 1e-6


@pytest.mark.parametrize("a,b", [(2e-3, 5e-4), (5e-4, 2e-3)])
def test_spectral_scheme_parts_hand_values(a, b):
    """Spectral split with a nonzero trace, principal strains (a, -b) rotated
    by 20 degrees: Psi_vol = lam/2 <a - b>_+^2 (S1's part), Psi_dev =
    mu <a>_+^2 (S2's part), Psi+ their sum (S3), Psi- = lam/2 <a - b>_-^2 +
    mu b^2.  Lame constants from the textbook formulas, not the oracle's."""
    lam = E * NU / ((1 + NU) * (1 - 2 * NU))
    mu = E / (2 * (1 + NU))
    th = np.deg2rad(20.0)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    T = R @ np.diag([a, -b]) @ R.T
    eps = np.array([[T[0, 0], T[1, 1], 2 * T[0, 1]]])
    p = C.Constitutive(E, NU, 1).parts(eps)
    t = a - b
    vol = 0.5 * lam * max(t, 0.0) ** 2
    dev = mu * a * a
    assert np.isclose(p["psi_vol"][0], vol, rtol=1e-12, atol=1e-18)
    assert np.isclose(p["psi_dev"][0], dev, rtol=1e-12)
    assert np.isclose(p["psi_minus"][0], 0.5 * lam * min(t, 0.0) ** 2 + mu * b * b, rtol=1e-12)
    for scheme, ref in ((1, vol), (2, dev), (3, vol + dev)):
        assert np.isclose(C.scheme_part(p, scheme)[0], ref, rtol=1e-12, atol=1e-18)
