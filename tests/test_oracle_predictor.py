"""Pins for the fixed-stress predictor (not GPU).

The paper's claim (Section 3.3): with the strain rescaled per eq:trdep /
eq:epdep, the stress keeps its first invariant (S1), its deviatoric
projection (S2), or both (S3) to first order in the phase increment.  The
checks below build the half-step 3-D strain with the oracle's scale factor,
evaluate a 3-D stress written here from the constitutive law (eq_sigma), and
require the held quantity to change only at O(Dd^2) -- a wrong factor a (for
example the factor-2 slip of the one-dimensional appendix) leaves an O(Dd)
change.  The energy of that strain must equal the oracle's predicted energy,
and the extra stiffness coefficient must be the derivative of the energy
update (eq:dpsi).
"""
import numpy as np
import pytest

from oracle import constitutive as C

E, NU, ETA = 2.1e5, 0.3, 1e-6
LAM, MU, K = C.lame(E, NU)


def strain3(eps):
    exx, eyy, g = eps
    return np.array([[exx, 0.5 * g, 0.0], [0.5 * g, eyy, 0.0], [0.0, 0.0, 0.0]])


def stress3(e3, d):
    """eq_sigma in 3-D: g [2 mu e_dev + K <t>_+ I] + K <t>_- I."""
    g = (1 - d) ** 2 + ETA
    t = np.trace(e3)
    dev = e3 - t / 3 * np.eye(3)
    return g * (2 * MU * dev + K * max(t, 0) * np.eye(3)) + K * min(t, 0) * np.eye(3)


def energy3(e3):
    t = np.trace(e3)
    dev = e3 - t / 3 * np.eye(3)
    return MU * np.sum(dev * dev) + 0.5 * K * max(t, 0) ** 2


def half_step_strain(e3, s, scheme):
    t = np.trace(e3)
    dev = e3 - t / 3 * np.eye(3)
    vol = t / 3 * np.eye(3)
    if scheme == 1:
        return dev + (s if t > 0 else 1.0) * vol
    if scheme == 2:
        return s * dev + vol
    return s * dev + (s if t > 0 else 1.0) * vol


def held_change(eps, d, dd, scheme):
    e3 = strain3(eps)
    s = C.strain_scale(d, ETA, dd)
    eh = half_step_strain(e3, s, scheme)
    dS = stress3(eh, d + dd) - stress3(e3, d)
    dev = e3 - np.trace(e3) / 3 * np.eye(3)
    return abs(np.trace(dS)), abs(np.sum(dS * dev))


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_invariants_held_to_second_order(scheme):
    rng = np.random.default_rng(100 + scheme)
    for _ in range(20):
        eps = rng.normal(size=3) * 1e-3
        if eps[0] + eps[1] <= 0:
            eps[:2] = np.abs(eps[:2])          # tension: the volumetric part is active
        d = rng.uniform(0.0, 0.8)
        dds = np.array([1e-3, 5e-4, 2.5e-4])
        ch = np.array([held_change(eps, d, x, scheme) for x in dds])
        for col, held in ((0, scheme in (1, 3)), (1, scheme in (2, 3))):
            if held:
                rates = np.log2(ch[:-1, col] / ch[1:, col])
                assert np.all(rates > 1.9), (scheme, col, rates)


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_predicted_energy_is_energy_of_half_step_strain(scheme):
    rng = np.random.default_rng(200 + scheme)
    cons = C.Constitutive(E, NU, 0)
    for _ in range(20):
        eps = rng.normal(size=3) * 1e-3
        d = rng.uniform(0, 0.9)
        dd = rng.uniform(0, 0.05)
        parts = cons.parts(eps[None])
        psi_s = C.scheme_part(parts, scheme)
        got = C.predicted_energy(parts["psi_plus"], psi_s, np.array([d]), ETA,
                                 np.array([dd]), np.array([True]))[0]
        e3 = strain3(eps)
        eh = half_step_strain(e3, C.strain_scale(d, ETA, dd), scheme)
        assert np.isclose(got, energy3(eh), rtol=1e-11)


def test_s3_identity():
    cons = C.Constitutive(E, NU, 0)
    eps = np.random.default_rng(1).normal(size=(50, 3)) * 1e-3
    parts = cons.parts(eps)
    d = np.random.default_rng(2).uniform(0, 0.9, 50)
    dd = np.random.default_rng(3).uniform(0, 0.1, 50)
    got = C.predicted_energy(parts["psi_plus"], C.scheme_part(parts, 3), d, ETA, dd, np.ones(50, bool))
    s = 1 + 2 * (1 - d) / ((1 - d) ** 2 + ETA) * dd
    np.testing.assert_allclose(got, s * s * parts["psi_plus"], rtol=1e-13)


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_coupling_coefficient_is_derivative_of_energy_update(scheme):
    """K~ = -c_S N N^T: c_S = 2(1-d) dPsi_hat/dDd at Dd = 0 (eq:dpsi)."""
    cons = C.Constitutive(E, NU, 0)
    eps = np.random.default_rng(9).normal(size=(40, 3)) * 1e-3
    parts = cons.parts(eps)
    d = np.random.default_rng(10).uniform(0, 0.9, 40)
    psi_s = C.scheme_part(parts, scheme)
    h = 1e-7
    on = np.ones(40, bool)
    fd = (C.predicted_energy(parts["psi_plus"], psi_s, d, ETA, np.full(40, h), on)
          - parts["psi_plus"]) / h
    cS = C.coupling_coefficient(d, ETA, psi_s)
    np.testing.assert_allclose(cS, 2 * (1 - d) * fd, rtol=1e-5, atol=1e-12)
    if scheme == 3:
        # printed form: 4 (1-d)^2/g [2 mu e_dev:e_dev + K <t>_+^2]
        g = (1 - d) ** 2 + ETA
        printed = 4 * (1 - d) ** 2 / g * (2 * MU * parts["devdev"] + K * np.maximum(parts["t"], 0) ** 2)
        np.testing.assert_allclose(cS, printed, rtol=1e-12)


def test_inactive_cases():
    psi = np.array([5.0, 5.0, 5.0])
    got = C.predicted_energy(psi, psi, np.array([0.1, 0.1, 0.1]), ETA,
                             np.array([-0.1, 0.1, 0.0]), np.array([True, False, True]))
    np.testing.assert_array_equal(got, psi)


def test_one_dimensional_reduction():
    """Appendix C: at eta = 0 the strain grows by 2 eps/(1-d) per unit Dd."""
    d, dd = 0.3, 1e-2
    s = C.strain_scale(d, 0.0, dd)
    assert np.isclose(s - 1.0, 2.0 / (1.0 - d) * dd, rtol=1e-14)


def test_trial_coefficient_hand_values():
    """Augmented block coefficient c - c_S, floored at theta*c, only where gated."""
    from oracle.assembly import trial_coefficient
    c = np.array([10.0, 10.0, 10.0, 10.0])
    cS = np.array([4.0, 9.5, 20.0, 4.0])
    gate = np.array([True, True, True, False])
    ct, hits = trial_coefficient(c, cS, gate, 0.1)
    np.testing.assert_array_equal(ct, [6.0, 1.0, 1.0, 10.0])
    assert hits == 2
