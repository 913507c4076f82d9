"""Pins for the oracle's 3-D hexahedral path (not GPU).

* Plane-strain equivalence: the 2-D notched panel extruded into a slab with
  u_z = 0 on both faces (one or two element layers) is plane strain; its
  fields are the 2-D oracle's on every node layer, its staggered counts the
  same, and its reaction force the 2-D force per unit thickness times the
  thickness.  This ties the 3-D kinematics, split, tangent, phase operator
  and staggered loop to the independently pinned 2-D oracle.
* Uniaxial stress: a cube on rollers pulled on one face has the affine
  displacement u = eps (-nu x, y, -nu z), Psi+ = E eps^2 / 2 (the trace
  eps (1 - 2 nu) is positive), so d = l E eps^2 / (Gc + l E eps^2) and the
  reaction force is g(d) E eps times the face area (textbook 3-D values,
  with E, not the plane-strain modulus).
* Spectral split in 3-D: the shear panel (spectral split) extruded into a
  slab matches the 2-D spectral oracle the same way (the out-of-plane
  principal strain is zero); a diagonal strain with mixed signs gives the
  energies and stresses by hand; rotating the strain rotates the stress and
  leaves the energies unchanged (catches a wrong engineering-shear factor);
  with every principal strain positive both splits give the undamaged
  energy lam/2 t^2 + mu eps:eps; the tangent is the stress's derivative.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from oracle.hex3d import Oracle3D, Spectral3D, VD3D


@pytest.mark.parametrize("nz", [1, 2])
@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_slab_is_plane_strain(scheme, nz):
    # steps 1-2: the second already runs gated trial solves (S1, S3)
    p2 = W.tension_panel(n=8, l=0.2, du=2e-3, steps=2)
    lz = 0.1
    p3 = W.slab_from_panel(p2, nz=nz, lz=lz)
    o2, o3 = Oracle(p2, scheme), Oracle3D(p3, scheme)
    P = (p2.nx + 1) * (p2.ny + 1)
    trials = 0
    for lam in p2.loads:
        s2, s3 = o2.load_step(float(lam)), o3.load_step(float(lam))
        assert s2.converged and s3.converged
        assert s2.n_stag == s3.n_stag, (scheme, lam, s2.n_stag, s3.n_stag)
        trials += s3.n_trial
        for k in range(nz + 1):
            lay = slice(k * P, (k + 1) * P)
            np.testing.assert_allclose(o3.d[lay], o2.d, rtol=1e-8, atol=1e-12)
            np.testing.assert_allclose(o3.u[3 * k * P:3 * (k + 1) * P][0::3], o2.u[0::2],
                                       rtol=1e-8, atol=1e-14)
            np.testing.assert_allclose(o3.u[3 * k * P:3 * (k + 1) * P][1::3], o2.u[1::2],
                                       rtol=1e-8, atol=1e-14)
        assert np.abs(o3.u[2::3]).max() < 1e-14
        assert np.isclose(s3.force, s2.force * lz, rtol=1e-8)
    if scheme != 0:
        assert trials > 0


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_uniaxial_bar3d_closed_form(scheme):
    p = W.uniaxial_bar3d(n=3, l=0.03, du=5e-3, steps=6)
    m = p.material
    o = Oracle3D(p, scheme)
    for lam in p.loads:
        st = o.load_step(float(lam))
        eps = lam / p.ly
        d_ref = m.l * m.E * eps ** 2 / (m.Gc + m.l * m.E * eps ** 2)
        F_ref = ((1 - d_ref) ** 2 + m.eta) * m.E * eps * p.lx * p.lz
        assert st.converged
        np.testing.assert_allclose(o.d, d_ref, rtol=1e-9)
        assert np.isclose(st.force, F_ref, rtol=1e-9)
        # lateral contraction: u_x = -nu eps x on the face x = 1
        nodes = np.arange(o.mesh.n_nodes)
        xface = nodes[(nodes % (p.nx + 1)) == p.nx]
        np.testing.assert_allclose(o.u[3 * xface], -m.nu * eps * p.lx, rtol=1e-9)
        if scheme == 0:
            assert st.n_stag == 2
        else:
            assert st.n_stag <= 3


def _assert_slab_matches(p2, scheme, nz, lz):
    o2, o3 = Oracle(p2, scheme), Oracle3D(W.slab_from_panel(p2, nz=nz, lz=lz), scheme)
    P = (p2.nx + 1) * (p2.ny + 1)
    trials = 0
    for lam in p2.loads:
        s2, s3 = o2.load_step(float(lam)), o3.load_step(float(lam))
        assert s2.converged and s3.converged
        assert s2.n_stag == s3.n_stag, (scheme, lam, s2.n_stag, s3.n_stag)
        trials += s3.n_trial
        for k in range(nz + 1):
            np.testing.assert_allclose(o3.d[k * P:(k + 1) * P], o2.d, rtol=1e-8, atol=1e-12)
            uk = o3.u[3 * k * P:3 * (k + 1) * P]
            np.testing.assert_allclose(uk[0::3], o2.u[0::2], rtol=1e-8, atol=1e-14)
            np.testing.assert_allclose(uk[1::3], o2.u[1::2], rtol=1e-8, atol=1e-14)
        assert np.abs(o3.u[2::3]).max() < 1e-14
        assert np.isclose(s3.force, s2.force * lz, rtol=1e-8)
    return trials


@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_spectral_slab_is_plane_strain(scheme):
    # shear panel, spectral split; the second step runs gated trial solves (S1, S3)
    p2 = W.shear_panel(n=8, l=0.2, du=4e-3, steps=2)
    assert p2.material.split == W.SPLIT_SPECTRAL
    trials = _assert_slab_matches(p2, scheme, nz=1, lz=0.1)
    if scheme != 0:
        assert trials > 0


def test_spectral_slab_two_layers():
    p2 = W.shear_panel(n=8, l=0.2, du=4e-3, steps=2)
    assert _assert_slab_matches(p2, 1, nz=2, lz=0.1) > 0


E, NU = 2.1e5, 0.3
LAM = E * NU / ((1 + NU) * (1 - 2 * NU))
MU = E / (2 * (1 + NU))


def _rotation(a, b, c):
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    Rx = np.array([[1, 0, 0], [0, np.cos(c), -np.sin(c)], [0, np.sin(c), np.cos(c)]])
    return Rz @ Ry @ Rx


def _voigt_strain(T):
    return np.array([T[0, 0], T[1, 1], T[2, 2], 2 * T[1, 2], 2 * T[0, 2], 2 * T[0, 1]])


def _stress_tensor(s):
    return np.array([[s[0], s[5], s[4]], [s[5], s[1], s[3]], [s[4], s[3], s[2]]])


def test_spectral3d_diagonal_hand_values():
    c = Spectral3D(E, NU)
    a, b, cz = 2e-3, -1e-3, 5e-4
    t = a + b + cz
    eps = np.array([[a, b, cz, 0.0, 0.0, 0.0]])
    g = np.array([0.36])
    P = c.parts(eps)
    assert np.isclose(P["psi_vol"][0], 0.5 * LAM * t * t, rtol=1e-13)
    assert np.isclose(P["psi_dev"][0], MU * (a * a + cz * cz), rtol=1e-13)
    assert np.isclose(P["psi_minus"][0], MU * b * b, rtol=1e-13)
    s = c.stress(eps, g)[0]
    ref = [g[0] * (LAM * t + 2 * MU * a), g[0] * LAM * t + 2 * MU * b,
           g[0] * (LAM * t + 2 * MU * cz), 0.0, 0.0, 0.0]
    np.testing.assert_allclose(s, ref, rtol=1e-12, atol=1e-9)
    # negative trace: the volumetric part goes undegraded
    eps_c = np.array([[-a, b, -cz, 0.0, 0.0, 0.0]])
    tc = -a + b - cz
    sc = c.stress(eps_c, g)[0]
    assert np.isclose(sc[0], LAM * tc + 2 * MU * (-a), rtol=1e-12)
    assert np.isclose(c.parts(eps_c)["psi_plus"][0], 0.0)


def test_spectral3d_rotation_covariance():
    c = Spectral3D(E, NU)
    D = np.diag([2e-3, -1e-3, 5e-4])
    eps0 = _voigt_strain(D)[None]
    g = np.array([0.5])
    P0, S0 = c.parts(eps0), _stress_tensor(c.stress(eps0, g)[0])
    for angles in [(0.3, 0.0, 0.0), (0.4, -0.7, 1.1), (2.0, 0.5, -0.9)]:
        R = _rotation(*angles)
        epsR = _voigt_strain(R @ D @ R.T)[None]
        PR = c.parts(epsR)
        for k in ("psi_vol", "psi_dev", "psi_minus"):
            assert np.isclose(PR[k][0], P0[k][0], rtol=1e-12)
        np.testing.assert_allclose(_stress_tensor(c.stress(epsR, g)[0]), R @ S0 @ R.T,
                                   rtol=1e-10, atol=1e-7)


def test_spectral_and_vd_agree_in_triaxial_tension():
    rng = np.random.default_rng(11)
    Q = _rotation(*rng.uniform(-np.pi, np.pi, 3))
    D = np.diag([3e-3, 1e-3, 2e-4])
    eps = _voigt_strain(Q @ D @ Q.T)[None]
    g = np.array([0.25])
    sp3, vd = Spectral3D(E, NU), VD3D(E, NU)
    t = 4.2e-3
    total = 0.5 * LAM * t * t + MU * np.sum(np.diag(D) ** 2)
    for c in (sp3, vd):
        P = c.parts(eps)
        assert np.isclose(P["psi_plus"][0], total, rtol=1e-12)
        assert P["psi_minus"][0] == pytest.approx(0.0, abs=1e-12 * total)
    np.testing.assert_allclose(sp3.stress(eps, g), vd.stress(eps, g), rtol=1e-10, atol=1e-8)
    np.testing.assert_allclose(sp3.tangent(eps, g), vd.tangent(eps, g), rtol=1e-10, atol=1e-6)


@pytest.mark.parametrize("seed", [0, 1])
def test_spectral3d_tangent_is_stress_derivative(seed):
    rng = np.random.default_rng(seed)
    c = Spectral3D(E, NU)
    eps = rng.normal(size=(6, 6)) * 1e-3
    g = rng.uniform(0.05, 1.0, 6)
    C = c.tangent(eps, g)
    h = 1e-8
    for k in range(6):
        dv = np.zeros(6)
        dv[k] = h
        fd = (c.stress(eps + dv, g) - c.stress(eps - dv, g)) / (2 * h)
        np.testing.assert_allclose(fd, C[:, :, k], rtol=0, atol=1e-8 * np.abs(C).max())


@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_uniaxial_bar3d_spectral_closed_form(scheme):
    """Uniaxial stress with the spectral split: the principal strains are
    eps (axial) and e_l twice (lateral, negative).  The lateral ones stay
    undegraded, so sigma_l = g lam t + 2 mu e_l = 0 with t = eps + 2 e_l,
    i.e. t = eps / (1 + g lam / mu); then Psi+ = lam/2 t^2 + mu eps^2 and
    the axial stress is g (lam t + 2 mu eps).  Psi+ grows with d, so d is
    the root of d = 2 l Psi+(d) / (Gc + 2 l Psi+(d)), which the staggered
    schemes reach as their common fixed point.  Steps 1-4 reach d = 0.50,
    beyond the stress peak (eps = 0.0127, d = 0.26); further on the
    softening bar also has non-uniform equilibria, and S3 lands on one at
    the next step, so the pin stops at step 4."""
    import dataclasses

    from scipy.optimize import brentq
    p = W.uniaxial_bar3d(n=2, l=0.03, du=5e-3, steps=4)
    m = dataclasses.replace(p.material, split=W.SPLIT_SPECTRAL)
    p = dataclasses.replace(p, material=m, tol_stag=1e-11, max_stag=200)
    lam = m.E * m.nu / ((1 + m.nu) * (1 - 2 * m.nu))
    mu = m.E / (2 * (1 + m.nu))
    o = Oracle3D(p, scheme)
    for lam_u in p.loads:
        st = o.load_step(float(lam_u))
        assert st.converged
        eps = lam_u / p.ly

        def parts(d):
            g = (1 - d) ** 2 + m.eta
            t = eps / (1 + g * lam / mu)
            return g, t, 0.5 * lam * t * t + mu * eps * eps

        d_ref = brentq(lambda d: d - 2 * m.l * parts(d)[2] / (m.Gc + 2 * m.l * parts(d)[2]),
                       0.0, 1.0, xtol=1e-15)
        g, t, _ = parts(d_ref)
        np.testing.assert_allclose(o.d, d_ref, rtol=1e-8)
        assert np.isclose(st.force, g * (lam * t + 2 * mu * eps) * p.lx * p.lz, rtol=1e-8)
        # lateral contraction e_l = (t - eps) / 2 on the faces x = lx and z = lz
        nodes = np.arange(o.mesh.n_nodes)
        xface = nodes[(nodes % (p.nx + 1)) == p.nx]
        np.testing.assert_allclose(o.u[3 * xface], 0.5 * (t - eps) * p.lx, rtol=1e-8)
    assert 0.45 < d_ref < 0.55


def _linear_field(mesh, A, b=None):
    """Nodal values of u(x) = A x (+ b) on the box mesh (interleaved dofs)."""
    P = (mesh.nx + 1) * (mesh.ny + 1)
    n = np.arange(mesh.n_nodes)
    k, r = n // P, n % P
    j, i = r // (mesh.nx + 1), r % (mesh.nx + 1)
    X = np.stack([i * mesh.lx / mesh.nx, j * mesh.ly / mesh.ny, k * mesh.lz / mesh.nz], axis=1)
    if A.ndim == 1:          # scalar field a . x + b
        return X @ A + (b or 0.0), X
    u = X @ A.T
    return u.reshape(-1), X


@pytest.mark.parametrize("split", [0, 1])
def test_patch_test_3d(split):
    """Trilinear hexahedra reproduce a linear displacement exactly: the
    strain at every point is sym(A), with engineering shears 2 eps_ij
    (this pins all six rows of B, the shear rows included, which the slab
    and the uniaxial cube leave untested); with uniform d the stress is
    uniform, so the internal force vanishes at interior nodes, and the
    stored energy integrates to volume x Psi(eps)."""
    from oracle.hex3d import Mesh3D, Spectral3D, VD3D, internal_force
    m = Mesh3D(3, 4, 2, 1.3, 0.7, 0.45)
    A = np.array([[1.0, 0.4, -0.3], [0.2, -0.6, 0.5], [-0.1, 0.7, 0.8]]) * 1e-3
    u, _ = _linear_field(m, A)
    S = 0.5 * (A + A.T)
    eps_ref = np.array([S[0, 0], S[1, 1], S[2, 2], 2 * S[1, 2], 2 * S[0, 2], 2 * S[0, 1]])
    eps = m.strain(u)
    np.testing.assert_allclose(eps, np.broadcast_to(eps_ref, eps.shape), rtol=0, atol=1e-15)
    cons = (VD3D if split == 0 else Spectral3D)(2.1e5, 0.3)
    d = np.full(m.n_nodes, 0.3)
    R = internal_force(m, cons, u, d, 1e-6).reshape(-1, 3)
    P = (m.nx + 1) * (m.ny + 1)
    n = np.arange(m.n_nodes)
    k, r = n // P, n % P
    j, i = r // (m.nx + 1), r % (m.nx + 1)
    interior = (i > 0) & (i < m.nx) & (j > 0) & (j < m.ny) & (k > 0) & (k < m.nz)
    assert interior.any()
    scale = np.abs(R).max()
    assert np.abs(R[interior]).max() <= 1e-12 * scale
    parts = cons.parts(eps)
    g = (1 - 0.3) ** 2 + 1e-6
    energy = np.sum(m.wdet * (g * parts["psi_plus"] + parts["psi_minus"]))
    ref = cons.parts(eps_ref[None])
    vol = m.lx * m.ly * m.lz
    assert np.isclose(energy, vol * (g * ref["psi_plus"][0] + ref["psi_minus"][0]), rtol=1e-12)


def test_phase_operator_3d_integrals():
    """The 3-D phase operator against integrals a linear field fixes: the
    mass part with coefficient c sums to c x volume; the gradient part
    annihilates constants, has zero interior rows on a linear d, and gives
    d^T L d = Gc l |grad d|^2 x volume (exact for a linear d), which pins
    the z-derivatives the slab's z-uniform fields never exercise."""
    from oracle.hex3d import Mesh3D, phase_matrix
    m = Mesh3D(3, 2, 4, 1.3, 0.7, 0.45)
    E = m.conn.shape[0]
    vol = m.lx * m.ly * m.lz
    c = 7.5
    M = phase_matrix(m, np.full((E, 8), c), 0.0, 1.0)          # mass only (Gc l = 0)
    one = np.ones(m.n_nodes)
    assert np.isclose(one @ (M @ one), c * vol, rtol=1e-13)
    Gc, l = 2.7, 0.05
    L = phase_matrix(m, np.zeros((E, 8)), Gc, l)               # gradient part only
    assert np.abs(L @ one).max() <= 1e-12 * Gc * l
    a = np.array([0.3, -1.1, 2.0])
    d, X = _linear_field(m, a, 0.25)
    Ld = L @ d
    P = (m.nx + 1) * (m.ny + 1)
    n = np.arange(m.n_nodes)
    k, r = n // P, n % P
    j, i = r // (m.nx + 1), r % (m.nx + 1)
    interior = (i > 0) & (i < m.nx) & (j > 0) & (j < m.ny) & (k > 0) & (k < m.nz)
    assert interior.any()
    assert np.abs(Ld[interior]).max() <= 1e-12 * np.abs(Ld).max()
    assert np.isclose(d @ Ld, Gc * l * (a @ a) * vol, rtol=1e-12)


@pytest.mark.parametrize("split", [0, 1])
def test_tangent_matrix_3d_is_force_jacobian(split):
    """The assembled 3-D tangent equals the central-difference Jacobian of
    the assembled internal force along random directions (both splits; the
    VD point tangent has no other pin of its own)."""
    from oracle.hex3d import Mesh3D, Spectral3D, VD3D, internal_force, tangent_matrix
    m = Mesh3D(2, 3, 2, 1.3, 0.7, 0.45)
    cons = (VD3D if split == 0 else Spectral3D)(2.1e5, 0.3)
    rng = np.random.default_rng(17 + split)
    u = rng.normal(size=3 * m.n_nodes) * 1e-3
    d = rng.uniform(0, 0.9, size=m.n_nodes)
    K = tangent_matrix(m, cons, u, d, 1e-6)
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()
    h = 1e-9
    for _ in range(3):
        p = rng.normal(size=u.size)
        fd = (internal_force(m, cons, u + h * p, d, 1e-6)
              - internal_force(m, cons, u - h * p, d, 1e-6)) / (2 * h)
        np.testing.assert_allclose(fd, K @ p, rtol=0, atol=1e-6 * np.abs(K @ p).max())
