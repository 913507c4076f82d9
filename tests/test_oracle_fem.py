"""Pins for the oracle's discretisation (not GPU).

* linear-displacement patch test (exact reproduction, d = 0 and uniform d);
* closed-form bilinear-rectangle mass and Laplacian element matrices;
* strain energy of a linear field against the textbook closed form;
* symmetry, rigid-body kernel, K_t against a finite-difference Jacobian of R_u;
* homogeneous AT2 closed form d = 2 l H / (Gc + 2 l H);
* manufactured solution of the AT2 equation with O(h^2) L2 convergence.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assembly as asm
from oracle.constitutive import Constitutive, lame
from oracle.fem import Mesh
from oracle.staggered import Oracle

E, NU = 2.1e5, 0.3
LAM, MU, K = lame(E, NU)


def test_rectangle_element_matrices_closed_form():
    a, b = 0.7, 0.3
    m = Mesh(1, 1, a, b)
    loc = m.conn[0]                       # global ids of local corners 0..3
    M = asm.phase_matrix(m, np.ones((1, 4)), 0.0, 0.0).toarray()[np.ix_(loc, loc)]
    Mref = a * b / 36 * np.array([[4, 2, 1, 2], [2, 4, 2, 1], [1, 2, 4, 2], [2, 1, 2, 4]])
    np.testing.assert_allclose(M, Mref, rtol=1e-13)
    L = asm.phase_matrix(m, np.zeros((1, 4)), 1.0, 1.0).toarray()[np.ix_(loc, loc)]
    Lx = b / (6 * a) * np.array([[2, -2, -1, 1], [-2, 2, 1, -1], [-1, 1, 2, -2], [1, -1, -2, 2]])
    Ly = a / (6 * b) * np.array([[2, 1, -1, -2], [1, 2, -2, -1], [-1, -2, 2, 1], [-2, -1, 1, 2]])
    np.testing.assert_allclose(L, Lx + Ly, rtol=1e-13, atol=1e-15)


def test_linear_field_strain_energy():
    m = Mesh(5, 3, 1.3, 0.9)
    cons = Constitutive(E, NU, 0)
    G = np.array([[1e-3, 4e-4], [-2e-4, 7e-4]])        # du_i/dx_j
    u = np.zeros(2 * m.n_nodes)
    u[0::2] = m.xy @ G[0]
    u[1::2] = m.xy @ G[1]
    Kt = asm.tangent_matrix(m, cons, u, np.zeros(m.n_nodes), 0.0)
    exx, eyy, exy = G[0, 0], G[1, 1], 0.5 * (G[0, 1] + G[1, 0])
    dens = 0.5 * LAM * (exx + eyy) ** 2 + MU * (exx ** 2 + eyy ** 2 + 2 * exy ** 2)
    # t > 0 and g = 1 -> the tangent is the linear-elastic one
    assert exx + eyy > 0
    assert np.isclose(0.5 * u @ (Kt @ u), dens * 1.3 * 0.9, rtol=1e-12)


@pytest.mark.parametrize("dval", [0.0, 0.4])
@pytest.mark.parametrize("split", [0, 1])
def test_patch_test(dval, split):
    nx, ny = 6, 5
    p = W.homogeneous_bar(nx=nx, ny=ny)
    m = Mesh(nx, ny, 1.0, 1.0)
    cons = Constitutive(E, NU, split)
    G = np.array([[2e-4, 3e-4], [1e-4, 9e-4]])
    exact = np.zeros(2 * m.n_nodes)
    exact[0::2] = m.xy @ G[0] + 1e-4
    exact[1::2] = m.xy @ G[1] - 2e-4
    # perturb node positions in u only, impose exact values on the boundary
    x, y = m.xy[:, 0], m.xy[:, 1]
    bnd = (x == 0) | (y == 0) | (np.isclose(x, 1)) | (np.isclose(y, 1))
    fixed = np.repeat(bnd, 2)
    free = ~fixed
    d = np.full(m.n_nodes, dval)
    u = exact.copy()
    u[free] = 0.0
    for _ in range(6):
        R = asm.internal_force(m, cons, u, d, 1e-6)[free]
        if np.linalg.norm(R) < 1e-12:
            break
        Kt = asm.tangent_matrix(m, cons, u, d, 1e-6)[free][:, free]
        u[free] += spla.spsolve(Kt.tocsc(), -R)
    np.testing.assert_allclose(u, exact, atol=1e-14, rtol=1e-11)
    del p


@pytest.mark.parametrize("split", [0, 1])
def test_tangent_symmetric_and_rigid_kernel(split):
    m = Mesh(4, 3, 1.0, 0.8)
    cons = Constitutive(E, NU, split)
    rng = np.random.default_rng(7)
    u = rng.normal(size=2 * m.n_nodes) * 1e-3
    d = rng.uniform(0, 1, size=m.n_nodes)
    Kt = asm.tangent_matrix(m, cons, u, d, 1e-6).toarray()
    np.testing.assert_allclose(Kt, Kt.T, rtol=1e-12, atol=1e-9)
    x, y = m.xy[:, 0], m.xy[:, 1]
    modes = []
    for mode in ("tx", "ty", "rot"):
        v = np.zeros(2 * m.n_nodes)
        if mode == "tx":
            v[0::2] = 1
        elif mode == "ty":
            v[1::2] = 1
        else:
            v[0::2] = -y
            v[1::2] = x
        modes.append(v)
        assert np.linalg.norm(Kt @ v) < 1e-9 * np.abs(Kt).max()
    # internal force is invariant under rigid translation
    R0 = asm.internal_force(m, cons, u, d, 1e-6)
    R1 = asm.internal_force(m, cons, u + 0.3 * modes[0], d, 1e-6)
    np.testing.assert_allclose(R0, R1, atol=1e-9)


@pytest.mark.parametrize("split", [0, 1])
def test_tangent_matches_fd_jacobian(split):
    m = Mesh(3, 3, 1.0, 1.0)
    cons = Constitutive(E, NU, split)
    rng = np.random.default_rng(11)
    u = rng.normal(size=2 * m.n_nodes) * 1e-3
    d = rng.uniform(0, 0.9, size=m.n_nodes)
    Kt = asm.tangent_matrix(m, cons, u, d, 1e-6).toarray()
    h = 1e-11
    J = np.zeros_like(Kt)
    for j in range(2 * m.n_nodes):
        up = u.copy(); up[j] += h
        um = u.copy(); um[j] -= h
        J[:, j] = (asm.internal_force(m, cons, up, d, 1e-6) - asm.internal_force(m, cons, um, d, 1e-6)) / (2 * h)
    np.testing.assert_allclose(J, Kt, rtol=1e-4, atol=1e-4 * np.abs(Kt).max())


def test_phase_operators_symmetric():
    m = Mesh(5, 4, 1.0, 1.0)
    rng = np.random.default_rng(3)
    c = rng.uniform(1, 10, size=(m.conn.shape[0], 4))
    A = asm.phase_matrix(m, c, 2.7, 0.03).toarray()
    np.testing.assert_allclose(A, A.T, rtol=1e-13, atol=1e-15)
    assert np.all(np.linalg.eigvalsh(A) > 0)


@pytest.mark.parametrize("H", [0.5, 30.0, 4e3])
def test_at2_homogeneous_closed_form(H):
    p = W.homogeneous_bar(nx=5, ny=7, Gc=2.7, l=0.03)
    o = Oracle(p)
    Hq = np.full_like(o.H, H)
    d = o.solve_phase(Hq, np.zeros(o.mesh.n_nodes))
    ref = 2 * 0.03 * H / (2.7 + 2 * 0.03 * H)
    np.testing.assert_allclose(d, ref, rtol=1e-12)


def _mms_error(n, Gc=1.0, l=0.1):
    m = Mesh(n, n, 1.0, 1.0)
    xq = m.xy[m.conn, 0] @ m.N.T
    yq = m.xy[m.conn, 1] @ m.N.T
    Hq = 1.0 + xq * yq
    A = asm.phase_matrix(m, asm.at2_coefficient(Hq, Gc, l), Gc, l)
    b = asm.phase_rhs(m, Hq)
    # extra source f = -Gc l Lap d* + (Gc/l + 2H) d* - 2H, integrated with 5x5 Gauss
    gx, gw = np.polynomial.legendre.leggauss(5)
    F = np.zeros(m.n_nodes)
    h = 1.0 / n
    for a, wa in zip(gx, gw):
        for bb, wb in zip(gx, gw):
            N = 0.25 * np.array([(1 - a) * (1 - bb), (1 + a) * (1 - bb), (1 + a) * (1 + bb), (1 - a) * (1 + bb)])
            X = m.xy[m.conn]
            x = X[:, :, 0] @ N
            y = X[:, :, 1] @ N
            ds = 0.5 + 0.25 * np.cos(np.pi * x) * np.cos(np.pi * y)
            lap = -0.25 * 2 * np.pi ** 2 * np.cos(np.pi * x) * np.cos(np.pi * y)
            H = 1.0 + x * y
            f = -Gc * l * lap + (Gc / l + 2 * H) * ds - 2 * H
            np.add.at(F, m.conn, (f * wa * wb * h * h / 4)[:, None] * N[None, :])
    d = spla.spsolve(A.tocsc(), b + F)
    # L2 error with 5x5 Gauss
    err = 0.0
    for a, wa in zip(gx, gw):
        for bb, wb in zip(gx, gw):
            N = 0.25 * np.array([(1 - a) * (1 - bb), (1 + a) * (1 - bb), (1 + a) * (1 + bb), (1 - a) * (1 + bb)])
            X = m.xy[m.conn]
            x = X[:, :, 0] @ N
            y = X[:, :, 1] @ N
            ds = 0.5 + 0.25 * np.cos(np.pi * x) * np.cos(np.pi * y)
            dh = d[m.conn] @ N
            err += np.sum((dh - ds) ** 2 * wa * wb * h * h / 4)
    return np.sqrt(err)


def test_at2_manufactured_solution_second_order():
    errs = [_mms_error(n) for n in (8, 16, 32, 64)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.9), rates
    assert errs[-1] < 1e-3
