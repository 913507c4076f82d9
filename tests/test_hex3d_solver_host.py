"""The 3-D load step (pf3d_solver.h) against the 3-D oracle, on the host
(not GPU).

A host-only build of tests/hex3d_solver_harness.cpp runs the solver's loop
on a backend that replays every launch's grid on the host and every
reduction with the device kernel's per-block tree and block order; the
loop, the functors and the per-index arithmetic are those the device build
runs.  It is compared with oracle/hex3d.py (direct solves) under the 2-D
parity protocol: staggered counts within one per step, rel-L2(u) <= 1e-7,
max |d - d_oracle| <= 1e-5 and the reaction within 1e-7 of its peak, on
the uniaxial cube (both splits, with its closed form through the oracle's
own pins), the notched tension panel extruded into a slab (one and two
element layers, the latter over several ragged blocks) for ST, S1 and S3,
the spectral shear slab, and a notched box whose damage varies through the
thickness.  The device build is compared by
tests/test_gpu_zz_hex3d.py.
"""
import ctypes
import dataclasses
import os
import subprocess

import numpy as np
import pytest

import paper_2209_07969_amd as pf
import workloads as W
from oracle.hex3d import Oracle3D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def solver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("h3s") / "libh3s.so")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "--offload-host-only", "-O1",
                    "-std=c++17", "-fPIC", "-shared", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "hex3d_solver_harness.cpp"), "-o", out],
                   check=True)
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    lib.h3s_create.restype = P
    lib.h3s_create.argtypes = [ctypes.POINTER(pf.Mesh3Desc), ctypes.POINTER(pf.MaterialDesc),
                               ctypes.POINTER(pf.SolverOpts)]
    lib.h3s_set_dirichlet_u.argtypes = [P, ctypes.c_int, ctypes.c_longlong, P, P, P]
    lib.h3s_set_dirichlet_d.argtypes = [P, ctypes.c_longlong, P, P]
    lib.h3s_load_step.argtypes = [P, ctypes.c_double, ctypes.POINTER(ctypes.c_longlong),
                                  ctypes.POINTER(ctypes.c_double)]
    lib.h3s_reaction.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.h3s_get_state.argtypes = [P, P, P, P]
    lib.h3s_set_state.argtypes = [P, P, P, P]
    lib.h3s_destroy.argtypes = [P]
    return lib


def opts_for(p, scheme):
    o = pf.default_opts()
    o.scheme = scheme
    for k in ("tol_stag", "tol_pcg", "tol_newton", "max_stag", "max_newton", "psi_crit",
              "d_gate", "trial_floor"):
        setattr(o, k, getattr(p, k))
    return o


def make(lib, p, scheme):
    m = p.material
    h = lib.h3s_create(pf.Mesh3Desc(p.nx, p.ny, p.nz, p.lx, p.ly, p.lz),
                       pf.MaterialDesc(m.E, m.nu, m.Gc, m.l, m.eta, int(m.split)),
                       opts_for(p, scheme))
    assert h
    for gi, g in enumerate(p.dir_u):
        n = np.ascontiguousarray(g.nodes, np.int64)
        c = np.ascontiguousarray(g.comps, np.int8)
        v = np.ascontiguousarray(g.values, np.float64)
        assert lib.h3s_set_dirichlet_u(h, gi, n.size, n.ctypes.data, c.ctypes.data,
                                       v.ctypes.data) == 0
    n = np.ascontiguousarray(p.dir_d_nodes, np.int64)
    v = np.ascontiguousarray(p.dir_d_values, np.float64)
    assert lib.h3s_set_dirichlet_d(h, n.size, n.ctypes.data, v.ctypes.data) == 0
    return h


def compare_history(lib, p, scheme, min_trials=0):
    h = make(lib, p, scheme)
    orc = Oracle3D(p, scheme)
    N = (p.nx + 1) * (p.ny + 1) * (p.nz + 1)
    forces, oforces, trials = [], [], 0
    try:
        for lam in p.loads:
            st = (ctypes.c_longlong * 10)()
            r = ctypes.c_double()
            lib.h3s_load_step(h, float(lam), st, ctypes.byref(r))
            so = orc.load_step(float(lam))
            assert st[9] == 1 and so.converged
            assert abs(st[0] - so.n_stag) <= 1, (lam, st[0], so.n_stag)
            trials += st[2]
            f = (ctypes.c_double * 3)()
            lib.h3s_reaction(h, p.load_group, f)
            forces.append(f[p.load_comp])
            oforces.append(so.force)
            if st[0] == so.n_stag:
                u, d = np.zeros(3 * N), np.zeros(N)
                lib.h3s_get_state(h, u.ctypes.data, d.ctypes.data, None)
                ou = np.concatenate([orc.u[0::3], orc.u[1::3], orc.u[2::3]])
                assert np.linalg.norm(u - ou) <= 1e-7 * np.linalg.norm(ou)
                assert np.abs(d - orc.d).max() <= 1e-5
    finally:
        lib.h3s_destroy(h)
    peak = max(abs(x) for x in oforces)
    np.testing.assert_allclose(forces, oforces, rtol=0, atol=1e-7 * peak)
    assert trials >= min_trials
    return trials


@pytest.mark.parametrize("scheme", [0, 1])
def test_uniaxial_cube(solver, scheme):
    compare_history(solver, W.uniaxial_bar3d(n=2, l=0.03, du=5e-3, steps=4), scheme)


def test_uniaxial_cube_spectral(solver):
    p = W.uniaxial_bar3d(n=2, l=0.03, du=5e-3, steps=4)
    p = dataclasses.replace(p, material=dataclasses.replace(p.material, split=W.SPLIT_SPECTRAL),
                            tol_stag=1e-9)
    compare_history(solver, p, 0)


@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_tension_slab(solver, scheme):
    p = W.slab_from_panel(W.tension_panel(n=8, l=0.2, du=2e-3, steps=2), nz=1, lz=0.1)
    compare_history(solver, p, scheme, min_trials=1 if scheme else 0)


def test_tension_slab_two_layers_ragged_blocks(solver):
    # 13 x 13 x 3 = 507 nodes and 288 elements: two blocks each, the second partial
    p = W.slab_from_panel(W.tension_panel(n=12, l=0.2, du=2e-3, steps=2), nz=2, lz=0.1)
    compare_history(solver, p, 1, min_trials=1)


def test_shear_slab_spectral(solver):
    p = W.slab_from_panel(W.shear_panel(n=8, l=0.2, du=4e-3, steps=2), nz=1, lz=0.1)
    compare_history(solver, p, 1, min_trials=1)


def test_options_outside_the_3d_path_are_refused(solver):
    p = W.uniaxial_bar3d(n=2)
    m = p.material
    mesh = pf.Mesh3Desc(p.nx, p.ny, p.nz, p.lx, p.ly, p.lz)
    mat = pf.MaterialDesc(m.E, m.nu, m.Gc, m.l, m.eta, 0)
    lib = pf.load_library()
    for field, value in (("precision", 1), ("precond", 1), ("phase_model", 1),
                         ("trial_operator", 1), ("trial_update", 1), ("scheme", 4),
                         ("trial_floor", 0.0), ("max_cg", 0)):
        o = opts_for(p, 1)
        setattr(o, field, value)
        assert not solver.h3s_create(mesh, mat, o), field
        h = ctypes.c_void_p()
        assert lib.pf3d_create(mesh, mat, o, None, ctypes.byref(h)) == 1, field
        assert not h.value


@pytest.mark.parametrize("scheme", [0, 1])
def test_unloading_keeps_the_history(solver, scheme):
    """Load, unload, reload: the committed history must hold d on the way
    down (Section 2, H = max over the history), which a monotone path
    cannot tell from H = Psi+."""
    p = W.uniaxial_bar3d(n=2, l=0.03, du=5e-3, steps=5)
    p = dataclasses.replace(p, loads=np.array([5e-3, 1e-2, 1.4e-2, 7e-3, 1.2e-2, 1.5e-2]))
    compare_history(solver, p, scheme)
    orc = Oracle3D(p, scheme)
    d_top = None
    for k, lam in enumerate(p.loads):
        orc.load_step(float(lam))
        if k == 2:
            d_top = orc.d.copy()
        if k in (3, 4):
            np.testing.assert_allclose(orc.d, d_top, rtol=1e-9)


def test_checkpoint_and_resume_is_exact(solver):
    """Saving the committed state after step 2 and resuming it in a fresh
    context reproduces step 3 of the uninterrupted run bit for bit."""
    p = W.slab_from_panel(W.tension_panel(n=8, l=0.2, du=2e-3, steps=3), nz=1, lz=0.1)
    N = (p.nx + 1) * (p.ny + 1) * (p.nz + 1)
    E = p.nx * p.ny * p.nz
    a, b = make(solver, p, 1), make(solver, p, 1)
    try:
        st = (ctypes.c_longlong * 10)()
        r = ctypes.c_double()
        for lam in p.loads[:2]:
            solver.h3s_load_step(a, float(lam), st, ctypes.byref(r))
        u, d, H = np.zeros(3 * N), np.zeros(N), np.zeros(8 * E)
        solver.h3s_get_state(a, u.ctypes.data, d.ctypes.data, H.ctypes.data)
        solver.h3s_set_state(b, u.ctypes.data, d.ctypes.data, H.ctypes.data)
        out = []
        for h in (a, b):
            solver.h3s_load_step(h, float(p.loads[2]), st, ctypes.byref(r))
            u2, d2, H2 = np.zeros(3 * N), np.zeros(N), np.zeros(8 * E)
            solver.h3s_get_state(h, u2.ctypes.data, d2.ctypes.data, H2.ctypes.data)
            out.append((list(st), r.value, u2, d2, H2))
        assert out[0][0] == out[1][0] and out[0][1] == out[1][1]
        for x, y in zip(out[0][2:], out[1][2:]):
            assert np.array_equal(x, y)
        assert out[0][0][2] > 0          # the resumed step ran gated trial solves
    finally:
        solver.h3s_destroy(a)
        solver.h3s_destroy(b)


@pytest.mark.parametrize("scheme", [0, 1])
def test_tilted_notched_box(solver, scheme):
    p = W.tilted_notched_box3d()
    trials = compare_history(solver, p, scheme, min_trials=1 if scheme else 0)
    orc = Oracle3D(p, scheme)
    for lam in p.loads:
        orc.load_step(float(lam))
    P = (p.nx + 1) * (p.ny + 1)
    # the fields really vary through the thickness
    d_front, d_back = orc.d[:P], orc.d[p.nz * P:]
    assert np.abs(d_back - d_front).max() > 0.1
    if scheme:
        assert trials > 0
