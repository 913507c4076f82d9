"""3-D operator kernels against the oracle's hexahedra, on the host (not GPU).

The kernels' arithmetic is __host__ __device__ (pf3d_ops.h).  A host-only
build of tests/hex3d_host_harness.cpp replays each launch's grid, block by
block and thread by thread, through the same per-index functions and the C
ABI's own mesh, material and gate checks.  This checks the indexing, the
element and Gauss-point tables and the arithmetic of every kernel against
the independently assembled oracle (oracle/hex3d.py), with either split,
on meshes that span
one block, several blocks with a ragged tail, and a single element.  Every
array sits between guard zones: inputs between NaNs (an out-of-bounds read
turns an output non-finite), outputs between sentinels that must survive
(an out-of-bounds write), and outputs start as NaN (an index the grid
misses stays NaN).  The device build of the same functions is compared
with the oracle by tests/test_gpu_zz_hex3d.py.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import paper_2209_07969_amd as pf
from oracle import hex3d as H3
from oracle.assembly import trial_coefficient
from oracle.constitutive import coupling_coefficient, predicted_energy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
GUARD = 64
SENT = 1.2345e300
SENT16 = 0xBEEF

# (4, 16, 9) spans two tiles of node columns in y and two chunks of node
# planes in z of the element-once tangent apply; (17, 5, 3) two tiles in x
MESHES = [(3, 2, 2), (9, 7, 5), (17, 5, 3), (1, 1, 1), (4, 16, 9)]
MAT = dict(E=2.1e5, nu=0.3, Gc=2.7, l=0.05, eta=1e-6)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("h3") / "libh3.so")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "--offload-host-only", "-O1",
                    "-std=c++17", "-fPIC", "-shared", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "hex3d_host_harness.cpp"), "-o", out],
                   check=True)
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    M3, MT = ctypes.POINTER(pf.Mesh3Desc), ctypes.POINTER(pf.MaterialDesc)
    lib.h3_internal_force.argtypes = [M3, MT, P, P, P]
    lib.h3_internal_force_tiled.argtypes = [M3, MT, P, P, P]
    lib.h3_tangent_apply.argtypes = [M3, MT, P, P, P, P]
    lib.h3_phase_apply.argtypes = [M3, MT, P, P, P]
    lib.h3_qp_update.argtypes = [M3, MT, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 P, P, P, P, P, P, ctypes.POINTER(ctypes.c_longlong)]
    lib.h3_predictor.argtypes = [M3, MT, P, P, P, P, P, P]
    lib.h3_tangent_diag.argtypes = [M3, MT, P, P, P]
    lib.h3_phase_diag.argtypes = [M3, MT, P, P]
    lib.h3_phase_rhs.argtypes = [M3, P, P]
    lib.h3_phase_coef.argtypes = [M3, MT, ctypes.c_int, ctypes.c_double, ctypes.c_int, P, P, P,
                                  P, P, ctypes.POINTER(ctypes.c_longlong)]
    for f in ("h3_internal_force", "h3_internal_force_tiled", "h3_tangent_apply",
              "h3_phase_apply", "h3_qp_update",
              "h3_predictor", "h3_tangent_diag", "h3_phase_diag", "h3_phase_rhs",
              "h3_phase_coef"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


class Guarded:
    """An array of n values between two guard zones."""

    def __init__(self, values=None, n=None, dtype=np.float64, guard=np.nan, init=np.nan):
        n = len(values) if values is not None else n
        self.buf = np.full(n + 2 * GUARD, guard, dtype=dtype)
        self.guard = guard
        self.n = n
        self.buf[GUARD:GUARD + n] = init if values is None else values

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.ctypes.data + GUARD * self.buf.itemsize)

    @property
    def val(self):
        return self.buf[GUARD:GUARD + self.n]

    def guards_intact(self):
        g = np.concatenate([self.buf[:GUARD], self.buf[GUARD + self.n:]])
        return bool(np.all(g == self.guard)) if self.guard == self.guard else bool(
            np.all(np.isnan(g)))


def out_f64(n):
    return Guarded(n=n, guard=SENT, init=np.nan)


def setup(nx, ny, nz, seed, split=0):
    lx, ly, lz = 1.3, 0.7, 0.45
    mesh = pf.Mesh3Desc(nx, ny, nz, lx, ly, lz)
    mat = pf.MaterialDesc(MAT["E"], MAT["nu"], MAT["Gc"], MAT["l"], MAT["eta"], split)
    om = H3.Mesh3D(nx, ny, nz, lx, ly, lz)
    rng = np.random.default_rng(seed)
    return mesh, mat, om, rng


def soa(v):
    return np.concatenate([v[0::3], v[1::3], v[2::3]])


def oracle_split(split):
    return (H3.VD3D if split == 0 else H3.Spectral3D)(MAT["E"], MAT["nu"])


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("shape", MESHES)
def test_internal_force_and_tangent(harness, shape, split):
    mesh, mat, om, rng = setup(*shape, seed=sum(shape), split=split)
    cons = oracle_split(split)
    N = om.n_nodes
    u = rng.normal(size=3 * N) * 1e-3
    d = rng.uniform(0, 1, size=N)
    p = rng.normal(size=3 * N)
    R_orc = soa(H3.internal_force(om, cons, u, d, MAT["eta"]))
    q_orc = soa(H3.tangent_matrix(om, cons, u, d, MAT["eta"]) @ p)
    uG, dG, pG = Guarded(soa(u)), Guarded(d), Guarded(soa(p))
    R, q = out_f64(3 * N), out_f64(3 * N)
    assert harness.h3_internal_force(mesh, mat, uG.ptr, dG.ptr, R.ptr) == 0
    assert harness.h3_tangent_apply(mesh, mat, uG.ptr, dG.ptr, pG.ptr, q.ptr) == 0
    for arr in (R, q):
        assert np.all(np.isfinite(arr.val)) and arr.guards_intact()
    np.testing.assert_allclose(R.val, R_orc, rtol=0, atol=1e-12 * np.abs(R_orc).max())
    np.testing.assert_allclose(q.val, q_orc, rtol=0, atol=1e-12 * np.abs(q_orc).max())
    # the element-once internal force (the ABI's choice once the tiles fill
    # the GPU, larger meshes than these) on the same inputs
    Rt = out_f64(3 * N)
    assert harness.h3_internal_force_tiled(mesh, mat, uG.ptr, dG.ptr, Rt.ptr) == 0
    assert np.all(np.isfinite(Rt.val)) and Rt.guards_intact()
    np.testing.assert_allclose(Rt.val, R_orc, rtol=0, atol=1e-12 * np.abs(R_orc).max())


@pytest.mark.parametrize("shape", MESHES)
def test_phase_apply(harness, shape):
    mesh, mat, om, rng = setup(*shape, seed=7 + sum(shape))
    N, E = om.n_nodes, om.conn.shape[0]
    coef = rng.uniform(0.1, 50.0, size=(E, 8))
    p = rng.normal(size=N)
    q_orc = H3.phase_matrix(om, coef, MAT["Gc"], MAT["l"]) @ p
    cG, pG, q = Guarded(coef.T.reshape(-1)), Guarded(p), out_f64(N)
    assert harness.h3_phase_apply(mesh, mat, cG.ptr, pG.ptr, q.ptr) == 0
    assert np.all(np.isfinite(q.val)) and q.guards_intact()
    np.testing.assert_allclose(q.val, q_orc, rtol=0, atol=1e-12 * np.abs(q_orc).max())


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(9, 7, 5), (2, 3, 1)])
def test_qp_update(harness, shape, scheme, split):
    mesh, mat, om, rng = setup(*shape, seed=100 + scheme, split=split)
    cons = oracle_split(split)
    N, E = om.n_nodes, om.conn.shape[0]
    u = rng.normal(size=3 * N) * 2e-3
    d = rng.uniform(0, 1, size=N)
    parts = cons.parts(om.strain(u))
    psi = parts["psi_plus"]
    Hprev = np.where(rng.uniform(size=psi.shape) < 0.5, psi * 0.5, psi * 1.5)
    psi_crit = MAT["Gc"] / (2 * MAT["l"])
    dq = om.interp(d)
    gate = (psi > psi_crit) & (psi > Hprev) & (dq < 0.95) & (scheme != 0)
    ps = {0: np.zeros_like(psi), 1: parts["psi_vol"], 2: parts["psi_dev"], 3: psi}[scheme]
    uG, dG, HpG = Guarded(soa(u)), Guarded(d), Guarded(Hprev.T.reshape(-1))
    Hout, PS = out_f64(8 * E), out_f64(8 * E)
    fl = Guarded(n=E, dtype=np.uint16, guard=SENT16, init=0)
    ng = ctypes.c_longlong(-1)
    assert harness.h3_qp_update(mesh, mat, scheme, -1.0, 0.95, uG.ptr, dG.ptr, HpG.ptr,
                                Hout.ptr, PS.ptr, fl.ptr, ctypes.byref(ng)) == 0
    for arr in (Hout, PS, fl):
        assert arr.guards_intact()
    assert np.all(np.isfinite(Hout.val)) and np.all(np.isfinite(PS.val))
    np.testing.assert_allclose(Hout.val.reshape(8, E).T, np.maximum(Hprev, psi), rtol=1e-12,
                               atol=0)
    np.testing.assert_allclose(PS.val.reshape(8, E).T, ps, rtol=1e-12,
                               atol=1e-14 * max(ps.max(), 1))
    bits_t = np.stack([(fl.val >> q) & 1 for q in range(8)], axis=1).astype(bool)
    bits_g = np.stack([(fl.val >> (q + 8)) & 1 for q in range(8)], axis=1).astype(bool)
    np.testing.assert_array_equal(bits_t, parts["t"] > 0)
    np.testing.assert_array_equal(bits_g, gate)
    assert ng.value == int(gate.sum())
    if scheme != 0 and shape == (9, 7, 5):
        assert 0 < ng.value < gate.size
    # predictor on the kernel's own H, psi_S and flags (checked above): a
    # random increment with both signs, so the Dd > 0 rule is exercised
    dd = rng.normal(size=N) * 0.05
    Hh = out_f64(8 * E)
    ddG = Guarded(dd)
    assert harness.h3_predictor(mesh, mat, dG.ptr, ddG.ptr, Hout.ptr, PS.ptr, fl.ptr,
                                Hh.ptr) == 0
    assert np.all(np.isfinite(Hh.val)) and Hh.guards_intact()
    H_orc = np.maximum(Hprev, psi)
    Hhat_orc = np.maximum(H_orc, predicted_energy(psi, ps, dq, MAT["eta"], om.interp(dd), gate))
    np.testing.assert_allclose(Hh.val.reshape(8, E).T, Hhat_orc, rtol=1e-12, atol=0)
    if scheme != 0 and shape == (9, 7, 5):
        moved = Hhat_orc > H_orc
        assert 0 < moved.sum() < gate.sum()


def test_checks_refuse_bad_arguments(harness):
    lib = pf.load_library()
    mat = pf.MaterialDesc(MAT["E"], MAT["nu"], MAT["Gc"], MAT["l"], MAT["eta"], 0)
    no_split = pf.MaterialDesc(MAT["E"], MAT["nu"], MAT["Gc"], MAT["l"], MAT["eta"], 2)
    x = Guarded(np.zeros(3 * 8))
    good = pf.Mesh3Desc(1, 1, 1, 1.0, 1.0, 1.0)
    null = ctypes.c_void_p()
    s = ctypes.c_void_p()
    bad_meshes = [pf.Mesh3Desc(0, 1, 1, 1.0, 1.0, 1.0), pf.Mesh3Desc(1, 1, 1, 1.0, -1.0, 1.0),
                  pf.Mesh3Desc(1024, 1024, 1024, 1.0, 1.0, 1.0),
                  pf.Mesh3Desc(2 ** 31 - 1, 1, 1, 1.0, 1.0, 1.0)]
    # the library's entry points refuse before any device call, and so does
    # the harness, through the same checks
    for m in bad_meshes:
        assert lib.pf3d_op_internal_force(m, mat, x.ptr, x.ptr, x.ptr, s) == 1
        assert harness.h3_internal_force(m, mat, x.ptr, x.ptr, x.ptr) == 1
    assert lib.pf3d_op_internal_force(good, no_split, x.ptr, x.ptr, x.ptr, s) == 1
    assert lib.pf3d_op_internal_force(good, mat, null, x.ptr, x.ptr, s) == 1
    assert lib.pf3d_op_phase_apply(good, mat, x.ptr, x.ptr, null, s) == 1
    ng = ctypes.c_longlong()
    for scheme, crit in ((4, -1.0), (-1, -1.0), (1, float("nan"))):
        assert lib.pf3d_op_qp_update(good, mat, scheme, crit, 0.95, x.ptr, x.ptr, x.ptr, x.ptr,
                                     x.ptr, x.ptr, s) == 1
        assert harness.h3_qp_update(good, mat, scheme, crit, 0.95, x.ptr, x.ptr, x.ptr, x.ptr,
                                    x.ptr, x.ptr, ctypes.byref(ng)) == 1
    # nothing was written by a refused call
    assert np.all(x.val == 0.0) and x.guards_intact()


def test_spectral_plane_fields(harness):
    """Fields independent of z with u_z = 0 (the slab's kinematics): one
    principal strain vanishes.  In exact arithmetic its z-shears cancel in
    pairs of corners; both sides sum them in their own order and keep about
    1e-18 of rounding, so that principal strain comes out near +-1e-33 with
    an arbitrary sign, and the strict tie rule may classify it differently
    on each side.  That choice only scales out-of-plane increments, so the
    tangent is driven by a plane increment, as in the slab, where both sides
    must agree."""
    mesh, mat, om, rng = setup(9, 7, 3, seed=5, split=1)
    cons = oracle_split(1)
    N = om.n_nodes
    P = (9 + 1) * (7 + 1)
    uxy = rng.normal(size=(2, P)) * 1e-3
    u = np.zeros(3 * N)
    for k in range(4):
        u[3 * (k * P + np.arange(P))] = uxy[0]
        u[3 * (k * P + np.arange(P)) + 1] = uxy[1]
    d = np.tile(rng.uniform(0, 1, size=P), 4)
    pxy = rng.normal(size=(2, P))
    p = np.zeros(3 * N)
    for k in range(4):
        p[3 * (k * P + np.arange(P))] = pxy[0]
        p[3 * (k * P + np.arange(P)) + 1] = pxy[1]
    R_orc = soa(H3.internal_force(om, cons, u, d, MAT["eta"]))
    q_orc = soa(H3.tangent_matrix(om, cons, u, d, MAT["eta"]) @ p)
    uG, dG, pG = Guarded(soa(u)), Guarded(d), Guarded(soa(p))
    R, q = out_f64(3 * N), out_f64(3 * N)
    assert harness.h3_internal_force(mesh, mat, uG.ptr, dG.ptr, R.ptr) == 0
    assert harness.h3_tangent_apply(mesh, mat, uG.ptr, dG.ptr, pG.ptr, q.ptr) == 0
    np.testing.assert_allclose(R.val, R_orc, rtol=0, atol=1e-12 * np.abs(R_orc).max())
    np.testing.assert_allclose(q.val, q_orc, rtol=0, atol=1e-12 * np.abs(q_orc).max())
    # the element-once internal force (the ABI's choice once the tiles fill
    # the GPU, larger meshes than these) on the same inputs
    Rt = out_f64(3 * N)
    assert harness.h3_internal_force_tiled(mesh, mat, uG.ptr, dG.ptr, Rt.ptr) == 0
    assert np.all(np.isfinite(Rt.val)) and Rt.guards_intact()
    np.testing.assert_allclose(Rt.val, R_orc, rtol=0, atol=1e-12 * np.abs(R_orc).max())


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("shape", [(9, 7, 5), (1, 1, 1)])
def test_diagonals_and_rhs(harness, shape, split):
    mesh, mat, om, rng = setup(*shape, seed=31 + sum(shape), split=split)
    cons = oracle_split(split)
    N, E = om.n_nodes, om.conn.shape[0]
    u = rng.normal(size=3 * N) * 1e-3
    d = rng.uniform(0, 1, size=N)
    coef = rng.uniform(0.1, 50.0, size=(E, 8))
    Hq = rng.uniform(0.0, 30.0, size=(E, 8))
    Dt_orc = soa(H3.tangent_matrix(om, cons, u, d, MAT["eta"]).diagonal())
    Dp_orc = H3.phase_matrix(om, coef, MAT["Gc"], MAT["l"]).diagonal()
    b_orc = H3.phase_rhs(om, Hq)
    Dt, Dp, b = out_f64(3 * N), out_f64(N), out_f64(N)
    assert harness.h3_tangent_diag(mesh, mat, Guarded(soa(u)).ptr, Guarded(d).ptr, Dt.ptr) == 0
    assert harness.h3_phase_diag(mesh, mat, Guarded(coef.T.reshape(-1)).ptr, Dp.ptr) == 0
    assert harness.h3_phase_rhs(mesh, Guarded(Hq.T.reshape(-1)).ptr, b.ptr) == 0
    for arr in (Dt, Dp, b):
        assert np.all(np.isfinite(arr.val)) and arr.guards_intact()
    np.testing.assert_allclose(Dt.val, Dt_orc, rtol=1e-12)
    np.testing.assert_allclose(Dp.val, Dp_orc, rtol=1e-12)
    np.testing.assert_allclose(b.val, b_orc, rtol=1e-12)


@pytest.mark.parametrize("floor", [1, 0])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_phase_coefficients(harness, scheme, floor):
    mesh, mat, om, rng = setup(9, 7, 5, seed=200 + scheme)
    cons = oracle_split(0)
    N, E = om.n_nodes, om.conn.shape[0]
    # this scale puts some gated points below theta c and leaves others above
    u = rng.normal(size=3 * N) * 5e-4
    d = rng.uniform(0, 0.9, size=N)
    parts = cons.parts(om.strain(u))
    psi = parts["psi_plus"]
    Hprev = np.where(rng.uniform(size=psi.shape) < 0.5, psi * 0.5, psi * 1.5)
    uG, dG, HpG = Guarded(soa(u)), Guarded(d), Guarded(Hprev.T.reshape(-1))
    Hout, PS = out_f64(8 * E), out_f64(8 * E)
    fl = Guarded(n=E, dtype=np.uint16, guard=SENT16, init=0)
    ng = ctypes.c_longlong()
    assert harness.h3_qp_update(mesh, mat, scheme, 0.0, 0.95, uG.ptr, dG.ptr, HpG.ptr, Hout.ptr,
                                PS.ptr, fl.ptr, ctypes.byref(ng)) == 0
    H = np.maximum(Hprev, psi)
    gate = (psi > 0.0) & (psi > Hprev) & (om.interp(d) < 0.95)
    ps = {1: parts["psi_vol"], 2: parts["psi_dev"], 3: psi}[scheme]
    c = MAT["Gc"] / MAT["l"] + 2.0 * H
    cS = coupling_coefficient(om.interp(d), MAT["eta"], ps)
    theta = 0.3
    ct_orc, hits = trial_coefficient(c, cS, gate, theta, floor=bool(floor))
    co, below = out_f64(8 * E), ctypes.c_longlong(-1)
    assert harness.h3_phase_coef(mesh, mat, 1, theta, floor, Hout.ptr, PS.ptr, fl.ptr, dG.ptr,
                                 co.ptr, ctypes.byref(below)) == 0
    assert np.all(np.isfinite(co.val)) and co.guards_intact()
    np.testing.assert_allclose(co.val.reshape(8, E).T, ct_orc, rtol=1e-12,
                               atol=1e-12 * np.abs(c).max())
    assert below.value == hits
    assert 0 < hits < gate.sum()
    # without the trial: the AT2 coefficient on every point
    c0 = out_f64(8 * E)
    assert harness.h3_phase_coef(mesh, mat, 0, theta, floor, Hout.ptr, PS.ptr, fl.ptr, dG.ptr,
                                 c0.ptr, ctypes.byref(below)) == 0
    np.testing.assert_allclose(c0.val.reshape(8, E).T, c, rtol=1e-14)
    assert below.value == 0
