"""3-D operator kernels on the GPU against the oracle's hexahedra, through
the C ABI (include/phasefield3d.h): internal force, tangent apply, phase
apply and the quadrature-point update, on meshes of one block, several
blocks with a ragged tail, and one element.  The same per-index functions
are checked on the host, grid by grid, by tests/test_hex3d_kernels_host.py.

Every index these kernels' grids compute has been checked against exact-
size buffers on the CPU (tests/hex3d_asan_main.cpp) before their first
device run.  PF_GPU3D=0 in the environment skips this file.
"""
import os

import numpy as np
import pytest

from oracle import hex3d as H3

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("PF_GPU3D") == "0",
                                 reason="3-D GPU tests switched off (PF_GPU3D=0)")]

MESHES = [(3, 2, 2), (9, 7, 5), (17, 5, 3), (1, 1, 1)]


class Box:
    def __init__(self, nx, ny, nz, split=0):
        import workloads as W
        self.nx, self.ny, self.nz = nx, ny, nz
        self.lx, self.ly, self.lz = 1.3, 0.7, 0.45
        self.material = W.Material(E=2.1e5, nu=0.3, Gc=2.7, l=0.05, eta=1e-6, split=split)


def soa(v):
    return np.concatenate([v[0::3], v[1::3], v[2::3]])


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def setup(gpu_lib, shape, seed, split=0):
    b = Box(*shape, split=split)
    ops = gpu_lib.Hex3DOps(b)
    om = H3.Mesh3D(b.nx, b.ny, b.nz, b.lx, b.ly, b.lz)
    return b, ops, om, np.random.default_rng(seed)


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("shape", MESHES)
def test_internal_force_and_tangent_3d(gpu_lib, shape, split):
    import torch
    b, ops, om, rng = setup(gpu_lib, shape, sum(shape), split)
    m = b.material
    cons = (H3.VD3D if split == 0 else H3.Spectral3D)(m.E, m.nu)
    N = om.n_nodes
    u = rng.normal(size=3 * N) * 1e-3
    d = rng.uniform(0, 1, size=N)
    p = rng.normal(size=3 * N)
    R_orc = soa(H3.internal_force(om, cons, u, d, m.eta))
    q_orc = soa(H3.tangent_matrix(om, cons, u, d, m.eta) @ p)
    R = torch.full((3 * N,), float("nan"), dtype=torch.float64, device="cuda")
    q = torch.full_like(R, float("nan"))
    ops.internal_force(dev(soa(u)), dev(d), R)
    ops.tangent_apply(dev(soa(u)), dev(d), dev(soa(p)), q)
    np.testing.assert_allclose(host(R), R_orc, rtol=0, atol=1e-12 * np.abs(R_orc).max())
    np.testing.assert_allclose(host(q), q_orc, rtol=0, atol=1e-12 * np.abs(q_orc).max())


@pytest.mark.parametrize("split", [0, 1])
def test_internal_force_3d_element_once_tiles(gpu_lib, split):
    """A mesh whose tiles fill the GPU (16 x 2 x 1020 elements: 2 x 1 tiles
    of node columns, 128 chunks of planes, ragged in x and z), where the
    internal force runs element-once instead of as a node gather."""
    import torch
    b, ops, om, rng = setup(gpu_lib, (16, 2, 1020), 1038 + split, split)
    m = b.material
    cons = (H3.VD3D if split == 0 else H3.Spectral3D)(m.E, m.nu)
    N = om.n_nodes
    u = rng.normal(size=3 * N) * 1e-3
    d = rng.uniform(0, 1, size=N)
    R_orc = soa(H3.internal_force(om, cons, u, d, m.eta))
    R = torch.full((3 * N,), float("nan"), dtype=torch.float64, device="cuda")
    ops.internal_force(dev(soa(u)), dev(d), R)
    np.testing.assert_allclose(host(R), R_orc, rtol=0, atol=1e-12 * np.abs(R_orc).max())


@pytest.mark.parametrize("shape", MESHES)
def test_phase_apply_3d(gpu_lib, shape):
    import torch
    b, ops, om, rng = setup(gpu_lib, shape, 7 + sum(shape))
    N, E = om.n_nodes, om.conn.shape[0]
    coef = rng.uniform(0.1, 50.0, size=(E, 8))
    p = rng.normal(size=N)
    q_orc = H3.phase_matrix(om, coef, b.material.Gc, b.material.l) @ p
    q = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    ops.phase_apply(dev(coef.T.reshape(-1)), dev(p), q)
    np.testing.assert_allclose(host(q), q_orc, rtol=0, atol=1e-12 * np.abs(q_orc).max())


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_qp_update_3d(gpu_lib, scheme, split):
    import torch
    b, ops, om, rng = setup(gpu_lib, (9, 7, 5), 100 + scheme, split)
    m = b.material
    cons = (H3.VD3D if split == 0 else H3.Spectral3D)(m.E, m.nu)
    N, E = om.n_nodes, om.conn.shape[0]
    u = rng.normal(size=3 * N) * 2e-3
    d = rng.uniform(0, 1, size=N)
    parts = cons.parts(om.strain(u))
    psi = parts["psi_plus"]
    Hprev = np.where(rng.uniform(size=psi.shape) < 0.5, psi * 0.5, psi * 1.5)
    gate = ((psi > m.Gc / (2 * m.l)) & (psi > Hprev) & (om.interp(d) < 0.95) & (scheme != 0))
    ps = {0: np.zeros_like(psi), 1: parts["psi_vol"], 2: parts["psi_dev"], 3: psi}[scheme]
    H = torch.full((8 * E,), float("nan"), dtype=torch.float64, device="cuda")
    PS = torch.full_like(H, float("nan"))
    fl = torch.zeros(E, dtype=torch.int16, device="cuda")
    ops.qp_update(scheme, -1.0, 0.95, dev(soa(u)), dev(d), dev(Hprev.T.reshape(-1)), H, PS, fl)
    np.testing.assert_allclose(host(H).reshape(8, E).T, np.maximum(Hprev, psi), rtol=1e-12, atol=0)
    np.testing.assert_allclose(host(PS).reshape(8, E).T, ps, rtol=1e-12,
                               atol=1e-14 * max(ps.max(), 1))
    flags = host(fl).view(np.uint16)
    bits_t = np.stack([(flags >> q) & 1 for q in range(8)], axis=1).astype(bool)
    bits_g = np.stack([(flags >> (q + 8)) & 1 for q in range(8)], axis=1).astype(bool)
    np.testing.assert_array_equal(bits_t, parts["t"] > 0)
    np.testing.assert_array_equal(bits_g, gate)
    from oracle.constitutive import predicted_energy
    dd = rng.normal(size=N) * 0.05
    Hh = torch.full_like(H, float("nan"))
    ops.predictor(dev(d), dev(dd), H, PS, fl, Hh)
    Hhat_orc = np.maximum(np.maximum(Hprev, psi),
                          predicted_energy(psi, ps, om.interp(d), m.eta, om.interp(dd), gate))
    np.testing.assert_allclose(host(Hh).reshape(8, E).T, Hhat_orc, rtol=1e-12, atol=0)


@pytest.mark.parametrize("split", [0, 1])
def test_diagonals_rhs_and_coefficients_3d(gpu_lib, split):
    import torch
    from oracle.assembly import trial_coefficient
    from oracle.constitutive import coupling_coefficient
    b, ops, om, rng = setup(gpu_lib, (9, 7, 5), 31, split)
    m = b.material
    cons = (H3.VD3D if split == 0 else H3.Spectral3D)(m.E, m.nu)
    N, E = om.n_nodes, om.conn.shape[0]
    u = rng.normal(size=3 * N) * 5e-4
    d = rng.uniform(0, 0.9, size=N)
    coef = rng.uniform(0.1, 50.0, size=(E, 8))
    Hq = rng.uniform(0.0, 30.0, size=(E, 8))
    Dt = torch.full((3 * N,), float("nan"), dtype=torch.float64, device="cuda")
    Dp = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    bb = torch.full_like(Dp, float("nan"))
    ops.tangent_diag(dev(soa(u)), dev(d), Dt)
    ops.phase_diag(dev(coef.T.reshape(-1)), Dp)
    ops.phase_rhs(dev(Hq.T.reshape(-1)), bb)
    np.testing.assert_allclose(host(Dt), soa(H3.tangent_matrix(om, cons, u, d, m.eta).diagonal()),
                               rtol=1e-12)
    np.testing.assert_allclose(host(Dp), H3.phase_matrix(om, coef, m.Gc, m.l).diagonal(),
                               rtol=1e-12)
    np.testing.assert_allclose(host(bb), H3.phase_rhs(om, Hq), rtol=1e-12)
    # trial coefficient from the kernel's own QP update (S3, floored)
    parts = cons.parts(om.strain(u))
    psi = parts["psi_plus"]
    Hprev = np.where(rng.uniform(size=psi.shape) < 0.5, psi * 0.5, psi * 1.5)
    H = torch.full((8 * E,), float("nan"), dtype=torch.float64, device="cuda")
    PS = torch.full_like(H, float("nan"))
    fl = torch.zeros(E, dtype=torch.int16, device="cuda")
    ops.qp_update(3, 0.0, 0.95, dev(soa(u)), dev(d), dev(Hprev.T.reshape(-1)), H, PS, fl)
    co = torch.full_like(H, float("nan"))
    ops.phase_coef(H, co, trial=(0.3, 1, PS, fl, dev(d)))
    Hn = np.maximum(Hprev, psi)
    gate = (psi > 0.0) & (psi > Hprev) & (om.interp(d) < 0.95)
    c = m.Gc / m.l + 2.0 * Hn
    ct, _ = trial_coefficient(c, coupling_coefficient(om.interp(d), m.eta, psi), gate, 0.3)
    np.testing.assert_allclose(host(co).reshape(8, E).T, ct, rtol=1e-11,
                               atol=1e-12 * np.abs(c).max())


@pytest.mark.parametrize("case", ["cube_s1", "cube_unload_s1", "slab_st", "slab_s3", "slab2_s1",
                                  "shear_s1", "tilted_st", "tilted_s1"])
def test_load_steps_3d(gpu_lib, case):
    """pf3d_load_step against the 3-D oracle under the 2-D parity protocol."""
    import dataclasses

    import workloads as W
    from oracle.hex3d import Oracle3D
    if case == "cube_s1":
        p, scheme = W.uniaxial_bar3d(n=2, l=0.03, du=5e-3, steps=4), 1
    elif case == "cube_unload_s1":
        p = W.uniaxial_bar3d(n=2, l=0.03, du=5e-3, steps=5)
        p = dataclasses.replace(p, loads=np.array([5e-3, 1e-2, 1.4e-2, 7e-3, 1.2e-2, 1.5e-2]))
        scheme = 1
    elif case == "shear_s1":
        p, scheme = W.slab_from_panel(W.shear_panel(n=8, l=0.2, du=4e-3, steps=2), 1, 0.1), 1
    elif case in ("tilted_st", "tilted_s1"):
        p, scheme = W.tilted_notched_box3d(), (0 if case == "tilted_st" else 1)
    elif case == "slab2_s1":
        p, scheme = W.slab_from_panel(W.tension_panel(n=12, l=0.2, du=2e-3, steps=2), 2, 0.1), 1
    else:
        p = W.slab_from_panel(W.tension_panel(n=8, l=0.2, du=2e-3, steps=2), 1, 0.1)
        scheme = 0 if case == "slab_st" else 3
    ctx = gpu_lib.Hex3DContext(p, scheme=scheme)
    orc = Oracle3D(p, scheme)
    forces, oforces = [], []
    for lam in p.loads:
        sg = ctx.load_step(float(lam))
        so = orc.load_step(float(lam))
        assert sg["converged"] and so.converged
        assert abs(sg["n_stag"] - so.n_stag) <= 1
        forces.append(ctx.reaction_force(p.load_group)[p.load_comp])
        oforces.append(so.force)
        if sg["n_stag"] == so.n_stag:
            u, d, _ = ctx.get_state()
            ou = np.stack([orc.u[0::3], orc.u[1::3], orc.u[2::3]])
            assert np.linalg.norm(u - ou) <= 1e-7 * np.linalg.norm(ou)
            assert np.abs(d - orc.d).max() <= 1e-5
    ctx.close()
    peak = max(abs(x) for x in oforces)
    np.testing.assert_allclose(forces, oforces, rtol=0, atol=1e-7 * peak)


def test_checkpoint_and_resume_3d(gpu_lib):
    """A state saved after step 2 and resumed in a fresh context reproduces
    step 3 of the uninterrupted run bit for bit (deterministic reductions)."""
    import workloads as W
    p = W.slab_from_panel(W.tension_panel(n=8, l=0.2, du=2e-3, steps=3), 1, 0.1)
    a, b = gpu_lib.Hex3DContext(p, scheme=1), gpu_lib.Hex3DContext(p, scheme=1)
    for lam in p.loads[:2]:
        a.load_step(float(lam))
    b.set_state(*a.get_state())
    sa, sb = a.load_step(float(p.loads[2])), b.load_step(float(p.loads[2]))
    assert sa["n_stag"] == sb["n_stag"] and sa["force"] == sb["force"] and sa["n_trial"] > 0
    for x, y in zip(a.get_state(), b.get_state()):
        assert np.array_equal(x, y)
    a.close()
    b.close()
