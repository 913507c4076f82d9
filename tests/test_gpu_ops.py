"""Kernel-level parity: each HIP operator against the oracle's assembled FP64
operator on the same seeded inputs (GPU).

Meshes are ragged (several wave strips and row chunks plus a partial one) and
one case masks out elements; both work decompositions run (column marching,
march_rows 0, and LDS tiles, march_rows 1).  Tolerances are relative to the
operator scale: both sides are FP64 and differ only in summation order.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assembly as asm
from oracle import constitutive as C
from oracle.staggered import Oracle

pytestmark = pytest.mark.gpu

SHAPES = [(37, 23), (130, 67), (5, 3)]


def to_soa(u_inter):
    return np.stack([u_inter[0::2], u_inter[1::2]]).reshape(-1)


def to_inter(u_soa, N):
    u = np.empty(2 * N)
    u[0::2] = u_soa[:N]
    u[1::2] = u_soa[N:]
    return u


def make(pf, nx, ny, masked=False, scheme=0, split=0, march_rows=0):
    p = W.tension_panel(n=4, l=0.05, split=split)
    p.nx, p.ny, p.lx, p.ly = nx, ny, 1.3, 0.7
    p.dir_u = [W.DirichletU(np.array([0], np.int64), np.array([0], np.int8), np.zeros(1)),
               W.DirichletU(np.array([1], np.int64), np.array([1], np.int8), np.zeros(1))]
    p.dir_d_nodes = np.zeros(0, np.int64)
    p.dir_d_values = np.zeros(0)
    if masked:
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        p.elem_active = (~((ii >= nx // 2) & (jj >= ny // 2))).astype(np.uint8).reshape(-1)
    ctx = pf.Context(p, scheme=scheme, march_rows=march_rows)
    orc = Oracle(p, scheme)
    return p, ctx, orc


def dev(x, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("rows", [0, 1])
@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("masked", [False, True])
def test_internal_force_and_tangent(gpu_lib, nx, ny, masked, split, rows):
    import torch
    p, ctx, orc = make(gpu_lib, nx, ny, masked, split=split, march_rows=rows)
    N = p.n_nodes
    rng = np.random.default_rng(nx * 100 + ny)
    u = rng.normal(size=2 * N) * 1e-3
    d = rng.uniform(0, 1, size=N)
    pv = rng.normal(size=2 * N)
    m = orc.mesh
    R_orc = asm.internal_force(m, orc.cons, u, d, p.material.eta)
    K = asm.tangent_matrix(m, orc.cons, u, d, p.material.eta)
    q_orc = K @ pv
    uG, dG, pG = dev(to_soa(u)), dev(d), dev(to_soa(pv))
    R = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
    q = torch.zeros_like(R)
    ctx.op_internal_force(uG, dG, R)
    ctx.op_tangent_apply(uG, dG, pG, q)
    R_gpu = to_inter(host(R), N)
    q_gpu = to_inter(host(q), N)
    scale_R = np.abs(R_orc).max()
    scale_q = np.abs(q_orc).max()
    np.testing.assert_allclose(R_gpu, R_orc, rtol=0, atol=1e-12 * scale_R)
    np.testing.assert_allclose(q_gpu, q_orc, rtol=0, atol=1e-12 * scale_q)
    ctx.close()


@pytest.mark.parametrize("rows", [0, 1])
@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("masked", [False, True])
def test_phase_apply(gpu_lib, nx, ny, masked, rows):
    import torch
    p, ctx, orc = make(gpu_lib, nx, ny, masked, march_rows=rows)
    N, E = p.n_nodes, p.n_elems
    rng = np.random.default_rng(7 + nx)
    coef_planes = rng.uniform(0.1, 50.0, size=(4, E))
    pv = rng.normal(size=N)
    m = orc.mesh
    A = asm.phase_matrix(m, coef_planes[:, m.elems].T, p.material.Gc, p.material.l)
    q_orc = A @ pv
    q = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.op_phase_apply(dev(coef_planes.reshape(-1)), dev(pv), q)
    np.testing.assert_allclose(host(q), q_orc, rtol=0, atol=1e-12 * np.abs(q_orc).max())
    ctx.close()


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_qp_update_and_predictor(gpu_lib, scheme, split):
    import torch
    nx, ny = 41, 19
    p, ctx, orc = make(gpu_lib, nx, ny, masked=False, scheme=scheme, split=split)
    N, E = p.n_nodes, p.n_elems
    rng = np.random.default_rng(100 + scheme)
    u = rng.normal(size=2 * N) * 2e-3
    d = rng.uniform(0, 1, size=N)
    m = orc.mesh
    parts = orc.energies(u, d)
    psi = parts["psi_plus"]
    # history: a mix of points below and above the current energy
    Hprev = np.where(rng.uniform(size=psi.shape) < 0.5, psi * 0.5, psi * 1.5)
    H_orc = np.maximum(Hprev, psi)
    psi_s = C.scheme_part(parts, scheme)
    dq = m.interp(d)
    psi_crit = p.material.Gc / (2 * p.material.l)
    gate = (psi > psi_crit) & (psi > Hprev) & (dq < 0.95) & (scheme != 0)
    tbit = parts["t"] > 0

    uG, dG = dev(to_soa(u)), dev(d)
    HpG = dev(Hprev.T.reshape(-1))
    H = torch.zeros(4 * E, dtype=torch.float64, device="cuda")
    PS = torch.zeros_like(H)
    fl = torch.zeros(E, dtype=torch.uint8, device="cuda")
    ng = ctx.op_qp_update(scheme, uG, dG, HpG, H, PS, fl)
    # spectral: the smaller eigenvalue t/2 - r cancels when |e2| << |e1|, so
    # the two sides' strain roundings (edge differences vs. B matrices) show
    # up at ~1e-12 relative in psi
    rt = 1e-13 if split == 0 else 1e-11
    np.testing.assert_allclose(host(H).reshape(4, E).T, H_orc, rtol=rt, atol=0)
    np.testing.assert_allclose(host(PS).reshape(4, E).T, psi_s, rtol=max(rt, 1e-12),
                               atol=1e-14 * max(psi_s.max(), 1))
    flags = host(fl)
    bits_t = np.stack([(flags >> q) & 1 for q in range(4)], axis=1).astype(bool)
    bits_g = np.stack([(flags >> (q + 4)) & 1 for q in range(4)], axis=1).astype(bool)
    np.testing.assert_array_equal(bits_t, tbit)
    np.testing.assert_array_equal(bits_g, gate)
    assert ng == int(gate.sum())
    if scheme != 0:
        assert ng > 0
        dd = rng.normal(size=N) * 0.05
        ddq = m.interp(dd)
        Hhat_orc = np.maximum(H_orc, C.predicted_energy(psi, psi_s, dq, p.material.eta, ddq, gate))
        Hh = torch.zeros_like(H)
        ctx.op_predictor(dG, dev(dd), H, PS, fl, Hh)
        np.testing.assert_allclose(host(Hh).reshape(4, E).T, Hhat_orc, rtol=max(rt, 1e-12), atol=0)
    ctx.close()
