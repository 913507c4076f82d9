"""3-D trilinear hexahedra for the oracle (Q1, 2x2x2 Gauss), plain FP64.
Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use it.

The same model and staggered schemes as the 2-D oracle, in three
dimensions: the volumetric-deviatoric split of Section 2 (eq_sigma) or the
spectral split named there, both with the full 3-D strain (principal strains
from a symmetric 3x3 eigendecomposition), AT2 with the history field, the standard scheme
(Section 3.1) and the fixed-stress schemes S1/S2/S3 with the floored trial
block, predictor and corrected solve (Sections 3.3-3.5).  The quadrature-
point algebra of the predictor (coupling coefficient, half-step energy) does
not depend on the dimension and is shared with the 2-D oracle.

A structured nx x ny x nz box; node (i, j, k) has id i + j (nx+1) +
k (nx+1)(ny+1); displacement DOFs are interleaved, dof = 3 node + comp.
Strains are engineering Voigt vectors [xx, yy, zz, 2yz, 2xz, 2xy].
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .constitutive import (coupling_coefficient, degradation, lame, neg, pos,
                           predicted_energy, scheme_part)
from .assembly import trial_coefficient

GP = 1.0 / np.sqrt(3.0)
CX = np.array([-1, 1, 1, -1, -1, 1, 1, -1], dtype=float)
CY = np.array([-1, -1, 1, 1, -1, -1, 1, 1], dtype=float)
CZ = np.array([-1, -1, -1, -1, 1, 1, 1, 1], dtype=float)


def shape(xi, eta, zeta):
    """N_a at one reference point, a = 0..7."""
    return 0.125 * (1 + CX * xi) * (1 + CY * eta) * (1 + CZ * zeta)


def shape_grad(xi, eta, zeta):
    """(dN/dxi, dN/deta, dN/dzeta) at one reference point."""
    return (0.125 * CX * (1 + CY * eta) * (1 + CZ * zeta),
            0.125 * CY * (1 + CX * xi) * (1 + CZ * zeta),
            0.125 * CZ * (1 + CX * xi) * (1 + CY * eta))


class Mesh3D:
    def __init__(self, nx, ny, nz, lx, ly, lz):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.ly, self.lz = float(lx), float(ly), float(lz)
        P = (nx + 1) * (ny + 1)
        self.n_nodes = P * (nz + 1)
        kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        n0 = (ii + jj * (nx + 1) + kk * P).reshape(-1)
        self.conn = np.stack([n0, n0 + 1, n0 + 1 + (nx + 1), n0 + (nx + 1),
                              n0 + P, n0 + 1 + P, n0 + 1 + (nx + 1) + P, n0 + (nx + 1) + P],
                             axis=1)
        E = self.conn.shape[0]
        hx, hy, hz = lx / nx, ly / ny, lz / nz
        self.N = np.zeros((8, 8))
        G = np.zeros((8, 3, 8))                          # [q, dir, a], same in every element
        for q in range(8):
            xi, eta, zeta = CX[q] * GP, CY[q] * GP, CZ[q] * GP
            self.N[q] = shape(xi, eta, zeta)
            dxi, deta, dzeta = shape_grad(xi, eta, zeta)
            G[q, 0], G[q, 1], G[q, 2] = dxi * 2 / hx, deta * 2 / hy, dzeta * 2 / hz
        self.G = G
        self.wdet = np.full((E, 8), hx * hy * hz / 8.0)
        B = np.zeros((8, 6, 24))
        for a in range(8):
            gx, gy, gz = G[:, 0, a], G[:, 1, a], G[:, 2, a]
            B[:, 0, 3 * a] = gx
            B[:, 1, 3 * a + 1] = gy
            B[:, 2, 3 * a + 2] = gz
            B[:, 3, 3 * a + 1], B[:, 3, 3 * a + 2] = gz, gy
            B[:, 4, 3 * a], B[:, 4, 3 * a + 2] = gz, gx
            B[:, 5, 3 * a], B[:, 5, 3 * a + 1] = gy, gx
        self.B = B                                       # [q, 6, 24]
        dofs = np.zeros((E, 24), dtype=np.int64)
        for c in range(3):
            dofs[:, c::3] = 3 * self.conn + c
        self.dofs = dofs

    def strain(self, u):
        return np.einsum("qij,ej->eqi", self.B, u[self.dofs])

    def interp(self, d):
        return d[self.conn] @ self.N.T


class VD3D:
    """Volumetric-deviatoric split with the full 3-D strain (Section 2)."""

    def __init__(self, E, nu):
        self.lam, self.mu, self.K = lame(E, nu)

    @staticmethod
    def _dev(eps):
        t = eps[..., 0] + eps[..., 1] + eps[..., 2]
        dn = eps[..., :3] - t[..., None] / 3.0
        dd = np.sum(dn * dn, axis=-1) + 0.5 * np.sum(eps[..., 3:] ** 2, axis=-1)
        return t, dn, dd

    def parts(self, eps):
        t, _, dd = self._dev(eps)
        pv = 0.5 * self.K * pos(t) ** 2
        pd = self.mu * dd
        return {"t": t, "psi_vol": pv, "psi_dev": pd, "psi_plus": pv + pd,
                "psi_minus": 0.5 * self.K * neg(t) ** 2}

    def stress(self, eps, g):
        """Voigt stress [xx, yy, zz, yz, xz, xy]."""
        t, dn, _ = self._dev(eps)
        s = np.zeros_like(eps)
        vol = g * self.K * pos(t) + self.K * neg(t)
        s[..., :3] = (g * 2 * self.mu)[..., None] * dn + vol[..., None]
        s[..., 3:] = (g * self.mu)[..., None] * eps[..., 3:]
        return s

    def tangent(self, eps, g):
        """C with sigma = C eps (engineering shears); tr eps > 0 strictly
        counts as active."""
        t = eps[..., 0] + eps[..., 1] + eps[..., 2]
        kf = self.K * np.where(t > 0.0, g, 1.0)
        C = np.zeros(eps.shape[:-1] + (6, 6))
        Pn = np.eye(3) - 1.0 / 3.0
        C[..., :3, :3] = (g * 2 * self.mu)[..., None, None] * Pn + kf[..., None, None]
        for i in range(3, 6):
            C[..., i, i] = g * self.mu
        return C


def _tensor3(v):
    """Engineering Voigt [xx, yy, zz, 2yz, 2xz, 2xy] -> symmetric 3x3 tensor."""
    T = np.zeros(v.shape[:-1] + (3, 3))
    T[..., 0, 0], T[..., 1, 1], T[..., 2, 2] = v[..., 0], v[..., 1], v[..., 2]
    T[..., 1, 2] = T[..., 2, 1] = 0.5 * v[..., 3]
    T[..., 0, 2] = T[..., 2, 0] = 0.5 * v[..., 4]
    T[..., 0, 1] = T[..., 1, 0] = 0.5 * v[..., 5]
    return T


def _voigt_stress(S):
    return np.stack([S[..., 0, 0], S[..., 1, 1], S[..., 2, 2], S[..., 1, 2], S[..., 0, 2],
                     S[..., 0, 1]], axis=-1)


class Spectral3D:
    """Spectral split with the full 3-D strain (named in Section 2): Psi+ =
    lam/2 <tr eps>_+^2 + mu sum <e_i>_+^2 over the principal strains e_i,
    sigma = g [lam <t>_+ I + 2 mu eps+] + lam <t>_- I + 2 mu eps-.  A trace or
    principal strain counts as positive only when strictly above zero."""

    def __init__(self, E, nu):
        self.lam, self.mu, self.K = lame(E, nu)

    def parts(self, eps):
        t = eps[..., 0] + eps[..., 1] + eps[..., 2]
        w = np.linalg.eigvalsh(_tensor3(eps))
        pv = 0.5 * self.lam * pos(t) ** 2
        pd = self.mu * np.sum(pos(w) ** 2, axis=-1)
        pm = 0.5 * self.lam * neg(t) ** 2 + self.mu * np.sum(neg(w) ** 2, axis=-1)
        return {"t": t, "psi_vol": pv, "psi_dev": pd, "psi_plus": pv + pd, "psi_minus": pm}

    def stress(self, eps, g):
        t = eps[..., 0] + eps[..., 1] + eps[..., 2]
        w, Q = np.linalg.eigh(_tensor3(eps))
        ep = np.einsum("...ik,...k,...jk->...ij", Q, pos(w), Q)
        en = np.einsum("...ik,...k,...jk->...ij", Q, neg(w), Q)
        I = np.eye(3)
        S = (g[..., None, None] * (self.lam * pos(t)[..., None, None] * I + 2 * self.mu * ep)
             + self.lam * neg(t)[..., None, None] * I + 2 * self.mu * en)
        return _voigt_stress(S)

    @staticmethod
    def _plus_map(w, Q, dE):
        """Directional derivative of eps+ = sum <e_i>_+ n_i n_i along dE: in
        the eigenbasis, entry (i, j) times (<e_i>_+ - <e_j>_+) / (e_i - e_j),
        whose limit at e_i = e_j is H(e_i)."""
        dEp = np.einsum("...ki,...kl,...lj->...ij", Q, dE, Q)
        h = (w > 0.0).astype(float)
        wi, wj = w[..., :, None], w[..., None, :]
        diff = wi - wj
        with np.errstate(divide="ignore", invalid="ignore"):
            th = np.where(diff != 0.0, (pos(wi) - pos(wj)) / np.where(diff == 0.0, 1.0, diff),
                          np.broadcast_to(h[..., :, None], diff.shape))
        return np.einsum("...ik,...kl,...jl->...ij", Q, th * dEp, Q)

    def tangent(self, eps, g):
        t = eps[..., 0] + eps[..., 1] + eps[..., 2]
        hp = (t > 0.0).astype(float)
        w, Q = np.linalg.eigh(_tensor3(eps))
        C = np.zeros(eps.shape[:-1] + (6, 6))
        I = np.eye(3)
        for col in range(6):
            dv = np.zeros(eps.shape)
            dv[..., col] = 1.0
            dt = dv[..., 0] + dv[..., 1] + dv[..., 2]
            dE = _tensor3(dv)
            dEp = self._plus_map(w, Q, dE)
            dS = (g[..., None, None] * (self.lam * (hp * dt)[..., None, None] * I
                                        + 2 * self.mu * dEp)
                  + self.lam * ((1 - hp) * dt)[..., None, None] * I
                  + 2 * self.mu * (dE - dEp))
            C[..., :, col] = _voigt_stress(dS)
        return C


def _csr(rows, cols, vals, n):
    return sp.csr_matrix((vals.reshape(-1), (rows.reshape(-1), cols.reshape(-1))), shape=(n, n))


def internal_force(mesh, cons, u, d, eta):
    eps = mesh.strain(u)
    g = degradation(mesh.interp(d), eta)
    s = cons.stress(eps, g)
    Re = np.einsum("qij,eqi,eq->ej", mesh.B, s, mesh.wdet)
    R = np.zeros(3 * mesh.n_nodes)
    np.add.at(R, mesh.dofs, Re)
    return R


def tangent_matrix(mesh, cons, u, d, eta):
    eps = mesh.strain(u)
    g = degradation(mesh.interp(d), eta)
    C = cons.tangent(eps, g)
    Ke = np.einsum("qia,eqij,qjb,eq->eab", mesh.B, C, mesh.B, mesh.wdet)
    rows = np.repeat(mesh.dofs[:, :, None], 24, axis=2)
    cols = np.repeat(mesh.dofs[:, None, :], 24, axis=1)
    return _csr(rows, cols, Ke, 3 * mesh.n_nodes)


def phase_matrix(mesh, coef, Gc, l):
    """sum [coef_q N N^T + Gc l grad N . grad N^T] w detJ."""
    mass = np.einsum("eq,qa,qb,eq->eab", coef, mesh.N, mesh.N, mesh.wdet)
    lap = np.einsum("qia,qib,eq->eab", mesh.G, mesh.G, mesh.wdet)
    Ke = mass + Gc * l * lap
    rows = np.repeat(mesh.conn[:, :, None], 8, axis=2)
    cols = np.repeat(mesh.conn[:, None, :], 8, axis=1)
    return _csr(rows, cols, Ke, mesh.n_nodes)


def phase_rhs(mesh, H):
    be = np.einsum("eq,qa,eq->ea", 2.0 * H, mesh.N, mesh.wdet)
    b = np.zeros(mesh.n_nodes)
    np.add.at(b, mesh.conn, be)
    return b


@dataclasses.dataclass
class StepStats3D:
    n_stag: int = 0
    n_trial: int = 0
    converged: bool = True
    r_stag: float = 0.0
    force: float = 0.0
    time_s: float = 0.0


class Oracle3D:
    """ST and S1/S2/S3 on a workloads.Problem3D (AT2, history field, floored
    trial block with predict -> correct), the 2-D oracle's steps in 3-D."""

    def __init__(self, problem, scheme=0):
        p = problem
        self.p, self.scheme = p, int(scheme)
        m = p.material
        self.mesh = Mesh3D(p.nx, p.ny, p.nz, p.lx, p.ly, p.lz)
        self.cons = VD3D(m.E, m.nu) if int(m.split) == 0 else Spectral3D(m.E, m.nu)
        self.Gc, self.l, self.eta = m.Gc, m.l, m.eta
        self.psi_crit = p.psi_crit if p.psi_crit >= 0 else m.Gc / (2.0 * m.l)
        nn = self.mesh.n_nodes
        self.u_fixed = np.zeros(3 * nn, dtype=bool)
        self.u_unit = np.zeros(3 * nn)
        for grp in p.dir_u:
            dofs = 3 * grp.nodes + grp.comps.astype(np.int64)
            self.u_fixed[dofs] = True
            self.u_unit[dofs] = grp.values
        self.u_free = ~self.u_fixed
        self.d_fixed = np.zeros(nn, dtype=bool)
        self.d_fixed[p.dir_d_nodes] = True
        self.d_val = np.zeros(nn)
        self.d_val[p.dir_d_nodes] = p.dir_d_values
        self.d_free = ~self.d_fixed
        self.u = np.zeros(3 * nn)
        self.d = self.d_val.copy()
        self.H = np.zeros((self.mesh.conn.shape[0], 8))

    def residual_u(self, u, d):
        return internal_force(self.mesh, self.cons, u, d, self.eta)

    def newton(self, u, d, R_ref):
        p, f, it = self.p, self.u_free, 0
        R = self.residual_u(u, d)[f]
        nr = np.linalg.norm(R)
        while nr > p.tol_newton * R_ref:
            if it >= p.max_newton:
                return u, it, False
            K = tangent_matrix(self.mesh, self.cons, u, d, self.eta)[f][:, f]
            delta = spla.spsolve(K.tocsc(), -R)
            alpha, halvings = 1.0, 0
            while True:
                ut = u.copy()
                ut[f] += alpha * delta
                Rt = self.residual_u(ut, d)[f]
                nt = np.linalg.norm(Rt)
                if nt < nr or halvings == 5:
                    break
                alpha *= 0.5
                halvings += 1
            u, R, nr = ut, Rt, nt
            it += 1
        return u, it, True

    def phase_system(self, H):
        K = phase_matrix(self.mesh, self.Gc / self.l + 2.0 * H, self.Gc, self.l)
        return K, phase_rhs(self.mesh, H)

    def stag_residual(self, d, H):
        K, b = self.phase_system(H)
        nR = np.linalg.norm((K @ d - b)[self.d_free])
        nb = np.linalg.norm(b[self.d_free])
        return nR / nb if nb > 0 else nR

    def solve_phase(self, H, d):
        K, b = self.phase_system(H)
        f = self.d_free
        out = d.copy()
        out[~f] = self.d_val[~f]
        out[f] = spla.spsolve(K[f][:, f].tocsc(), b[f] - K[f][:, ~f] @ out[~f])
        return out

    def trial_increment(self, d, H, gate, psi_s):
        dq = self.mesh.interp(d)
        c = self.Gc / self.l + 2.0 * H
        ct, _ = trial_coefficient(c, coupling_coefficient(dq, self.eta, psi_s), gate,
                                  self.p.trial_floor)
        A = phase_matrix(self.mesh, ct, self.Gc, self.l)
        K, b = self.phase_system(H)
        f = self.d_free
        dd = np.zeros_like(d)
        dd[f] = spla.spsolve(A[f][:, f].tocsc(), -(K @ d - b)[f])
        return dd

    def load_step(self, lam):
        p, t0, st = self.p, time.perf_counter(), StepStats3D()
        H_prev = self.H
        u = self.u.copy()
        u[self.u_fixed] = lam * self.u_unit[self.u_fixed]
        d = self.d.copy()
        d[self.d_fixed] = self.d_val[self.d_fixed]
        R0 = np.linalg.norm(self.residual_u(u, d)[self.u_free])
        R_ref = R0 if R0 > 0 else 1.0
        u, _, ok = self.newton(u, d, R_ref)
        st.converged &= ok
        st.n_stag = 1
        parts = self.cons.parts(self.mesh.strain(u))
        H = np.maximum(H_prev, parts["psi_plus"])
        r = self.stag_residual(d, H)
        while r > p.tol_stag and st.n_stag < p.max_stag:
            H_hat = H
            if self.scheme != 0:
                dq = self.mesh.interp(d)
                psi = parts["psi_plus"]
                gate = (psi > self.psi_crit) & (psi > H_prev) & (dq < p.d_gate)
                if np.any(gate):
                    psi_s = scheme_part(parts, self.scheme)
                    dd = self.trial_increment(d, H, gate, psi_s)
                    st.n_trial += 1
                    psi_hat = predicted_energy(psi, psi_s, dq, self.eta, self.mesh.interp(dd),
                                               gate)
                    H_hat = np.maximum(H, psi_hat)
            d = self.solve_phase(H_hat, d)
            u, _, ok = self.newton(u, d, R_ref)
            st.converged &= ok
            st.n_stag += 1
            parts = self.cons.parts(self.mesh.strain(u))
            H = np.maximum(H_prev, parts["psi_plus"])
            r = self.stag_residual(d, H)
        st.r_stag = r
        st.converged &= bool(r <= p.tol_stag)
        self.u, self.d, self.H = u, d, H
        R = self.residual_u(u, d)
        grp = p.dir_u[p.load_group]
        dofs = 3 * grp.nodes + grp.comps.astype(np.int64)
        st.force = float(np.sum(R[dofs[grp.comps == p.load_comp]]))
        st.time_s = time.perf_counter() - t0
        return st
