"""Staggered load stepping of the oracle: ST (Section 3.1) and S1/S2/S3
(Sections 3.3-3.5), FP64, assembled CSR matrices, direct sparse solves.

One load step n at load factor lambda_n, from the committed state
(u_{n-1}, d_{n-1}, H_{n-1}):

0. Impose the Dirichlet data: u_D = lambda_n * unit values, d_D fixed.
1. k = 0: the phase-field solve is skipped (Section 3.1: it cannot change d
   before the displacement has moved); Newton for u at fixed d.  H is the
   history max(H_{n-1}, Psi^+(u)); the staggered residual
   r = ||R_d(d; H)|| / ||b(H)|| over free phase DOFs.
2. While r > TOL_ST: for S1/S2/S3, evaluate the softening gate
   (Section 3.5, condition_update) -- Psi^+ > Psi_crit, Psi^+ > Psi_max and
   d < 0.95, with Psi_max read as H_{n-1} and the undefined phi read as d --
   and, if any point is gated, do the first Newton iteration of the
   evolution equation with the augmented block K_dd + K~ (trial increment
   Dd); update the active energy from Dd by the half-step formulas, only
   where the gate holds and Dd > 0 (Section 3.5); then solve the evolution
   equation with that energy frozen (the AT2 equation is linear, so this
   is one solve).  ST skips the trial.  Then Newton for u at the new d, and
   recompute H and r.  The count N_stag includes the k = 0 u-solve.
   Two literal readings of the trial are options of the problem:
   * trial_operator = 1 keeps the mass coefficient c - c_S of K_dd + K~
     unfloored, so the block may be indefinite (Section 3.4 prints no floor);
     the direct solve gives its exact solution;
   * trial_update = 1 takes d^{k+1} = d^k + Dd as the phase update and skips
     the energy update and the corrected solve (the end of Section 3.5 notes
     that AT2 with a history variable needs no energy update because its
     equation is linear).  Ungated iterations take the standard solve, which
     is the same update with K~ = 0.
   phase_model = 1 swaps the evolution equation for AT1 with penalised
   irreversibility (Section 2, eq_evolution_equation; oracle/at1.py): the
   driving energy is Psi+ of the current displacement, the phase solve is a
   semismooth Newton iteration on F_d, the trial block is its matrix plus K~
   (the floor relative to its mass coefficient 2 Psi+ + gamma chi), and the
   staggered residual is ||F_d|| / ||sum 2 Psi+ N||.  The committed maximum
   of Psi+ is kept only as the gate's Psi_max, and d_{n-1} for the penalty.
3. Commit u_n, d_n, H_n = max(H_{n-1}, Psi^+(u_n)) (the predicted energy is
   never stored) and the reaction force of the loaded Dirichlet group.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.sparse.linalg as spla

from . import assembly as asm
from . import at1
from .constitutive import (Constitutive, coupling_coefficient, degradation,
                           predicted_energy, scheme_part)
from .fem import Mesh


@dataclasses.dataclass
class StepStats:
    n_stag: int = 0
    n_newton: int = 0
    n_trial: int = 0
    gated_max: int = 0
    floor_hits: int = 0
    r_stag: float = 0.0
    converged: bool = True
    force: float = 0.0
    force_xy: tuple = (0.0, 0.0)
    time_s: float = 0.0
    # size of the last staggered iteration (reporting only): ||u^k - u^{k-1}||
    # / ||u^k|| and max |d^k - d^{k-1}|; both 0 when the step took k = 0 only
    last_du: float = 0.0
    last_dd: float = 0.0


class Oracle:
    """Plain FP64 staggered solver for one workloads.Problem."""

    def __init__(self, problem, scheme=0):
        p = problem
        self.p = p
        self.scheme = int(scheme)
        m = p.material
        self.mesh = Mesh(p.nx, p.ny, p.lx, p.ly, p.elem_active)
        self.cons = Constitutive(m.E, m.nu, m.split)
        self.Gc, self.l, self.eta = m.Gc, m.l, m.eta
        self.model = int(getattr(p, "phase_model", 0))
        if self.model == 1:
            self.gamma = at1.penalty_gamma(m.Gc, m.l, p.tol_ir)
            crit = at1.psi_crit(m.Gc, m.l)
        else:
            crit = m.Gc / (2.0 * m.l)
        self.psi_crit = p.psi_crit if p.psi_crit >= 0 else crit
        nn = self.mesh.n_nodes
        # constrained displacement DOFs and their unit values
        self.u_fixed = np.zeros(2 * nn, dtype=bool)
        self.u_unit = np.zeros(2 * nn)
        for grp in p.dir_u:
            dofs = 2 * grp.nodes + grp.comps.astype(np.int64)
            self.u_fixed[dofs] = True
            self.u_unit[dofs] = grp.values
        inactive = ~self.mesh.node_active
        self.u_fixed[0::2] |= inactive
        self.u_fixed[1::2] |= inactive
        self.u_free = ~self.u_fixed
        # constrained phase DOFs
        self.d_fixed = inactive.copy()
        self.d_fixed[p.dir_d_nodes] = True
        self.d_val = np.zeros(nn)
        self.d_val[p.dir_d_nodes] = p.dir_d_values
        self.d_free = ~self.d_fixed
        grp = p.dir_u[p.load_group]
        self.load_dofs = 2 * grp.nodes + grp.comps.astype(np.int64)
        # state
        self.u = np.zeros(2 * nn)
        self.d = self.d_val.copy()
        self.d_prev = self.d.copy()          # committed d (AT1 penalty)
        Ea = self.mesh.conn.shape[0]
        self.H = np.zeros((Ea, 4))
        self.step_index = 0

    # ---------------------------------------------------------------- state
    def get_state(self):
        """(u as [2][N] SoA, d [N], H as [4][nx*ny] planes over all elements)."""
        nn = self.mesh.n_nodes
        u = np.stack([self.u[0::2], self.u[1::2]])
        Hf = np.zeros((4, self.p.nx * self.p.ny))
        Hf[:, self.mesh.elems] = self.H.T
        return u.reshape(2, nn).copy(), self.d.copy(), Hf

    def set_state(self, u_soa, d, H_planes):
        self.u = np.empty(2 * self.mesh.n_nodes)
        self.u[0::2] = u_soa[0]
        self.u[1::2] = u_soa[1]
        self.d = np.array(d, dtype=float)
        self.d_prev = self.d.copy()
        self.H = np.asarray(H_planes)[:, self.mesh.elems].T.copy()

    # ---------------------------------------------------------- components
    def residual_u(self, u, d):
        return asm.internal_force(self.mesh, self.cons, u, d, self.eta)

    def newton(self, u, d, R_ref):
        """Newton for the momentum balance at fixed d (reading: criterion
        ||R_u|| <= tol_newton * R_ref, at most 5 step halvings, max_newton)."""
        p = self.p
        f = self.u_free
        it = 0
        R = self.residual_u(u, d)[f]
        nr = np.linalg.norm(R)
        while nr > p.tol_newton * R_ref:
            if it >= p.max_newton:
                return u, it, False
            K = asm.tangent_matrix(self.mesh, self.cons, u, d, self.eta)[f][:, f]
            delta = spla.spsolve(K.tocsc(), -R)
            alpha = 1.0
            halvings = 0
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

    def energies(self, u, d):
        eps = self.mesh.strain(u)
        return self.cons.parts(eps)

    def phase_system(self, H):
        c = asm.at2_coefficient(H, self.Gc, self.l)
        K = asm.phase_matrix(self.mesh, c, self.Gc, self.l)
        b = asm.phase_rhs(self.mesh, H)
        return K, b

    def stag_residual(self, d, H):
        if self.model == 1:
            R = at1.residual(self.mesh, H, d, self.d_prev, self.Gc, self.l, self.gamma)
            nR = np.linalg.norm(R[self.d_free])
            nb = at1.driving_scale(self.mesh, H, self.d_free)
            return nR / nb if nb > 0 else nR
        K, b = self.phase_system(H)
        R = (K @ d - b)[self.d_free]
        nb = np.linalg.norm(b[self.d_free])
        nR = np.linalg.norm(R)
        return nR / nb if nb > 0 else nR

    def solve_phase(self, H, d):
        """Solve K_dd(H) d = b(H) with the Dirichlet values of d imposed
        (AT1: F_d(d; H) = 0 by semismooth Newton, H being Psi+)."""
        f = self.d_free
        out = d.copy()
        out[~f] = self.d_val[~f]
        if self.model == 1:
            out, _, ok = at1.solve(self.mesh, H, out, self.d_prev, self.Gc, self.l, self.gamma, f)
            if not ok:
                raise RuntimeError("AT1 phase solve: active set did not settle")
            return out
        K, b = self.phase_system(H)
        rhs = b[f] - K[f][:, ~f] @ out[~f]
        out[f] = spla.spsolve(K[f][:, f].tocsc(), rhs)
        return out

    def trial_increment(self, d, H, gate, psi_s):
        """First Newton iteration of the evolution equation with the augmented
        block K_dd + K~ (eq_staggered_NR), K~ only on gated points; its mass
        coefficient floored at theta c unless trial_operator = 1.  With AT1
        (phase_model = 1) K_dd is the semismooth Newton matrix of F_d at d
        and the right-hand side is -F_d(d); H is then Psi+."""
        dq = self.mesh.interp(d)
        cS = coupling_coefficient(dq, self.eta, psi_s)
        literal = int(getattr(self.p, "trial_operator", 0)) == 1
        if self.model == 1:
            chi = at1.active(self.mesh, d, self.d_prev)
            c = at1.jacobian_coefficient(H, chi, self.gamma)
            ct, hits = asm.trial_coefficient(c, cS, gate, self.p.trial_floor, floor=not literal)
            A = at1.matrix(self.mesh, ct, self.Gc, self.l)
            Rd = at1.residual(self.mesh, H, d, self.d_prev, self.Gc, self.l, self.gamma)
        else:
            c = asm.at2_coefficient(H, self.Gc, self.l)
            ct, hits = asm.trial_coefficient(c, cS, gate, self.p.trial_floor, floor=not literal)
            A = asm.phase_matrix(self.mesh, ct, self.Gc, self.l)
            K, b = self.phase_system(H)
            Rd = K @ d - b
        f = self.d_free
        dd = np.zeros_like(d)
        dd[f] = spla.spsolve(A[f][:, f].tocsc(), -Rd[f])
        return dd, hits

    def reaction(self, u, d):
        R = self.residual_u(u, d)
        grp = self.p.dir_u[self.p.load_group]
        comps = grp.comps.astype(np.int64)
        dofs = 2 * grp.nodes + comps
        fx = float(np.sum(R[dofs[comps == 0]]))
        fy = float(np.sum(R[dofs[comps == 1]]))
        return fx, fy

    # ------------------------------------------------------------ load step
    def load_step(self, lam):
        p = self.p
        t0 = time.perf_counter()
        st = StepStats()
        H_prev = self.H
        u = self.u.copy()
        u[self.u_fixed] = lam * self.u_unit[self.u_fixed]
        d = self.d.copy()
        d[self.d_fixed] = self.d_val[self.d_fixed]
        R0 = np.linalg.norm(self.residual_u(u, d)[self.u_free])
        R_ref = R0 if R0 > 0 else 1.0
        u, nit, ok = self.newton(u, d, R_ref)
        st.n_newton += nit
        st.converged &= ok
        st.n_stag = 1
        parts = self.energies(u, d)
        H = np.maximum(H_prev, parts["psi_plus"])
        drive = parts["psi_plus"] if self.model == 1 else H
        r = self.stag_residual(d, drive)
        trial_only = int(getattr(p, "trial_update", 0)) == 1
        while r > p.tol_stag and st.n_stag < p.max_stag:
            u_before, d_before = u.copy(), d.copy()
            H_hat = drive
            ng = 0
            if self.scheme != 0:
                dq = self.mesh.interp(d)
                psi = parts["psi_plus"]
                gate = (psi > self.psi_crit) & (psi > H_prev) & (dq < p.d_gate)
                ng = int(np.count_nonzero(gate))
                st.gated_max = max(st.gated_max, ng)
                if ng > 0:
                    psi_s = scheme_part(parts, self.scheme)
                    dd, hits = self.trial_increment(d, drive, gate, psi_s)
                    st.n_trial += 1
                    st.floor_hits += hits
                    if trial_only:
                        d = d + dd
                    else:
                        ddq = self.mesh.interp(dd)
                        psi_hat = predicted_energy(psi, psi_s, dq, self.eta, ddq, gate)
                        H_hat = np.maximum(drive, psi_hat)
            if not (trial_only and ng > 0):
                d = self.solve_phase(H_hat, d)
            u, nit, ok = self.newton(u, d, R_ref)
            st.n_newton += nit
            st.converged &= ok
            st.n_stag += 1
            parts = self.energies(u, d)
            H = np.maximum(H_prev, parts["psi_plus"])
            drive = parts["psi_plus"] if self.model == 1 else H
            r = self.stag_residual(d, drive)
            nu_ = np.linalg.norm(u)
            st.last_du = float(np.linalg.norm(u - u_before) / (nu_ if nu_ > 0 else 1.0))
            st.last_dd = float(np.abs(d - d_before).max()) if d.size else 0.0
        st.r_stag = r
        st.converged &= bool(r <= p.tol_stag)
        self.u, self.d, self.H = u, d, H
        self.d_prev = d.copy()
        self.step_index += 1
        fx, fy = self.reaction(u, d)
        st.force_xy = (fx, fy)
        st.force = fy if p.load_comp == 1 else fx
        st.time_s = time.perf_counter() - t0
        return st

    def run(self, n_steps=None, callback=None):
        loads = self.p.loads if n_steps is None else self.p.loads[:n_steps]
        out = []
        for lam in loads:
            st = self.load_step(float(lam))
            out.append(st)
            if callback is not None:
                callback(self, st)
        return out


__all__ = ["Oracle", "StepStats", "degradation"]
