"""AT1 phase field with penalised irreversibility for the oracle (plain FP64,
assembled CSR, direct sparse solves).  Test infrastructure: only the tests,
the smoke check and the benchmark's CPU baseline use it.

Section 2 (eq_evolution_equation) replaces the history field by a penalty on
decreasing damage, for AT1 as well as AT2.  With AT1, w(d) = d and
c_w = 8/3, and the weak form printed in Section 3.2 (F_d) reads, per
quadrature point q of every element,

    F_d = sum_q { N [-2 (1 - d_q) Psi+_q + Gc / (c_w l)
                     + gamma <d_q - d_{n-1,q}>_-]
                  + (2 Gc l / c_w) grad N . grad d } w detJ,

with <x>_- = min(x, 0) and gamma = 27 Gc / (64 l tol_ir^2) (Section 2,
tol_ir = 0.01).  Psi+ is the active energy of the current displacement:
the penalty, not a history maximum, keeps d from decreasing.

F_d is piecewise linear in d, with kinks where d_q crosses d_{n-1,q}.  Its
derivative (the semismooth Newton matrix) is

    J = sum_q [(2 Psi+_q + gamma chi_q) N N^T + (2 Gc l / c_w) grad N grad N^T] w detJ,

chi_q = 1 where d_q < d_{n-1,q}.  Newton with J is exact once the active
set stops changing, so the solve stops when two successive iterates have
the same active set.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import assembly as asm

C_W = 8.0 / 3.0


def penalty_gamma(Gc, l, tol_ir):
    """gamma = 27 Gc / (64 l tol_ir^2) (Section 2)."""
    return 27.0 * Gc / (64.0 * l * tol_ir ** 2)


def psi_crit(Gc, l):
    """Psi_crit = Gc / (c_w l) of the gate (Section 3.5) for AT1."""
    return Gc / (C_W * l)


def _lap_coef(Gc, l):
    return 2.0 * Gc * l / C_W


def residual(mesh, psi, d, d_prev, Gc, l, gamma):
    """Nodal F_d(d; Psi+) (the printed AT1 form, boundary term zero)."""
    dq = mesh.interp(d)
    dpq = mesh.interp(d_prev)
    f = -2.0 * (1.0 - dq) * psi + Gc / (C_W * l) + gamma * np.minimum(dq - dpq, 0.0)
    be = np.einsum("eq,qa,eq->ea", f, mesh.N, mesh.wdet)
    de = d[mesh.conn]                                           # (Ea, 4)
    gx = np.einsum("eqa,ea->eq", mesh.dNdx, de)
    gy = np.einsum("eqa,ea->eq", mesh.dNdy, de)
    le = (np.einsum("eqa,eq,eq->ea", mesh.dNdx, gx, mesh.wdet)
          + np.einsum("eqa,eq,eq->ea", mesh.dNdy, gy, mesh.wdet))
    R = np.zeros(mesh.n_nodes)
    np.add.at(R, mesh.conn, be + _lap_coef(Gc, l) * le)
    return R


def active(mesh, d, d_prev):
    """chi_q = 1 where the penalty acts (d_q < d_{n-1,q})."""
    return mesh.interp(d) < mesh.interp(d_prev)


def jacobian_coefficient(psi, chi, gamma):
    """Mass coefficient 2 Psi+_q + gamma chi_q of J."""
    return 2.0 * psi + gamma * chi


def matrix(mesh, coef, Gc, l):
    """sum [coef_q N N^T + (2 Gc l / c_w) grad N grad N^T] w detJ."""
    return asm.phase_matrix(mesh, coef, Gc, l, lap=_lap_coef(Gc, l))


def driving_scale(mesh, psi, free):
    """||sum_q 2 Psi+_q N w detJ|| over free phase DOFs: the staggered
    residual's normaliser, the AT2 right-hand side's counterpart."""
    return float(np.linalg.norm(asm.phase_rhs(mesh, psi)[free]))


def solve(mesh, psi, d0, d_prev, Gc, l, gamma, free, max_it=60):
    """Semismooth Newton for F_d(d; Psi+) = 0 from d0 (fixed DOFs kept).
    Returns (d, iterations, converged)."""
    d = d0.copy()
    chi = active(mesh, d, d_prev)
    for it in range(1, max_it + 1):
        R = residual(mesh, psi, d, d_prev, Gc, l, gamma)
        J = matrix(mesh, jacobian_coefficient(psi, chi, gamma), Gc, l)
        d[free] -= spla.spsolve(J[free][:, free].tocsc(), R[free])
        chi_new = active(mesh, d, d_prev)
        if np.array_equal(chi_new, chi):
            return d, it, True
        chi = chi_new
    return d, max_it, False
