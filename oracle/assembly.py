"""Assembled residuals and Jacobians (scipy.sparse CSR), oracle side.

* Momentum balance (Section 3.2, weak form F_u without tractions):
  R_u(u; d) = sum_e sum_q B_q^T sigma(eps_q, g(d_q)) w_q detJ_q,
  K_t       = sum_e sum_q B_q^T C_t(eps_q, g(d_q)) B_q w_q detJ_q.
* AT2 evolution with the history field H (Section 2, the governing
  inequality with g' = -2(1-d), w = d^2, c_w = 2; history substitution as in
  the remark after the stress equation).  Dividing nothing out:
  K_dd(H) = sum [(Gc/l + 2 H_q) N N^T + Gc l grad N grad N^T] w detJ,
  b(H)    = sum 2 H_q N w detJ,
  R_d     = K_dd(H) d - b(H).
  (The printed F_d of Section 3.2 is in AT1/penalty form; for AT2 the term
  Gc/(c_w l) w'(d) becomes Gc d / l -- the reading recorded in the design
  notes.)
* Augmented phase-field block (Section 3.4, eq_staggered_NR): K_dd + K~ with
  K~ = -sum c_S N N^T w detJ.  The trial operator floors the mass coefficient
  at theta * c_q, c_q = Gc/l + 2 H_q (reading of the indefinite block).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _csr(rows, cols, vals, n):
    return sp.coo_matrix((vals.reshape(-1), (rows.reshape(-1), cols.reshape(-1))),
                         shape=(n, n)).tocsr()


def internal_force(mesh, cons, u, d, eta):
    """R_u(u; d) on all displacement DOFs (length 2*n_nodes)."""
    eps = mesh.strain(u)
    g = (1.0 - mesh.interp(d)) ** 2 + eta
    sig = cons.stress(eps, g)                                  # (Ea, 4, 3)
    fe = np.einsum("eqij,eqi,eq->ej", mesh.B(), sig, mesh.wdet)
    R = np.zeros(2 * mesh.n_nodes)
    np.add.at(R, mesh.u_dofs(), fe)
    return R


def tangent_matrix(mesh, cons, u, d, eta):
    """K_t(u; d) on all displacement DOFs (CSR)."""
    eps = mesh.strain(u)
    g = (1.0 - mesh.interp(d)) ** 2 + eta
    C = cons.tangent(eps, g)                                   # (Ea, 4, 3, 3)
    B = mesh.B()
    Ke = np.einsum("eqki,eqkl,eqlj,eq->eij", B, C, B, mesh.wdet)
    dofs = mesh.u_dofs()
    rows = np.repeat(dofs[:, :, None], 8, axis=2)
    cols = np.repeat(dofs[:, None, :], 8, axis=1)
    return _csr(rows, cols, Ke, 2 * mesh.n_nodes)


def phase_matrix(mesh, coef, Gc, l, lap=None):
    """sum [coef_q N N^T + Gc l grad N . grad N^T] w detJ, coef per QP (Ea, 4);
    lap replaces the Laplacian's factor Gc l where given (AT1: 2 Gc l / c_w)."""
    N = mesh.N                                                  # (4, 4) [q, a]
    mass = np.einsum("eq,qa,qb,eq->eab", coef, N, N, mesh.wdet)
    L = (np.einsum("eqa,eqb,eq->eab", mesh.dNdx, mesh.dNdx, mesh.wdet)
         + np.einsum("eqa,eqb,eq->eab", mesh.dNdy, mesh.dNdy, mesh.wdet))
    Ke = mass + (Gc * l if lap is None else lap) * L
    c = mesh.conn
    rows = np.repeat(c[:, :, None], 4, axis=2)
    cols = np.repeat(c[:, None, :], 4, axis=1)
    return _csr(rows, cols, Ke, mesh.n_nodes)


def phase_rhs(mesh, H):
    """b(H) = sum 2 H_q N w detJ."""
    be = np.einsum("eq,qa,eq->ea", 2.0 * H, mesh.N, mesh.wdet)
    b = np.zeros(mesh.n_nodes)
    np.add.at(b, mesh.conn, be)
    return b


def at2_coefficient(H, Gc, l):
    """c_q = Gc/l + 2 H_q, the mass coefficient of K_dd."""
    return Gc / l + 2.0 * H


def trial_coefficient(c, cS, gate, theta, floor=True):
    """Mass coefficient of K_dd + K~ (Section 3.4): c - c_S on gated points,
    c elsewhere.  With floor, a gated coefficient below theta*c is raised to
    theta*c; without, it is kept as it is (it may be negative, and K_dd + K~
    indefinite).  hits counts the gated points below theta*c either way."""
    below = gate & (c - cS < theta * c)
    if floor:
        ct = np.where(gate, np.maximum(c - cS, theta * c), c)
    else:
        ct = np.where(gate, c - cS, c)
    return ct, int(np.count_nonzero(below))
