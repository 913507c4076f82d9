"""Q1 (bilinear quadrilateral) geometry for the oracle.

Generic isoparametric element: shape functions N_a(xi, eta) on [-1,1]^2, the
Jacobian from the element's nodal coordinates, and 2x2 Gauss quadrature with
points (-,-), (+,-), (+,+), (-,+) at +-1/sqrt(3), weights 1.  The paper uses
Q1 elements in deal.II and is silent on quadrature; 2x2 Gauss is the reading
recorded in the design notes.

Displacement DOFs are interleaved: dof(node, comp) = 2*node + comp.
"""
from __future__ import annotations

import numpy as np

GP = 1.0 / np.sqrt(3.0)
QP_XI = np.array([-GP, GP, GP, -GP])
QP_ETA = np.array([-GP, -GP, GP, GP])
QP_W = np.ones(4)

# reference corner coordinates of nodes 0..3
CORNER_XI = np.array([-1.0, 1.0, 1.0, -1.0])
CORNER_ETA = np.array([-1.0, -1.0, 1.0, 1.0])


def shape(xi, eta):
    """N_a(xi, eta), a = 0..3 -> array (..., 4)."""
    xi = np.asarray(xi, dtype=float)[..., None]
    eta = np.asarray(eta, dtype=float)[..., None]
    return 0.25 * (1.0 + CORNER_XI * xi) * (1.0 + CORNER_ETA * eta)


def shape_ref_grad(xi, eta):
    """(dN/dxi, dN/deta) -> arrays (..., 4) each."""
    xi = np.asarray(xi, dtype=float)[..., None]
    eta = np.asarray(eta, dtype=float)[..., None]
    dxi = 0.25 * CORNER_XI * (1.0 + CORNER_ETA * eta)
    deta = 0.25 * CORNER_ETA * (1.0 + CORNER_XI * xi)
    return dxi, deta


class Mesh:
    """Structured nx x ny rectangle with an optional element mask."""

    def __init__(self, nx, ny, lx, ly, elem_active=None):
        self.nx, self.ny, self.lx, self.ly = int(nx), int(ny), float(lx), float(ly)
        self.n_nodes = (nx + 1) * (ny + 1)
        jj, ii = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
        self.xy = np.stack([(ii * (lx / nx)).reshape(-1), (jj * (ly / ny)).reshape(-1)], axis=1)
        ej, ei = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        ei = ei.reshape(-1)
        ej = ej.reshape(-1)
        n0 = ei + ej * (nx + 1)
        self.conn_all = np.stack([n0, n0 + 1, n0 + 1 + (nx + 1), n0 + (nx + 1)], axis=1)
        if elem_active is None:
            self.active = np.ones(nx * ny, dtype=bool)
        else:
            self.active = np.asarray(elem_active).astype(bool).reshape(-1)
        self.elems = np.nonzero(self.active)[0]          # ids of active elements
        self.conn = self.conn_all[self.elems]            # (Ea, 4)
        node_active = np.zeros(self.n_nodes, dtype=bool)
        node_active[self.conn.reshape(-1)] = True
        self.node_active = node_active
        self._geometry()

    def _geometry(self):
        X = self.xy[self.conn]                           # (Ea, 4, 2)
        Ea = X.shape[0]
        self.N = np.zeros((4, 4))                        # N[q, a]
        self.dNdx = np.zeros((Ea, 4, 4))                 # [e, q, a]
        self.dNdy = np.zeros((Ea, 4, 4))
        self.wdet = np.zeros((Ea, 4))
        for q in range(4):
            self.N[q] = shape(QP_XI[q], QP_ETA[q])
            dxi, deta = shape_ref_grad(QP_XI[q], QP_ETA[q])
            J11 = X[:, :, 0] @ dxi        # dx/dxi
            J12 = X[:, :, 1] @ dxi        # dy/dxi
            J21 = X[:, :, 0] @ deta       # dx/deta
            J22 = X[:, :, 1] @ deta       # dy/deta
            det = J11 * J22 - J12 * J21
            # [dN/dx; dN/dy] = J^{-T} [dN/dxi; dN/deta]
            inv11 = J22 / det
            inv12 = -J12 / det
            inv21 = -J21 / det
            inv22 = J11 / det
            self.dNdx[:, q, :] = inv11[:, None] * dxi[None, :] + inv12[:, None] * deta[None, :]
            self.dNdy[:, q, :] = inv21[:, None] * dxi[None, :] + inv22[:, None] * deta[None, :]
            self.wdet[:, q] = QP_W[q] * det

    def B(self):
        """Strain-displacement matrices B[e, q, 3, 8] (engineering shear)."""
        Ea = self.conn.shape[0]
        B = np.zeros((Ea, 4, 3, 8))
        B[:, :, 0, 0::2] = self.dNdx
        B[:, :, 1, 1::2] = self.dNdy
        B[:, :, 2, 0::2] = self.dNdy
        B[:, :, 2, 1::2] = self.dNdx
        return B

    def u_dofs(self):
        """Element DOF map (Ea, 8) for interleaved displacement DOFs."""
        c = self.conn
        out = np.zeros((c.shape[0], 8), dtype=np.int64)
        out[:, 0::2] = 2 * c
        out[:, 1::2] = 2 * c + 1
        return out

    def strain(self, u):
        """Engineering strain at every active QP: (Ea, 4, 3)."""
        ue = u[self.u_dofs()]                           # (Ea, 8)
        return np.einsum("eqij,ej->eqi", self.B(), ue)

    def interp(self, d):
        """Nodal scalar field interpolated to the QPs: (Ea, 4)."""
        return d[self.conn] @ self.N.T
