"""Quadrature-point functions of the oracle (FP64, vectorised over points).

Strain input is the in-plane engineering strain (exx, eyy, gxy = 2 exy) of a
plane-strain state (ezz = 0).  Stress output is (sxx, syy, sxy).  All tangents
are 3x3 matrices acting on engineering strain, so that the element stiffness
is B^T C B.

Sources in the paper:
* volumetric-deviatoric energies and stress: Section 2 (energy split equation,
  whose second line is the inactive part Psi^-; stress equation eq_sigma);
* tie rule for the indicators: Section 3.3, eq_definition_+ (trace > 0 strictly
  counts as active);
* degradation g(d) = (1-d)^2 + eta: Section 2, table of AT1/AT2 parameters;
* fixed-invariant relations eq:trdep, eq:epdep and the half-step updates
  eq:epn1 and e_dev_1/2 (Section 3.3), which give the scale factor
  (1 + a*Dd) with a = 2(1-d)/g(d) applied to <tr eps>_+ and to |eps_dev|;
* the extra stiffness K~ (eq:dpsi, Section 3.4), rewritten as a coefficient
  c_S = 8 (1-d)^2 / g * Psi_S per scheme;
* spectral split: named in Section 2 as an extension; the formulas are the
  standard Miehe split (reading recorded in the design notes).
"""
from __future__ import annotations

import numpy as np


def lame(E, nu):
    """Lame constants and the 3-D bulk modulus K = lambda + 2 mu / 3."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    K = lam + 2.0 * mu / 3.0
    return lam, mu, K


def degradation(d, eta):
    """g(d) = (1 - d)^2 + eta (AT1 and AT2 alike)."""
    return (1.0 - d) ** 2 + eta


def pos(x):
    return 0.5 * (x + np.abs(x))


def neg(x):
    return 0.5 * (x - np.abs(x))


# --------------------------------------------------------------------------
# Volumetric-deviatoric split
# --------------------------------------------------------------------------

def vd_parts(eps, mu, K):
    """Energy parts of the VD split at each point.

    eps: (..., 3) engineering strain.  Returns dict with trace t, the deviatoric
    square e_dev:e_dev (3-D deviator with ezz = 0), psi_vol = K/2 <t>_+^2,
    psi_dev = mu e_dev:e_dev, psi_plus = psi_vol + psi_dev and
    psi_minus = K/2 <t>_-^2.
    """
    exx, eyy, gxy = eps[..., 0], eps[..., 1], eps[..., 2]
    exy = 0.5 * gxy
    t = exx + eyy
    m = t / 3.0
    devdev = (exx - m) ** 2 + (eyy - m) ** 2 + m ** 2 + 2.0 * exy ** 2
    psi_vol = 0.5 * K * pos(t) ** 2
    psi_dev = mu * devdev
    return {
        "t": t,
        "devdev": devdev,
        "psi_vol": psi_vol,
        "psi_dev": psi_dev,
        "psi_plus": psi_vol + psi_dev,
        "psi_minus": 0.5 * K * neg(t) ** 2,
    }


def vd_stress(eps, g, mu, K):
    """sigma = g [2 mu e_dev + K <t>_+ I] + K <t>_- I, in-plane components."""
    exx, eyy, gxy = eps[..., 0], eps[..., 1], eps[..., 2]
    t = exx + eyy
    m = t / 3.0
    vol = np.where(t > 0.0, g * K * t, K * t)
    sxx = 2.0 * mu * g * (exx - m) + vol
    syy = 2.0 * mu * g * (eyy - m) + vol
    sxy = mu * g * gxy
    return np.stack([sxx, syy, sxy], axis=-1)


def vd_tangent(eps, g, mu, K):
    """d sigma / d eps (engineering), with the indicator taken at eps (t > 0 active)."""
    t = eps[..., 0] + eps[..., 1]
    kap = np.where(t > 0.0, g * K, K)
    a = 2.0 * mu * g
    C = np.zeros(eps.shape[:-1] + (3, 3))
    C[..., 0, 0] = a * (2.0 / 3.0) + kap
    C[..., 1, 1] = a * (2.0 / 3.0) + kap
    C[..., 0, 1] = -a / 3.0 + kap
    C[..., 1, 0] = -a / 3.0 + kap
    C[..., 2, 2] = 0.5 * a
    return C


# --------------------------------------------------------------------------
# Spectral split (in-plane eigenvalues; the out-of-plane one is zero)
# --------------------------------------------------------------------------

def _eig2(eps):
    exx, eyy, exy = eps[..., 0], eps[..., 1], 0.5 * eps[..., 2]
    t = exx + eyy
    r = np.sqrt((0.5 * (exx - eyy)) ** 2 + exy ** 2)
    e1 = 0.5 * t + r
    e2 = 0.5 * t - r
    # unit eigenvector of e1
    theta = 0.5 * np.arctan2(2.0 * exy, exx - eyy)
    n1 = np.stack([np.cos(theta), np.sin(theta)], axis=-1)
    n2 = np.stack([-np.sin(theta), np.cos(theta)], axis=-1)
    return t, e1, e2, n1, n2


def spectral_parts(eps, lam, mu):
    t, e1, e2, _, _ = _eig2(eps)
    psi_vol = 0.5 * lam * pos(t) ** 2
    psi_dev = mu * (pos(e1) ** 2 + pos(e2) ** 2)
    return {
        "t": t, "e1": e1, "e2": e2,
        "psi_vol": psi_vol,
        "psi_dev": psi_dev,
        "psi_plus": psi_vol + psi_dev,
        "psi_minus": 0.5 * lam * neg(t) ** 2 + mu * (neg(e1) ** 2 + neg(e2) ** 2),
    }


def _tensor(v):
    """Engineering 3-vector -> symmetric 2x2 tensor."""
    T = np.zeros(v.shape[:-1] + (2, 2))
    T[..., 0, 0] = v[..., 0]
    T[..., 1, 1] = v[..., 1]
    T[..., 0, 1] = T[..., 1, 0] = 0.5 * v[..., 2]
    return T


def _spectral_plus_map(eps, dv):
    """Directional derivative of eps^+ = sum <e_i>_+ n_i n_i along dv (engineering).

    In the eigenbasis the diagonal entries are multiplied by H(e_i) and the
    off-diagonal entry by (<e1>_+ - <e2>_+)/(e1 - e2), whose limit at e1 = e2 is
    H(e1).  Returns the tensor (2x2) derivative.
    """
    t, e1, e2, n1, n2 = _eig2(eps)
    Q = np.stack([n1, n2], axis=-1)              # columns n1, n2
    dE = _tensor(dv)
    dEp = np.einsum("...ji,...jk,...kl->...il", Q, dE, Q)
    h1 = (e1 > 0.0).astype(float)
    h2 = (e2 > 0.0).astype(float)
    diff = e1 - e2
    with np.errstate(divide="ignore", invalid="ignore"):
        th = np.where(np.abs(diff) > 0.0, (pos(e1) - pos(e2)) / np.where(diff == 0, 1.0, diff), h1)
    out = np.zeros_like(dEp)
    out[..., 0, 0] = h1 * dEp[..., 0, 0]
    out[..., 1, 1] = h2 * dEp[..., 1, 1]
    out[..., 0, 1] = th * dEp[..., 0, 1]
    out[..., 1, 0] = th * dEp[..., 1, 0]
    return np.einsum("...ij,...jk,...lk->...il", Q, out, Q)


def spectral_stress(eps, g, lam, mu):
    """sigma = g [lam <t>_+ I + 2 mu eps^+] + lam <t>_- I + 2 mu eps^-."""
    t, e1, e2, n1, n2 = _eig2(eps)
    P1 = np.einsum("...i,...j->...ij", n1, n1)
    P2 = np.einsum("...i,...j->...ij", n2, n2)
    ep = pos(e1)[..., None, None] * P1 + pos(e2)[..., None, None] * P2
    en = neg(e1)[..., None, None] * P1 + neg(e2)[..., None, None] * P2
    I = np.eye(2)
    S = (g[..., None, None] * (lam * pos(t)[..., None, None] * I + 2.0 * mu * ep)
         + lam * neg(t)[..., None, None] * I + 2.0 * mu * en)
    return np.stack([S[..., 0, 0], S[..., 1, 1], S[..., 0, 1]], axis=-1)


def spectral_tangent(eps, g, lam, mu):
    t = eps[..., 0] + eps[..., 1]
    C = np.zeros(eps.shape[:-1] + (3, 3))
    hp = (t > 0.0).astype(float)
    for col in range(3):
        dv = np.zeros(eps.shape)
        dv[..., col] = 1.0
        dt = dv[..., 0] + dv[..., 1]
        dEp = _spectral_plus_map(eps, dv)
        dE = _tensor(dv)
        dEn = dE - dEp
        I = np.eye(2)
        dS = (g[..., None, None] * (lam * (hp * dt)[..., None, None] * I + 2.0 * mu * dEp)
              + lam * ((1.0 - hp) * dt)[..., None, None] * I + 2.0 * mu * dEn)
        C[..., 0, col] = dS[..., 0, 0]
        C[..., 1, col] = dS[..., 1, 1]
        C[..., 2, col] = dS[..., 0, 1]
    return C


# --------------------------------------------------------------------------
# Split dispatch
# --------------------------------------------------------------------------

class Constitutive:
    """Material point functions for one material and split."""

    def __init__(self, E, nu, split):
        self.lam, self.mu, self.K = lame(E, nu)
        self.split = int(split)

    def parts(self, eps):
        if self.split == 0:
            return vd_parts(eps, self.mu, self.K)
        return spectral_parts(eps, self.lam, self.mu)

    def stress(self, eps, g):
        if self.split == 0:
            return vd_stress(eps, g, self.mu, self.K)
        return spectral_stress(eps, g, self.lam, self.mu)

    def tangent(self, eps, g):
        if self.split == 0:
            return vd_tangent(eps, g, self.mu, self.K)
        return spectral_tangent(eps, g, self.lam, self.mu)


# --------------------------------------------------------------------------
# Fixed-stress predictor pieces (Sections 3.3-3.5)
# --------------------------------------------------------------------------

def scheme_part(parts, scheme):
    """Psi_S: the part of Psi^+ whose strain invariant the scheme rescales.

    S1 holds the first stress invariant (rescales <tr eps>_+, i.e. psi_vol),
    S2 the second (rescales |eps_dev|, i.e. psi_dev), S3 both (psi_plus).
    """
    if scheme == 1:
        return parts["psi_vol"]
    if scheme == 2:
        return parts["psi_dev"]
    if scheme == 3:
        return parts["psi_plus"]
    return np.zeros_like(parts["psi_plus"])


def strain_scale(d, eta, dd):
    """1 + a*Dd with a = 2(1-d)/g(d): the factor eq:trdep/eq:epdep put on
    <tr eps>_+ and on |eps_dev| over a phase increment Dd (eq:epn1, e_dev_1/2)."""
    a = 2.0 * (1.0 - d) / degradation(d, eta)
    return 1.0 + a * dd


def coupling_coefficient(d, eta, psi_s):
    """c_S = 8 (1-d)^2 / g(d) * Psi_S, so that K~ = -c_S N N^T (eq:dpsi;
    2 mu e_dev:e_dev + K <t>_+^2 = 2 Psi^+ for the VD split)."""
    return 8.0 * (1.0 - d) ** 2 / degradation(d, eta) * psi_s


def predicted_energy(psi_plus, psi_s, d, eta, dd, active):
    """Half-step active energy: Psi^+ + ((1 + a Dd)^2 - 1) Psi_S where the
    softening gate holds and Dd > 0 (Section 3.5), else Psi^+."""
    s = strain_scale(d, eta, dd)
    upd = psi_plus + (s * s - 1.0) * psi_s
    return np.where(active & (dd > 0.0), upd, psi_plus)
