// Trilinear hexahedra (Q1, 2x2x2 Gauss) on a structured box: the per-node
// and per-element arithmetic of the 3-D operators.  The device kernels in
// pf3d_kernels.hip call these functions once per grid index; the functions
// are __host__ __device__ so that a host build can replay a kernel's grid
// index by index.
//
// Model (Section 2), with the full 3-D strain: the volumetric-deviatoric
// split sigma = g(d) [K <tr eps>_+ I + 2 mu eps_dev] + K <tr eps>_- I, or the
// spectral split sigma = g(d) [lam <tr eps>_+ I + 2 mu eps+] + lam <tr eps>_-
// I + 2 mu eps- over the principal strains; AT2 phase operator coef N N^T +
// Gc l grad N . grad N^T; history H = max(H_n, Psi+).
//
// Layout in device memory (structure of arrays):
//   node (i, j, k) has id n = i + j (nx+1) + k (nx+1)(ny+1);
//   element (ie, je, ke) has id e = ie + je nx + ke nx ny;
//   displacement-like fields [3N]: the x plane, then y, then z;
//   nodal scalars [N]; quadrature-point fields [8E]: plane q holds point q
//   of every element (index e + q E); flags [E] (uint16).
// Corner a of an element sits at offsets (di, dj, dk) = (((a+1)>>1)&1,
// (a>>1)&1, a>>2), i.e. the bottom face counter-clockwise, then the top
// face; Gauss point q sits at the reference coordinates (2 di - 1,
// 2 dj - 1, 2 dk - 1) / sqrt(3) of corner q.
#pragma once

#include "../../include/phasefield3d.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace pf3d {

struct Grid3 {
  int nx, ny, nz;
  int N, E;             // nodes, elements
  double hx, hy, hz;    // element edge lengths
};

struct Mat3 {
  double lam, mu, K;    // Lame constants, bulk modulus K = lam + 2 mu / 3
  double Gcl;           // Gc l, the phase operator's gradient factor
  double eta;           // residual stiffness of g(d) = (1 - d)^2 + eta
  int split;            // PF_SPLIT_VD or PF_SPLIT_SPECTRAL
  double Gc_l;          // Gc / l, the AT2 mass coefficient's constant part
};

struct Qp3 {
  int scheme;           // 0 ST, 1 S1 (psi_vol), 2 S2 (psi_dev), 3 S3 (psi+)
  double psi_crit;      // softening threshold of the gate
  double d_gate;        // gate only where d_q < d_gate
};

constexpr int kTpb3 = 256;

__host__ __device__ inline int corner_di(int a) { return ((a + 1) >> 1) & 1; }
__host__ __device__ inline int corner_dj(int a) { return (a >> 1) & 1; }
__host__ __device__ inline int corner_dk(int a) { return a >> 2; }

// One-dimensional factor (1 + s_a s_q / sqrt 3) / 2 of the shape function
// N_a at Gauss point q along one axis (s = +-1).
__host__ __device__ inline double axis_factor(int oa, int oq) {
  const double c = 0.28867513459481287;   // 1 / (2 sqrt 3)
  return (oa == oq) ? 0.5 + c : 0.5 - c;
}

// N_a and grad N_a at Gauss point q of a box element with edges hx, hy, hz.
struct ShapeAt {
  double N, gx, gy, gz;
};

__host__ __device__ inline ShapeAt shape_at(const Grid3 &g, int a, int q) {
  const double fx = axis_factor(corner_di(a), corner_di(q));
  const double fy = axis_factor(corner_dj(a), corner_dj(q));
  const double fz = axis_factor(corner_dk(a), corner_dk(q));
  const double sx = corner_di(a) ? 1.0 : -1.0, sy = corner_dj(a) ? 1.0 : -1.0,
               sz = corner_dk(a) ? 1.0 : -1.0;
  return ShapeAt{fx * fy * fz, sx / g.hx * fy * fz, sy / g.hy * fx * fz, sz / g.hz * fx * fy};
}

__host__ __device__ inline int node_id(const Grid3 &g, int i, int j, int k) {
  return i + j * (g.nx + 1) + k * (g.nx + 1) * (g.ny + 1);
}

// Node of corner b of the element whose first corner is node (ie, je, ke).
__host__ __device__ inline int corner_node(const Grid3 &g, int ie, int je, int ke, int b) {
  return node_id(g, ie + corner_di(b), je + corner_dj(b), ke + corner_dk(b));
}

__host__ __device__ inline double degrade(double d, double eta) {
  return (1.0 - d) * (1.0 - d) + eta;
}

// Strain (engineering Voigt [xx, yy, zz, 2yz, 2xz, 2xy]) at Gauss point q
// from the element's corner displacements u[b], u[8+b], u[16+b].
__host__ __device__ inline void strain_at(const Grid3 &g, int q, const double *ue,
                                          double eps[6]) {
  for (int c = 0; c < 6; ++c) eps[c] = 0.0;
  for (int b = 0; b < 8; ++b) {
    const ShapeAt s = shape_at(g, b, q);
    const double ux = ue[b], uy = ue[8 + b], uz = ue[16 + b];
    eps[0] += s.gx * ux;
    eps[1] += s.gy * uy;
    eps[2] += s.gz * uz;
    eps[3] += s.gz * uy + s.gy * uz;
    eps[4] += s.gz * ux + s.gx * uz;
    eps[5] += s.gy * ux + s.gx * uy;
  }
}

// Split stress (Voigt [xx, yy, zz, yz, xz, xy]) at degradation gd; the
// volumetric part is degraded only under expansion (tr eps > 0 strictly).
__host__ __device__ inline void vd_stress(const Mat3 &m, const double eps[6], double gd,
                                          double sig[6]) {
  const double t = eps[0] + eps[1] + eps[2], m3 = t / 3.0;
  const double vol = t > 0.0 ? gd * m.K * t : m.K * t;
  for (int c = 0; c < 3; ++c) sig[c] = gd * 2.0 * m.mu * (eps[c] - m3) + vol;
  for (int c = 3; c < 6; ++c) sig[c] = gd * m.mu * eps[c];
}

// Tangent of the split stress at the strain eps, applied to a strain
// increment de: the volumetric factor is g K where tr eps > 0 (act), else K.
__host__ __device__ inline void vd_tangent_apply_act(const Mat3 &m, bool act, double gd,
                                                     const double de[6], double ds[6]) {
  const double kf = act ? gd * m.K : m.K;
  const double dt = de[0] + de[1] + de[2];
  for (int c = 0; c < 3; ++c) ds[c] = gd * 2.0 * m.mu * (de[c] - dt / 3.0) + kf * dt;
  for (int c = 3; c < 6; ++c) ds[c] = gd * m.mu * de[c];
}
__host__ __device__ inline void vd_tangent_apply(const Mat3 &m, const double eps[6], double gd,
                                                 const double de[6], double ds[6]) {
  vd_tangent_apply_act(m, eps[0] + eps[1] + eps[2] > 0.0, gd, de, ds);
}

// Energy parts: psi_vol = K/2 <t>_+^2, psi_dev = mu eps_dev : eps_dev.
__host__ __device__ inline void vd_parts(const Mat3 &m, const double eps[6], double *t_out,
                                         double *pvol, double *pdev) {
  const double t = eps[0] + eps[1] + eps[2], m3 = t / 3.0;
  double dd = 0.0;
  for (int c = 0; c < 3; ++c) dd += (eps[c] - m3) * (eps[c] - m3);
  for (int c = 3; c < 6; ++c) dd += 0.5 * eps[c] * eps[c];
  const double tp = t > 0.0 ? t : 0.0;
  *t_out = t;
  *pvol = 0.5 * m.K * tp * tp;
  *pdev = m.mu * dd;
}

// ---- spectral split

// Symmetric 3x3 eigen-decomposition A = Q diag(w) Q^T by cyclic Jacobi
// rotations: each rotation in the (p, r) plane annihilates A_pr, with the
// tangent of the angle taken as the smaller root.  The sweeps stop once the
// off-diagonal mass is below 1e-32 of the whole (quadratic convergence
// reaches that in a few sweeps) and never exceed 16.  Exact zeros
// off the diagonal are left alone, so a block-diagonal strain keeps its
// block's eigenvalue exactly.  eps is an engineering Voigt strain.
__host__ __device__ inline void sym3_eig(const double eps[6], double w[3], double Q[3][3]) {
  double a[3][3] = {{eps[0], 0.5 * eps[5], 0.5 * eps[4]},
                    {0.5 * eps[5], eps[1], 0.5 * eps[3]},
                    {0.5 * eps[4], 0.5 * eps[3], eps[2]}};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Q[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off == 0.0 || off <= 1e-32 * (dia + 2.0 * off)) break;
    for (int pr = 0; pr < 3; ++pr) {
      const int p = pr == 2 ? 1 : 0, r = pr == 0 ? 1 : 2;
      const double apr = a[p][r];
      if (apr == 0.0) continue;
      const double theta = (a[r][r] - a[p][p]) / (2.0 * apr);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      const int o = 3 - p - r;   // the third index
      const double aop = a[o][p], aor = a[o][r];
      a[p][p] -= t * apr;
      a[r][r] += t * apr;
      a[p][r] = a[r][p] = 0.0;
      a[o][p] = a[p][o] = c * aop - s * aor;
      a[o][r] = a[r][o] = s * aop + c * aor;
      for (int k = 0; k < 3; ++k) {
        const double qp = Q[k][p], qr = Q[k][r];
        Q[k][p] = c * qp - s * qr;
        Q[k][r] = s * qp + c * qr;
      }
    }
  }
  for (int i = 0; i < 3; ++i) w[i] = a[i][i];
}

__host__ __device__ inline double pos_part(double x) { return x > 0.0 ? x : 0.0; }

// sum_k f_k Q[:,k] Q[:,k]^T as a Voigt stress-like vector [xx, yy, zz, yz, xz, xy].
__host__ __device__ inline void spectral_sum(const double Q[3][3], const double f[3],
                                             double out[6]) {
  const int I[6] = {0, 1, 2, 1, 0, 0}, J[6] = {0, 1, 2, 2, 2, 1};
  for (int c = 0; c < 6; ++c) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += f[k] * Q[I[c]][k] * Q[J[c]][k];
    out[c] = s;
  }
}

__host__ __device__ inline void spectral_stress(const Mat3 &m, const double eps[6], double gd,
                                                double sig[6]) {
  double w[3], Q[3][3];
  sym3_eig(eps, w, Q);
  const double t = eps[0] + eps[1] + eps[2];
  const double fp[3] = {pos_part(w[0]), pos_part(w[1]), pos_part(w[2])};
  const double fn[3] = {w[0] - fp[0], w[1] - fp[1], w[2] - fp[2]};
  double ep[6], en[6];
  spectral_sum(Q, fp, ep);
  spectral_sum(Q, fn, en);
  const double vol = t > 0.0 ? gd * m.lam * t : m.lam * t;
  for (int c = 0; c < 6; ++c) sig[c] = gd * 2.0 * m.mu * ep[c] + 2.0 * m.mu * en[c];
  for (int c = 0; c < 3; ++c) sig[c] += vol;
}

// Tangent of the spectral stress at eps applied to de: with dE the tensor
// of de in the eigenbasis, deps+ = Q (theta o dE) Q^T with theta_ij =
// (<e_i>_+ - <e_j>_+) / (e_i - e_j), or H(e_i) where e_i = e_j; then
// dsigma = g [lam H(t) dt I + 2 mu deps+] + lam (1 - H(t)) dt I + 2 mu
// (de - deps+).  H counts strictly positive values.
__host__ __device__ inline void spectral_tangent_apply(const Mat3 &m, const double eps[6],
                                                       double gd, const double de[6],
                                                       double ds[6]) {
  double w[3], Q[3][3];
  sym3_eig(eps, w, Q);
  const double D[3][3] = {{de[0], 0.5 * de[5], 0.5 * de[4]},
                          {0.5 * de[5], de[1], 0.5 * de[3]},
                          {0.5 * de[4], 0.5 * de[3], de[2]}};
  // B = theta o (Q^T D Q)
  double B[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) s += Q[k][i] * D[k][l] * Q[l][j];
      const double diff = w[i] - w[j];
      const double th = diff != 0.0 ? (pos_part(w[i]) - pos_part(w[j])) / diff
                                    : (w[i] > 0.0 ? 1.0 : 0.0);
      B[i][j] = th * s;
    }
  // deps+ = Q B Q^T, as a Voigt tensor [xx, yy, zz, yz, xz, xy]
  const int I[6] = {0, 1, 2, 1, 0, 0}, J[6] = {0, 1, 2, 2, 2, 1};
  double dp[6];
  for (int c = 0; c < 6; ++c) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) s += Q[I[c]][k] * B[k][l] * Q[J[c]][l];
    dp[c] = s;
  }
  const double t = eps[0] + eps[1] + eps[2], dt = de[0] + de[1] + de[2];
  const double lv = t > 0.0 ? gd * m.lam * dt : m.lam * dt;
  // the Voigt shear entries of de are engineering strains (twice the tensor)
  const double dten[6] = {de[0], de[1], de[2], 0.5 * de[3], 0.5 * de[4], 0.5 * de[5]};
  for (int c = 0; c < 6; ++c) ds[c] = gd * 2.0 * m.mu * dp[c] + 2.0 * m.mu * (dten[c] - dp[c]);
  for (int c = 0; c < 3; ++c) ds[c] += lv;
}

// Energy parts of the spectral split: psi_vol = lam/2 <t>_+^2, psi_dev =
// mu sum <e_i>_+^2.
__host__ __device__ inline void spectral_parts(const Mat3 &m, const double eps[6],
                                               double *t_out, double *pvol, double *pdev) {
  double w[3], Q[3][3];
  sym3_eig(eps, w, Q);
  const double t = eps[0] + eps[1] + eps[2], tp = pos_part(t);
  *t_out = t;
  *pvol = 0.5 * m.lam * tp * tp;
  *pdev = m.mu * (pos_part(w[0]) * pos_part(w[0]) + pos_part(w[1]) * pos_part(w[1]) +
                  pos_part(w[2]) * pos_part(w[2]));
}

// The split's stress, tangent apply and energy parts.
__host__ __device__ inline void split_stress(const Mat3 &m, const double eps[6], double gd,
                                             double sig[6]) {
  if (m.split == 1) spectral_stress(m, eps, gd, sig);
  else vd_stress(m, eps, gd, sig);
}

__host__ __device__ inline void split_tangent_apply(const Mat3 &m, const double eps[6],
                                                    double gd, const double de[6],
                                                    double ds[6]) {
  if (m.split == 1) spectral_tangent_apply(m, eps, gd, de, ds);
  else vd_tangent_apply(m, eps, gd, de, ds);
}

__host__ __device__ inline void split_parts(const Mat3 &m, const double eps[6], double *t,
                                            double *pvol, double *pdev) {
  if (m.split == 1) spectral_parts(m, eps, t, pvol, pdev);
  else vd_parts(m, eps, t, pvol, pdev);
}

// Load the 8 corner values of nodal planes (ncomp planes of N values) of
// element (ie, je, ke) into out[c * 8 + b].
__host__ __device__ inline void gather_corners(const Grid3 &g, int ie, int je, int ke,
                                               const double *f, int ncomp, double *out) {
  for (int b = 0; b < 8; ++b) {
    const int nb = corner_node(g, ie, je, ke, b);
    for (int c = 0; c < ncomp; ++c) out[c * 8 + b] = f[nb + c * g.N];
  }
}

__host__ __device__ inline double interp_at(const Grid3 &g, int q, const double *fe) {
  double s = 0.0;
  for (int b = 0; b < 8; ++b) s += shape_at(g, b, q).N * fe[b];
  return s;
}

// The elements that hold node n, each with the corner a that n is in it:
// calls visit(ie, je, ke, a) for every such element inside the box.
template <class F>
__host__ __device__ inline void for_node_elements(const Grid3 &g, int n, F &&visit) {
  const int P = (g.nx + 1) * (g.ny + 1);
  const int k = n / P, r = n - k * P, j = r / (g.nx + 1), i = r - j * (g.nx + 1);
  for (int a = 0; a < 8; ++a) {
    const int ie = i - corner_di(a), je = j - corner_dj(a), ke = k - corner_dk(a);
    if (ie < 0 || je < 0 || ke < 0 || ie >= g.nx || je >= g.ny || ke >= g.nz) continue;
    visit(ie, je, ke, a);
  }
}

// Internal force at node n: R_n = sum over its elements and their Gauss
// points of B_a^T sigma(eps(u), g(d_q)) w, written to R[n], R[N+n], R[2N+n].
__host__ __device__ inline void node_internal_force(const Grid3 &g, const Mat3 &m, int n,
                                                    const double *u, const double *d,
                                                    double *R) {
  const double w = g.hx * g.hy * g.hz / 8.0;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for_node_elements(g, n, [&](int ie, int je, int ke, int a) {
    double ue[24], de[8];
    gather_corners(g, ie, je, ke, u, 3, ue);
    gather_corners(g, ie, je, ke, d, 1, de);
    for (int q = 0; q < 8; ++q) {
      double eps[6], sig[6];
      strain_at(g, q, ue, eps);
      split_stress(m, eps, degrade(interp_at(g, q, de), m.eta), sig);
      const ShapeAt s = shape_at(g, a, q);
      fx += w * (s.gx * sig[0] + s.gz * sig[4] + s.gy * sig[5]);
      fy += w * (s.gy * sig[1] + s.gz * sig[3] + s.gx * sig[5]);
      fz += w * (s.gz * sig[2] + s.gy * sig[3] + s.gx * sig[4]);
    }
  });
  R[n] = fx;
  R[g.N + n] = fy;
  R[2 * g.N + n] = fz;
}

// Tangent apply at node n: (K_t(u; d) p)_n with the tangent taken at u.
__host__ __device__ inline void node_tangent_apply(const Grid3 &g, const Mat3 &m, int n,
                                                   const double *u, const double *d,
                                                   const double *p, double *out) {
  const double w = g.hx * g.hy * g.hz / 8.0;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for_node_elements(g, n, [&](int ie, int je, int ke, int a) {
    double ue[24], pe[24], de[8];
    gather_corners(g, ie, je, ke, u, 3, ue);
    gather_corners(g, ie, je, ke, p, 3, pe);
    gather_corners(g, ie, je, ke, d, 1, de);
    for (int q = 0; q < 8; ++q) {
      double eps[6], dep[6], ds[6];
      strain_at(g, q, ue, eps);
      strain_at(g, q, pe, dep);
      split_tangent_apply(m, eps, degrade(interp_at(g, q, de), m.eta), dep, ds);
      const ShapeAt s = shape_at(g, a, q);
      fx += w * (s.gx * ds[0] + s.gz * ds[4] + s.gy * ds[5]);
      fy += w * (s.gy * ds[1] + s.gz * ds[3] + s.gx * ds[5]);
      fz += w * (s.gz * ds[2] + s.gy * ds[3] + s.gx * ds[4]);
    }
  });
  out[n] = fx;
  out[g.N + n] = fy;
  out[2 * g.N + n] = fz;
}

// Phase operator at node n: sum w [coef_q N_a (N . p) + Gc l grad N_a .
// grad(N . p)] with the per-point coefficient coef[e + q E].
__host__ __device__ inline void node_phase_apply(const Grid3 &g, const Mat3 &m, int n,
                                                 const double *coef, const double *p,
                                                 double *out) {
  const double w = g.hx * g.hy * g.hz / 8.0;
  double acc = 0.0;
  for_node_elements(g, n, [&](int ie, int je, int ke, int a) {
    const int e = ie + je * g.nx + ke * g.nx * g.ny;
    double pe[8];
    gather_corners(g, ie, je, ke, p, 1, pe);
    for (int q = 0; q < 8; ++q) {
      double pq = 0.0, px = 0.0, py = 0.0, pz = 0.0;
      for (int b = 0; b < 8; ++b) {
        const ShapeAt s = shape_at(g, b, q);
        pq += s.N * pe[b];
        px += s.gx * pe[b];
        py += s.gy * pe[b];
        pz += s.gz * pe[b];
      }
      const ShapeAt s = shape_at(g, a, q);
      acc += w * (coef[e + q * g.E] * s.N * pq + m.Gcl * (s.gx * px + s.gy * py + s.gz * pz));
    }
  });
  out[n] = acc;
}

// Diagonal of the tangent at node n: for each component c, the sum over
// its elements and points of w (B_a,c)^T C_t(eps(u)) B_a,c, i.e. the tangent
// applied to the strain of a unit displacement of corner a along c.
__host__ __device__ inline void node_tangent_diag(const Grid3 &g, const Mat3 &m, int n,
                                                  const double *u, const double *d,
                                                  double *D) {
  const double w = g.hx * g.hy * g.hz / 8.0;
  double dx = 0.0, dy = 0.0, dz = 0.0;
  for_node_elements(g, n, [&](int ie, int je, int ke, int a) {
    double ue[24], de[8];
    gather_corners(g, ie, je, ke, u, 3, ue);
    gather_corners(g, ie, je, ke, d, 1, de);
    for (int q = 0; q < 8; ++q) {
      double eps[6];
      strain_at(g, q, ue, eps);
      const double gd = degrade(interp_at(g, q, de), m.eta);
      const ShapeAt s = shape_at(g, a, q);
      const double bx[6] = {s.gx, 0.0, 0.0, 0.0, s.gz, s.gy};
      const double by[6] = {0.0, s.gy, 0.0, s.gz, 0.0, s.gx};
      const double bz[6] = {0.0, 0.0, s.gz, s.gy, s.gx, 0.0};
      double ds[6];
      split_tangent_apply(m, eps, gd, bx, ds);
      dx += w * (s.gx * ds[0] + s.gz * ds[4] + s.gy * ds[5]);
      split_tangent_apply(m, eps, gd, by, ds);
      dy += w * (s.gy * ds[1] + s.gz * ds[3] + s.gx * ds[5]);
      split_tangent_apply(m, eps, gd, bz, ds);
      dz += w * (s.gz * ds[2] + s.gy * ds[3] + s.gx * ds[4]);
    }
  });
  D[n] = dx;
  D[g.N + n] = dy;
  D[2 * g.N + n] = dz;
}

// Diagonal of the phase operator at node n: sum w [coef_q N_a^2 + Gc l
// |grad N_a|^2].
__host__ __device__ inline void node_phase_diag(const Grid3 &g, const Mat3 &m, int n,
                                                const double *coef, double *D) {
  const double w = g.hx * g.hy * g.hz / 8.0;
  double acc = 0.0;
  for_node_elements(g, n, [&](int ie, int je, int ke, int a) {
    const int e = ie + je * g.nx + ke * g.nx * g.ny;
    for (int q = 0; q < 8; ++q) {
      const ShapeAt s = shape_at(g, a, q);
      acc += w * (coef[e + q * g.E] * s.N * s.N +
                  m.Gcl * (s.gx * s.gx + s.gy * s.gy + s.gz * s.gz));
    }
  });
  D[n] = acc;
}

// AT2 right-hand side at node n: b_n = sum w 2 H_q N_a.
__host__ __device__ inline void node_phase_rhs(const Grid3 &g, int n, const double *H,
                                               double *b) {
  const double w = g.hx * g.hy * g.hz / 8.0;
  double acc = 0.0;
  for_node_elements(g, n, [&](int ie, int je, int ke, int a) {
    const int e = ie + je * g.nx + ke * g.nx * g.ny;
    for (int q = 0; q < 8; ++q) acc += w * 2.0 * H[e + q * g.E] * shape_at(g, a, q).N;
  });
  b[n] = acc;
}

// Mass coefficient of the phase block at the points of element e: the AT2
// coefficient c = Gc/l + 2H (Section 2), or with trial = 1 that of the
// trial block K_dd + K~ (Section 3.4): c - c_S at gated points, c_S = 8
// (1 - d_q)^2 / g(d_q) psi_S, raised to theta c where it falls below
// (floor = 1) or kept as it is (floor = 0).  Returns the gated points below
// theta c.
__host__ __device__ inline int elem_phase_coef(const Grid3 &g, const Mat3 &m, int e, int trial,
                                               double theta, int floor, const double *H,
                                               const double *psi_s, const uint16_t *flags,
                                               const double *d, double *coef) {
  const unsigned fl = trial ? flags[e] : 0u;
  double de[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (fl >> 8) {
    const int ke = e / (g.nx * g.ny), r = e - ke * g.nx * g.ny, je = r / g.nx,
              ie = r - je * g.nx;
    gather_corners(g, ie, je, ke, d, 1, de);
  }
  int below = 0;
  for (int q = 0; q < 8; ++q) {
    const double c = m.Gc_l + 2.0 * H[e + q * g.E];
    double ct = c;
    if ((fl >> (q + 8)) & 1u) {
      const double om = 1.0 - interp_at(g, q, de);
      const double cS = 8.0 * om * om / (om * om + m.eta) * psi_s[e + q * g.E];
      ct = c - cS;
      if (ct < theta * c) {
        if (floor) ct = theta * c;
        ++below;
      }
    }
    coef[e + q * g.E] = ct;
  }
  return below;
}

// Quadrature-point update of element e (Sections 2, 3.5): H = max(H_prev,
// psi+), the scheme part psi_S, and flags bit q = tr eps > 0 at point q,
// bit 8 + q = the softening gate at point q (a fixed-stress scheme, psi+
// above psi_crit and above H_prev, d_q below d_gate).  Returns the number
// of gated points.
__host__ __device__ inline int elem_qp_update(const Grid3 &g, const Mat3 &m, const Qp3 &qp,
                                              int e, const double *u, const double *d,
                                              const double *Hprev, double *H, double *psi_s,
                                              uint16_t *flags) {
  const int ke = e / (g.nx * g.ny), r = e - ke * g.nx * g.ny, je = r / g.nx,
            ie = r - je * g.nx;
  double ue[24], de[8];
  gather_corners(g, ie, je, ke, u, 3, ue);
  gather_corners(g, ie, je, ke, d, 1, de);
  unsigned fl = 0;
  int ng = 0;
  for (int q = 0; q < 8; ++q) {
    double eps[6], t, pv, pd;
    strain_at(g, q, ue, eps);
    split_parts(m, eps, &t, &pv, &pd);
    const double pplus = pv + pd, hp = Hprev[e + q * g.E];
    H[e + q * g.E] = pplus > hp ? pplus : hp;
    double ps = 0.0;
    if (qp.scheme == 1) ps = pv;
    else if (qp.scheme == 2) ps = pd;
    else if (qp.scheme == 3) ps = pplus;
    psi_s[e + q * g.E] = ps;
    if (t > 0.0) fl |= 1u << q;
    const double dq = interp_at(g, q, de);
    if (qp.scheme != 0 && pplus > qp.psi_crit && pplus > hp && dq < qp.d_gate) {
      fl |= 1u << (q + 8);
      ++ng;
    }
  }
  flags[e] = uint16_t(fl);
  return ng;
}

// Fixed-stress predictor of element e (Sections 3.3, 3.5): at gated points
// (flag bit 8 + q) with Dd_q > 0, Hhat = max(H, H + ((1 + a Dd_q)^2 - 1)
// psi_S) with a = 2 (1 - d_q) / g(d_q), the factor that eq:epn1 and
// e_dev_1/2 put on the scheme's strain invariant; elsewhere Hhat = H.  At a
// gated point H = psi+, so this is the half-step active energy.
__host__ __device__ inline void elem_predictor(const Grid3 &g, const Mat3 &m, int e,
                                               const double *d, const double *dd,
                                               const double *H, const double *psi_s,
                                               const uint16_t *flags, double *Hhat) {
  const unsigned fl = flags[e];
  if ((fl >> 8) == 0) {
    for (int q = 0; q < 8; ++q) Hhat[e + q * g.E] = H[e + q * g.E];
    return;
  }
  const int ke = e / (g.nx * g.ny), r = e - ke * g.nx * g.ny, je = r / g.nx,
            ie = r - je * g.nx;
  double de[8], dde[8];
  gather_corners(g, ie, je, ke, d, 1, de);
  gather_corners(g, ie, je, ke, dd, 1, dde);
  for (int q = 0; q < 8; ++q) {
    const double h = H[e + q * g.E];
    double out = h;
    const double ddq = interp_at(g, q, dde);
    if (((fl >> (q + 8)) & 1u) && ddq > 0.0) {
      const double om = 1.0 - interp_at(g, q, de);
      const double a = 2.0 * om / (om * om + m.eta);
      const double sc = 1.0 + a * ddq;
      const double ph = h + (sc * sc - 1.0) * psi_s[e + q * g.E];
      out = ph > h ? ph : h;
    }
    Hhat[e + q * g.E] = out;
  }
}

// ---- element-once operators: tiles of node columns marching in z
//
// The node-gather operators above evaluate every element once for each of
// its eight nodes.  For the internal force and the tangent apply, whose
// element is costly, a block instead owns a tile of kT3 x kT3 node columns and a
// chunk of kT3Z node planes, and marches through the element layers that
// touch its planes.  For each layer ke it stages node plane ke + 1 in LDS
// (plane ke was staged for the layer before; the first layer stages both),
// and its kTpb3 threads take the (kT3 + 1)^2 elements of the layer that touch
// the tile, each computing its element's eight corner contributions once.
// An owned node of plane ke then adds the four contributions from the layer
// below (carried in its thread) and the four from this layer, in a fixed
// order; the top plane of the mesh has only the layer below.  Every output is
// written by one thread: deterministic, no atomics.  The phases are
// functions of one thread index, so a host build can replay a block by
// running each phase for all threads between the block's barriers.
//
// An element operator Op provides the staged node record Op::Node (value-
// initialised to zero outside the box), its output components Op::NC,
//   Node stage(const Grid3 &, int node) const
//   void element(const Grid3 &, const Mat3 &, int e, const Node *c[8],
//                double out[8 * NC]) const     (out[NC * a + comp])
// and the output array q (component c of node n at q[n + c N]).
constexpr int kT3 = 15;         // owned node columns per tile side
constexpr int kT3E = kT3 + 1;   // element columns per tile side
constexpr int kT3N = kT3 + 2;   // staged node columns per side
constexpr int kT3Z = 8;         // node planes per block
static_assert(kT3E * kT3E == kTpb3, "one element column per thread");

template <class Node, int NC>
struct T3LdsT {
  Node plane[2][kT3N * kT3N];   // two node planes, slot k & 1
  double f[4][NC][kTpb3];       // four corners of each element of the layer
};

__host__ __device__ inline int t3_tiles_x(const Grid3 &g) { return (g.nx + kT3) / kT3; }
__host__ __device__ inline int t3_tiles_y(const Grid3 &g) { return (g.ny + kT3) / kT3; }
__host__ __device__ inline int t3_chunks_z(const Grid3 &g) { return (g.nz + kT3Z) / kT3Z; }
inline int t3_blocks(const Grid3 &g) { return t3_tiles_x(g) * t3_tiles_y(g) * t3_chunks_z(g); }

// Tangent apply of one element: out[3a + c] = sum_q w (B_a^T C_t(eps_q(u),
// g(d_q)) eps_q(p))_c, the element's share of node_tangent_apply at corner a.
// SPL is the split (0 volumetric-deviatoric, 1 spectral).  The VD tangent
// depends on u only through the sign of tr eps_q(u), so those eight signs
// are taken first and u is not held through the main loop (the same
// operations in the same order as the spectral form, so the same result).
template <int SPL>
__host__ __device__ inline void elem_tangent_apply(const Grid3 &g, const Mat3 &m,
                                                   const double *ue, const double *pe,
                                                   const double *de, double out[24]) {
  const double w = g.hx * g.hy * g.hz / 8.0;
  for (int x = 0; x < 24; ++x) out[x] = 0.0;
  unsigned act = 0;
  if constexpr (SPL == 0) {
    for (int q = 0; q < 8; ++q) {
      double eps[6];
      strain_at(g, q, ue, eps);
      if (eps[0] + eps[1] + eps[2] > 0.0) act |= 1u << q;
    }
  }
  for (int q = 0; q < 8; ++q) {
    double dep[6], ds[6];
    strain_at(g, q, pe, dep);
    const double gd = degrade(interp_at(g, q, de), m.eta);
    if constexpr (SPL == 0) {
      vd_tangent_apply_act(m, ((act >> q) & 1u) != 0u, gd, dep, ds);
    } else {
      double eps[6];
      strain_at(g, q, ue, eps);
      spectral_tangent_apply(m, eps, gd, dep, ds);
    }
    for (int a = 0; a < 8; ++a) {
      const ShapeAt s = shape_at(g, a, q);
      out[3 * a + 0] += w * (s.gx * ds[0] + s.gz * ds[4] + s.gy * ds[5]);
      out[3 * a + 1] += w * (s.gy * ds[1] + s.gz * ds[3] + s.gx * ds[5]);
      out[3 * a + 2] += w * (s.gz * ds[2] + s.gy * ds[3] + s.gx * ds[4]);
    }
  }
}

// Internal force of one element: out[3a + c] = sum_q w (B_a^T sigma(eps_q(u),
// g(d_q)))_c, the element's share of node_internal_force at corner a.
template <int SPL>
__host__ __device__ inline void elem_internal_force(const Grid3 &g, const Mat3 &m,
                                                    const double *ue, const double *de,
                                                    double out[24]) {
  const double w = g.hx * g.hy * g.hz / 8.0;
  for (int x = 0; x < 24; ++x) out[x] = 0.0;
  for (int q = 0; q < 8; ++q) {
    double eps[6], sig[6];
    strain_at(g, q, ue, eps);
    const double gd = degrade(interp_at(g, q, de), m.eta);
    if constexpr (SPL == 0) vd_stress(m, eps, gd, sig);
    else spectral_stress(m, eps, gd, sig);
    for (int a = 0; a < 8; ++a) {
      const ShapeAt s = shape_at(g, a, q);
      out[3 * a + 0] += w * (s.gx * sig[0] + s.gz * sig[4] + s.gy * sig[5]);
      out[3 * a + 1] += w * (s.gy * sig[1] + s.gz * sig[3] + s.gx * sig[5]);
      out[3 * a + 2] += w * (s.gz * sig[2] + s.gy * sig[3] + s.gx * sig[4]);
    }
  }
}

// The element operators of the tiled kernels.
struct T3Node {
  double ux, uy, uz, px, py, pz, d;
};
template <int SPL>
struct T3TangentOp {
  using Node = T3Node;
  static constexpr int NC = 3;
  const double *u, *d, *p;
  double *q;
  __host__ __device__ Node stage(const Grid3 &g, int id) const {
    return Node{u[id], u[id + g.N], u[id + 2 * g.N], p[id], p[id + g.N], p[id + 2 * g.N], d[id]};
  }
  __host__ __device__ void element(const Grid3 &g, const Mat3 &m, int, const Node *const c[8],
                                   double out[24]) const {
    double ue[24], pe[24], de[8];
    for (int b = 0; b < 8; ++b) {
      ue[b] = c[b]->ux; ue[8 + b] = c[b]->uy; ue[16 + b] = c[b]->uz;
      pe[b] = c[b]->px; pe[8 + b] = c[b]->py; pe[16 + b] = c[b]->pz;
      de[b] = c[b]->d;
    }
    elem_tangent_apply<SPL>(g, m, ue, pe, de, out);
  }
};
struct T3UdNode {
  double ux, uy, uz, d;
};
template <int SPL>
struct T3ForceOp {
  using Node = T3UdNode;
  static constexpr int NC = 3;
  const double *u, *d;
  double *q;
  __host__ __device__ Node stage(const Grid3 &g, int id) const {
    return Node{u[id], u[id + g.N], u[id + 2 * g.N], d[id]};
  }
  __host__ __device__ void element(const Grid3 &g, const Mat3 &m, int, const Node *const c[8],
                                   double out[24]) const {
    double ue[24], de[8];
    for (int b = 0; b < 8; ++b) {
      ue[b] = c[b]->ux; ue[8 + b] = c[b]->uy; ue[16 + b] = c[b]->uz;
      de[b] = c[b]->d;
    }
    elem_internal_force<SPL>(g, m, ue, de, out);
  }
};
// Thread t stages its entries of node plane k (columns i0 - 1 .. i0 + kT3,
// j0 - 1 .. j0 + kT3) into slot s; nodes outside the box are zero.
template <class Op>
__host__ __device__ inline void t3_stage(const Op &op, const Grid3 &g, int i0, int j0, int k,
                                         int s, int t, T3LdsT<typename Op::Node, Op::NC> &sm) {
  for (int c = t; c < kT3N * kT3N; c += kTpb3) {
    const int i = i0 - 1 + c % kT3N, j = j0 - 1 + c / kT3N;
    typename Op::Node n{};
    if (i >= 0 && i <= g.nx && j >= 0 && j <= g.ny && k >= 0 && k <= g.nz)
      n = op.stage(g, node_id(g, i, j, k));
    sm.plane[s][c] = n;
  }
}

// Thread t computes element t of layer ke (zero outside the box).
template <class Op>
__host__ __device__ inline void t3_element(const Op &op, const Grid3 &g, const Mat3 &m, int i0,
                                           int j0, int ke, int t,
                                           const T3LdsT<typename Op::Node, Op::NC> &sm,
                                           double out[8 * Op::NC]) {
  const int el = t % kT3E, ej = t / kT3E;
  const int ie = i0 - 1 + el, je = j0 - 1 + ej;
  if (ie < 0 || ie >= g.nx || je < 0 || je >= g.ny || ke < 0 || ke >= g.nz) {
    for (int x = 0; x < 8 * Op::NC; ++x) out[x] = 0.0;
    return;
  }
  const typename Op::Node *c[8];
  for (int b = 0; b < 8; ++b)
    c[b] = &sm.plane[(ke + corner_dk(b)) & 1][(ej + corner_dj(b)) * kT3N + el + corner_di(b)];
  op.element(g, m, ie + je * g.nx + ke * g.nx * g.ny, c, out);
}

// Thread t stores the corners of plane ke (h = 0: corners 0-3) or of plane
// ke + 1 (h = 1: corners 4-7) of its element.
template <int NC, class Node>
__host__ __device__ inline void t3_put(const double *out, int h, int t, T3LdsT<Node, NC> &sm) {
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < NC; ++c) sm.f[a][c][t] = out[NC * (4 * h + a) + c];
}

// Owned node column t (< kT3^2): the four stored corner values at its node,
// corner 2 of element (li, lj), 3 of (li+1, lj), 1 of (li, lj+1) and 0 of
// (li+1, lj+1) (corners 6, 7, 5, 4 for the upper half).
template <int NC, class Node>
__host__ __device__ inline void t3_gather(const T3LdsT<Node, NC> &sm, int t, double *s) {
  const int li = t % kT3, lj = t / kT3, e = lj * kT3E + li;
  for (int c = 0; c < NC; ++c)
    s[c] = sm.f[2][c][e] + sm.f[3][c][e + 1] + sm.f[1][c][e + kT3E] + sm.f[0][c][e + kT3E + 1];
}

// One block of an element-once operator, played by NT threads t0 .. t0+NT-1
// (the device runs one per thread, NT = 1; a host replay runs the block's
// kTpb3 threads in one call).  sync() is the block's barrier.
template <class Op, int NT, class Sync>
__host__ __device__ inline void t3_block(const Op &op, const Grid3 &g, const Mat3 &m, int blk,
                                         int t0, T3LdsT<typename Op::Node, Op::NC> &sm,
                                         double (&out)[NT][8 * Op::NC],
                                         double (&carry)[NT][Op::NC], const Sync &sync) {
  constexpr int NC = Op::NC;
  const int nxt = t3_tiles_x(g), nyt = t3_tiles_y(g);
  const int i0 = (blk % nxt) * kT3, j0 = ((blk / nxt) % nyt) * kT3;
  const int k0 = (blk / (nxt * nyt)) * kT3Z;
  const int k1 = (k0 + kT3Z < g.nz + 1) ? k0 + kT3Z : g.nz + 1;   // owned planes [k0, k1)
  const int kb = k0 > 0 ? k0 - 1 : 0;                              // element layers [kb, kl]
  const int kl = (k1 - 1 < g.nz - 1) ? k1 - 1 : g.nz - 1;
  for (int r = 0; r < NT; ++r)
    for (int c = 0; c < NC; ++c) carry[r][c] = 0.0;
  for (int ke = kb; ke <= kl; ++ke) {
    if (ke == kb)
      for (int r = 0; r < NT; ++r) t3_stage(op, g, i0, j0, ke, ke & 1, t0 + r, sm);
    for (int r = 0; r < NT; ++r) t3_stage(op, g, i0, j0, ke + 1, (ke + 1) & 1, t0 + r, sm);
    sync();
    for (int r = 0; r < NT; ++r) {
      t3_element(op, g, m, i0, j0, ke, t0 + r, sm, out[r]);
      t3_put<NC>(out[r], 0, t0 + r, sm);
    }
    sync();
    if (ke >= k0)
      for (int r = 0; r < NT; ++r) {
        const int t = t0 + r, i = i0 + t % kT3, j = j0 + t / kT3;
        if (t < kT3 * kT3 && i <= g.nx && j <= g.ny) {
          double s[NC];
          t3_gather<NC>(sm, t, s);
          const int id = node_id(g, i, j, ke);
          for (int c = 0; c < NC; ++c) op.q[id + c * g.N] = carry[r][c] + s[c];
        }
      }
    sync();
    for (int r = 0; r < NT; ++r) t3_put<NC>(out[r], 1, t0 + r, sm);
    sync();
    for (int r = 0; r < NT; ++r)
      if (t0 + r < kT3 * kT3) t3_gather<NC>(sm, t0 + r, carry[r]);
  }
  // the top plane of the box has the layer below only
  if (g.nz >= k0 && g.nz < k1)
    for (int r = 0; r < NT; ++r) {
      const int t = t0 + r, i = i0 + t % kT3, j = j0 + t / kT3;
      if (t < kT3 * kT3 && i <= g.nx && j <= g.ny) {
        const int id = node_id(g, i, j, g.nz);
        for (int c = 0; c < NC; ++c) op.q[id + c * g.N] = carry[r][c];
      }
    }
}

// Host replay of an element-once operator over its whole grid (tests only).
struct T3HostSync {
  void operator()() const {}
};
template <class Op>
inline void t3_host(const Op &op, const Grid3 &g, const Mat3 &m) {
  static T3LdsT<typename Op::Node, Op::NC> sm;
  static double out[kTpb3][8 * Op::NC], carry[kTpb3][Op::NC];
  for (int b = 0; b < t3_blocks(g); ++b)
    t3_block<Op, kTpb3>(op, g, m, b, 0, sm, out, carry, T3HostSync{});
}
inline void t3_tangent_host(const Grid3 &g, const Mat3 &m, const double *u, const double *d,
                            const double *p, double *q) {
  if (m.split == 1) t3_host(T3TangentOp<1>{u, d, p, q}, g, m);
  else t3_host(T3TangentOp<0>{u, d, p, q}, g, m);
}
// The tiled internal force pays only once the tiles fill the GPU: on fewer
// blocks the node gather, one thread per node, is faster (45 tiles at 32^3:
// 69 us tiled against 45 us gathered; 225 tiles at 64^3: 74 us against
// 164 us).
constexpr int kT3ForceMinBlocks = 128;
inline bool t3_force_tiled(const Grid3 &g) { return t3_blocks(g) >= kT3ForceMinBlocks; }

inline void t3_force_host(const Grid3 &g, const Mat3 &m, const double *u, const double *d,
                          double *R) {
  if (m.split == 1) t3_host(T3ForceOp<1>{u, d, R}, g, m);
  else t3_host(T3ForceOp<0>{u, d, R}, g, m);
}

// Grid of a one-index-per-thread launch over count indices.
__host__ __device__ inline int grid_index(int block, int thread) {
  return block * kTpb3 + thread;
}

inline int grid_blocks(int count) { return (count + kTpb3 - 1) / kTpb3; }

// ---- host side: mesh and material checks of the C ABI

// largest 3N and 8E: 32-bit indices with room for rounding up to whole blocks
constexpr long long kMaxIndexCount = (1LL << 31) - (1LL << 16);

inline pf_status make_grid(const pf3d_mesh *mesh, Grid3 *g) {
  if (!mesh || mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1 || !(mesh->lx > 0) ||
      !(mesh->ly > 0) || !(mesh->lz > 0) || !std::isfinite(mesh->lx) ||
      !std::isfinite(mesh->ly) || !std::isfinite(mesh->lz))
    return PF_E_INVALID_ARG;
  // bound the partial product before the third factor so that nothing
  // overflows 64 bits (each side is below 2^31)
  const long long nxy = ((long long)mesh->nx + 1) * ((long long)mesh->ny + 1);
  if (nxy > kMaxIndexCount / 3) return PF_E_INVALID_ARG;
  const long long N = nxy * ((long long)mesh->nz + 1);
  const long long E = (long long)mesh->nx * mesh->ny * mesh->nz;   // E < N
  if (N > kMaxIndexCount / 3 || E > kMaxIndexCount / 8) return PF_E_INVALID_ARG;
  *g = Grid3{mesh->nx, mesh->ny, mesh->nz, (int)N, (int)E, mesh->lx / mesh->nx,
             mesh->ly / mesh->ny, mesh->lz / mesh->nz};
  return PF_OK;
}

inline pf_status make_mat(const pf_material *mat, Mat3 *m) {
  if (!mat || !(mat->E > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->Gc > 0) ||
      !(mat->l > 0) || !(mat->eta >= 0) || !std::isfinite(mat->E) || !std::isfinite(mat->Gc) ||
      !std::isfinite(mat->l) || !std::isfinite(mat->eta) ||
      (mat->split != PF_SPLIT_VD && mat->split != PF_SPLIT_SPECTRAL))
    return PF_E_INVALID_ARG;
  const double mu = mat->E / (2.0 * (1.0 + mat->nu));
  const double lam = mat->E * mat->nu / ((1.0 + mat->nu) * (1.0 - 2.0 * mat->nu));
  *m = Mat3{lam,       mu,         lam + 2.0 * mu / 3.0, mat->Gc * mat->l,
            mat->eta,  mat->split, mat->Gc / mat->l};
  return PF_OK;
}

// Gate parameters; psi_crit < 0 means Gc / (c_w l) with c_w = 2 (AT2).
inline pf_status make_qp(int scheme, double psi_crit, double d_gate, const pf_material *mat,
                         Qp3 *qp) {
  if (!mat || scheme < 0 || scheme > 3 || std::isnan(psi_crit) || std::isnan(d_gate))
    return PF_E_INVALID_ARG;
  *qp = Qp3{scheme, psi_crit >= 0 ? psi_crit : mat->Gc / (2.0 * mat->l), d_gate};
  return PF_OK;
}

}  // namespace pf3d
