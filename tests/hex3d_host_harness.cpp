// Host replay of the 3-D kernels' grids, for the tests only: each launch of
// pf3d_kernels.hip becomes one loop over the same blocks and threads, and
// every index runs the same function of pf3d_ops.h, after the same mesh,
// material and gate checks as the C ABI.  Built host-only (no device code,
// no HIP calls), so it runs without a GPU.
#include "../paper_2209_07969_amd/csrc/pf3d_ops.h"

using namespace pf3d;

namespace {

template <class F>
void replay(int count, F &&body) {
  for (int b = 0; b < grid_blocks(count); ++b)
    for (int t = 0; t < kTpb3; ++t) {
      const int i = grid_index(b, t);
      if (i < count) body(i);
    }
}

}  // namespace

extern "C" {

int h3_internal_force(const pf3d_mesh *mesh, const pf_material *mat, const double *u,
                      const double *d, double *R) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  // the launch the C ABI makes: element-once tiles where they fill the GPU
  if (t3_force_tiled(g)) t3_force_host(g, m, u, d, R);
  else replay(g.N, [&](int n) { node_internal_force(g, m, n, u, d, R); });
  return PF_OK;
}

int h3_internal_force_tiled(const pf3d_mesh *mesh, const pf_material *mat, const double *u,
                            const double *d, double *R) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  t3_force_host(g, m, u, d, R);   // the element-once grid at any size
  return PF_OK;
}

int h3_internal_force_gather(const pf3d_mesh *mesh, const pf_material *mat, const double *u,
                             const double *d, double *R) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  replay(g.N, [&](int n) { node_internal_force(g, m, n, u, d, R); });
  return PF_OK;
}

int h3_tangent_apply(const pf3d_mesh *mesh, const pf_material *mat, const double *u,
                     const double *d, const double *p, double *q) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  t3_tangent_host(g, m, u, d, p, q);   // the element-once kernel's grid
  return PF_OK;
}

int h3_tangent_apply_gather(const pf3d_mesh *mesh, const pf_material *mat, const double *u,
                            const double *d, const double *p, double *q) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  replay(g.N, [&](int n) { node_tangent_apply(g, m, n, u, d, p, q); });
  return PF_OK;
}

int h3_phase_apply(const pf3d_mesh *mesh, const pf_material *mat, const double *coef,
                   const double *p, double *q) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  replay(g.N, [&](int n) { node_phase_apply(g, m, n, coef, p, q); });
  return PF_OK;
}

int h3_qp_update(const pf3d_mesh *mesh, const pf_material *mat, int scheme, double psi_crit,
                 double d_gate, const double *u, const double *d, const double *H_prev,
                 double *H, double *psi_s, uint16_t *flags, long long *n_gated) {
  Grid3 g;
  Mat3 m;
  Qp3 qp;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK ||
      make_qp(scheme, psi_crit, d_gate, mat, &qp) != PF_OK)
    return PF_E_INVALID_ARG;
  long long ng = 0;
  replay(g.E, [&](int e) { ng += elem_qp_update(g, m, qp, e, u, d, H_prev, H, psi_s, flags); });
  *n_gated = ng;
  return PF_OK;
}

int h3_predictor(const pf3d_mesh *mesh, const pf_material *mat, const double *d,
                 const double *dd, const double *H, const double *psi_s, const uint16_t *flags,
                 double *Hhat) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  replay(g.E, [&](int e) { elem_predictor(g, m, e, d, dd, H, psi_s, flags, Hhat); });
  return PF_OK;
}

int h3_tangent_diag(const pf3d_mesh *mesh, const pf_material *mat, const double *u,
                    const double *d, double *D) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  replay(g.N, [&](int n) { node_tangent_diag(g, m, n, u, d, D); });
  return PF_OK;
}

int h3_phase_diag(const pf3d_mesh *mesh, const pf_material *mat, const double *coef,
                  double *D) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  replay(g.N, [&](int n) { node_phase_diag(g, m, n, coef, D); });
  return PF_OK;
}

int h3_phase_rhs(const pf3d_mesh *mesh, const double *H, double *b) {
  Grid3 g;
  if (make_grid(mesh, &g) != PF_OK) return PF_E_INVALID_ARG;
  replay(g.N, [&](int n) { node_phase_rhs(g, n, H, b); });
  return PF_OK;
}

int h3_phase_coef(const pf3d_mesh *mesh, const pf_material *mat, int trial, double theta,
                  int floor, const double *H, const double *psi_s, const uint16_t *flags,
                  const double *d, double *coef, long long *below) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK) return PF_E_INVALID_ARG;
  long long nb = 0;
  replay(g.E, [&](int e) {
    nb += elem_phase_coef(g, m, e, trial, theta, floor, H, psi_s, flags, d, coef);
  });
  *below = nb;
  return PF_OK;
}

}  // extern "C"
