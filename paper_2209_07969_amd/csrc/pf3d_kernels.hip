// 3-D operator kernels (trilinear hexahedra) and their C ABI.
//
// One thread per node (operators) or per element (quadrature-point
// update); a node gathers the contributions of its up to eight elements, so
// every output is written by one thread in a fixed order (deterministic,
// no atomics).  The arithmetic lives in pf3d_ops.h.

#include "../../include/phasefield3d.h"
#include "pf3d_ops.h"

#include <hip/hip_runtime.h>

#include <cmath>

using namespace pf3d;

namespace {

__global__ void __launch_bounds__(kTpb3) k3_internal_force(Grid3 g, Mat3 m, const double *u,
                                                           const double *d, double *R) {
  const int n = grid_index(blockIdx.x, threadIdx.x);
  if (n < g.N) node_internal_force(g, m, n, u, d, R);
}

__global__ void __launch_bounds__(kTpb3) k3_tangent_apply(Grid3 g, Mat3 m, const double *u,
                                                          const double *d, const double *p,
                                                          double *q) {
  const int n = grid_index(blockIdx.x, threadIdx.x);
  if (n < g.N) node_tangent_apply(g, m, n, u, d, p, q);
}

__global__ void __launch_bounds__(kTpb3) k3_phase_apply(Grid3 g, Mat3 m, const double *coef,
                                                        const double *p, double *q) {
  const int n = grid_index(blockIdx.x, threadIdx.x);
  if (n < g.N) node_phase_apply(g, m, n, coef, p, q);
}

__global__ void __launch_bounds__(kTpb3) k3_qp_update(Grid3 g, Mat3 m, Qp3 qp, const double *u,
                                                      const double *d, const double *Hprev,
                                                      double *H, double *psi_s,
                                                      uint16_t *flags) {
  const int e = grid_index(blockIdx.x, threadIdx.x);
  if (e < g.E) (void)elem_qp_update(g, m, qp, e, u, d, Hprev, H, psi_s, flags);
}

__global__ void __launch_bounds__(kTpb3) k3_predictor(Grid3 g, Mat3 m, const double *d,
                                                      const double *dd, const double *H,
                                                      const double *psi_s,
                                                      const uint16_t *flags, double *Hhat) {
  const int e = grid_index(blockIdx.x, threadIdx.x);
  if (e < g.E) elem_predictor(g, m, e, d, dd, H, psi_s, flags, Hhat);
}

__global__ void __launch_bounds__(kTpb3) k3_tangent_diag(Grid3 g, Mat3 m, const double *u,
                                                         const double *d, double *D) {
  const int n = grid_index(blockIdx.x, threadIdx.x);
  if (n < g.N) node_tangent_diag(g, m, n, u, d, D);
}

__global__ void __launch_bounds__(kTpb3) k3_phase_diag(Grid3 g, Mat3 m, const double *coef,
                                                       double *D) {
  const int n = grid_index(blockIdx.x, threadIdx.x);
  if (n < g.N) node_phase_diag(g, m, n, coef, D);
}

__global__ void __launch_bounds__(kTpb3) k3_phase_rhs(Grid3 g, const double *H, double *b) {
  const int n = grid_index(blockIdx.x, threadIdx.x);
  if (n < g.N) node_phase_rhs(g, n, H, b);
}

__global__ void __launch_bounds__(kTpb3) k3_phase_coef(Grid3 g, Mat3 m, int trial, double theta,
                                                       int floor, const double *H,
                                                       const double *psi_s,
                                                       const uint16_t *flags, const double *d,
                                                       double *coef) {
  const int e = grid_index(blockIdx.x, threadIdx.x);
  if (e < g.E) (void)elem_phase_coef(g, m, e, trial, theta, floor, H, psi_s, flags, d, coef);
}

pf_status launched() {
  return hipGetLastError() == hipSuccess ? PF_OK : PF_E_HIP;
}

}  // namespace

extern "C" {

pf_status pf3d_op_internal_force(const pf3d_mesh *mesh, const pf_material *mat,
                                 const double *u, const double *d, double *R,
                                 void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!u || !d || !R || make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_internal_force, dim3(grid_blocks(g.N)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, m, u, d, R);
  return launched();
}

pf_status pf3d_op_tangent_apply(const pf3d_mesh *mesh, const pf_material *mat,
                                const double *u, const double *d, const double *p,
                                double *q, void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!u || !d || !p || !q || make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_tangent_apply, dim3(grid_blocks(g.N)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, m, u, d, p, q);
  return launched();
}

pf_status pf3d_op_phase_apply(const pf3d_mesh *mesh, const pf_material *mat,
                              const double *coef, const double *p, double *q,
                              void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!coef || !p || !q || make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_phase_apply, dim3(grid_blocks(g.N)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, m, coef, p, q);
  return launched();
}

pf_status pf3d_op_qp_update(const pf3d_mesh *mesh, const pf_material *mat, int32_t scheme,
                            double psi_crit, double d_gate, const double *u,
                            const double *d, const double *H_prev, double *H,
                            double *psi_s, uint16_t *flags, void *hip_stream) {
  Grid3 g;
  Mat3 m;
  Qp3 qp;
  if (!u || !d || !H_prev || !H || !psi_s || !flags || make_grid(mesh, &g) != PF_OK ||
      make_mat(mat, &m) != PF_OK || make_qp(scheme, psi_crit, d_gate, mat, &qp) != PF_OK)
    return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_qp_update, dim3(grid_blocks(g.E)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, m, qp, u, d, H_prev, H, psi_s,
                     flags);
  return launched();
}

pf_status pf3d_op_predictor(const pf3d_mesh *mesh, const pf_material *mat, const double *d,
                            const double *dd, const double *H, const double *psi_s,
                            const uint16_t *flags, double *Hhat, void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!d || !dd || !H || !psi_s || !flags || !Hhat || make_grid(mesh, &g) != PF_OK ||
      make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_predictor, dim3(grid_blocks(g.E)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, m, d, dd, H, psi_s, flags, Hhat);
  return launched();
}

pf_status pf3d_op_tangent_diag(const pf3d_mesh *mesh, const pf_material *mat, const double *u,
                               const double *d, double *D, void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!u || !d || !D || make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_tangent_diag, dim3(grid_blocks(g.N)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, m, u, d, D);
  return launched();
}

pf_status pf3d_op_phase_diag(const pf3d_mesh *mesh, const pf_material *mat, const double *coef,
                             double *D, void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!coef || !D || make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_phase_diag, dim3(grid_blocks(g.N)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, m, coef, D);
  return launched();
}

pf_status pf3d_op_phase_rhs(const pf3d_mesh *mesh, const double *H, double *b,
                            void *hip_stream) {
  Grid3 g;
  if (!H || !b || make_grid(mesh, &g) != PF_OK) return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_phase_rhs, dim3(grid_blocks(g.N)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, H, b);
  return launched();
}

pf_status pf3d_op_phase_coef(const pf3d_mesh *mesh, const pf_material *mat, int32_t trial,
                             double theta, int32_t floor, const double *H, const double *psi_s,
                             const uint16_t *flags, const double *d, double *coef,
                             void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!H || !coef || (trial && (!psi_s || !flags || !d)) || trial < 0 || trial > 1 ||
      floor < 0 || floor > 1 || !(theta >= 0.0 && theta <= 1.0) ||
      make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  hipLaunchKernelGGL(k3_phase_coef, dim3(grid_blocks(g.E)), dim3(kTpb3), 0,
                     static_cast<hipStream_t>(hip_stream), g, m, trial, theta, floor, H, psi_s,
                     flags, d, coef);
  return launched();
}

}  // extern "C"
