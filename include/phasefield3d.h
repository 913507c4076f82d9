/* phasefield3d.h - C ABI of the 3-D path: trilinear hexahedra (Q1, 2x2x2
 * Gauss) on a structured box, the volumetric-deviatoric or the spectral
 * split of Section 2 with the full 3-D strain, and the AT2 phase operator,
 * as in the paper's one-element-thick slab (Section 4) or a full 3-D panel.
 * Two parts: the element and node operators of the 2-D path (internal
 * force, tangent apply and diagonal, phase apply, diagonal, right-hand side
 * and mass coefficients, quadrature-point update, predictor), and below
 * them a load step built on those operators (pf3d_create ... pf3d_load_step).
 *
 * The operator entry points (pf3d_op_*) are stateless: each takes the mesh
 * and material by value (read on the host), device pointers for the
 * fields, and a hipStream_t (void *, NULL = the null stream) on which its
 * one kernel is enqueued; it returns once the kernel is enqueued, without
 * synchronising.  Fields are
 * structure-of-arrays in device memory, all FP64 unless stated:
 *   node (i, j, k) has id n = i + j (nx+1) + k (nx+1)(ny+1), N nodes;
 *   element (ie, je, ke) has id e = ie + je nx + ke nx ny, E elements;
 *   displacement-like fields [3N]: the x plane, then y, then z;
 *   nodal scalars [N]; quadrature-point fields [8E], plane q holding point
 *   q of every element (index e + q E).  Corner a of an element sits at
 *   offsets (((a+1)>>1)&1, (a>>1)&1, a>>2) from its first node, and Gauss
 *   point q at reference coordinates (2 di - 1, 2 dj - 1, 2 dk - 1)/sqrt 3
 *   of corner q.
 * The caller owns every buffer; outputs must not alias inputs.  No Dirichlet
 * masking is applied.  Errors: PF_E_INVALID_ARG for a null pointer, a bad
 * mesh (nx, ny, nz >= 1, lengths > 0, 3N and 8E at most 2^31 - 2^16) or a
 * bad material; PF_E_HIP if the launch fails.  Nothing is written on error.
 * The spectral split takes the principal strains of the full 3x3 strain
 * (cyclic Jacobi rotations); a principal strain counts as positive only
 * when strictly above zero, as does the trace.
 */
#ifndef PHASEFIELD3D_H
#define PHASEFIELD3D_H

#include "phasefield.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf3d_mesh {
  int32_t nx, ny, nz;      /* elements per direction, >= 1 */
  double lx, ly, lz;       /* box size [mm], > 0           */
} pf3d_mesh;

/* Internal force R = sum_e sum_q B^T sigma(eps(u), g(d_q)) w detJ with the
 * split stress of Section 2 (eq_sigma; spectral: g [lam <t>_+ I + 2 mu
 * eps+] + lam <t>_- I + 2 mu eps-), g(d) = (1-d)^2 + eta.
 * u [3N], d [N] -> R [3N]. */
pf_status pf3d_op_internal_force(const pf3d_mesh *mesh, const pf_material *mat,
                                 const double *u, const double *d, double *R,
                                 void *hip_stream);

/* Tangent apply q = K_t(u; d) p of the split stress at u (eq_definition_+):
 * VD, volumetric factor g K where tr eps(u) > 0 strictly, else K; spectral,
 * the derivative of eps+ with the divided differences (<e_i>_+ - <e_j>_+) /
 * (e_i - e_j) between principal strains, H(e_i) where they coincide.
 * u, p, q [3N]; d [N]. */
pf_status pf3d_op_tangent_apply(const pf3d_mesh *mesh, const pf_material *mat,
                                const double *u, const double *d, const double *p,
                                double *q, void *hip_stream);

/* Phase operator q = sum [coef_q N N^T + Gc l grad N . grad N^T] w detJ p
 * with a per-point coefficient coef [8E] (K_dd uses Gc/l + 2H, the trial
 * block of Section 3.4 a reduced one).  p, q [N]. */
pf_status pf3d_op_phase_apply(const pf3d_mesh *mesh, const pf_material *mat,
                              const double *coef, const double *p, double *q,
                              void *hip_stream);

/* Quadrature-point update (Sections 2, 3.5): from u [3N], d [N] and the
 * committed history H_prev [8E], write H = max(H_prev, psi+) [8E], the
 * scheme part psi_S [8E] (scheme 0 ST: 0; 1 S1: psi_vol; 2 S2: psi_dev;
 * 3 S3: psi+, with psi_vol = K/2 <tr eps>_+^2 and psi_dev = mu eps_dev:eps_dev
 * for VD, lam/2 <tr eps>_+^2 and mu sum <e_i>_+^2 for the spectral split) and per element a flag
 * word flags [E] (uint16): bit q = tr eps > 0 at point q, bit 8+q = the
 * softening gate at point q (scheme != 0, psi+ > psi_crit, psi+ > H_prev
 * and d_q < d_gate).  psi_crit < 0 means Gc / (2 l). */
pf_status pf3d_op_qp_update(const pf3d_mesh *mesh, const pf_material *mat, int32_t scheme,
                            double psi_crit, double d_gate, const double *u,
                            const double *d, const double *H_prev, double *H,
                            double *psi_s, uint16_t *flags, void *hip_stream);

/* Fixed-stress predictor (Section 3.3 half-step update, Section 3.5 gate and
 * positive-increment rule): Hhat = max(H, H + ((1 + a Dd)^2 - 1) psi_S) at
 * gated points with Dd_q > 0, else H; a = 2(1-d_q)/g(d_q).  d, dd [N];
 * H, psi_s, Hhat [8E]; flags [E] as written by pf3d_op_qp_update. */
pf_status pf3d_op_predictor(const pf3d_mesh *mesh, const pf_material *mat, const double *d,
                            const double *dd, const double *H, const double *psi_s,
                            const uint16_t *flags, double *Hhat, void *hip_stream);

/* Diagonal of the tangent K_t(u; d) (the Jacobi preconditioner of the
 * displacement solve).  u [3N], d [N] -> D [3N]. */
pf_status pf3d_op_tangent_diag(const pf3d_mesh *mesh, const pf_material *mat, const double *u,
                               const double *d, double *D, void *hip_stream);

/* Diagonal of the phase operator with the per-point coefficient coef [8E]:
 * D_n = sum [coef_q N_n^2 + Gc l |grad N_n|^2] w detJ.  -> D [N]. */
pf_status pf3d_op_phase_diag(const pf3d_mesh *mesh, const pf_material *mat, const double *coef,
                             double *D, void *hip_stream);

/* Right-hand side of the AT2 evolution equation (Section 2 with w = d^2):
 * b = sum 2 H_q N w detJ.  H [8E] -> b [N]. */
pf_status pf3d_op_phase_rhs(const pf3d_mesh *mesh, const double *H, double *b,
                            void *hip_stream);

/* Mass coefficient of the phase block at every point, coef [8E]: with
 * trial = 0 the AT2 coefficient Gc/l + 2H; with trial = 1 that of the trial
 * block K_dd + K~ (Section 3.4): at gated points (flags bit 8+q, from
 * pf3d_op_qp_update) c - c_S with c_S = 8 (1-d_q)^2 / g(d_q) psi_S, and
 * where that falls below theta c it is raised to theta c (floor = 1) or kept
 * (floor = 0, the unfloored block, possibly indefinite).  psi_s, flags and
 * d are read only with trial = 1 (may be NULL otherwise).  0 <= theta <= 1. */
pf_status pf3d_op_phase_coef(const pf3d_mesh *mesh, const pf_material *mat, int32_t trial,
                             double theta, int32_t floor, const double *H, const double *psi_s,
                             const uint16_t *flags, const double *d, double *coef,
                             void *hip_stream);

/* ---------------------------------------------------------------------------
 * 3-D load steps (Sections 3.1, 3.3-3.5 on hexahedra): the staggered loop of
 * pf_load_step with these operators, in FP64 with Jacobi PCG for every
 * linear solve, AT2 with the history field and, for S1/S2/S3, the floored
 * trial block with predict -> correct.  pf3d_create takes pf_solver_opts
 * (NULL: defaults) and refuses, with PF_E_INVALID_ARG, precision other than
 * PF_FP64, precond other than PF_PC_JACOBI, phase_model AT1, the literal
 * trial readings, and the 2-D checks' bad values.  The context owns its
 * device memory (hipMalloc) and runs on hip_stream; calls on one context
 * must not overlap.  Host arrays are copied before the call returns.
 * Every reduction is summed per block by a fixed tree and over the blocks
 * in order on the host, so results are deterministic.
 * ------------------------------------------------------------------------- */
typedef struct pf3d_ctx pf3d_ctx;

pf_status pf3d_create(const pf3d_mesh *mesh, const pf_material *mat,
                      const pf_solver_opts *opts, void *hip_stream, pf3d_ctx **out);

/* Frees every buffer; NULL is accepted. */
pf_status pf3d_destroy(pf3d_ctx *ctx);

/* Displacement Dirichlet data of one group (0 <= group < 8): component
 * comp[k] (0 = x, 1 = y, 2 = z) of node node[k] is load_factor *
 * value_per_unit_load[k].  Replaces the group's previous data.  Group 1 is
 * the loaded group whose reaction the step statistics carry (group 0 if
 * group 1 is empty).  Errors: PF_E_INVALID_ARG for out-of-range nodes,
 * components or groups, PF_E_NONFINITE for non-finite values. */
pf_status pf3d_set_dirichlet_u(pf3d_ctx *ctx, int32_t group, int64_t n, const int64_t *node,
                               const int8_t *comp, const double *value_per_unit_load);

/* Phase-field Dirichlet data: node[k] keeps value[k] (imposed at once). */
pf_status pf3d_set_dirichlet_d(pf3d_ctx *ctx, int64_t n, const int64_t *node,
                               const double *value);

/* One load step at load_factor, committed at the end (H_n = max(H_{n-1},
 * Psi+(u_n))).  stats (may be NULL): counts as for pf_load_step, force[0]
 * and force[1] the x and y reactions of the loaded group (all three from
 * pf3d_reaction_force).  Returns PF_E_NOT_CONVERGED, not fatal, if the loop
 * ended at max_stag or a Newton solve at max_newton (the step is committed
 * either way); PF_E_NONFINITE if the staggered residual is not finite;
 * PF_E_HIP on a device error (the state is then undefined). */
pf_status pf3d_load_step(pf3d_ctx *ctx, double load_factor, pf_step_stats *stats);

/* Reaction of a Dirichlet group at the committed state: the internal force
 * summed over its entries per component, force[3] = (x, y, z). */
pf_status pf3d_reaction_force(pf3d_ctx *ctx, int32_t group, double force[3]);

/* Committed state to host arrays (each may be NULL): u [3N] (x, y, z
 * planes), d [N], H [8E] (plane q = point q of every element). */
pf_status pf3d_get_state(pf3d_ctx *ctx, double *u, double *d, double *H);

/* Committed state from host arrays in the same layouts (each may be NULL,
 * keeping that field): checkpoint and resume.  The phase field's Dirichlet
 * values are imposed on d.  Errors: PF_E_NONFINITE for NaN/Inf (nothing is
 * written then). */
pf_status pf3d_set_state(pf3d_ctx *ctx, const double *u, const double *d, const double *H);

#ifdef __cplusplus
}
#endif

#endif /* PHASEFIELD3D_H */
