/*
 * phasefield.h -- C ABI of the MI355X phase-field fracture library.
 *
 * The library advances a brittle-fracture problem (AT2 phase field with a
 * history field, plane strain, structured Q1 mesh) one load step at a time
 * with the standard staggered scheme (Luo, Section 3.1) or one of the
 * fixed-stress schemes S1/S2/S3 (Sections 3.3-3.5).  Every numerical step
 * runs in HIP kernels on the device; the host only drives the loops and reads
 * back scalars (norms, counts).
 *
 * Conventions
 *   - Mesh: [0,lx] x [0,ly], nx x ny elements.  Node (i,j) has id i + j*(nx+1),
 *     N = (nx+1)*(ny+1).  Element (i,j) has id i + j*nx, E = nx*ny; its corners
 *     are (i,j), (i+1,j), (i+1,j+1), (i,j+1).
 *   - Quadrature: 2x2 Gauss, points ordered (-,-), (+,-), (+,+), (-,+).
 *   - Displacement arrays are structure-of-arrays: u[0..N) = u_x, u[N..2N) = u_y.
 *   - Per-quadrature-point arrays are QP-major planes: H[q*E + e], q = 0..3.
 *   - Units: N, mm, MPa.  Forces are per unit thickness.
 *   - Host arrays passed in are caller-owned and copied before the call
 *     returns.  Device pointers (the pf_op_* calls) are caller-owned, must hold
 *     the stated number of elements and must be valid on the context's device;
 *     those calls are stream-ordered on the context's stream and do not
 *     synchronise.
 *   - Every call returns a pf_status; on failure pf_last_error(ctx) holds a
 *     message.  A context is not thread-safe.
 */
#ifndef PHASEFIELD_H
#define PHASEFIELD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_ctx pf_ctx;

typedef enum {
  PF_OK = 0,
  PF_E_INVALID_ARG = 1,   /* bad size, pointer, index or option            */
  PF_E_OOM = 2,           /* device allocation failed                      */
  PF_E_HIP = 3,           /* a HIP runtime call failed                     */
  PF_E_STATE = 4,         /* call not valid in the context's current state */
  PF_E_NOT_CONVERGED = 5, /* max_stag / max_newton reached; state is kept  */
  PF_E_BREAKDOWN = 6,     /* CG saw p.Ap <= 0                              */
  PF_E_NONFINITE = 7      /* a norm became NaN or Inf                      */
} pf_status;

/* Staggered schemes: ST (Section 3.1) and the fixed-stress schemes holding the
 * first stress invariant (S1), the second (S2) or both (S3) (Section 3.4,
 * table of assumptions). */
typedef enum { PF_ST = 0, PF_S1 = 1, PF_S2 = 2, PF_S3 = 3 } pf_scheme;

/* Energy split: volumetric-deviatoric (Section 2, used throughout the paper)
 * or spectral (named in Section 2 as an extension). */
typedef enum { PF_SPLIT_VD = 0, PF_SPLIT_SPECTRAL = 1 } pf_split;

/* Precision of the inner linear solves.  PF_FP64: everything in FP64.
 * PF_MIXED: CG vectors and operator data in FP32 inside FP64 outer loops
 * (Newton for u, iterative refinement for d); history, norms and the
 * reaction force stay FP64. */
typedef enum { PF_FP64 = 0, PF_MIXED = 1 } pf_precision;

/* Preconditioner of the linear solves: Jacobi, or Jacobi-Chebyshev (m
 * Chebyshev steps on D^-1 A over [lambda_max/30, lambda_max], lambda_max times
 * 1.2 from a power iteration that continues from the previous solve's vector
 * for every solve). */
typedef enum { PF_PC_JACOBI = 0, PF_PC_JACOBI_CHEBYSHEV = 1 } pf_precond;

/* Trial block K_dd + K~ of S1/S2/S3 (Section 3.4).  FLOORED raises a gated
 * mass coefficient c - c_S below theta*c (trial_floor) to theta*c, so the
 * block stays SPD and is solved by PCG.  UNFLOORED keeps c - c_S as it is:
 * the block may be indefinite and is solved by MINRES in FP64 with
 * M = |diag| (tol_pcg on the M^-1 norm of the residual, at most max_cg
 * iterations). */
typedef enum { PF_TRIAL_FLOORED = 0, PF_TRIAL_UNFLOORED = 1 } pf_trial_operator;

/* What the trial increment Dd feeds.  PREDICT_CORRECT: the predicted
 * energy (Sections 3.3, 3.5), then the evolution solve with it frozen.
 * TRIAL_ONLY: d^{k+1} = d^k + Dd directly, with no energy update and no
 * corrected solve (the end of Section 3.5 notes that linear AT2 with a
 * history variable needs no energy update); ungated iterations take the
 * standard solve.  The trial-only increment is computed in FP64 in either
 * precision. */
typedef enum { PF_TRIAL_PREDICT_CORRECT = 0, PF_TRIAL_ONLY = 1 } pf_trial_update;

/* Evolution equation (Section 2).  AT2_HISTORY: AT2 (w = d^2, c_w = 2) driven
 * by the history field H = max(H, Psi+).  AT1_PENALTY: AT1 (w = d,
 * c_w = 8/3) driven by Psi+ of the current displacement, with the penalty
 * gamma <d - d_{n-1}>_-, gamma = 27 Gc / (64 l tol_ir^2), as the
 * irreversibility constraint (eq_evolution_equation); its phase solve is a
 * semismooth Newton iteration (FP64 in either precision, at most 60 steps,
 * PF_E_NOT_CONVERGED beyond) that ends when ||F_d|| is within tol_pcg of the
 * solve's starting residual, or when the penalty's active points have
 * stopped changing and a step no longer halves ||F_d|| (its rounding
 * floor); its staggered residual is ||F_d|| / ||sum 2 Psi+ N||.  H is still
 * kept as the gate's Psi_max, and Psi_crit defaults to Gc / (c_w l). */
typedef enum { PF_AT2_HISTORY = 0, PF_AT1_PENALTY = 1 } pf_phase_model;

typedef struct {
  int32_t nx, ny;              /* elements per direction, >= 1              */
  double lx, ly;               /* domain size [mm], > 0                     */
  const uint8_t *elem_active;  /* nx*ny flags (1 = active) or NULL = all    */
} pf_mesh_desc;

/* Material (Section 2): g(d) = (1-d)^2 + eta; the crack model (AT2 or AT1)
 * is pf_solver_opts::phase_model. */
typedef struct {
  double E, nu;    /* Young's modulus [MPa], Poisson ratio                   */
  double Gc, l;    /* fracture toughness [N/mm], length scale [mm]           */
  double eta;      /* residual stiffness                                     */
  int32_t split;   /* pf_split                                               */
} pf_material;

typedef struct {
  int32_t scheme;       /* pf_scheme                                          */
  int32_t precision;    /* pf_precision                                       */
  int32_t precond;      /* pf_precond                                         */
  int32_t cheb_degree;  /* Chebyshev steps m (1..16) for PF_PC_JACOBI_CHEBYSHEV; odd
                           m keeps the preconditioner SPD even if the
                           estimated lambda_max is too low                   */
  double tol_stag;      /* staggered tolerance on ||R_d||/||b|| (Section 3.1) */
  double tol_pcg;       /* relative tolerance of each linear correction solve */
  double tol_newton;    /* Newton: ||R_u|| <= tol_newton * ||R_u(lifted)||    */
  double tol_inner;     /* PF_MIXED: tightest relative tolerance of an FP32   */
                        /* inner CG.  A displacement solve asks for          */
                        /* min(0.1, max(tol_inner, 0.1 tol/||R_u||)), tol    */
                        /* being the Newton target (inexact Newton)          */
  int32_t max_stag;     /* max u-solves per load step (k = 0 included)        */
  int32_t max_newton;   /* max Newton iterations per u-solve                  */
  int32_t max_cg;       /* max CG iterations per linear solve                 */
  int32_t cg_check;     /* CG iterations enqueued between convergence polls   */
  double psi_crit;      /* softening threshold; < 0 means Gc/(c_w l)          */
  double d_gate;        /* gate: predictor only where d < d_gate (0.95)       */
  double trial_floor;   /* theta: trial mass coefficient >= theta*(Gc/l+2H)   */
  int32_t march_rows;   /* node rows per work item of the operator kernels:   */
                        /* 2, 4 or 8; 0 = chosen from the mesh size           */
  int32_t cg_kernels;   /* CG formulation: 0 = by precision (FP64: one kernel  */
                        /* per iteration, FP32: two), 1 = one kernel per      */
                        /* iteration (Chronopoulos-Gear recurrences, one      */
                        /* reduction), 2 = two kernels (standard recurrences) */
  double cheb_ratio;    /* Jacobi-Chebyshev interval [lmax/ratio, lmax]; 0 = 30 */
  int32_t trial_operator; /* pf_trial_operator                                */
  int32_t trial_update;   /* pf_trial_update                                  */
  double tol_ir;          /* AT1_PENALTY: irreversibility tolerance (0.01)    */
  int32_t phase_model;    /* pf_phase_model                                   */
  int32_t guess_vectors;  /* 0..4: displacement CG solves whose relative      */
                          /* tolerance is below 1e-3 start from the Galerkin  */
                          /* projection of their right-hand side onto the     */
                          /* last guess_vectors such solutions (two-kernel CG */
                          /* on the context's stream only; 0 = off)           */
} pf_solver_opts;

typedef struct {
  int32_t n_stag;       /* u-solves in the step, k = 0 included               */
  int32_t n_newton;     /* Newton linear solves                               */
  int32_t n_trial;      /* trial (augmented) phase solves                     */
  int32_t n_dsolve;     /* corrected / standard phase solves                  */
  int64_t n_cg_u;       /* CG iterations, displacement solves                 */
  int64_t n_cg_d;       /* CG iterations, phase solves                        */
  int64_t n_cg_trial;   /* CG iterations, trial solves                        */
  int64_t gated_max;    /* max gated quadrature points over the iterations    */
  int64_t floor_hits;   /* gated points whose trial coefficient was floored   */
  double r_stag;        /* staggered residual at exit                         */
  double force[2];      /* reaction of the load group (x, y) at exit          */
  double time_ms;       /* host wall time of the call                         */
  double dof_updates;   /* sum over CG solves of free DOFs x iterations       */
  int32_t converged;    /* 1 if r_stag <= tol_stag and Newton converged       */
  int32_t cg_not_converged; /* linear solves that hit max_cg                  */
  double time_u_ms;     /* host wall time of the displacement solves (Newton, */
                        /* k = 0 included)                                    */
  double time_d_ms;     /* host wall time of the phase part of k >= 1: trial, */
                        /* predictor and evolution solve (the paper's split   */
                        /* of wall time into d- and u-solves, Section 4.4)    */
} pf_step_stats;

/* Fill *opts with defaults: ST, FP64, Jacobi (cheb_degree 3), tol_stag 1e-5, tol_pcg 1e-10,
 * tol_newton 1e-9, tol_inner 1e-5, max_stag 500, max_newton 25,
 * max_cg 200000, cg_check 32, psi_crit -1, d_gate 0.95, trial_floor 0.1,
 * march_rows 0, cg_kernels 0, cheb_ratio 0 (30), trial_operator FLOORED,
 * trial_update PREDICT_CORRECT, tol_ir 0.01, phase_model AT2_HISTORY,
 * guess_vectors 0. */
void pf_default_opts(pf_solver_opts *opts);

/* Create a context on the current HIP device.  hip_stream is a hipStream_t
 * (NULL = the null stream) on which every kernel of this context runs.  All
 * device memory is owned by the context.  Size limit (32-bit kernel
 * indices): 2 (nx+1)(ny+1) and 4 nx ny at most 2^31 - 2^16, i.e. up to
 * about 23170 x 23170 elements.  Errors: PF_E_INVALID_ARG for bad sizes or
 * options (checked before any device call), PF_E_OOM, PF_E_HIP. */
pf_status pf_create(const pf_mesh_desc *mesh, const pf_material *mat,
                    const pf_solver_opts *opts, void *hip_stream, pf_ctx **out);

/* Release every device buffer (through the release callback when an
 * allocator is installed) and the context itself. */
pf_status pf_destroy(pf_ctx *ctx);

/* Device-memory allocator for the context's buffers, e.g. a framework's
 * caching allocator.  alloc(bytes, user) returns device memory on the
 * context's device, aligned to 256 bytes, or NULL; release(ptr, user) takes
 * it back.  The call moves every buffer the context already holds to memory
 * from alloc (contents copied on the context's stream, then synchronised)
 * and returns the old buffers to the previous allocator; later allocations
 * and pf_destroy use the new pair.  Both NULL restores hipMalloc/hipFree.
 * The callbacks and user must stay valid until pf_destroy or the next
 * pf_set_allocator.  Captured CG batches are discarded and re-captured on
 * first use.  Errors: PF_E_INVALID_ARG if exactly one callback is NULL,
 * PF_E_STATE inside an open step, PF_E_OOM if alloc returns NULL or
 * misaligned memory (the context then keeps its old buffers). */
typedef void *(*pf_alloc_fn)(size_t bytes, void *user);
typedef void (*pf_release_fn)(void *ptr, void *user);
pf_status pf_set_allocator(pf_ctx *ctx, pf_alloc_fn alloc, pf_release_fn release, void *user);

/* Displacement Dirichlet data of one group (0 <= group < 8).  Entry k fixes
 * component comp[k] (0 = x, 1 = y) of node node[k] to
 * load_factor * value_per_unit_load[k].  Replaces the group's previous data.
 * Nodes of masked-out regions are fixed to zero automatically.
 * Errors: PF_E_INVALID_ARG for out-of-range nodes/components. */
pf_status pf_set_dirichlet_u(pf_ctx *ctx, int32_t group, int64_t n,
                             const int64_t *node, const int8_t *comp,
                             const double *value_per_unit_load);

/* Phase-field Dirichlet data (e.g. a notch d = 1): node[k] keeps value[k]. */
pf_status pf_set_dirichlet_d(pf_ctx *ctx, int64_t n, const int64_t *node,
                             const double *value);

/* One load step at load_factor (Section 3.1 / 3.3-3.5): staggered
 * iterations until r_stag <= tol_stag or max_stag u-solves, then commit
 * (u_n, d_n, H_n) and evaluate the reaction forces.  PF_E_NOT_CONVERGED is
 * not fatal: the step is committed and stats are filled. */
pf_status pf_load_step(pf_ctx *ctx, double load_factor, pf_step_stats *stats);

/* Finer-grained stepping.  The first call after a commit opens a step at
 * load_factor and performs k = 0 (the displacement solve only); each later
 * call performs one staggered iteration k >= 1 (trial + predictor for S*,
 * phase solve, displacement solve).  stats accumulates over the open step
 * and stats->r_stag is the staggered residual after this call.
 * pf_commit_step closes the step.  Errors: PF_E_STATE if load_factor
 * differs from the open step's. */
pf_status pf_staggered_iterate(pf_ctx *ctx, double load_factor, pf_step_stats *stats);
/* Commits the open step: H_n, d_{n-1} (AT1) and the reaction force of the
 * load group (reported by the next pf_reaction_force).  Errors: PF_E_STATE
 * when no step is open. */
pf_status pf_commit_step(pf_ctx *ctx);

/* Reaction force of a Dirichlet group: the sum over its entries of the
 * internal force sum_e int B^T sigma (Section 3.2, weak form F_u) at the
 * committed state, split by component into force[0] (x) and force[1] (y). */
pf_status pf_reaction_force(pf_ctx *ctx, int32_t group, double force[2]);

/* Committed state, host arrays: u [2N] SoA, d [N], H [4E] QP planes (the
 * history max(H_{n-1}, psi+) of the last committed step).  Any pointer may
 * be NULL to skip it. */
pf_status pf_get_state(pf_ctx *ctx, double *u, double *d, double *H);
/* Overwrite the committed state (any pointer may be NULL).  Errors:
 * PF_E_NONFINITE if an input holds NaN/Inf, PF_E_STATE inside an open step. */
pf_status pf_set_state(pf_ctx *ctx, const double *u, const double *d, const double *H);

const char *pf_status_string(pf_status s);
const char *pf_last_error(const pf_ctx *ctx);

/* Number of free displacement / phase DOFs (after Dirichlet data and mask). */
pf_status pf_free_dofs(pf_ctx *ctx, int64_t *n_free_u, int64_t *n_free_d);

/* ---------------------------------------------------------------------------
 * Batched sweeps: many independent problems advanced together (a parameter
 * sweep of uneven instances).  Each member context should have its own HIP
 * stream (pf_create's hip_stream).  Two modes:
 *  - shared launches (default): one host thread per member runs its load
 *    step; its FP32 Jacobi CG solves (mixed precision) go to a service
 *    thread that keeps one CG loop running over every queued system: per CG
 *    iteration one apply launch per (operator, split, work-item height) and
 *    one update launch, over a table of the systems, each keeping the
 *    blocks it would have on its own.  Every few iterations (at the status
 *    poll) finished systems return to their members and newly queued ones
 *    join, so no member waits for another's solve to end.  Other solves
 *    (FP64, Jacobi-Chebyshev) run on the member's stream.  The tables live
 *    in memory of the batch's own (hipMalloc and hipHostMalloc), not in a
 *    member's installed allocator.
 *  - concurrent streams: a pool of host threads (4 unless
 *    pf_batch_set_workers says otherwise) runs the members' steps, whose
 *    kernels overlap on the GPU.
 * Results are bit-identical to stepping the members one by one in either
 * mode.  The batch borrows its members: destroy it first.
 * ------------------------------------------------------------------------- */
typedef struct pf_batch pf_batch;
/* n >= 1 distinct, non-NULL members.  Errors: PF_E_INVALID_ARG. */
pf_status pf_batch_create(int32_t n, pf_ctx *const *members, pf_batch **out);
/* enable = 1: shared launches (default); 0: concurrent streams. */
pf_status pf_batch_set_shared_launches(pf_batch *b, int32_t enable);
/* Host threads of the concurrent-stream mode (>= 1; default 4). */
pf_status pf_batch_set_workers(pf_batch *b, int32_t workers);
/* load_factors[n], stats[n] (may be NULL).  Returns PF_OK, or
 * PF_E_NOT_CONVERGED if any member did not converge (all members are still
 * committed), or the first error of a member. */
pf_status pf_batch_load_step(pf_batch *b, const double *load_factors, pf_step_stats *stats);
/* Frees the batch and its shared-launch tables (its host threads live only
 * inside each pf_batch_load_step call); the members stay valid and are
 * destroyed by their owner afterwards.  NULL is accepted. */
pf_status pf_batch_destroy(pf_batch *b);

/* Autotuning of the operator kernels' work-item height (2, 4 or 8 node rows
 * per wave): times `reps` launches of the displacement CG kernel for each
 * candidate on the current state and keeps the fastest; *chosen receives it.
 * Must be called outside an open step. */
pf_status pf_autotune(pf_ctx *ctx, int32_t reps, int32_t *chosen);

/* Kernel timing for measurement.  When enabled, the CG drivers time a sample
 * of the CG kernel launches with HIP events on the context's stream: in one
 * enqueued CG batch of every eight of the displacement solves and of the
 * phase solves (counted from enabling, the first included), the first
 * iteration's operator kernel (idempotent: it only reads buffers it does not
 * write) is launched four times back to back between one event pair.  Launch counts and elapsed times accumulate.
 * Single-kernel CG solves time that kernel (a whole iteration); two-kernel
 * CG solves time the fused operator apply and their vector update.  The
 * update is one launch between the events, except with Jacobi-Chebyshev of
 * degree >= 2, where it is fused with the first polynomial step (with the
 * first two steps on LDS tiles, degree >= 3) into a repeatable operator
 * kernel timed like the apply.  The next separate polynomial step of the
 * displacement solves (repeatable) is timed too.
 * kernel: 0 = elasticity CG kernel, 1 = phase CG kernel, 2 = vector update
 * (fused with the first Chebyshev step where it applies) of the
 * displacement solves, 3 = elasticity Chebyshev step.  Enabling resets the
 * counters. */
pf_status pf_set_profiling(pf_ctx *ctx, int32_t enable);
/* Outputs (each may be NULL): timed launches, their summed milliseconds, and
 * the nodes one launch covers.  Errors: PF_E_INVALID_ARG for a kernel id
 * outside 0..3. */
pf_status pf_kernel_time(pf_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms,
                         int64_t *nodes_per_launch);

/* ---------------------------------------------------------------------------
 * Operator-level entry points (device pointers, FP64).  They run the same
 * kernels the solver uses, on the context's mesh, material and masks, and
 * exist for verification and measurement.  No Dirichlet masking is applied
 * unless stated.
 * ------------------------------------------------------------------------- */

/* Internal force R = sum_e sum_q B^T sigma(eps(u), g(d)) w detJ with the
 * split stress (Section 2, eq_sigma).  u [2N], d [N] -> R [2N]. */
pf_status pf_op_internal_force(pf_ctx *ctx, const double *u, const double *d, double *R);

/* Tangent apply q = K_t(u; d) p: the split tangent with its active
 * indicators (eq_definition_+) taken at u.  u, p, q [2N]; d [N]. */
pf_status pf_op_tangent_apply(pf_ctx *ctx, const double *u, const double *d,
                              const double *p, double *q);

/* Phase operator q = sum [coef_q N N^T + Gc l grad N grad N^T] w detJ p with
 * an arbitrary per-QP coefficient coef [4E] (K_dd uses Gc/l + 2H, the
 * augmented block of Section 3.4 a reduced one).  p, q [N]. */
pf_status pf_op_phase_apply(pf_ctx *ctx, const double *coef, const double *p, double *q);

/* Quadrature-point update (Sections 2, 3.5): from u [2N], d [N] and the
 * committed history H_prev [4E], write H = max(H_prev, psi+) [4E], the
 * scheme part psi_S [4E] (psi_vol for S1, psi_dev for S2, psi+ for S3) and
 * per element a flag byte [E]: bits 0-3 = tr eps > 0 at QP q, bits 4-7 =
 * softening gate at QP q.  Returns the number of gated points in *n_gated. */
pf_status pf_op_qp_update(pf_ctx *ctx, int32_t scheme, const double *u, const double *d,
                          const double *H_prev, double *H, double *psi_s,
                          uint8_t *flags, int64_t *n_gated);

/* Fixed-stress predictor (Section 3.3 half-step update, Section 3.5 gate and
 * positive-increment rule): Hhat = max(H, H + ((1 + a Dd)^2 - 1) psi_S) at
 * gated points with Dd_q > 0, else H; a = 2(1-d_q)/g(d_q).  d, dd [N];
 * H, psi_s, Hhat [4E]; flags [E] as written by pf_op_qp_update. */
pf_status pf_op_predictor(pf_ctx *ctx, const double *d, const double *dd,
                          const double *H, const double *psi_s,
                          const uint8_t *flags, double *Hhat);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc.
 *
 * pf_tangent_apply_noalloc: q = K_t(u; d) p as pf_op_tangent_apply computes
 * it (same kernels, the work decomposition of a context with default
 * options), without a context and without allocating: no hipMalloc, hipFree
 * or allocating library call.  The per-element indicator bytes (tr eps > 0
 * at each quadrature point) go to a static device array of the library,
 * PF_NOALLOC_MAX_ELEMENTS bytes on each device it runs on, held until the
 * process ends and shared by every call on that device; each call rewrites
 * the nx*ny bytes it uses.  Calls that overlap on one device (different
 * streams) therefore race; calls on one stream do not.
 *   mesh: nx, ny, lx, ly as for pf_create, but elem_active is NULL or a
 *         DEVICE pointer to nx*ny flags (nothing is copied);
 *   mat:  E, nu, eta and split are used;
 *   u, p, q [2N], d [N]: device pointers on the current device (N =
 *         (nx+1)(ny+1)); q is overwritten;
 *   hip_stream: the stream the kernels run on (NULL = the null stream).
 * Stream-ordered, does not synchronise.  Errors: PF_E_INVALID_ARG for a
 * null pointer, a bad mesh or material, or nx*ny > PF_NOALLOC_MAX_ELEMENTS
 * (checked before any device call); PF_E_HIP if the scratch address cannot
 * be found or a launch fails.
 * ------------------------------------------------------------------------- */
#define PF_NOALLOC_MAX_ELEMENTS (16 * 1024 * 1024)
pf_status pf_tangent_apply_noalloc(const pf_mesh_desc *mesh, const pf_material *mat,
                                   const double *u, const double *d, const double *p,
                                   double *q, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PHASEFIELD_H */
