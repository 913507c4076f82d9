// Internal declarations shared by the HIP kernels (pf_kernels.hip) and the
// host runtime (pf_solver.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pf {

// Structured-grid geometry: nx x ny Q1 elements on [0,lx] x [0,ly].
struct Grid {
  int nx, ny;     // elements per direction
  int N, E;       // nodes (nx+1)(ny+1), elements nx*ny
  double hx, hy;  // element size
};

// Material constants (Section 2): mu, bulk modulus K = lam + 2mu/3, lam.
struct Mat {
  double mu, K, lam, Gc, l, eta;
  int split;      // 0 = volumetric-deviatoric, 1 = spectral
};

// Per-solve CG state in device memory.  The CG loop has no communication
// between blocks of one kernel: each kernel writes block partials with plain
// stores, and every block of the next kernel reduces them in a fixed order in
// its prologue, so all blocks hold bit-identical scalars.  Block 0 records
// the scalars for later kernels in the half of this struct the current
// kernel does not read (A = written by the operator apply, B = written by the
// vector update / init), each half on its own 128-byte line.
struct alignas(128) CgHalfA {
  double rz;      // r.z entering this iteration
  double rr;      // r.r entering this iteration
  double rr0;     // r.r of the initial residual
  int done;       // 0 running, 1 converged, 2 breakdown/non-finite, 3 maxit
  int iters;      // completed iterations
};
struct alignas(128) CgHalfB {
  double rz_prev; // r.z of the previous iteration (for beta)
  double rr0;
  double tol2;    // squared relative tolerance of the solve (set by the init)
  double rr_abs;  // > 0: converged at r.r <= rr_abs instead (a warm start)
  int done;
  int iters;
  int first;      // 1 before the first direction
};
struct CgState {
  CgHalfA a;
  CgHalfB b;
};

// Node flag bits
constexpr uint8_t NF_UX = 1;   // u_x fixed (Dirichlet or inactive node)
constexpr uint8_t NF_UY = 2;   // u_y fixed
constexpr uint8_t NF_D = 4;    // d fixed

// Column-marching launch shape for the node-accumulating operators.
// Work decomposition of the operator kernels.  ch = 2, 4 or 8: column
// marching, one wave per (strip of 62 node columns, chunk of ch node rows).
// ch = 1: LDS tiles, one block per tile of 15 x 15 owned nodes (nstrips x
// nchunks tiles), one element per thread.
struct March {
  int nstrips;    // marching: wave strips across x; tiles: tiles across x
  int nchunks;    // marching: row chunks along y;   tiles: tiles along y
  int ch;         // node rows per marching item, or 1 for LDS tiles
};

// Scratch for block reductions.  Kernels that reduce run at most kPMax
// blocks (8 waves per SIMD at four waves per block) and write one partial
// per block and value.
constexpr int kPMax = 2048;
struct RedScratch {
  double *partR;               // [4 * kPMax]  block partials
  unsigned long long *icount;  // [kICounters] integer counters (atomic adds)
  double *scal;                // [kScal]      finalised scalars
};
constexpr int kICounters = 8;
constexpr int kScal = 16;

// Slots in RedScratch::scal and ::icount
enum ScalSlot {
  SC_NORM_A = 0,    // ||R||^2 of the last residual kernel
  SC_NORM_B = 1,    // ||b||^2 (phase residual)
  SC_SUM_X = 2,     // group reaction x
  SC_SUM_Y = 3,     // group reaction y
};
enum ICounter { IC_GATED = 0, IC_FLOOR = 1, IC_CHI = 2 };

// Single-kernel CG (Chronopoulos-Gear recurrences): one kernel per iteration.
// Kernel K_i reduces the partials of K_{i-1} (gamma = r.u, delta = w.u,
// r.r) in its prologue, applies the pending recurrences of iteration i-1 to
// the vectors it reads and computes w_i = A u_i.  Vectors read at halo nodes
// and everything the kernel writes are double-buffered by iteration parity,
// so the kernel only reads parity i-1 and writes parity i: it is idempotent.
struct alignas(128) Cg1State {
  double alpha_prev;   // alpha of the update applied by this kernel
  double gamma_prev;   // gamma of that update
  double rr0;          // r.r of the initial residual
  double rr;           // r.r entering this kernel
  int done;            // 0 running, 1 converged, 2 breakdown/non-finite, 3 maxit
  int iters;           // completed updates of x
  int first;           // 1 after the initial kernel
  int pad;
};

template <class T>
struct CgVecs {
  T *R[2], *W[2], *S[2], *X[2], *P[2];
  const T *Dinv;
};

struct Cg1Args {
  Cg1State *st;        // [2] by parity
  double *part;        // [2][3][kPMax] by parity
  int np;              // number of blocks (partials) of every CG kernel
  double tol2;
  int maxit;
  int parity;          // i & 1
  int init;            // 1 for K_0
};

// Launch geometry of one CG solve: grid sizes of the apply (ga) and of the
// vector kernels (gb); each kernel's prologue reduces the other's partials.
struct CgArgs {
  CgState *st;
  double *partA;
  double *partB;
  int ga, gb;
  double tol2;
  int maxit;
  int ext;    // 1: z comes from an external preconditioner (Chebyshev), which
              // also writes the (r.z, r.r) partials; the vector kernels then
              // update only x and r
  int npb;    // number of (r.z, r.r) partials the apply prologue reduces
  int warm;   // 1: x holds a starting guess and r its residual (the init keeps x)
  double rr_abs;  // > 0: absolute convergence target for r.r (a warm start)
};

// Starting guess of a displacement solve from earlier solutions (the
// Galerkin projection of the right-hand side onto their span, with the
// current operator): up to kGuessMax stored solutions v_j and w_j = K v_j.
constexpr int kGuessMax = 4;
// v_j . w_k (j <= k), v_j . b, b . b
constexpr int kGuessDots = kGuessMax * (kGuessMax + 1) / 2 + kGuessMax + 1;
template <class T>
struct GuessArgs {
  const T *v[kGuessMax];
  const T *w[kGuessMax];
  int m, n;
};
struct GuessCoef {
  double c[kGuessMax];
};

// One step of the Jacobi-Chebyshev polynomial (z = p(D^-1 A) D^-1 r by
// Chebyshev iteration on A y = r from y = 0): d_0 = D^-1 r / theta;
// d_k = c1 d_{k-1} + c2 D^-1 res_k; y_{k+1} = y_k + d_k;
// res_{k+1} = res_k - A d_k.  The coefficients live in
// device memory (coef[0] = 1/theta, coef[2k-1], coef[2k] = c1, c2 of step
// k >= 1), so captured CG batches stay valid when lambda_max is
// re-estimated; `last` marks the step that writes the r.z, r.r partials.
constexpr int kChebCoefs = 33;   // 1 + 2 x (16 - 1) + 2 spare
struct ChebStep {
  const double *coef;
  int k;
  int last;
};

// Preconditioned MINRES (Paige and Saunders) for the symmetric, possibly
// indefinite phase trial block, FP64, M = |diag A| (SPD).  Lanczos step j
// (1-based) applies A to v_j = y_{j-1} / beta_j, where y_{j-1} = M^-1 r_j and
// beta_j^2 = r_j . y_{j-1}; the Givens rotation that advances x by step j
// needs beta_{j+1}, so x and w of step j are updated in the apply of step
// j + 1.  Two kernels per step, like the CG: the apply (prologue: reduce
// beta_j, rotate for step j - 1, test convergence; q = A v_j, w and x of
// step j - 1, partials of alpha_j = v_j . q) and the vector kernel
// (r_{j+1} = q - alpha_j / beta_j r_j - beta_j / beta_{j-1} r_{j-1},
// y_j = M^-1 r_{j+1}, partials of beta_{j+1}^2).  The apply writes half a,
// the vector kernel half b, each reading the other's.
struct MrHalf {
  double beta, oldb, alfa;            // beta_j, beta_{j-1}, alpha_j
  double cs, sn, dbar, epsln, phibar;  // rotation state
  double beta1;                        // beta_1 = ||b||_{M^-1}
  int done;    // 0 running, 1 converged, 2 breakdown, 3 iteration cap
  int iters;   // steps whose x update has been applied
  int first;   // set by the init kernel: the next apply is step 1
  int pad;
};
struct MrState {
  MrHalf a;
  MrHalf b;
};
struct MrArgs {
  MrState *st;
  double *partA;   // alpha partials (apply blocks)
  double *partB;   // beta^2 partials (init / vector kernel blocks)
  int ga, gb;      // block counts of the apply and of the vector kernels
  double tol;      // stop at phibar <= tol * beta_1
  int maxit;
};
// Vectors of one MINRES solve (length N): x, w_j in w[j & 1], y_j in
// y[j & 1], r_j in r[j & 1], q = A v_j, M^-1 = Dinv (0 on fixed nodes).
struct MrVecs {
  double *x;
  double *w[2];
  double *y[2];
  double *r[2];
  double *q;
  const double *Dinv;
};

// Operator coefficients passed by value.
struct ElasCoef {
  double two_mu, K, lam, mu, eta;
  double ihx, ihy;   // 1/hx, 1/hy
  double sx, sy;     // hy/4, hx/4 (w detJ / hx, w detJ / hy)
};
struct PhaseCoef {
  double Gcl;        // Gc * l
  double Gc_l;       // Gc / l
  double wdet;       // hx hy / 4
  double ihx, ihy, sx, sy;
};

// ---------------------------------------------------------------- launches
// All launches are stream-ordered on `s` and return the launch status.

March march_shape(const Grid &g, int ch_override);

// CG (T = double or float).  p_old/p_new are the two direction buffers; the
// apply computes p_new = z + beta p_old on the fly and q = A p_new.
CgArgs cg_args(const Grid &g, const March &m, int n, CgState *st, RedScratch rs, double tol,
               int maxit);
template <class T>
hipError_t cg_init(hipStream_t s, int n, T *x, T *r, T *z, T *p_old, const T *Dinv,
                   const CgArgs &ca);
// ---- batched CG: the systems of many contexts advanced by shared launches.
// Every system keeps the blocks it has in a launch of its own (same work
// items, same partial slots, so its results are bit-identical); bmap[b] is
// the table entry of block b of a shared launch and entry.b0 its first block.
constexpr int kBatchEntryBytes = 512;   // stride of an apply-table entry
template <class T>
struct BatchUpdateEntry {
  T *x, *r, *z;
  const T *p, *q, *Dinv;
  CgArgs ca;
  int n, b0, nb;
  int *status;   // [2]: done and iteration count after this update
};
// Apply-table entry of one system (written to dst, kBatchEntryBytes bytes),
// with the operands of tangent_cg_apply / phase_cg_apply.
template <class T>
void tangent_batch_entry(void *dst, const Grid &g, const March &m, const ElasCoef &c, int split,
                         const T *ulin, const T *d, const uint8_t *qflag, const uint8_t *eact,
                         const uint8_t *nflag, const T *z, const T *p_old, T *p_new, T *q,
                         const CgArgs &ca, int b0, int nb);
template <class T>
void phase_batch_entry(void *dst, const Grid &g, const March &m, const PhaseCoef &c,
                       const T *coef, const uint8_t *eact, const uint8_t *nflag, const T *z,
                       const T *p_old, T *p_new, T *q, const CgArgs &ca, int b0, int nb);
// Shared launches: one apply over the entries of one (operator, split, work
// item height), one update over any entries.
template <class T>
hipError_t tangent_cg_apply_batch(hipStream_t s, int split, int ch, const void *tab,
                                  const int *bmap, int nblocks);
template <class T>
hipError_t phase_cg_apply_batch(hipStream_t s, int ch, const void *tab, const int *bmap,
                                int nblocks);
template <class T>
hipError_t cg_update_batch(hipStream_t s, const BatchUpdateEntry<T> *tab, const int *bmap,
                           int nblocks);

// First Chebyshev step fused into the CG update (Jacobi-Chebyshev only):
// d0 = z = D^-1 r / theta and res = r; the partials r.z, r.r are written
// when the polynomial has degree 1.  d0 == nullptr: no fused step.
template <class T>
struct ChebFuse {
  T *d0;
  T *res;
  const double *coef;   // coef[0] = 1/theta
  int last;
};
template <class T>
hipError_t cg_update(hipStream_t s, int n, T *x, T *r, T *z, const T *p, const T *q,
                     const T *Dinv, const CgArgs &ca, const ChebFuse<T> &cf);
// split = 1 (spectral): the tangent is re-derived per QP from the
// linearisation point ulin [2N] instead of the indicator bits.
template <class T>
hipError_t tangent_cg_apply(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                            int split, const T *ulin, const T *d, const uint8_t *qflag,
                            const uint8_t *eact, const uint8_t *nflag, const T *z,
                            const T *p_old, T *p_new, T *q, const CgArgs &ca);
template <class T>
hipError_t phase_cg_apply(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const T *coef, const uint8_t *eact, const uint8_t *nflag,
                          const T *z, const T *p_old, T *p_new, T *q, const CgArgs &ca);
// Jacobi-Chebyshev preconditioner kernels (two-kernel CG, ext = 1).
template <class T>
hipError_t cheb_init(hipStream_t s, int n, const T *r, const T *Dinv, T *d0, T *z, T *res,
                     const CgArgs &ca, const ChebStep &cs);
// One Chebyshev step: reads z_in/res_in, writes z_out/res_out (distinct
// buffers, so a launch can be repeated).
template <class T>
hipError_t tangent_cheb_step(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                             int split, const T *ulin, const T *d, const uint8_t *qflag,
                             const uint8_t *eact, const uint8_t *nflag, const T *dprev, T *dnext,
                             const T *z_in, T *z_out, const T *res_in, T *res_out, const T *r,
                             const T *Dinv, const CgArgs &ca, const ChebStep &cs);
template <class T>
hipError_t phase_cheb_step(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                           const T *coef, const uint8_t *eact, const uint8_t *nflag,
                           const T *dprev, T *dnext, const T *z_in, T *z_out, const T *res_in,
                           T *res_out, const T *r, const T *Dinv, const CgArgs &ca,
                           const ChebStep &cs);
// CG vector update fused with the first Chebyshev step (degree >= 2):
// x_out = x_in + alpha p and r_out = r_in - alpha q (out of place, so the
// launch can be repeated); d1 -> dnext, z1 -> z_out, res1 -> res_out; s0 the
// polynomial's initial step (1/theta), s1 its first step.
template <class T>
hipError_t tangent_updcheb(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                           int split, const T *ulin, const T *d, const uint8_t *qflag,
                           const uint8_t *eact, const uint8_t *nflag, const T *x_in, T *x_out,
                           const T *r_in, T *r_out, const T *p, const T *q, const T *Dinv,
                           T *dnext, T *z_out, T *res_out, const CgArgs &ca, const ChebStep &s0,
                           const ChebStep &s1);
template <class T>
hipError_t phase_updcheb(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                         const T *coef, const uint8_t *eact, const uint8_t *nflag,
                         const T *x_in, T *x_out, const T *r_in, T *r_out, const T *p,
                         const T *q, const T *Dinv, T *dnext, T *z_out, T *res_out,
                         const CgArgs &ca, const ChebStep &s0, const ChebStep &s1);
// The same update fused with the first two Chebyshev steps (LDS tiles only,
// m.ch == 1; degree >= 3): writes x_out, r_out, z_out and, unless s2 is the
// last step, d2 into dnext and res2 into res_out; s2 is step 2 of the
// polynomial.
template <class T>
hipError_t tangent_updcheb2(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                            int split, const T *ulin, const T *d, const uint8_t *qflag,
                            const uint8_t *eact, const uint8_t *nflag, const T *x_in, T *x_out,
                            const T *r_in, T *r_out, const T *p, const T *q, const T *Dinv,
                            T *dnext, T *z_out, T *res_out, const CgArgs &ca,
                            const ChebStep &s2);
template <class T>
hipError_t phase_updcheb2(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const T *coef, const uint8_t *eact, const uint8_t *nflag,
                          const T *x_in, T *x_out, const T *r_in, T *r_out, const T *p,
                          const T *q, const T *Dinv, T *dnext, T *z_out, T *res_out,
                          const CgArgs &ca, const ChebStep &s2);
// Power iteration step for lambda_max(D^-1 A): vnext = D^-1 A (scale v);
// scal[SC_NORM_A] = v'Av and scal[SC_NORM_B] = v'Dv (of the scaled v).
template <class T>
hipError_t tangent_power_step(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                              int split, const T *ulin, const T *d, const uint8_t *qflag,
                              const uint8_t *eact, const uint8_t *nflag, const T *v, T *vnext,
                              const T *Dinv, double scale, RedScratch rs);
template <class T>
hipError_t phase_power_step(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                            const T *coef, const uint8_t *eact, const uint8_t *nflag, const T *v,
                            T *vnext, const T *Dinv, double scale, RedScratch rs);
template <class T>
hipError_t power_start(hipStream_t s, int n, const T *Dinv, T *v);

// Single-kernel CG iteration for the elasticity tangent / the phase operator.
template <class T>
hipError_t tangent_cg1(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                       int split, const T *ulin, const T *d, const uint8_t *qflag,
                       const uint8_t *eact, const uint8_t *nflag, const CgVecs<T> &v,
                       const Cg1Args &a);
template <class T>
hipError_t phase_cg1(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                     const T *coef, const uint8_t *eact, const uint8_t *nflag,
                     const CgVecs<T> &v, const Cg1Args &a);
int cg1_blocks(const March &m);

template <class T>
hipError_t tangent_diag(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                        int split, const T *ulin, const T *d, const uint8_t *qflag,
                        const uint8_t *eact, const uint8_t *nflag, T *Dinv);
template <class T>
hipError_t phase_diag(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                      const T *coef, const uint8_t *eact, const uint8_t *nflag, T *Dinv,
                      int absdiag = 0);

// MINRES on the phase operator with coefficient coef (FP64; m a marching
// shape, not tiles).  mr_init: r_1 = rhs, x = w = 0, y_0 = M^-1 rhs.
hipError_t mr_init(hipStream_t s, int n, const double *rhs, const MrVecs &v, const MrArgs &a);
hipError_t phase_mr_apply(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const double *coef, const uint8_t *eact, const uint8_t *nflag,
                          const MrVecs &v, const MrArgs &a, int j);
hipError_t mr_update(hipStream_t s, int n, const MrVecs &v, const MrArgs &a, int j);
int vec_block_count(int n);

// q = K_t p in the CG's precision, zero on fixed displacement entries.
template <class T>
hipError_t tangent_apply_masked(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                                int split, const T *ulin, const T *d, const uint8_t *qflag,
                                const uint8_t *eact, const uint8_t *nflag, const T *p, T *q);
// The kGuessDots sums of a starting guess (b = the right-hand side), block
// partials then finalised into out[0 .. kGuessDots).
template <class T>
hipError_t guess_dots(hipStream_t s, const GuessArgs<T> &a, const T *b, double *part,
                      double *out);
// x = sum_j c_j v_j and r = b - sum_j c_j w_j, in place of b.
template <class T>
hipError_t guess_combine(hipStream_t s, const GuessArgs<T> &a, const GuessCoef &c, T *x, T *rb);

// Plain operator applies (no CG fusion, no masking) for the op entry points.
hipError_t tangent_apply_plain(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                               int split, const double *ulin, const double *d,
                               const uint8_t *qflag, const uint8_t *eact, const double *p,
                               double *q);
hipError_t phase_apply_plain(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                             const double *coef, const uint8_t *eact, const double *p,
                             double *q);

// FP64 residuals.  internal_force: R = sum B^T sigma; if nflag != nullptr the
// fixed DOFs are zeroed, optionally negated (neg), and ||R||^2 over free DOFs
// goes to scal[SC_NORM_A].
hipError_t internal_force(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                          int split, const double *u, const double *d, const uint8_t *eact,
                          const uint8_t *nflag, bool neg, double *R, RedScratch rs);
// Phase residual R_d = K_dd(H) d - b(H) on free nodes (0 on fixed), written
// negated if neg; ||R_d||^2 -> scal[SC_NORM_A], ||b||^2 -> scal[SC_NORM_B].
hipError_t phase_residual(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const double *H, const double *d, const uint8_t *eact,
                          const uint8_t *nflag, bool neg, double *R, RedScratch rs);
// AT1 with the penalty: F_d(d; psi) (c.Gc_l = Gc/(c_w l), c.Gcl = 2 Gc l/c_w),
// norms as phase_residual with b = sum 2 psi N.
hipError_t phase_residual_at1(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                              const double *psi, const double *d, const double *dprev,
                              double gamma, const uint8_t *eact, const uint8_t *nflag, bool neg,
                              double *R, RedScratch rs);
// AT1 Newton matrix coefficient 2 psi + gamma chi into coef; chi updated,
// changed points counted in icount[IC_CHI]; at_kink: d_q = d_{n-1,q} counts
// as active.
hipError_t at1_coef(hipStream_t s, const Grid &g, double gamma, const double *psi,
                    const double *d, const double *dprev, const uint8_t *eact, double *coef,
                    uint8_t *chi, int at_kink, RedScratch rs);

// Element-wise kernels.
struct QpParams {
  int scheme;
  double psi_crit, d_gate;
};
// psi_out (may be null): Psi+ of the current displacement per point.
hipError_t qp_update(hipStream_t s, const Grid &g, const Mat &mt, const QpParams &qp,
                     const double *u, const double *d, const uint8_t *eact,
                     const double *H_prev, double *H, double *psi_s, uint8_t *qflag,
                     double *psi_out, RedScratch rs);
hipError_t tangent_flags(hipStream_t s, const Grid &g, const double *u, const uint8_t *eact,
                         uint8_t *qflag);
template <class T>
// cbase (may be null, may alias coef): the block's own mass coefficient;
// null means the AT2 coefficient Gc/l + 2H.
hipError_t trial_coef(hipStream_t s, const Grid &g, const Mat &mt, double theta, int floor,
                      const double *H, const double *psi_s, const uint8_t *qflag,
                      const double *d, const uint8_t *eact, const T *cbase, T *coef,
                      RedScratch rs);
template <class T>
hipError_t at2_coef(hipStream_t s, const Grid &g, const Mat &mt, const double *H,
                    const uint8_t *eact, T *coef);
template <class TD>
hipError_t predictor(hipStream_t s, const Grid &g, const Mat &mt, const double *d,
                     const TD *dd, const double *H, const double *psi_s, const uint8_t *qflag,
                     const uint8_t *eact, double *Hhat);

// Vector helpers.
hipError_t lift_dirichlet(hipStream_t s, int n, const uint8_t *fixedmask, uint8_t bits,
                          int nmask, const double *unit, double lam, double *u);
template <class TS>
hipError_t axpy_into(hipStream_t s, int n, double *out, const double *x, double alpha,
                     const TS *y);
template <class TO, class TI>
hipError_t convert(hipStream_t s, int n, TO *out, const TI *in);
hipError_t group_sum(hipStream_t s, int n, const int64_t *dof, const int8_t *comp,
                     const double *R, RedScratch rs);
hipError_t fill_zero_bytes(hipStream_t s, void *p, size_t bytes);

}  // namespace pf
