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

// Per-solve CG scalars, resident in device memory.  Written by the last
// block of a kernel (thread 0, vector store), read by the following kernels.
struct CgScal {
  double rz;      // r.z of the current residual
  double pq;      // p.Ap of the current direction
  double alpha;   // rz / pq
  double beta;    // rz_new / rz_old (0 on the first iteration)
  double rr;      // r.r of the current residual
  double rr0;     // r.r of the initial residual
  double tol2;    // converged when rr <= tol2 * rr0
  int done;       // 0 running, 1 converged, 2 breakdown (pq <= 0), 3 maxit
  int iters;      // completed iterations
  int maxit;
  int pad;
};

// Node flag bits
constexpr uint8_t NF_UX = 1;   // u_x fixed (Dirichlet or inactive node)
constexpr uint8_t NF_UY = 2;   // u_y fixed
constexpr uint8_t NF_D = 4;    // d fixed

// Column-marching launch shape for the node-accumulating operators.
struct March {
  int nstrips;    // wave strips across x (63 owned node columns each)
  int nchunks;    // row chunks along y
  int ch;         // node rows owned per wave
};

// Scratch for block reductions with last-block finalisation.
struct RedScratch {
  double *part;        // [kRedSlots * kMaxBlocks]
  unsigned *counter;   // [kRedCounters]
  unsigned long long *icount;  // [kICounters] integer counters
  double *scal;        // [kScal] generic reduced scalars
};
constexpr int kMaxBlocks = 4096;
constexpr int kRedSlots = 4;
constexpr int kRedCounters = 8;
constexpr int kICounters = 8;
constexpr int kScal = 16;

// Generic scalar slots in RedScratch::scal
enum ScalSlot {
  SC_NORM_A = 0,    // ||R||^2 of the last residual kernel
  SC_NORM_B = 1,    // ||b||^2 (phase residual)
  SC_SUM_X = 2,     // group reaction x
  SC_SUM_Y = 3,     // group reaction y
};
enum ICounter { IC_GATED = 0, IC_FLOOR = 1 };

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
template <class T>
hipError_t cg_init(hipStream_t s, int n, T *x, T *r, T *z, T *p_old, const T *Dinv,
                   CgScal *sc, double tol, int maxit, RedScratch rs);
template <class T>
hipError_t cg_update(hipStream_t s, int n, T *x, T *r, T *z, const T *p, const T *q,
                     const T *Dinv, CgScal *sc, RedScratch rs);
template <class T>
hipError_t tangent_cg_apply(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                            const T *d, const uint8_t *qflag, const uint8_t *eact,
                            const uint8_t *nflag, const T *z, const T *p_old, T *p_new,
                            T *q, CgScal *sc, RedScratch rs);
template <class T>
hipError_t phase_cg_apply(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const T *coef, const uint8_t *eact, const uint8_t *nflag,
                          const T *z, const T *p_old, T *p_new, T *q, CgScal *sc,
                          RedScratch rs);
template <class T>
hipError_t tangent_diag(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                        const T *d, const uint8_t *qflag, const uint8_t *eact,
                        const uint8_t *nflag, T *Dinv);
template <class T>
hipError_t phase_diag(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                      const T *coef, const uint8_t *eact, const uint8_t *nflag, T *Dinv);

// Plain operator applies (no CG fusion, no masking) for the op entry points.
hipError_t tangent_apply_plain(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                               const double *d, const uint8_t *qflag, const uint8_t *eact,
                               const double *p, double *q);
hipError_t phase_apply_plain(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                             const double *coef, const uint8_t *eact, const double *p,
                             double *q);

// FP64 residuals.  internal_force: R = sum B^T sigma; if nflag != nullptr the
// fixed DOFs are zeroed, optionally negated (neg), and ||R||^2 over free DOFs
// goes to scal[SC_NORM_A].
hipError_t internal_force(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                          const double *u, const double *d, const uint8_t *eact,
                          const uint8_t *nflag, bool neg, double *R, RedScratch rs);
// Phase residual R_d = K_dd(H) d - b(H) on free nodes (0 on fixed), written
// negated if neg; ||R_d||^2 -> scal[SC_NORM_A], ||b||^2 -> scal[SC_NORM_B].
hipError_t phase_residual(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const double *H, const double *d, const uint8_t *eact,
                          const uint8_t *nflag, bool neg, double *R, RedScratch rs);

// Element-wise kernels.
struct QpParams {
  int scheme;
  double psi_crit, d_gate;
};
hipError_t qp_update(hipStream_t s, const Grid &g, const Mat &mt, const QpParams &qp,
                     const double *u, const double *d, const uint8_t *eact,
                     const double *H_prev, double *H, double *psi_s, uint8_t *qflag,
                     RedScratch rs);
hipError_t tangent_flags(hipStream_t s, const Grid &g, const double *u, const uint8_t *eact,
                         uint8_t *qflag);
template <class T>
hipError_t trial_coef(hipStream_t s, const Grid &g, const Mat &mt, double theta,
                      const double *H, const double *psi_s, const uint8_t *qflag,
                      const double *d, const uint8_t *eact, T *coef, RedScratch rs);
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
