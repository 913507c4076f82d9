// 3-D load step (trilinear hexahedra, FP64): Newton for u with Jacobi PCG,
// the AT2 phase solve, and for S1/S2/S3 the floored trial solve and the
// predictor, in the staggered loop of Sections 3.1 and 3.3-3.5.
//
// The loop is written once over a backend B that runs per-index functors:
//   B::each(count, f)   calls f(i) for i < count, one grid index per thread;
//   B::sum(count, f)    returns the sum of f(i) over i < count, reduced per
//                       block of kTpb3 indices by a fixed binary tree and then
//                       over the blocks in order, so that every backend gives
//                       the same bits;
//   B::sum_into(count, f, slot)  the same sum, left in device memory at slot
//                       (no host synchronisation);
//   B::sum2_into(count, f, slot_a, slot_b, post)  the two sums of a functor
//                       returning Sum2, in the same order, left at the two
//                       slots, after which post(0) runs once (one thread);
//   B::replay(key), B::capture_begin(blocks), B::capture_end(key)  an
//                       optional record-and-replay of a CG batch: replay
//                       launches the batch recorded under key if it is still
//                       valid; capture_begin (which first reserves `blocks`
//                       reduction partials) starts recording, or returns
//                       false, and the batch then runs as it is enqueued;
//   B::alloc/release/upload/download for the buffers.
// The device backend (pf3d_kernels.hip) launches one kernel per call; a host
// backend that replays the same grid serves the tests.
#pragma once

#include "pf3d_ops.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace pf3d {

// ---- per-index functors

struct FTangentDiag {
  Grid3 g; Mat3 m; const double *u, *d; double *D;
  __host__ __device__ void operator()(int n) const { node_tangent_diag(g, m, n, u, d, D); }
};
struct FPhaseDiag {
  Grid3 g; Mat3 m; const double *coef; double *D;
  __host__ __device__ void operator()(int n) const { node_phase_diag(g, m, n, coef, D); }
};
struct FPhaseRhs {
  Grid3 g; const double *H; double *b;
  __host__ __device__ void operator()(int n) const { node_phase_rhs(g, n, H, b); }
};
struct FPhaseCoef {
  Grid3 g; Mat3 m; int trial; double theta; const double *H, *psi_s; const uint16_t *flags;
  const double *d; double *coef;
  __host__ __device__ void operator()(int e) const {
    (void)elem_phase_coef(g, m, e, trial, theta, 1, H, psi_s, flags, d, coef);
  }
};
// gated points of element e whose trial coefficient is floored
struct FFloorHits {
  Grid3 g; Mat3 m; double theta; const double *H, *psi_s; const uint16_t *flags;
  const double *d; double *scratch;
  __host__ __device__ double operator()(int e) const {
    return double(elem_phase_coef(g, m, e, 1, theta, 1, H, psi_s, flags, d, scratch));
  }
};
struct FQp {
  Grid3 g; Mat3 m; Qp3 qp; const double *u, *d, *Hprev; double *H, *psi_s; uint16_t *flags;
  __host__ __device__ void operator()(int e) const {
    (void)elem_qp_update(g, m, qp, e, u, d, Hprev, H, psi_s, flags);
  }
};
struct FPredictor {
  Grid3 g; Mat3 m; const double *d, *dd, *H, *psi_s; const uint16_t *flags; double *Hhat;
  __host__ __device__ void operator()(int e) const {
    elem_predictor(g, m, e, d, dd, H, psi_s, flags, Hhat);
  }
};
// out = a + s b, zero on fixed entries (fixed may be null)
struct FAxpy {
  const double *a, *b; double s; const uint8_t *fixed; double *out;
  __host__ __device__ void operator()(int i) const {
    out[i] = (fixed && fixed[i]) ? 0.0 : a[i] + s * b[i];
  }
};
// out = a + s b on free entries; fixed entries keep a
struct FUpdate {
  const double *a, *b; double s; const uint8_t *fixed; double *out;
  __host__ __device__ void operator()(int i) const {
    out[i] = (fixed && fixed[i]) ? a[i] : a[i] + s * b[i];
  }
};
// out = v everywhere
struct FFill {
  double v; double *out;
  __host__ __device__ void operator()(int i) const { out[i] = v; }
};
// out = s a, zero on fixed entries
struct FScale {
  const double *a; double s; const uint8_t *fixed; double *out;
  __host__ __device__ void operator()(int i) const { out[i] = fixed[i] ? 0.0 : s * a[i]; }
};
// out = w v elementwise
struct FMul {
  const double *w, *v; double *out;
  __host__ __device__ void operator()(int i) const { out[i] = w[i] * v[i]; }
};
// Dinv = 1 / D on free entries, 0 on fixed ones
struct FInvDiag {
  const double *D; const uint8_t *fixed; double *Dinv;
  __host__ __device__ void operator()(int i) const {
    Dinv[i] = (fixed[i] || D[i] == 0.0) ? 0.0 : 1.0 / D[i];
  }
};
// x = value on fixed entries (value = s * val)
struct FSetFixed {
  const uint8_t *fixed; const double *val; double s; double *x;
  __host__ __device__ void operator()(int i) const {
    if (fixed[i]) x[i] = s * val[i];
  }
};
// a . b over free entries (fixed may be null)
struct FDot {
  const double *a, *b; const uint8_t *fixed;
  __host__ __device__ double operator()(int i) const {
    return (fixed && fixed[i]) ? 0.0 : a[i] * b[i];
  }
};
// gated points of element e
struct FGated {
  const uint16_t *flags;
  __host__ __device__ double operator()(int e) const {
    unsigned v = flags[e] >> 8, c = 0;
    for (; v; v &= v - 1) ++c;
    return double(c);
  }
};
// R[dof[k]] over a Dirichlet group's entries of one component
struct FGroupSum {
  const double *R; const int64_t *dof; const int8_t *comp; int c;
  __host__ __device__ double operator()(int k) const {
    return comp[k] == c ? R[dof[k]] : 0.0;
  }
};

constexpr int kGroups3 = 8;

// Iterations enqueued between two polls of the CG state.
constexpr int kCgBatch3 = 16;

// Scalars of one CG solve, kept in device memory between its launches.
// done: 0 running, 1 converged, 2 breakdown (p.q <= 0), 3 at max_cg,
// 4 zero right-hand side.
struct CgState3 {
  double bb, rz, pq, rr, rz_new, beta, tol2;
  int iters, maxit, done, pad;
};

struct FCgStart {
  CgState3 *s; double tol; int maxit;
  __host__ __device__ void operator()(int) const {
    s->tol2 = tol * tol * s->bb;
    s->iters = 0;
    s->maxit = maxit;
    s->done = s->bb == 0.0 ? 4 : 0;
  }
};
// q = 0 on fixed entries; returns p . q
struct FMaskDot {
  double *q; const double *p; const uint8_t *fixed;
  __host__ __device__ double operator()(int i) const {
    if (fixed[i]) {
      q[i] = 0.0;
      return 0.0;
    }
    return p[i] * q[i];
  }
};
// Two sums of one pass (see B::sum2_into).
struct Sum2 {
  double a, b;
};
// One pass of the CG update: with alpha = rz / pq, x += alpha p and
// r -= alpha q on free entries while the solve runs and p.q > 0; then
// z = D^-1 r.  Returns (r_i^2, r_i z_i), (0, 0) on fixed entries.  Every
// thread forms the same alpha from the same two scalars.
struct FCgUpdate {
  const CgState3 *s; double *x, *r, *z; const double *p, *q, *Dinv; const uint8_t *fixed;
  __host__ __device__ Sum2 operator()(int i) const {
    if (!fixed[i] && !s->done && s->pq > 0.0) {
      const double alpha = s->rz / s->pq;
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    const double zi = Dinv[i] * r[i];
    z[i] = zi;
    if (fixed[i]) return Sum2{0.0, 0.0};
    return Sum2{r[i] * r[i], r[i] * zi};
  }
};
// After the update's sums: a breakdown (p.q <= 0) ends the solve; else
// counts the iteration, tests ||r||^2 <= tol^2 ||b||^2 and max_cg, forms beta
struct FCgBeta {
  CgState3 *s;
  __host__ __device__ void operator()(int) const {
    if (s->done) return;
    if (!(s->pq > 0.0)) {
      s->done = 2;
      return;
    }
    s->iters += 1;
    if (s->rr <= s->tol2) {
      s->done = 1;
      return;
    }
    if (s->iters >= s->maxit) {
      s->done = 3;
      return;
    }
    s->beta = s->rz_new / s->rz;
    s->rz = s->rz_new;
  }
};
struct FCgP {
  const CgState3 *s; double *p; const double *z; const uint8_t *fixed;
  __host__ __device__ void operator()(int i) const {
    if (s->done) return;
    p[i] = fixed[i] ? 0.0 : z[i] + s->beta * p[i];
  }
};

// The options the 3-D load step takes: FP64 with Jacobi PCG, AT2 with the
// history field, the floored trial block with predict -> correct; the
// tolerances and limits as for the 2-D path.
inline pf_status check_opts3(const pf_solver_opts *o) {
  if (!o || o->scheme < 0 || o->scheme > 3 || o->precision != PF_FP64 ||
      o->precond != PF_PC_JACOBI || o->phase_model != PF_AT2_HISTORY ||
      o->trial_operator != PF_TRIAL_FLOORED || o->trial_update != PF_TRIAL_PREDICT_CORRECT)
    return PF_E_INVALID_ARG;
  if (!(o->tol_stag > 0) || !(o->tol_pcg > 0) || !(o->tol_newton > 0) || o->max_stag < 1 ||
      o->max_newton < 1 || o->max_cg < 1 || !(o->trial_floor > 0) || o->trial_floor > 1 ||
      std::isnan(o->psi_crit) || std::isnan(o->d_gate))
    return PF_E_INVALID_ARG;
  return PF_OK;
}

struct Counts3 {
  int n_stag = 0, n_newton = 0, n_trial = 0, n_dsolve = 0;
  long long n_cg_u = 0, n_cg_d = 0, n_cg_trial = 0, gated_max = 0, floor_hits = 0;
  long long cg_not_converged = 0;
  double r_stag = 0.0, dof_updates = 0.0;
  bool converged = true;
};

template <class B>
class Solver3 {
 public:
  Solver3(B &be, const Grid3 &g, const Mat3 &m, const pf_solver_opts &o)
      : be_(be), g_(g), m_(m), o_(o) {}

  ~Solver3() {
    for (void *p : owned_) be_.release(p);
    for (int k = 0; k < kGroups3; ++k) {
      if (gdof_[k]) be_.release(gdof_[k]);
      if (gcomp_dev_[k]) be_.release(gcomp_dev_[k]);
    }
  }

  // Allocate every buffer; false if the backend could not.
  bool init() {
    const size_t N = g_.N, N3 = 3 * N, E8 = 8 * (size_t)g_.E;
    for (double **p : {&u_, &ut_, &R_, &Rt_, &x_, &r_, &z_, &p_, &q_, &Dinv_, &D_, &unit_})
      if (!(*p = alloc<double>(N3))) return false;
    for (double **p : {&d_, &dd_, &Rd_, &b_, &dval_})
      if (!(*p = alloc<double>(N))) return false;
    for (double **p : {&Hc_, &H_, &Hhat_, &psi_, &coef_, &ctr_})
      if (!(*p = alloc<double>(E8))) return false;
    if (!(flags_ = alloc<uint16_t>(g_.E)) || !(fu_ = alloc<uint8_t>(N3)) ||
        !(fd_ = alloc<uint8_t>(N)) || !(cs_ = alloc<CgState3>(1)))
      return false;
    host_fu_.assign(N3, 0);
    host_fd_.assign(N, 0);
    host_unit_.assign(N3, 0.0);
    host_dval_.assign(N, 0.0);
    zero(u_, N3);
    zero(d_, N);
    zero(Hc_, E8);
    return upload_constraints();
  }

  // Group k's entries: node, component (0..2), value per unit load.
  bool set_dirichlet_u(int grp, int64_t n, const int64_t *node, const int8_t *comp,
                       const double *val) {
    gnode_[grp].assign(node, node + n);
    gcomp_[grp].assign(comp, comp + n);
    gval_[grp].assign(val, val + n);
    return upload_constraints();
  }

  bool set_dirichlet_d(int64_t n, const int64_t *node, const double *val) {
    dnode_.assign(node, node + n);
    dvalue_.assign(val, val + n);
    if (!upload_constraints()) return false;
    be_.each(g_.N, FSetFixed{fd_, dval_, 1.0, d_});   // impose on the committed state
    return true;
  }

  // One load step at load factor lam; returns false if the loop ended at
  // max_stag or Newton did not converge (the step is committed either way).
  bool load_step(double lam, Counts3 *st) {
    *st = Counts3{};
    const int N = g_.N, N3 = 3 * N;
    be_.each(N3, FSetFixed{fu_, unit_, lam, u_});
    be_.each(N, FSetFixed{fd_, dval_, 1.0, d_});
    const double R0 = residual_u(u_, R_);
    const double Rref = R0 > 0.0 ? R0 : 1.0;
    st->converged &= newton(Rref, st);
    st->n_stag = 1;
    double r = qp_and_residual();
    while (r > o_.tol_stag && st->n_stag < o_.max_stag) {
      const double *Hs = H_;
      if (o_.scheme != 0 && gated_ > 0) {
        trial(st);
        Hs = Hhat_;
      }
      phase_solve(Hs, st);
      st->converged &= newton(Rref, st);
      st->n_stag += 1;
      r = qp_and_residual();
    }
    st->r_stag = r;
    st->converged &= r <= o_.tol_stag;
    // commit: H_n = H (the predicted energy is never stored)
    std::swap(Hc_, H_);
    return st->converged;
  }

  // Reaction of group grp: the internal force summed over its entries.
  void reaction(int grp, double f[3]) {
    be_.internal_force(g_, m_, u_, d_, Rt_);
    for (int c = 0; c < 3; ++c)
      f[c] = gn_[grp] ? be_.sum(gn_[grp], FGroupSum{Rt_, gdof_[grp], gcomp_dev_[grp], c}) : 0.0;
  }

  // Committed state from host arrays (each may be null); the phase field's
  // Dirichlet values are imposed on the new d.
  void set_state(const double *u, const double *d, const double *H) {
    if (u) be_.upload(u_, u, 3 * (size_t)g_.N * sizeof(double));
    if (d) {
      be_.upload(d_, d, (size_t)g_.N * sizeof(double));
      be_.each(g_.N, FSetFixed{fd_, dval_, 1.0, d_});
    }
    if (H) be_.upload(Hc_, H, 8 * (size_t)g_.E * sizeof(double));
  }

  void get_state(double *u, double *d, double *H) {
    if (u) be_.download(u, u_, 3 * (size_t)g_.N * sizeof(double));
    if (d) be_.download(d, d_, (size_t)g_.N * sizeof(double));
    if (H) be_.download(H, Hc_, 8 * (size_t)g_.E * sizeof(double));
  }

 private:
  template <class T>
  T *alloc(size_t n) {
    T *p = static_cast<T *>(be_.alloc(std::max<size_t>(n, 1) * sizeof(T)));
    if (p) owned_.push_back(p);
    return p;
  }
  void zero(double *p, size_t n) {
    std::vector<double> z(n, 0.0);
    be_.upload(p, z.data(), n * sizeof(double));
  }

  bool upload_constraints() {
    const size_t N = g_.N;
    std::fill(host_fu_.begin(), host_fu_.end(), 0);
    std::fill(host_unit_.begin(), host_unit_.end(), 0.0);
    std::fill(host_fd_.begin(), host_fd_.end(), 0);
    std::fill(host_dval_.begin(), host_dval_.end(), 0.0);
    for (int k = 0; k < kGroups3; ++k) {
      std::vector<int64_t> dof(gnode_[k].size());
      for (size_t i = 0; i < dof.size(); ++i) {
        dof[i] = gnode_[k][i] + gcomp_[k][i] * (int64_t)N;
        host_fu_[dof[i]] = 1;
        host_unit_[dof[i]] = gval_[k][i];
      }
      if (gdof_[k]) be_.release(gdof_[k]);
      if (gcomp_dev_[k]) be_.release(gcomp_dev_[k]);
      gdof_[k] = nullptr;
      gcomp_dev_[k] = nullptr;
      gn_[k] = (int)dof.size();
      if (gn_[k]) {
        gdof_[k] = static_cast<int64_t *>(be_.alloc(dof.size() * sizeof(int64_t)));
        gcomp_dev_[k] = static_cast<int8_t *>(be_.alloc(dof.size()));
        if (!gdof_[k] || !gcomp_dev_[k]) return false;
        be_.upload(gdof_[k], dof.data(), dof.size() * sizeof(int64_t));
        be_.upload(gcomp_dev_[k], gcomp_[k].data(), dof.size());
      }
    }
    for (size_t i = 0; i < dnode_.size(); ++i) {
      host_fd_[dnode_[i]] = 1;
      host_dval_[dnode_[i]] = dvalue_[i];
    }
    be_.upload(fu_, host_fu_.data(), host_fu_.size());
    be_.upload(unit_, host_unit_.data(), host_unit_.size() * sizeof(double));
    be_.upload(fd_, host_fd_.data(), host_fd_.size());
    be_.upload(dval_, host_dval_.data(), host_dval_.size() * sizeof(double));
    nfree_u_ = 0;
    for (uint8_t f : host_fu_) nfree_u_ += !f;
    nfree_d_ = 0;
    for (uint8_t f : host_fd_) nfree_d_ += !f;
    return true;
  }

  // R = internal force at (u, d_), zero on fixed DOFs; returns ||R||.
  double residual_u(const double *u, double *R) {
    const int N3 = 3 * g_.N;
    be_.internal_force(g_, m_, u, d_, R);
    be_.each(N3, FAxpy{R, R, 0.0, fu_, R});
    return std::sqrt(be_.sum(N3, FDot{R, R, fu_}));
  }

  // Jacobi PCG on the free entries: x = A^-1 rhs to ||r|| <= tol ||rhs||,
  // with A applied by apply(p, q) and the inverse diagonal in Dinv_.  The
  // scalars stay in device memory (CgState3); batches of kCgBatch3
  // iterations are enqueued between polls of the state, and the launches of
  // a batch after the solve has ended change nothing.
  // key names the call site (its buffers and operator), under which the
  // backend may keep the batch as a replayable graph.
  template <class Apply>
  int pcg(int key, int n, const double *rhs, const uint8_t *fixed, double tol, Apply &&apply,
          Counts3 *st) {
    be_.each(n, FFill{0.0, x_});
    be_.each(n, FAxpy{rhs, rhs, 0.0, fixed, r_});            // r = rhs on free entries
    be_.sum_into(n, FDot{r_, r_, fixed}, &cs_->bb);
    be_.each(n, FMul{Dinv_, r_, z_});
    be_.each(n, FAxpy{z_, z_, 0.0, fixed, p_});
    be_.sum_into(n, FDot{r_, z_, fixed}, &cs_->rz);
    be_.each(1, FCgStart{cs_, tol, o_.max_cg});
    CgState3 h{};
    be_.download(&h, cs_, sizeof h);
    while (!h.done) {
      if (!be_.replay(key)) {
        // every launch of a batch reads and writes the same buffers, so the
        // backend can record the batch once and replay it
        const bool rec = be_.capture_begin(2 * grid_blocks(n));
        for (int k = 0; k < kCgBatch3; ++k) {
          apply(p_, q_);
          be_.sum_into(n, FMaskDot{q_, p_, fixed}, &cs_->pq);
          be_.sum2_into(n, FCgUpdate{cs_, x_, r_, z_, p_, q_, Dinv_, fixed}, &cs_->rr,
                        &cs_->rz_new, FCgBeta{cs_});
          be_.each(n, FCgP{cs_, p_, z_, fixed});
        }
        if (rec) be_.capture_end(key);
      }
      be_.download(&h, cs_, sizeof h);
      if (!be_.ok()) break;
    }
    if (h.done == 3) st->cg_not_converged += 1;
    return h.iters;
  }

  // Newton for u at fixed d (Section 3.1), line search of at most 5
  // halvings; false if max_newton was reached.
  bool newton(double Rref, Counts3 *st) {
    const int N3 = 3 * g_.N;
    double nr = residual_u(u_, R_);
    int it = 0;
    while (nr > o_.tol_newton * Rref) {
      if (it >= o_.max_newton) {
        st->n_newton += it;
        return false;
      }
      be_.each(g_.N, FTangentDiag{g_, m_, u_, d_, D_});
      be_.each(N3, FInvDiag{D_, fu_, Dinv_});
      const double *u = u_;
      // the line search swaps u_ and ut_, so the batch's graph depends on
      // which of the two buffers holds the Newton point
      const int cg = pcg(u_ < ut_ ? 0 : 3, N3, R_, fu_, o_.tol_pcg,
                         [&](const double *p, double *q) {
        be_.tangent_apply(g_, m_, u, d_, p, q, &cs_->done);
      }, st);
      st->n_cg_u += cg;
      st->dof_updates += double(cg) * double(nfree_u_);
      // x solves K x = R; the step is -x
      double alpha = 1.0, nt = 0.0;
      for (int halv = 0;; ++halv) {
        be_.each(N3, FUpdate{u_, x_, -alpha, fu_, ut_});
        nt = residual_u(ut_, Rt_);
        if (nt < nr || halv == 5) break;
        alpha *= 0.5;
      }
      std::swap(u_, ut_);
      std::swap(R_, Rt_);
      nr = nt;
      ++it;
    }
    st->n_newton += it;
    return true;
  }

  // R_d = K_dd(Hs) d - b(Hs) on free entries (coefficient left in coef_);
  // returns ||R_d|| and ||b|| over the free entries.
  void phase_residual(const double *Hs, double *nR, double *nb) {
    const int N = g_.N;
    be_.each(g_.E, FPhaseCoef{g_, m_, 0, 0.0, Hs, nullptr, nullptr, nullptr, coef_});
    be_.each(N, FPhaseRhs{g_, Hs, b_});
    be_.phase_apply(g_, m_, coef_, d_, Rd_, nullptr);
    be_.each(N, FAxpy{Rd_, b_, -1.0, fd_, Rd_});
    *nR = std::sqrt(be_.sum(N, FDot{Rd_, Rd_, fd_}));
    *nb = std::sqrt(be_.sum(N, FDot{b_, b_, fd_}));
  }

  // QP update and the staggered residual ||R_d(d; H)|| / ||b(H)||.
  double qp_and_residual() {
    const Qp3 qp{o_.scheme, o_.psi_crit >= 0 ? o_.psi_crit : m_.Gc_l / 2.0, o_.d_gate};
    be_.each(g_.E, FQp{g_, m_, qp, u_, d_, Hc_, H_, psi_, flags_});
    gated_ = (long long)be_.sum(g_.E, FGated{flags_});
    double nR = 0.0, nb = 0.0;
    phase_residual(H_, &nR, &nb);
    return nb > 0.0 ? nR / nb : nR;
  }

  // Phase solve K_dd(Hs) d = b(Hs): d += K^-1 (-R_d).
  void phase_solve(const double *Hs, Counts3 *st) {
    const int N = g_.N;
    double nR = 0.0, nb = 0.0;
    phase_residual(Hs, &nR, &nb);
    be_.each(N, FPhaseDiag{g_, m_, coef_, D_});
    be_.each(N, FInvDiag{D_, fd_, Dinv_});
    const int cg = pcg(1, N, Rd_, fd_, o_.tol_pcg, [&](const double *p, double *q) {
      be_.phase_apply(g_, m_, coef_, p, q, &cs_->done);
    }, st);
    st->n_cg_d += cg;
    st->dof_updates += double(cg) * double(nfree_d_);
    be_.each(N, FUpdate{d_, x_, -1.0, fd_, d_});
    st->n_dsolve += 1;
  }

  // Trial solve with the floored block K_dd + K~ (Section 3.4) and the
  // predictor (Sections 3.3, 3.5) into Hhat_.
  void trial(Counts3 *st) {
    const int N = g_.N;
    st->gated_max = std::max(st->gated_max, gated_);
    double nR = 0.0, nb = 0.0;
    phase_residual(H_, &nR, &nb);
    st->floor_hits += (long long)be_.sum(
        g_.E, FFloorHits{g_, m_, o_.trial_floor, H_, psi_, flags_, d_, ctr_});
    be_.each(N, FPhaseDiag{g_, m_, ctr_, D_});
    be_.each(N, FInvDiag{D_, fd_, Dinv_});
    const int cg = pcg(2, N, Rd_, fd_, o_.tol_pcg, [&](const double *p, double *q) {
      be_.phase_apply(g_, m_, ctr_, p, q, &cs_->done);
    }, st);
    st->n_cg_trial += cg;
    st->dof_updates += double(cg) * double(nfree_d_);
    // the increment is -x (x solves A x = R_d), zero on fixed nodes
    be_.each(N, FScale{x_, -1.0, fd_, dd_});
    be_.each(g_.E, FPredictor{g_, m_, d_, dd_, H_, psi_, flags_, Hhat_});
    st->n_trial += 1;
  }

  B &be_;
  Grid3 g_;
  Mat3 m_;
  pf_solver_opts o_;
  std::vector<void *> owned_;
  double *u_ = nullptr, *ut_ = nullptr, *R_ = nullptr, *Rt_ = nullptr, *x_ = nullptr,
         *r_ = nullptr, *z_ = nullptr, *p_ = nullptr, *q_ = nullptr, *Dinv_ = nullptr,
         *D_ = nullptr, *unit_ = nullptr;
  double *d_ = nullptr, *dd_ = nullptr, *Rd_ = nullptr, *b_ = nullptr, *dval_ = nullptr;
  double *Hc_ = nullptr, *H_ = nullptr, *Hhat_ = nullptr, *psi_ = nullptr, *coef_ = nullptr,
         *ctr_ = nullptr;
  uint16_t *flags_ = nullptr;
  uint8_t *fu_ = nullptr, *fd_ = nullptr;
  CgState3 *cs_ = nullptr;
  std::vector<uint8_t> host_fu_, host_fd_;
  std::vector<double> host_unit_, host_dval_;
  std::vector<int64_t> gnode_[kGroups3];
  std::vector<int8_t> gcomp_[kGroups3];
  std::vector<double> gval_[kGroups3];
  int64_t *gdof_[kGroups3] = {};
  int8_t *gcomp_dev_[kGroups3] = {};
  int gn_[kGroups3] = {};
  std::vector<int64_t> dnode_;
  std::vector<double> dvalue_;
  long long gated_ = 0, nfree_u_ = 0, nfree_d_ = 0;
};

}  // namespace pf3d
