// Host runtime and C ABI: context, Dirichlet data, Newton for u, PCG drivers,
// iterative refinement for d, the staggered controller and the op entry
// points.  Every numerical step is a kernel from pf_kernels.hip; the host
// reads back only norms, counts and CG status words.

#include "../../include/phasefield.h"
#include "pf_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

using namespace pf;

namespace {

constexpr int kGroups = 8;

struct Group {
  std::vector<int64_t> node;
  std::vector<int8_t> comp;
  std::vector<double> val;
  int64_t *d_dof = nullptr;
  int8_t *d_comp = nullptr;
  int n = 0;
};

struct Allocator {
  pf_alloc_fn alloc = nullptr;
  pf_release_fn release = nullptr;
  void *user = nullptr;
};

// Work vectors of one precision.
template <class T>
struct CgBuf {
  // single-kernel CG vectors, double-buffered by iteration parity; the
  // right-hand side of a solve goes into R[0]
  T *R[2] = {nullptr, nullptr}, *W[2] = {nullptr, nullptr}, *S[2] = {nullptr, nullptr},
    *X[2] = {nullptr, nullptr}, *P[2] = {nullptr, nullptr};
  T *Dinv = nullptr;
  T *d = nullptr;      // d in this precision (operator data of the tangent)
  T *ulin = nullptr;   // [2N] linearisation point of the spectral tangent
  T *zc = nullptr, *rc = nullptr;   // second z and residual of the Chebyshev steps
  T *dc = nullptr;                  // second Chebyshev step vector
  T *pv[2] = {nullptr, nullptr};    // power-iteration vectors per operator kind
  T *coef = nullptr;   // [4E] phase coefficient
  T *gv[kGuessMax] = {};   // [2N] stored displacement solutions (starting guesses)
  T *gw[kGuessMax] = {};   // [2N] K v_j with the current operator
};

struct BatchSvc;

}  // namespace

struct pf_ctx {
  Grid g{};
  Mat mt{};
  pf_solver_opts opts{};
  ElasCoef ec{};
  PhaseCoef pc{};
  March ms{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;

  Group groups[kGroups];
  std::vector<int64_t> dnode;
  std::vector<double> dval;
  std::vector<uint8_t> eact_h;
  std::vector<uint8_t> nflag_h;

  // device state
  double *u = nullptr, *u_try = nullptr, *d = nullptr;
  double *H_prev = nullptr, *H = nullptr, *Hhat = nullptr, *psi_s = nullptr;
  double *Ru = nullptr, *Ru_try = nullptr, *Rd = nullptr, *Rfull = nullptr;
  double *u_unit = nullptr, *d_fix = nullptr;
  uint8_t *nflag = nullptr, *qflag = nullptr, *tflag = nullptr, *eact = nullptr;
  CgBuf<double> bd;
  CgBuf<float> bf;
  Cg1State *cgs = nullptr;     // [2]
  CgState *cgs2 = nullptr;      // two-kernel CG state
  CgState *cgs2_h = nullptr;    // [2]: the polls of two batches in flight
  int guess_m = 0, guess_next = 0;   // stored solutions, ring position
  double *guess_part = nullptr;      // [kGuessDots * kPMax] block partials
  double *guess_out = nullptr;       // [kGuessDots] finalised sums
  double *guess_h = nullptr;         // host copy
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  double *cgpart = nullptr;     // [2][3][kPMax]
  RedScratch rs{};
  // pinned host mirrors
  Cg1State *cgs_h = nullptr;   // [2]
  double *scal_h = nullptr;
  unsigned long long *icount_h = nullptr;
  // every library-owned device buffer: the field that holds it and its size
  struct Buf {
    void **field;
    size_t bytes;
  };
  std::vector<Buf> bufs;
  // installed device allocator (null callbacks: hipMalloc / hipFree)
  Allocator al{};

  // captured CG batches (hipGraph), keyed by solve kind and precision
  struct GraphEntry {
    int kind, fp32, niter, variant;
    double tol;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;
  bool use_graphs = true;

  // Jacobi-Chebyshev: lambda_max(D^-1 A) per [kind][fp32], re-estimated
  // for every solve from the previous power vector (0: no usable vector,
  // the next estimate starts cold); the polynomial's coefficients in device
  // memory (slot 2 kind + fp32) and a pinned mirror
  double lmax[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  double pscale[2][2] = {{1.0, 1.0}, {1.0, 1.0}};
  double *cheb_dev = nullptr;
  double *cheb_h = nullptr;

  // MINRES of the unfloored trial block: state and its pinned mirror
  MrState *mrs = nullptr;
  MrState *mrs_h = nullptr;

  // AT1 with the penalty: Psi+ of the current displacement (the driving
  // energy), the committed d, the penalty's active points, gamma
  bool at1 = false;
  double *psi_p = nullptr;
  double *d_prev = nullptr;
  uint8_t *chi = nullptr;
  double gamma = 0.0;

  // shared CG launches of a batch (set only inside pf_batch_load_step)
  BatchSvc *svc = nullptr;
  hipEvent_t ready_ev = nullptr;

  // sampled kernel timing
  bool profiling = false;
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t prof_launches[4] = {0, 0, 0, 0};
  int64_t prof_tick[2] = {0, 0};   // CG batches enqueued while timing is on, per kind
  double prof_ms[4] = {0.0, 0.0, 0.0, 0.0};

  // step state
  bool step_open = false;
  double step_load = 0.0;
  double R_ref = 1.0;
  int64_t gated_last = 0;
  int64_t n_free_u = 0, n_free_d = 0;
  pf_step_stats acc{};
  std::chrono::steady_clock::time_point t_open;
};

namespace {

pf_status fail(pf_ctx *c, pf_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

#define PF_HIP(ctx, ...)                                                                 \
  do {                                                                                   \
    hipError_t e_ = (__VA_ARGS__);                                                       \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, PF_E_HIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define PF_TRY(expr)                \
  do {                              \
    pf_status s_ = (expr);          \
    if (s_ != PF_OK) return s_;     \
  } while (0)

// Device memory from an installed allocator, or hipMalloc.
hipError_t raw_alloc(const Allocator &al, void **p, size_t bytes) {
  *p = nullptr;
  if (!al.alloc) return hipMalloc(p, bytes);
  void *v = al.alloc(bytes, al.user);
  if (!v) return hipErrorOutOfMemory;
  if (reinterpret_cast<uintptr_t>(v) % 256 != 0) {
    al.release(v, al.user);
    return hipErrorOutOfMemory;
  }
  *p = v;
  return hipSuccess;
}

void raw_free(const Allocator &al, void *p) {
  if (!p) return;
  if (al.release) al.release(p, al.user);
  else (void)hipFree(p);
}

template <class T>
pf_status dalloc(pf_ctx *c, T **p, size_t count) {
  void *v = nullptr;
  size_t bytes = std::max<size_t>(count * sizeof(T), 16);
  if (raw_alloc(c->al, &v, bytes) != hipSuccess) return fail(c, PF_E_OOM, "device allocation failed");
  c->bufs.push_back({reinterpret_cast<void **>(p), bytes});
  *p = static_cast<T *>(v);
  hipError_t e = fill_zero_bytes(c->stream, v, bytes);
  if (e != hipSuccess) return fail(c, PF_E_HIP, "zero fill failed");
  return PF_OK;
}

pf_status sync(pf_ctx *c) {
  PF_HIP(c, hipStreamSynchronize(c->stream));
  return PF_OK;
}

// Read scal[] and integer counters back to the host.
pf_status read_scal(pf_ctx *c) {
  PF_HIP(c, hipMemcpyAsync(c->scal_h, c->rs.scal, kScal * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  PF_HIP(c, hipMemcpyAsync(c->icount_h, c->rs.icount, kICounters * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

pf_status zero_icount(pf_ctx *c) {
  PF_HIP(c, fill_zero_bytes(c->stream, c->rs.icount, kICounters * sizeof(unsigned long long)));
  return PF_OK;
}

bool is_finite(double x) { return std::isfinite(x); }

// Rebuild node flags and Dirichlet value arrays from the host-side data.
pf_status upload_constraints(pf_ctx *c) {
  const Grid &g = c->g;
  std::vector<uint8_t> nf(g.N, 0);
  std::vector<double> unit(2 * (size_t)g.N, 0.0), dfix(g.N, 0.0);
  // inactive nodes: not touched by any active element
  if (!c->eact_h.empty()) {
    std::vector<uint8_t> touched(g.N, 0);
    for (int je = 0; je < g.ny; ++je)
      for (int ie = 0; ie < g.nx; ++ie)
        if (c->eact_h[ie + (size_t)je * g.nx]) {
          int n0 = ie + je * (g.nx + 1);
          touched[n0] = touched[n0 + 1] = touched[n0 + 1 + g.nx + 1] = touched[n0 + g.nx + 1] = 1;
        }
    for (int k = 0; k < g.N; ++k)
      if (!touched[k]) nf[k] = NF_UX | NF_UY | NF_D;
  }
  for (int gi = 0; gi < kGroups; ++gi) {
    const Group &gr = c->groups[gi];
    for (size_t k = 0; k < gr.node.size(); ++k) {
      const int64_t n = gr.node[k];
      nf[n] |= (gr.comp[k] == 0) ? NF_UX : NF_UY;
      unit[(size_t)n + (gr.comp[k] == 0 ? 0 : (size_t)g.N)] = gr.val[k];
    }
  }
  for (size_t k = 0; k < c->dnode.size(); ++k) {
    nf[c->dnode[k]] |= NF_D;
    dfix[c->dnode[k]] = c->dval[k];
  }
  // inactive nodes keep zero values
  if (!c->eact_h.empty()) {
    std::vector<uint8_t> touched(g.N, 0);
    for (int je = 0; je < g.ny; ++je)
      for (int ie = 0; ie < g.nx; ++ie)
        if (c->eact_h[ie + (size_t)je * g.nx]) {
          int n0 = ie + je * (g.nx + 1);
          touched[n0] = touched[n0 + 1] = touched[n0 + 1 + g.nx + 1] = touched[n0 + g.nx + 1] = 1;
        }
    for (int k = 0; k < g.N; ++k)
      if (!touched[k]) {
        unit[k] = 0.0;
        unit[k + (size_t)g.N] = 0.0;
        dfix[k] = 0.0;
      }
  }
  c->nflag_h = nf;
  int64_t fu = 0, fd = 0;
  for (int k = 0; k < g.N; ++k) {
    fu += !(nf[k] & NF_UX);
    fu += !(nf[k] & NF_UY);
    fd += !(nf[k] & NF_D);
  }
  c->n_free_u = fu;
  c->n_free_d = fd;
  PF_HIP(c, hipMemcpyAsync(c->nflag, nf.data(), g.N, hipMemcpyHostToDevice, c->stream));
  PF_HIP(c, hipMemcpyAsync(c->u_unit, unit.data(), unit.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  PF_HIP(c, hipMemcpyAsync(c->d_fix, dfix.data(), dfix.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  // group DOF lists (SoA index node + comp*N)
  for (int gi = 0; gi < kGroups; ++gi) {
    Group &gr = c->groups[gi];
    gr.n = (int)gr.node.size();
    if (gr.n == 0) continue;
    std::vector<int64_t> dof(gr.n);
    for (int k = 0; k < gr.n; ++k) dof[k] = gr.node[k] + (gr.comp[k] ? (int64_t)g.N : 0);
    PF_TRY(sync(c));
    raw_free(c->al, gr.d_dof);
    raw_free(c->al, gr.d_comp);
    gr.d_dof = nullptr;
    gr.d_comp = nullptr;
    void *vd = nullptr, *vc = nullptr;
    if (raw_alloc(c->al, &vd, gr.n * sizeof(int64_t)) != hipSuccess)
      return fail(c, PF_E_OOM, "device allocation failed");
    gr.d_dof = static_cast<int64_t *>(vd);
    if (raw_alloc(c->al, &vc, std::max(gr.n, 16)) != hipSuccess)
      return fail(c, PF_E_OOM, "device allocation failed");
    gr.d_comp = static_cast<int8_t *>(vc);
    PF_HIP(c, hipMemcpy(gr.d_dof, dof.data(), gr.n * sizeof(int64_t), hipMemcpyHostToDevice));
    PF_HIP(c, hipMemcpy(gr.d_comp, gr.comp.data(), gr.n, hipMemcpyHostToDevice));
  }
  return sync(c);
}

// ------------------------------------------------------------------ PCG

enum Kind { K_ELASTIC = 0, K_PHASE = 1 };
// A two-kernel CG solve from a starting guess: x already holds it and the
// right-hand side buffer its residual; the solve ends at r.r <= rr_abs.
struct CgStart {
  int warm = 0;
  double rr_abs = 0.0;
};
constexpr int kTimedRepeat = 4;
// With timing on, one enqueued CG batch in kProfEvery of each kind (the
// first included) carries the timed launches, so the sample adds little to
// the time of the steps it samples.
constexpr int kProfEvery = 8;
// Jacobi-Chebyshev interval [lambda_max / kChebRatio, lambda_max] with
// lambda_max = kChebSafety x the power-iteration estimate; power-iteration
// steps of a cold and of a warm estimate
constexpr double kChebRatio = 30.0;
constexpr double kChebSafety = 1.2;
constexpr int kPowerCold = 20;
constexpr int kPowerWarm = 6;
// FP64 iterative refinement of the phase solve (mixed precision): floor of
// the attainable residual relative to ||b||, and the reduction per pass
// below which the passes are taken to have stalled
constexpr double kRefineFloor = 1e-13;
constexpr double kRefineStall = 0.5;
// AT1: c_w of w(d) = d
constexpr double kAt1Cw = 8.0 / 3.0;
// largest 2N and 4E a context accepts: 32-bit indices with room for rounding
// up to whole blocks
constexpr long long kMaxIndexCount = (1LL << 31) - (1LL << 16);

template <class T>
CgBuf<T> &buf(pf_ctx *c);
template <>
CgBuf<double> &buf<double>(pf_ctx *c) { return c->bd; }
template <>
CgBuf<float> &buf<float>(pf_ctx *c) { return c->bf; }

template <class T>
CgVecs<T> cg_vecs(CgBuf<T> &b) {
  CgVecs<T> v;
  for (int k = 0; k < 2; ++k) {
    v.R[k] = b.R[k];
    v.W[k] = b.W[k];
    v.S[k] = b.S[k];
    v.X[k] = b.X[k];
    v.P[k] = b.P[k];
  }
  v.Dinv = b.Dinv;
  return v;
}

template <class T>
pf_status launch_k(pf_ctx *c, hipStream_t st, Kind kind, const Cg1Args &a) {
  CgBuf<T> &b = buf<T>(c);
  const CgVecs<T> v = cg_vecs(b);
  if (kind == K_ELASTIC) {
    PF_HIP(c, tangent_cg1<T>(st, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d, c->tflag, c->eact,
                             c->nflag, v, a));
  } else {
    PF_HIP(c, phase_cg1<T>(st, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag, v, a));
  }
  return PF_OK;
}

// Enqueue `iters` CG iterations (one kernel each) starting at parity 1
// (iters is even, so the batch ends at parity 0).  With time_first, the first
// kernel (idempotent: it reads parity-0 buffers and writes parity-1 ones) is
// launched kTimedRepeat times between one event pair.
template <class T>
pf_status enqueue_iters(pf_ctx *c, hipStream_t st, Kind kind, Cg1Args a, int iters,
                        bool time_first) {
  for (int k = 0; k < iters; ++k) {
    a.parity = (k + 1) & 1;
    a.init = 0;
    const bool t = time_first && k == 0;
    if (t) PF_HIP(c, hipEventRecord(c->ev[0], st));
    for (int rep = 0; rep < (t ? kTimedRepeat : 1); ++rep) PF_TRY(launch_k<T>(c, st, kind, a));
    if (t) PF_HIP(c, hipEventRecord(c->ev[1], st));
  }
  return PF_OK;
}

// Graph of `niter` CG iterations for this solve kind, captured on a private
// stream the first time it is needed and launched on the context's stream.
template <class T>
pf_status cg_graph(pf_ctx *c, Kind kind, const Cg1Args &a, double tol, int niter,
                   hipGraphExec_t *out) {
  const int fp32 = std::is_same<T, float>::value ? 1 : 0;
  for (auto &e : c->graphs)
    if (e.kind == kind && e.fp32 == fp32 && e.niter == niter && e.tol == tol && e.variant == 1) {
      *out = e.exec;
      return PF_OK;
    }
  if (!c->cap_stream) PF_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  PF_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  pf_status s = enqueue_iters<T>(c, c->cap_stream, kind, a, niter, false);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  if (s != PF_OK) return s;
  if (e != hipSuccess) return fail(c, PF_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(c, PF_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  c->graphs.push_back({kind, fp32, niter, 1, tol, ex});
  *out = ex;
  return PF_OK;
}

// ---- two-kernel CG (standard recurrences), used for the FP32 inner solves.
// Buffers: x = X[0], r = R[0], z = W[0], p_old/p_new = P[0]/P[1], q = S[0].
// lambda_max(D^-1 A) by power iteration (Rayleigh quotient in the D inner
// product); b.Dinv must be set and W[1] serves as scratch.  The first
// estimate runs kPowerCold steps from a fixed start, renormalising after
// each.  Later ones continue from the previous vector for kPowerWarm steps,
// so the estimate follows the operator as the damage grows; they keep the
// previous normalisation (the operator changes little between solves, and
// the Rayleigh quotient does not depend on the scale), so their launches
// queue back to back and only the last step's sums are read.  A warm
// estimate that comes out degenerate falls back to a cold one.  Both step
// counts are even, so the latest vector ends in b.pv[kind].
template <class T>
pf_status power_step(pf_ctx *c, Kind kind, const T *v, T *vn, double scale) {
  CgBuf<T> &b = buf<T>(c);
  if (kind == K_ELASTIC) {
    PF_HIP(c, tangent_power_step<T>(c->stream, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d,
                                    c->tflag, c->eact, c->nflag, v, vn, b.Dinv, scale, c->rs));
  } else {
    PF_HIP(c, phase_power_step<T>(c->stream, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag, v,
                                  vn, b.Dinv, scale, c->rs));
  }
  return PF_OK;
}

template <class T>
pf_status estimate_lmax(pf_ctx *c, Kind kind, double *out) {
  CgBuf<T> &b = buf<T>(c);
  const int n = (kind == K_ELASTIC) ? 2 * c->g.N : c->g.N;
  const int fp32 = std::is_same<T, float>::value ? 1 : 0;
  T *v = b.pv[kind], *vn = b.W[1];
  if (c->lmax[kind][fp32] > 0.0) {
    const double scale = c->pscale[kind][fp32];
    for (int it = 0; it < kPowerWarm; ++it) {
      PF_TRY(power_step<T>(c, kind, v, vn, scale));
      std::swap(v, vn);
    }
    PF_TRY(read_scal(c));
    const double A = c->scal_h[SC_NORM_A], B = c->scal_h[SC_NORM_B];
    if (B > 0.0 && A > 0.0 && std::isfinite(A) && std::isfinite(B)) {
      const double lam = A / B;
      c->pscale[kind][fp32] = 1.0 / (lam * std::sqrt(B));
      c->lmax[kind][fp32] = lam;
      *out = lam;
      return PF_OK;
    }
  }
  PF_HIP(c, power_start<T>(c->stream, n, b.Dinv, b.pv[kind]));
  v = b.pv[kind];
  vn = b.W[1];
  double scale = 1.0, lam = 0.0;
  for (int it = 0; it < kPowerCold; ++it) {
    PF_TRY(power_step<T>(c, kind, v, vn, scale));
    PF_TRY(read_scal(c));
    const double A = c->scal_h[SC_NORM_A], B = c->scal_h[SC_NORM_B];
    if (!(B > 0.0) || !(A > 0.0) || !std::isfinite(A) || !std::isfinite(B)) {
      // a degenerate operator (nothing free): no vector to continue from
      c->lmax[kind][fp32] = 0.0;
      *out = lam > 0.0 ? lam : 4.0;
      return PF_OK;
    }
    lam = A / B;
    scale = 1.0 / (lam * std::sqrt(B));
    std::swap(v, vn);
  }
  c->pscale[kind][fp32] = scale;
  c->lmax[kind][fp32] = lam;
  *out = lam;
  return PF_OK;
}

// Chebyshev coefficients for degree m on [lmax / ratio, lmax], written to
// host[] (coef layout of ChebStep); the steps point at the device copy dev.
void cheb_steps(double lmax, int m, double ratio, const double *dev, double *host,
                std::vector<ChebStep> *out) {
  const double hi = lmax, lo = lmax / ratio;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  out->clear();
  double rho = 1.0 / sigma;
  host[0] = 1.0 / theta;
  out->push_back(ChebStep{dev, 0, m == 1 ? 1 : 0});
  for (int k = 1; k < m; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    host[2 * k - 1] = rn * rho;
    host[2 * k] = 2.0 * rn / delta;
    out->push_back(ChebStep{dev, k, k == m - 1 ? 1 : 0});
    rho = rn;
  }
}

// z = Chebyshev(r) (partials r.z, r.r from the last step)
template <class T>
pf_status enqueue_cheb(pf_ctx *c, hipStream_t st, Kind kind, const CgArgs &ca, int n,
                       const std::vector<ChebStep> &cs, bool init, size_t kfirst, bool timed,
                       const T *rcur) {
  CgBuf<T> &b = buf<T>(c);
  T *D[2] = {b.W[1], b.dc};
  // z and the residual alternate between two buffers; the first step
  // starts from the buffer that makes the last one end in W[0]
  T *zb[2] = {b.W[0], b.zc}, *rb[2] = {b.S[1], b.rc};
  const int i0 = (int)((cs.size() - 1) & 1);
  if (init) PF_HIP(c, cheb_init<T>(st, n, rcur, b.Dinv, D[0], zb[i0], rb[i0], ca, cs[0]));
  for (size_t k = kfirst; k < cs.size(); ++k) {
    const int in = i0 ^ (int)((k - 1) & 1), out = i0 ^ (int)(k & 1);
    // the steps leave their inputs intact: the timed sample repeats the first
    const bool t = timed && k == kfirst;
    if (t) PF_HIP(c, hipEventRecord(c->ev[3], st));
    for (int rep = 0; rep < (t ? kTimedRepeat : 1); ++rep) {
      if (kind == K_ELASTIC) {
        PF_HIP(c, tangent_cheb_step<T>(st, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d,
                                       c->tflag, c->eact, c->nflag, D[(k - 1) & 1], D[k & 1],
                                       zb[in], zb[out], rb[in], rb[out], rcur, b.Dinv, ca,
                                       cs[k]));
      } else {
        PF_HIP(c, phase_cheb_step<T>(st, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag,
                                     D[(k - 1) & 1], D[k & 1], zb[in], zb[out], rb[in], rb[out],
                                     rcur, b.Dinv, ca, cs[k]));
      }
    }
    if (t) PF_HIP(c, hipEventRecord(c->ev[4], st));
  }
  return PF_OK;
}

template <class T>
pf_status enqueue_iters2(pf_ctx *c, hipStream_t st, Kind kind, const CgArgs &ca, int n, int iters,
                         bool time_first, const std::vector<ChebStep> *cs) {
  CgBuf<T> &b = buf<T>(c);
  T *pold = b.P[0], *pnew = b.P[1];
  // Jacobi-Chebyshev of degree >= 2: the update is fused with the first
  // polynomial step and writes x and r to the other buffer of each pair, so
  // iteration k (counted from an even start) reads X[k&1], R[k&1]
  const bool fused = cs && cs->size() >= 2;
  for (int k = 0; k < iters; ++k) {
    // the apply kernel is idempotent (it rewrites p_new, q and its partials
    // from inputs it does not modify): the timed sample repeats it
    const bool t = time_first && k == 0;
    if (t) PF_HIP(c, hipEventRecord(c->ev[0], st));
    for (int rep = 0; rep < (t ? kTimedRepeat : 1); ++rep) {
      if (kind == K_ELASTIC) {
        PF_HIP(c, tangent_cg_apply<T>(st, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d, c->tflag,
                                      c->eact, c->nflag, b.W[0], pold, pnew, b.S[0], ca));
      } else {
        PF_HIP(c, phase_cg_apply<T>(st, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag, b.W[0],
                                    pold, pnew, b.S[0], ca));
      }
    }
    if (t) PF_HIP(c, hipEventRecord(c->ev[1], st));
    if (fused && cs->size() >= 3 && c->ms.ch == 1) {
      // LDS tiles: the update and the first two polynomial steps are one
      // kernel; step 2's z, residual and direction land where step 2 of the
      // separate kernels puts them (zb[i0], rb[i0], W[1])
      const int par = k & 1;
      const int i0 = (int)((cs->size() - 1) & 1);
      T *zb[2] = {b.W[0], b.zc}, *rb[2] = {b.S[1], b.rc};
      for (int rep = 0; rep < (t ? kTimedRepeat : 1); ++rep) {
        if (kind == K_ELASTIC) {
          PF_HIP(c, tangent_updcheb2<T>(st, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d,
                                        c->tflag, c->eact, c->nflag, b.X[par], b.X[par ^ 1],
                                        b.R[par], b.R[par ^ 1], pnew, b.S[0], b.Dinv, b.W[1],
                                        zb[i0], rb[i0], ca, (*cs)[2]));
        } else {
          PF_HIP(c, phase_updcheb2<T>(st, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag,
                                      b.X[par], b.X[par ^ 1], b.R[par], b.R[par ^ 1], pnew,
                                      b.S[0], b.Dinv, b.W[1], zb[i0], rb[i0], ca, (*cs)[2]));
        }
      }
      if (t) PF_HIP(c, hipEventRecord(c->ev[2], st));
      PF_TRY(enqueue_cheb<T>(c, st, kind, ca, n, *cs, false, 3, t && cs->size() > 3,
                             b.R[par ^ 1]));
    } else if (fused) {
      const int par = k & 1;
      const int i0 = (int)((cs->size() - 1) & 1);
      T *zb[2] = {b.W[0], b.zc}, *rb[2] = {b.S[1], b.rc};
      for (int rep = 0; rep < (t ? kTimedRepeat : 1); ++rep) {
        if (kind == K_ELASTIC) {
          PF_HIP(c, tangent_updcheb<T>(st, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d, c->tflag,
                                       c->eact, c->nflag, b.X[par], b.X[par ^ 1], b.R[par],
                                       b.R[par ^ 1], pnew, b.S[0], b.Dinv, b.dc, zb[i0 ^ 1],
                                       rb[i0 ^ 1], ca, (*cs)[0], (*cs)[1]));
        } else {
          PF_HIP(c, phase_updcheb<T>(st, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag,
                                     b.X[par], b.X[par ^ 1], b.R[par], b.R[par ^ 1], pnew, b.S[0],
                                     b.Dinv, b.dc, zb[i0 ^ 1], rb[i0 ^ 1], ca, (*cs)[0],
                                     (*cs)[1]));
        }
      }
      if (t) PF_HIP(c, hipEventRecord(c->ev[2], st));
      PF_TRY(enqueue_cheb<T>(c, st, kind, ca, n, *cs, false, 2, t && cs->size() > 2,
                             b.R[par ^ 1]));
    } else {
      // Jacobi, or Chebyshev of degree 1: the update also takes the
      // polynomial's only step (z and residual into W[0] and S[1])
      ChebFuse<T> cf{nullptr, nullptr, nullptr, 0};
      if (cs) cf = ChebFuse<T>{b.W[1], b.S[1], (*cs)[0].coef, (*cs)[0].last};
      PF_HIP(c, cg_update<T>(st, n, b.X[0], b.R[0], b.W[0], pnew, b.S[0], b.Dinv, ca, cf));
      if (t) PF_HIP(c, hipEventRecord(c->ev[2], st));
    }
    std::swap(pold, pnew);
  }
  return PF_OK;
}

// ------------------------------------------------ shared CG launches

// One FP32 Jacobi CG solve served by shared launches.
struct CgRequest {
  pf_ctx *c = nullptr;
  Kind kind = K_ELASTIC;
  double tol = 0.0;
  int iters = 0, status = 0;
  bool done = false;
  pf_status err = PF_OK;
  std::string msg;
};

// A request inside the running shared CG loop.
struct ActiveCg {
  CgRequest *r;
  CgArgs ca;
  int n, split, ch;
};

// Batch service (continuous batching of CG solves): member threads queue
// their solves; a service thread keeps one CG loop running over every active
// system, two shared launches (one apply per operator kind, split and
// work-item height, one update) per iteration.  At each status poll, every
// `check` iterations, finished systems are handed back to their members and
// queued ones join, so no member waits for another's solve.
struct BatchSvc {
  std::mutex mu;
  std::condition_variable work_cv;   // service: new requests or stop
  std::condition_variable done_cv;   // members: a request finished
  std::vector<CgRequest *> pending;
  bool stop = false;
  hipStream_t stream = nullptr;
  char *dblob = nullptr, *hblob = nullptr;
  size_t cap = 0;
  int check = 32;
  // launch layout of the current active set
  struct Launch {
    int kind, split, ch, nb;
    size_t tab, map, count;
  };
  std::vector<Launch> applies;
  size_t utab = 0, umap = 0, stat = 0;
  int ublocks = 0;

  ~BatchSvc() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (dblob) (void)hipFree(dblob);
    if (hblob) (void)hipHostFree(hblob);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Start a request's CG on the service stream (after its member's right-hand
// side is in place).
hipError_t admit(BatchSvc *svc, CgRequest *r, ActiveCg *a) {
  pf_ctx *c = r->c;
  CgBuf<float> &b = c->bf;
  a->r = r;
  a->n = (r->kind == K_ELASTIC) ? 2 * c->g.N : c->g.N;
  a->ca = cg_args(c->g, c->ms, a->n, c->cgs2, c->rs, r->tol, c->opts.max_cg);
  a->split = (r->kind == K_ELASTIC) ? c->mt.split : 0;
  a->ch = c->ms.ch;
  hipError_t e = hipStreamWaitEvent(svc->stream, c->ready_ev, 0);
  if (e != hipSuccess) return e;
  return cg_init<float>(svc->stream, a->n, b.X[0], b.R[0], b.W[0], b.P[0], b.Dinv, a->ca);
}

// Tables and block maps of the active set, uploaded to the device.  Each
// system keeps the blocks of its own launch.  Systems join at even shared
// iteration counts, so iteration k of every system uses direction buffers
// of parity k & 1 (two tables).
hipError_t rebuild(BatchSvc *svc, const std::vector<ActiveCg> &act) {
  std::map<std::tuple<int, int, int>, std::vector<int>> groups;
  for (int i = 0; i < (int)act.size(); ++i)
    groups[std::make_tuple((int)act[i].r->kind, act[i].split, act[i].ch)].push_back(i);
  const size_t nr = act.size();
  svc->applies.clear();
  std::vector<std::vector<int>> members;
  size_t off = 0;
  for (auto &kv : groups) {
    BatchSvc::Launch L{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), 0,
                       off, 0, kv.second.size()};
    for (int i : kv.second) L.nb += act[i].ca.ga;
    off += 2 * L.count * (size_t)kBatchEntryBytes;
    svc->applies.push_back(L);
    members.push_back(kv.second);
  }
  svc->utab = align_up(off, 256);
  off = svc->utab + 2 * nr * sizeof(BatchUpdateEntry<float>);
  for (auto &L : svc->applies) {
    L.map = align_up(off, 256);
    off = L.map + (size_t)L.nb * sizeof(int);
  }
  svc->ublocks = 0;
  for (auto &a : act) svc->ublocks += a.ca.gb;
  svc->umap = align_up(off, 256);
  off = svc->umap + (size_t)svc->ublocks * sizeof(int);
  svc->stat = align_up(off, 256);
  const size_t total = svc->stat + 2 * nr * sizeof(int);
  if (total > svc->cap) {
    if (svc->dblob) (void)hipFree(svc->dblob);
    if (svc->hblob) (void)hipHostFree(svc->hblob);
    svc->dblob = svc->hblob = nullptr;
    svc->cap = 0;
    const size_t want = align_up(total * 2, 1 << 16);
    hipError_t e = hipMalloc((void **)&svc->dblob, want);
    if (e != hipSuccess) return e;
    e = hipHostMalloc((void **)&svc->hblob, want);
    if (e != hipSuccess) return e;
    svc->cap = want;
  }
  char *h = svc->hblob;
  int *dstat = reinterpret_cast<int *>(svc->dblob + svc->stat);
  std::memset(h, 0, total);
  for (size_t gi = 0; gi < svc->applies.size(); ++gi) {
    const BatchSvc::Launch &L = svc->applies[gi];
    int *map = reinterpret_cast<int *>(h + L.map);
    int b0 = 0;
    for (size_t j = 0; j < L.count; ++j) {
      const ActiveCg &a = act[members[gi][j]];
      pf_ctx *c = a.r->c;
      CgBuf<float> &b = c->bf;
      for (int par = 0; par < 2; ++par) {
        void *e = h + L.tab + (par * L.count + j) * (size_t)kBatchEntryBytes;
        float *pold = b.P[par], *pnew = b.P[par ^ 1];
        if (L.kind == K_ELASTIC)
          tangent_batch_entry<float>(e, c->g, c->ms, c->ec, L.split, b.ulin, b.d, c->tflag,
                                     c->eact, c->nflag, b.W[0], pold, pnew, b.S[0], a.ca, b0,
                                     a.ca.ga);
        else
          phase_batch_entry<float>(e, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag, b.W[0],
                                   pold, pnew, b.S[0], a.ca, b0, a.ca.ga);
      }
      for (int k = 0; k < a.ca.ga; ++k) map[b0 + k] = (int)j;
      b0 += a.ca.ga;
    }
  }
  auto *ut = reinterpret_cast<BatchUpdateEntry<float> *>(h + svc->utab);
  int *umap = reinterpret_cast<int *>(h + svc->umap);
  int b0 = 0;
  for (size_t i = 0; i < nr; ++i) {
    const ActiveCg &a = act[i];
    CgBuf<float> &b = a.r->c->bf;
    for (int par = 0; par < 2; ++par)
      ut[par * nr + i] = BatchUpdateEntry<float>{b.X[0], b.R[0], b.W[0], b.P[par ^ 1], b.S[0],
                                                 b.Dinv, a.ca, a.n, b0, a.ca.gb,
                                                 dstat + 2 * i};
    for (int k = 0; k < a.ca.gb; ++k) umap[b0 + k] = (int)i;
    b0 += a.ca.gb;
  }
  return hipMemcpyAsync(svc->dblob, h, total, hipMemcpyHostToDevice, svc->stream);
}

// `check` shared iterations of the active set from iteration K (even).
hipError_t run_iters(BatchSvc *svc, size_t nr) {
  char *d = svc->dblob;
  const auto *dut = reinterpret_cast<const BatchUpdateEntry<float> *>(d + svc->utab);
  const int *dumap = reinterpret_cast<const int *>(d + svc->umap);
  for (int k = 0; k < svc->check; ++k) {
    const int par = k & 1;
    for (const auto &L : svc->applies) {
      const void *tab = d + L.tab + par * L.count * (size_t)kBatchEntryBytes;
      const int *map = reinterpret_cast<const int *>(d + L.map);
      const hipError_t e = L.kind == K_ELASTIC
                               ? tangent_cg_apply_batch<float>(svc->stream, L.split, L.ch, tab,
                                                               map, L.nb)
                               : phase_cg_apply_batch<float>(svc->stream, L.ch, tab, map, L.nb);
      if (e != hipSuccess) return e;
    }
    const hipError_t e = cg_update_batch<float>(svc->stream, dut + par * nr, dumap, svc->ublocks);
    if (e != hipSuccess) return e;
  }
  int *hstat = reinterpret_cast<int *>(svc->hblob + svc->stat);
  const int *dstat = reinterpret_cast<const int *>(d + svc->stat);
  hipError_t e = hipMemcpyAsync(hstat, dstat, 2 * nr * sizeof(int), hipMemcpyDeviceToHost,
                                svc->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(svc->stream);
}

// Service thread: admit, iterate, hand back, until stopped with nothing left.
void service_loop(BatchSvc *svc) {
  std::vector<ActiveCg> act;
  std::unique_lock<std::mutex> lk(svc->mu);
  for (;;) {
    svc->work_cv.wait(lk, [&] { return !act.empty() || !svc->pending.empty() || svc->stop; });
    if (act.empty() && svc->pending.empty()) break;   // stopped
    std::vector<CgRequest *> add;
    add.swap(svc->pending);
    lk.unlock();
    hipError_t e = hipSuccess;
    for (CgRequest *r : add) {
      ActiveCg a{};
      if (e == hipSuccess) e = admit(svc, r, &a);
      a.r = r;
      act.push_back(a);
    }
    if (e == hipSuccess && !add.empty()) e = rebuild(svc, act);
    if (e == hipSuccess) e = run_iters(svc, act.size());
    std::vector<ActiveCg> keep;
    bool removed = false;
    lk.lock();
    if (e != hipSuccess) {
      for (auto &a : act) {
        a.r->err = PF_E_HIP;
        a.r->msg = hipGetErrorString(e);
        a.r->done = true;
      }
      act.clear();
    } else {
      const int *hstat = reinterpret_cast<const int *>(svc->hblob + svc->stat);
      for (size_t i = 0; i < act.size(); ++i) {
        if (hstat[2 * i] != 0) {
          act[i].r->status = hstat[2 * i];
          act[i].r->iters = hstat[2 * i + 1];
          act[i].r->done = true;
          removed = true;
        } else {
          keep.push_back(act[i]);
        }
      }
      act.swap(keep);
    }
    svc->done_cv.notify_all();
    if (removed && !act.empty() && svc->pending.empty()) {
      lk.unlock();
      e = rebuild(svc, act);
      lk.lock();
      if (e != hipSuccess) {
        for (auto &a : act) {
          a.r->err = PF_E_HIP;
          a.r->msg = hipGetErrorString(e);
          a.r->done = true;
        }
        act.clear();
        svc->done_cv.notify_all();
      }
    }
  }
}

// Queue this context's FP32 Jacobi solve with the batch service and wait.
pf_status shared_pcg(pf_ctx *c, Kind kind, double tol, int *iters, int *status, float **xout) {
  if (!c->ready_ev) PF_HIP(c, hipEventCreateWithFlags(&c->ready_ev, hipEventDisableTiming));
  PF_HIP(c, hipEventRecord(c->ready_ev, c->stream));
  CgRequest req;
  req.c = c;
  req.kind = kind;
  req.tol = tol;
  BatchSvc *svc = c->svc;
  {
    std::unique_lock<std::mutex> lk(svc->mu);
    svc->pending.push_back(&req);
    svc->work_cv.notify_one();
    svc->done_cv.wait(lk, [&] { return req.done; });
  }
  if (req.err != PF_OK) return fail(c, req.err, "shared CG launch: " + req.msg);
  *iters = req.iters;
  *status = req.status;
  *xout = c->bf.X[0];
  return PF_OK;
}

template <class T>
pf_status pcg2(pf_ctx *c, Kind kind, double tol, int *iters, int *status, T **xout,
               const CgStart &start = CgStart{}) {
  if constexpr (std::is_same<T, float>::value) {
    if (c->svc && c->opts.precond == PF_PC_JACOBI && !c->profiling)
      return shared_pcg(c, kind, tol, iters, status, xout);
  }
  CgBuf<T> &b = buf<T>(c);
  const int n = (kind == K_ELASTIC) ? 2 * c->g.N : c->g.N;
  CgArgs ca = cg_args(c->g, c->ms, n, c->cgs2, c->rs, tol, c->opts.max_cg);
  const int fp32 = std::is_same<T, float>::value ? 1 : 0;
  const bool cheb = c->opts.precond == PF_PC_JACOBI_CHEBYSHEV;
  std::vector<ChebStep> cs;
  if (cheb) {
    double est = 0.0;
    PF_TRY(estimate_lmax<T>(c, kind, &est));
    const int slot = 2 * (int)kind + fp32;
    double *dev = c->cheb_dev + slot * kChebCoefs, *host = c->cheb_h + slot * kChebCoefs;
    cheb_steps(kChebSafety * est, std::max(1, c->opts.cheb_degree),
               c->opts.cheb_ratio > 0 ? c->opts.cheb_ratio : kChebRatio, dev, host, &cs);
    // the previous solve of this kind has finished, so its copy has too
    PF_HIP(c, hipMemcpyAsync(dev, host, kChebCoefs * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
    ca.ext = 1;
    ca.npb = cs.size() > 1 ? cg1_blocks(c->ms) : ca.gb;
  }
  ca.warm = start.warm;
  ca.rr_abs = start.rr_abs;
  PF_HIP(c, cg_init<T>(c->stream, n, b.X[0], b.R[0], b.W[0], b.P[0], b.Dinv, ca));
  if (cheb) PF_TRY(enqueue_cheb<T>(c, c->stream, kind, ca, n, cs, true, 1, false, b.R[0]));
  int batch = std::max(4, c->opts.cg_check);
  batch += batch & 1;
  const int kid = (kind == K_ELASTIC) ? 0 : 1;
  const bool timed = c->profiling;
  const int ngraph = timed ? batch - 2 : batch;
  const int variant = cheb ? 3 : 2;
  hipGraphExec_t ex = nullptr;
  if (c->use_graphs) {
    for (auto &e : c->graphs)
      // the tolerance is read from the CG state, which the init (outside
      // the graph) sets, so one graph serves every tolerance
      if (e.kind == kind && e.fp32 == fp32 && e.niter == ngraph && e.variant == variant)
        ex = e.exec;
    if (!ex) {
      if (!c->cap_stream) PF_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      PF_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      pf_status s = enqueue_iters2<T>(c, c->cap_stream, kind, ca, n, ngraph, false,
                                      cheb ? &cs : nullptr);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
      if (s != PF_OK) return s;
      if (e != hipSuccess) return fail(c, PF_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(c, PF_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      c->graphs.push_back({kind, fp32, ngraph, variant, tol, ex});
    }
  }
  // A batch, then a copy of the CG state to one of two host slots and an
  // event after it.  While the residual's decay between polls says that the
  // solve needs well over another batch, the next batch and its poll are
  // enqueued before the host waits for the current one, so the GPU does not
  // idle through the round trip.  A batch enqueued after convergence exits
  // in its kernels' prologues, as the rest of a batch does.
  auto enqueue_batch = [&](bool tb, int slot) -> pf_status {
    if (tb) PF_TRY(enqueue_iters2<T>(c, c->stream, kind, ca, n, 2, true, cheb ? &cs : nullptr));
    if (ex) {
      PF_HIP(c, hipGraphLaunch(ex, c->stream));
    } else {
      PF_TRY(enqueue_iters2<T>(c, c->stream, kind, ca, n, ngraph, false, cheb ? &cs : nullptr));
    }
    PF_HIP(c, hipMemcpyAsync(c->cgs2_h + slot, c->cgs2, sizeof(CgState), hipMemcpyDeviceToHost,
                             c->stream));
    PF_HIP(c, hipEventRecord(c->poll_ev[slot], c->stream));
    return PF_OK;
  };
  const double tol2 = tol * tol;
  int slot = 0;
  bool ahead = false;               // the batch of `slot` is already enqueued
  double rr_last = -1.0, rr0 = 0.0; // r.r, the initial r.r and the iteration count
  int it_last = 0;                  // at the previous poll
  double log_rate = 0.0;            // log of the per-iteration decay of r.r (< 0)
  const int per_batch = ngraph + (timed ? 2 : 0);
  for (;;) {
    bool tb = false;
    if (!ahead) {
      tb = timed && (c->prof_tick[kid]++ % kProfEvery) == 0;
      PF_TRY(enqueue_batch(tb, slot));
    }
    bool next_ahead = false;
    // the batch of `slot` runs iterations it_last .. it_last + per_batch;
    // one enqueued ahead would run the next per_batch
    const double target = tol2 * rr0;
    if (!tb && rr_last > target && target > 0.0 && log_rate < 0.0 &&
        std::log(target / rr_last) / log_rate > 2.5 * per_batch) {
      PF_TRY(enqueue_batch(false, slot ^ 1));
      next_ahead = true;
    }
    PF_HIP(c, hipEventSynchronize(c->poll_ev[slot]));
    const CgState &h = c->cgs2_h[slot];
    if (tb) {
      float a = 0.f, u = 0.f;
      PF_HIP(c, hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
      PF_HIP(c, hipEventElapsedTime(&u, c->ev[1], c->ev[2]));
      c->prof_launches[kid] += kTimedRepeat;
      c->prof_ms[kid] += a;
      // displacement solves only; the fused update + first Chebyshev step
      // is repeated like the apply
      if (kind == K_ELASTIC) {
        c->prof_launches[2] += (cheb && cs.size() > 1) ? kTimedRepeat : 1;
        c->prof_ms[2] += u;
      }
      // the first separate polynomial step (timed by enqueue_cheb) is step 3
      // where the update kernel takes two steps (LDS tiles), else step 2
      const size_t first_sep = (cheb && cs.size() >= 3 && c->ms.ch == 1) ? 3 : 2;
      if (cheb && cs.size() > first_sep && kind == K_ELASTIC) {
        float q = 0.f;
        PF_HIP(c, hipEventElapsedTime(&q, c->ev[3], c->ev[4]));
        c->prof_launches[3] += kTimedRepeat;
        c->prof_ms[3] += q;
      }
    }
    // a batch enqueued ahead finishes in stream order: it writes the other
    // slot and no buffer the caller reads
    if (h.b.done != 0) break;
    if (rr_last > 0.0 && h.a.rr > 0.0 && h.a.iters > it_last)
      log_rate = std::log(h.a.rr / rr_last) / double(h.a.iters - it_last);
    rr_last = h.a.rr;
    rr0 = h.a.rr0;
    it_last = h.a.iters;
    if (next_ahead) slot ^= 1;
    ahead = next_ahead;
  }
  const CgState &fin = c->cgs2_h[slot];
  *iters = fin.b.iters;
  *status = fin.b.done;
  // the fused update alternates the x buffers: the last active iteration
  // wrote X[iters & 1]
  *xout = (cheb && cs.size() >= 2) ? b.X[*iters & 1] : b.X[0];
  return PF_OK;
}

// Solve A x = r0 (r0 in b.R[0], zero on fixed DOFs) from x = 0 with Jacobi
// PCG (single-kernel CG) to ||r|| <= tol ||r0||.  b.Dinv holds the inverse
// diagonal.  Batches of cg_check iterations are enqueued (as a captured
// graph) between polls of the device-side status; kernels after convergence
// exit in their prologue.  *xout points to the solution buffer.
template <class T>
pf_status pcg(pf_ctx *c, Kind kind, double tol, int *iters, int *status, T **xout,
              const CgStart &start = CgStart{}) {
  // the single-kernel formulation marches columns; LDS tiles use two kernels
  const bool two = c->opts.cg_kernels == 2 || c->ms.ch == 1 ||
                   (c->opts.cg_kernels == 0 && std::is_same<T, float>::value);
  if (two || c->opts.precond == PF_PC_JACOBI_CHEBYSHEV)
    return pcg2<T>(c, kind, tol, iters, status, xout, start);
  CgBuf<T> &b = buf<T>(c);
  Cg1Args a;
  a.st = c->cgs;
  a.part = c->cgpart;
  a.np = cg1_blocks(c->ms);
  a.tol2 = tol * tol;
  a.maxit = c->opts.max_cg;
  a.parity = 0;
  a.init = 1;
  PF_TRY(launch_k<T>(c, c->stream, kind, a));
  int batch = std::max(4, c->opts.cg_check);
  batch += batch & 1;
  const int kid = (kind == K_ELASTIC) ? 0 : 1;
  const bool timed = c->profiling;
  hipGraphExec_t ex = nullptr;
  const int ngraph = timed ? batch - 2 : batch;
  if (c->use_graphs) PF_TRY(cg_graph<T>(c, kind, a, tol, ngraph, &ex));
  for (;;) {
    const bool tb = timed && (c->prof_tick[kid]++ % kProfEvery) == 0;
    if (tb) PF_TRY(enqueue_iters<T>(c, c->stream, kind, a, 2, true));
    if (ex) {
      PF_HIP(c, hipGraphLaunch(ex, c->stream));
    } else {
      PF_TRY(enqueue_iters<T>(c, c->stream, kind, a, ngraph, false));
    }
    PF_HIP(c, hipMemcpyAsync(c->cgs_h, c->cgs, 2 * sizeof(Cg1State), hipMemcpyDeviceToHost,
                             c->stream));
    PF_TRY(sync(c));
    if (tb) {
      float ms = 0.f;
      PF_HIP(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
      c->prof_launches[kid] += kTimedRepeat;
      c->prof_ms[kid] += ms;
    }
    if (c->cgs_h[0].done != 0) break;
  }
  *iters = c->cgs_h[0].iters;
  *status = c->cgs_h[0].done;
  *xout = b.X[*iters & 1];
  return PF_OK;
}

// ------------------------------------------------------- displacement

pf_status residual_u(pf_ctx *c, const double *u, double *R, double *norm) {
  PF_HIP(c, internal_force(c->stream, c->g, c->ms, c->ec, c->mt.split, u, c->d, c->eact,
                           c->nflag, true, R, c->rs));
  PF_TRY(read_scal(c));
  *norm = std::sqrt(c->scal_h[SC_NORM_A]);
  if (!is_finite(*norm)) return fail(c, PF_E_NONFINITE, "displacement residual is not finite");
  return PF_OK;
}

// Inexact Newton for the mixed path: an FP32 inner solve only has to bring
// the FP64 residual ||R|| down to the Newton target tol, so it is asked for a
// relative reduction of kForcing * tol / ||R||, no tighter than tol_inner
// (what FP32 CG resolves) and no looser than kForcingMax.  A step that
// starts near the target then costs a short solve instead of a full one.
// With the split's piecewise-linear stress a Newton step inside one active
// set is exact up to the linear solve, so the step lands about a factor
// kForcing below the target: a margin for the FP32 solve's rounding, and
// room for the staggered iteration, which carries the displacement's
// remaining error into the next phase solve (a missed target costs one
// more short step).
constexpr double kForcing = 0.1;
constexpr double kForcingMax = 0.1;

inline double inner_tolerance(double tol_inner, double target, double nr) {
  return std::min(kForcingMax, std::max(tol_inner, kForcing * target / nr));
}

// ---- starting guesses of the displacement solves
//
// Consecutive displacement solves of a load history have nearly the same
// operator, and their solutions (the response to a load increment, to the
// change of d in one staggered iteration) point in nearly the same
// directions.  A solve whose relative tolerance is below kGuessTol starts
// from x0 = V c, the Galerkin projection of its right-hand side b onto the
// span of the last stored solutions V with the current operator K:
// (V' K V) c = V' b, the x0 of least energy error in that span.  Its
// residual b - K V c replaces b, and the solve ends at the same absolute
// target, tol ||b||, as a solve from zero.
constexpr double kGuessTol = 1e-3;

template <class T>
bool guess_applies(const pf_ctx *c, double tol) {
  if (c->opts.guess_vectors <= 0 || tol >= kGuessTol) return false;
  if (c->opts.precond == PF_PC_JACOBI_CHEBYSHEV) return true;
  const bool two = c->opts.cg_kernels == 2 || c->ms.ch == 1 ||
                   (c->opts.cg_kernels == 0 && std::is_same<T, float>::value);
  // FP32 Jacobi solves of a batch member go to the shared launches
  const bool shared = std::is_same<T, float>::value && c->svc && !c->profiling;
  return two && !shared;
}

// Solve G c = g for a symmetric positive semidefinite m x m Gram matrix:
// symmetric Gaussian elimination on the unit-diagonal scaling, where a
// direction whose pivot falls below kGuessPivot (a stored solution nearly in
// the span of the ones before it) is left out (c_j = 0).
constexpr double kGuessPivot = 1e-10;
void guess_solve(int m, const double *G, const double *g, double *cout) {
  double sc[kGuessMax], A[kGuessMax][kGuessMax], y[kGuessMax];
  bool use[kGuessMax];
  for (int i = 0; i < m; ++i) {
    use[i] = G[i * m + i] > 0.0 && std::isfinite(G[i * m + i]);
    sc[i] = use[i] ? 1.0 / std::sqrt(G[i * m + i]) : 0.0;
  }
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) A[i][j] = sc[i] * sc[j] * G[i * m + j];
    y[i] = sc[i] * g[i];
  }
  for (int k = 0; k < m; ++k) {
    if (!use[k] || !(A[k][k] > kGuessPivot)) {
      use[k] = false;
      continue;
    }
    for (int i = k + 1; i < m; ++i) {
      if (!use[i]) continue;
      const double f = A[i][k] / A[k][k];
      for (int j = k; j < m; ++j) A[i][j] -= f * A[k][j];
      y[i] -= f * y[k];
    }
  }
  for (int k = m - 1; k >= 0; --k) {
    double v = 0.0;
    if (use[k]) {
      v = y[k];
      for (int j = k + 1; j < m; ++j) v -= A[k][j] * y[j];
      v /= A[k][k];
    }
    y[k] = v;   // the scaled solution, back-substituted in place
  }
  for (int i = 0; i < m; ++i) cout[i] = std::isfinite(y[i]) ? sc[i] * y[i] : 0.0;
}

// x0 into X[0] and its residual into R[0] (which holds b); *start tells
// the CG about it.
template <class T>
pf_status guess_start(pf_ctx *c, double tol, CgStart *start) {
  CgBuf<T> &b = buf<T>(c);
  const int m = c->guess_m;
  GuessArgs<T> a{};
  a.m = m;
  a.n = 2 * c->g.N;
  for (int j = 0; j < m; ++j) {
    PF_HIP(c, tangent_apply_masked<T>(c->stream, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d,
                                      c->tflag, c->eact, c->nflag, b.gv[j], b.gw[j]));
    a.v[j] = b.gv[j];
    a.w[j] = b.gw[j];
  }
  PF_HIP(c, guess_dots<T>(c->stream, a, b.R[0], c->guess_part, c->guess_out));
  PF_HIP(c, hipMemcpyAsync(c->guess_h, c->guess_out, kGuessDots * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  PF_TRY(sync(c));
  // the sums come in the order v_j . w_k (j <= k, row by row of the
  // kGuessMax x kGuessMax triangle), v_j . b, b . b
  double G[kGuessMax * kGuessMax], gb[kGuessMax];
  int k = 0;
  for (int j = 0; j < kGuessMax; ++j)
    for (int l = j; l < kGuessMax; ++l, ++k)
      if (j < m && l < m) G[j * m + l] = G[l * m + j] = c->guess_h[k];
  for (int j = 0; j < kGuessMax; ++j, ++k)
    if (j < m) gb[j] = c->guess_h[k];
  const double bb = c->guess_h[k];
  if (!(bb > 0.0) || !std::isfinite(bb)) return PF_OK;   // nothing to solve: start from 0
  GuessCoef cf{};
  guess_solve(m, G, gb, cf.c);
  PF_HIP(c, guess_combine<T>(c->stream, a, cf, b.X[0], b.R[0]));
  start->warm = 1;
  start->rr_abs = tol * tol * bb;
  return PF_OK;
}

// Keep the solution of a solve that took the guess path (the ring's oldest
// entry is replaced once it is full).
template <class T>
pf_status guess_store(pf_ctx *c, const T *x) {
  CgBuf<T> &b = buf<T>(c);
  const int cap = c->opts.guess_vectors;
  PF_HIP(c, hipMemcpyAsync(b.gv[c->guess_next], x, 2 * (size_t)c->g.N * sizeof(T),
                           hipMemcpyDeviceToDevice, c->stream));
  c->guess_next = (c->guess_next + 1) % cap;
  if (c->guess_m < cap) ++c->guess_m;
  return PF_OK;
}

template <class T>
pf_status newton_impl(pf_ctx *c, pf_step_stats *st, bool *ok) {
  *ok = true;
  double nr = 0.0;
  PF_TRY(residual_u(c, c->u, c->Ru, &nr));
  const double tol = c->opts.tol_newton * c->R_ref;
  const bool mixed = std::is_same<T, float>::value;
  int it = 0;
  CgBuf<T> &b = buf<T>(c);
  const int n2 = 2 * c->g.N;
  while (nr > tol) {
    if (it >= c->opts.max_newton) {
      *ok = false;
      break;
    }
    PF_HIP(c, tangent_flags(c->stream, c->g, c->u, c->eact, c->tflag));
    if (mixed) {
      PF_HIP(c, convert<float, double>(c->stream, c->g.N, c->bf.d, c->d));
      PF_HIP(c, convert<float, double>(c->stream, n2, c->bf.R[0], c->Ru));
      if (c->mt.split == 1) PF_HIP(c, convert<float, double>(c->stream, n2, c->bf.ulin, c->u));
    } else {
      PF_HIP(c, hipMemcpyAsync(c->bd.R[0], c->Ru, n2 * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    }
    if (!mixed && c->mt.split == 1)   // the Newton point, in a buffer whose address captured
                                     // graphs can keep (u is swapped by the line search)
      PF_HIP(c, hipMemcpyAsync(c->bd.ulin, c->u, n2 * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    PF_HIP(c, tangent_diag<T>(c->stream, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d, c->tflag,
                              c->eact, c->nflag, b.Dinv));
    int iters = 0, status = 0;
    T *xs = nullptr;
    const double tol_lin =
        mixed ? inner_tolerance(c->opts.tol_inner, tol, nr) : c->opts.tol_pcg;
    const bool guess = guess_applies<T>(c, tol_lin);
    CgStart start;
    if (guess && c->guess_m > 0) PF_TRY(guess_start<T>(c, tol_lin, &start));
    PF_TRY(pcg<T>(c, K_ELASTIC, tol_lin, &iters, &status, &xs, start));
    if (guess && status != 2) PF_TRY(guess_store<T>(c, xs));
    st->n_cg_u += iters;
    st->dof_updates += (double)iters * (double)c->n_free_u;
    if (status == 3) st->cg_not_converged += 1;
    if (status == 2 && iters == 0)
      return fail(c, PF_E_BREAKDOWN, "displacement CG breakdown");
    double alpha = 1.0, nt = 0.0;
    int halv = 0;
    for (;;) {
      PF_HIP(c, axpy_into<T>(c->stream, n2, c->u_try, c->u, alpha, xs));
      PF_TRY(residual_u(c, c->u_try, c->Ru_try, &nt));
      if (nt < nr || halv == 5) break;
      alpha *= 0.5;
      ++halv;
    }
    std::swap(c->u, c->u_try);
    std::swap(c->Ru, c->Ru_try);
    nr = nt;
    ++it;
  }
  st->n_newton += it;
  return PF_OK;
}

pf_status newton(pf_ctx *c, pf_step_stats *st, bool *ok) {
  if (c->opts.precision == PF_MIXED) return newton_impl<float>(c, st, ok);
  return newton_impl<double>(c, st, ok);
}

// ------------------------------------------------------------- phase

pf_status phase_res(pf_ctx *c, const double *Hs, bool neg, double *nR, double *nb) {
  PF_HIP(c, phase_residual(c->stream, c->g, c->ms, c->pc, Hs, c->d, c->eact, c->nflag, neg,
                           c->Rd, c->rs));
  PF_TRY(read_scal(c));
  *nR = std::sqrt(c->scal_h[SC_NORM_A]);
  *nb = std::sqrt(c->scal_h[SC_NORM_B]);
  if (!is_finite(*nR) || !is_finite(*nb)) return fail(c, PF_E_NONFINITE, "phase residual is not finite");
  return PF_OK;
}

pf_status phase_res_at1(pf_ctx *c, const double *psi, bool neg, double *nR, double *nb) {
  PF_HIP(c, phase_residual_at1(c->stream, c->g, c->ms, c->pc, psi, c->d, c->d_prev, c->gamma,
                               c->eact, c->nflag, neg, c->Rd, c->rs));
  PF_TRY(read_scal(c));
  *nR = std::sqrt(c->scal_h[SC_NORM_A]);
  *nb = std::sqrt(c->scal_h[SC_NORM_B]);
  if (!is_finite(*nR) || !is_finite(*nb)) return fail(c, PF_E_NONFINITE, "phase residual is not finite");
  return PF_OK;
}

// AT1 with the penalty: F_d(d; psi) = 0 by semismooth Newton in FP64.  Each
// step solves J delta = -F_d with J's mass coefficient 2 psi + gamma chi for
// the active points chi of the current d.  F_d is linear for a fixed active
// set, so with exact solves the iteration could end when a step leaves chi
// unchanged.  The CG solves are exact only to tol_pcg of the step's own
// residual, and points that sit at the kink (d_q = d_{n-1,q} in the exact
// solution) then keep flipping in and out of chi at that error level, so
// the iteration ends on the residual instead: ||F_d|| within tol_pcg of the
// solve's starting residual (or kRefineFloor of ||b||).  A solve that starts
// from an already converged d (a later staggered iteration) can ask for less
// than the rounding floor of F_d, whose terms are of order Gc/(c_w l) while
// ||b|| and the start residual may be orders smaller; so once the active set
// has stopped changing and a step whose CG solve converged no longer shrinks
// ||F_d|| by kRefineStall, the residual is at that floor and the solve ends
// (with an unchanged active set F_d is linear, and a converged solve would
// otherwise cut it by about tol_pcg).  A CG solve that stopped at max_cg
// proves nothing about the floor, so after one the loop goes on.  The first step takes
// points at the kink (d_q = d_{n-1,q}, which is everywhere d has not moved
// since the last commit) as active: the penalty's stiffness then bounds that
// step, where the other choice would solve a nearly singular Laplacian
// wherever Psi+ vanishes and overshoot by orders of magnitude.
constexpr int kAt1MaxNewton = 60;
pf_status phase_solve_at1(pf_ctx *c, const double *psi, pf_step_stats *st) {
  CgBuf<double> &b = c->bd;
  const int n = c->g.N;
  double nR0 = 0.0, nR_prev = 0.0;
  int last_status = 0;
  for (int it = 0;; ++it) {
    PF_TRY(zero_icount(c));
    PF_HIP(c, at1_coef(c->stream, c->g, c->gamma, psi, c->d, c->d_prev, c->eact, b.coef, c->chi,
                       it == 0 ? 1 : 0, c->rs));
    double nR = 0.0, nb = 0.0;
    PF_TRY(phase_res_at1(c, psi, true, &nR, &nb));   // also reads icount (chi changes)
    if (it == 0) nR0 = nR;
    const double target = std::max(c->opts.tol_pcg * nR0, kRefineFloor * nb);
    if (it > 0 && nR <= target) break;
    if (it > 0 && c->icount_h[IC_CHI] == 0 && last_status == 1 && nR > kRefineStall * nR_prev)
      break;
    if (nR == 0.0) break;
    if (it >= kAt1MaxNewton)
      return fail(c, PF_E_NOT_CONVERGED, "AT1 phase solve: active set did not settle");
    PF_HIP(c, phase_diag<double>(c->stream, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag,
                                 b.Dinv));
    PF_HIP(c, hipMemcpyAsync(b.R[0], c->Rd, n * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    int iters = 0, status = 0;
    double *xs = nullptr;
    PF_TRY(pcg<double>(c, K_PHASE, c->opts.tol_pcg, &iters, &status, &xs));
    last_status = status;
    st->n_cg_d += iters;
    st->dof_updates += (double)iters * (double)c->n_free_d;
    if (status == 3) st->cg_not_converged += 1;
    if (status == 2) return fail(c, PF_E_BREAKDOWN, "AT1 phase CG breakdown");
    PF_HIP(c, axpy_into<double>(c->stream, n, c->d, c->d, 1.0, xs));
    nR_prev = nR;
  }
  st->n_dsolve += 1;
  return PF_OK;
}

// Evolution solve K_dd(Hs) d = b(Hs): correction solves d += delta with
// delta from PCG on the residual; FP64: one solve, mixed: refinement until
// ||R_d|| <= tol_pcg ||R_d(start)||.
template <class T>
pf_status phase_solve_impl(pf_ctx *c, const double *Hs, pf_step_stats *st) {
  const bool mixed = std::is_same<T, float>::value;
  CgBuf<T> &b = buf<T>(c);
  const int n = c->g.N;
  PF_HIP(c, at2_coef<T>(c->stream, c->g, c->mt, Hs, c->eact, b.coef));
  PF_HIP(c, phase_diag<T>(c->stream, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag, b.Dinv));
  double nR0 = 0.0, nb = 0.0;
  PF_TRY(phase_res(c, Hs, true, &nR0, &nb));
  double nR = nR0, nR_prev = 0.0;
  const int max_refine = mixed ? 30 : 1;
  // refinement target: tol_pcg relative to the initial residual, but not
  // below what an FP64 residual of this system can resolve (kRefineFloor of
  // ||b||); passes that stop reducing the residual end the loop too
  const double target = std::max(c->opts.tol_pcg * nR0, kRefineFloor * nb);
  for (int k = 0; k < max_refine; ++k) {
    if (nR == 0.0) break;
    if (mixed && k > 0 && (nR <= target || nR > kRefineStall * nR_prev)) break;
    nR_prev = nR;
    if (mixed) {
      PF_HIP(c, convert<float, double>(c->stream, n, c->bf.R[0], c->Rd));
    } else {
      PF_HIP(c, hipMemcpyAsync(c->bd.R[0], c->Rd, n * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    }
    int iters = 0, status = 0;
    T *xs = nullptr;
    PF_TRY(pcg<T>(c, K_PHASE, mixed ? c->opts.tol_inner : c->opts.tol_pcg, &iters, &status, &xs));
    st->n_cg_d += iters;
    st->dof_updates += (double)iters * (double)c->n_free_d;
    if (status == 3) st->cg_not_converged += 1;
    PF_HIP(c, axpy_into<T>(c->stream, n, c->d, c->d, 1.0, xs));
    if (mixed) PF_TRY(phase_res(c, Hs, true, &nR, &nb));
  }
  st->n_dsolve += 1;
  return PF_OK;
}

pf_status phase_solve(pf_ctx *c, const double *Hs, pf_step_stats *st) {
  if (c->at1) return phase_solve_at1(c, Hs, st);
  if (c->opts.precision == PF_MIXED) return phase_solve_impl<float>(c, Hs, st);
  return phase_solve_impl<double>(c, Hs, st);
}

// MINRES on the phase block held in bd.coef / bd.Dinv (M = |diag|) with
// right-hand side c->Rd; the increment ends in bd.X[0].
pf_status minres_phase(pf_ctx *c, double tol, int *iters, int *status, double **xout) {
  CgBuf<double> &b = c->bd;
  const int n = c->g.N;
  // the kernels march in columns; LDS tiles fall back to 2-row marching
  const March m = c->ms.ch == 1 ? march_shape(c->g, 2) : c->ms;
  const MrVecs v{b.X[0], {b.W[0], b.W[1]}, {b.P[0], b.P[1]}, {b.R[0], b.R[1]}, b.S[0], b.Dinv};
  const MrArgs a{c->mrs, c->rs.partR, c->rs.partR + 2 * kPMax, cg1_blocks(m),
                 vec_block_count(n), tol, c->opts.max_cg};
  PF_HIP(c, mr_init(c->stream, n, c->Rd, v, a));
  const int batch = std::max(4, c->opts.cg_check);
  for (int j = 1;;) {
    for (int k = 0; k < batch; ++k, ++j) {
      PF_HIP(c, phase_mr_apply(c->stream, c->g, m, c->pc, b.coef, c->eact, c->nflag, v, a, j));
      PF_HIP(c, mr_update(c->stream, n, v, a, j));
    }
    PF_HIP(c, hipMemcpyAsync(c->mrs_h, c->mrs, sizeof(MrState), hipMemcpyDeviceToHost, c->stream));
    PF_TRY(sync(c));
    const MrHalf &h = c->mrs_h->b;
    if (h.done != 0) {
      *iters = h.iters;
      *status = h.done;
      *xout = b.X[0];
      return PF_OK;
    }
  }
}

// Trial increment with the augmented block K_dd + K~ (Section 3.4), then
// either the predictor (Sections 3.3, 3.5), which writes Hhat, or, for the
// trial-only update, d += increment.  The floored block is SPD and solved by
// PCG; the unfloored one may be indefinite and is solved by MINRES in FP64.
template <class T>
pf_status trial_impl(pf_ctx *c, pf_step_stats *st) {
  CgBuf<T> &b = buf<T>(c);
  const bool mixed = std::is_same<T, float>::value;
  const bool literal = c->opts.trial_operator == PF_TRIAL_UNFLOORED;
  const int n = c->g.N;
  // MINRES and AT1 run in FP64 only; trial() never sends them here
  if (mixed && (literal || c->at1)) return fail(c, PF_E_STATE, "this trial needs the FP64 path");
  // AT2: the history field drives the evolution equation; AT1: Psi+ itself
  const double *drive = c->at1 ? c->psi_p : c->H;
  PF_TRY(zero_icount(c));
  const T *cbase = nullptr;
  if constexpr (std::is_same<T, double>::value) {
    if (c->at1) {
      // the semismooth Newton matrix at d^k is the block's base
      PF_HIP(c, at1_coef(c->stream, c->g, c->gamma, c->psi_p, c->d, c->d_prev, c->eact, b.coef,
                         c->chi, 0, c->rs));
      cbase = b.coef;
    }
  }
  PF_HIP(c, trial_coef<T>(c->stream, c->g, c->mt, c->opts.trial_floor, literal ? 0 : 1, c->H,
                          c->psi_s, c->qflag, c->d, c->eact, cbase, b.coef, c->rs));
  PF_HIP(c, phase_diag<T>(c->stream, c->g, c->ms, c->pc, b.coef, c->eact, c->nflag, b.Dinv,
                          literal ? 1 : 0));
  double nR = 0.0, nb = 0.0;
  if (c->at1) {
    PF_TRY(phase_res_at1(c, drive, true, &nR, &nb));   // also reads icount (floor hits)
  } else {
    PF_TRY(phase_res(c, c->H, true, &nR, &nb));
  }
  st->floor_hits += (int64_t)c->icount_h[IC_FLOOR];
  int iters = 0, status = 0;
  T *xs = nullptr;
  if constexpr (std::is_same<T, double>::value) {
    if (literal) PF_TRY(minres_phase(c, c->opts.tol_pcg, &iters, &status, &xs));
  }
  if (!literal) {
    if (mixed) {
      PF_HIP(c, convert<float, double>(c->stream, n, c->bf.R[0], c->Rd));
    } else {
      PF_HIP(c, hipMemcpyAsync(c->bd.R[0], c->Rd, n * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    }
    PF_TRY(pcg<T>(c, K_PHASE, mixed ? c->opts.tol_inner : c->opts.tol_pcg, &iters, &status, &xs));
  }
  st->n_cg_trial += iters;
  st->dof_updates += (double)iters * (double)c->n_free_d;
  if (status == 3) st->cg_not_converged += 1;
  if (status == 2) return fail(c, PF_E_BREAKDOWN, literal ? "trial MINRES breakdown" : "trial CG breakdown");
  if (c->opts.trial_update == PF_TRIAL_ONLY) {
    PF_HIP(c, axpy_into<T>(c->stream, n, c->d, c->d, 1.0, xs));
  } else {
    PF_HIP(c, predictor<T>(c->stream, c->g, c->mt, c->d, xs, drive, c->psi_s, c->qflag,
                           c->eact, c->Hhat));
  }
  st->n_trial += 1;
  return PF_OK;
}

// The FP32 trial serves only the floored predictor; the trial-only update
// is the phase update itself, and MINRES runs in FP64, so both take the
// FP64 path in either precision.
pf_status trial(pf_ctx *c, pf_step_stats *st) {
  if (c->opts.precision == PF_MIXED && c->opts.trial_operator == PF_TRIAL_FLOORED &&
      c->opts.trial_update == PF_TRIAL_PREDICT_CORRECT && !c->at1)
    return trial_impl<float>(c, st);
  return trial_impl<double>(c, st);
}

// Softening threshold of the gate: the option, or Psi_crit = Gc / (c_w l)
// with c_w = 2 (AT2) or 8/3 (AT1).
double psi_crit_of(const pf_ctx *c) {
  if (c->opts.psi_crit >= 0) return c->opts.psi_crit;
  const double cw = c->at1 ? kAt1Cw : 2.0;
  return c->mt.Gc / (cw * c->mt.l);
}

// QP update from the current (u, d) and the staggered residual.
pf_status qp_and_residual(pf_ctx *c, double *r) {
  PF_TRY(zero_icount(c));
  QpParams qp{c->opts.scheme, psi_crit_of(c), c->opts.d_gate};
  PF_HIP(c, qp_update(c->stream, c->g, c->mt, qp, c->u, c->d, c->eact, c->H_prev, c->H, c->psi_s,
                      c->qflag, c->at1 ? c->psi_p : nullptr, c->rs));
  double nR = 0.0, nb = 0.0;
  if (c->at1) {
    PF_TRY(phase_res_at1(c, c->psi_p, false, &nR, &nb));   // reads icount too
  } else {
    PF_TRY(phase_res(c, c->H, false, &nR, &nb));
  }
  c->gated_last = (int64_t)c->icount_h[IC_GATED];
  *r = (nb > 0.0) ? nR / nb : nR;
  return PF_OK;
}

pf_status reaction(pf_ctx *c, int group, double f[2]) {
  Group &gr = c->groups[group];
  if (gr.n == 0) {
    f[0] = f[1] = 0.0;
    return PF_OK;
  }
  PF_HIP(c, internal_force(c->stream, c->g, c->ms, c->ec, c->mt.split, c->u, c->d, c->eact,
                           nullptr, false, c->Rfull, c->rs));
  PF_HIP(c, group_sum(c->stream, gr.n, gr.d_dof, gr.d_comp, c->Rfull, c->rs));
  PF_TRY(read_scal(c));
  f[0] = c->scal_h[SC_SUM_X];
  f[1] = c->scal_h[SC_SUM_Y];
  return PF_OK;
}

int load_group_of(pf_ctx *c) {
  // the loaded group is group 1 by convention (group 0 = support)
  return c->groups[1].n > 0 ? 1 : 0;
}

pf_status open_step(pf_ctx *c, double lam) {
  c->acc = pf_step_stats{};
  c->acc.converged = 1;
  c->t_open = std::chrono::steady_clock::now();
  const int n2 = 2 * c->g.N;
  PF_HIP(c, lift_dirichlet(c->stream, n2, c->nflag, NF_UX | (NF_UY << 4), c->g.N, c->u_unit, lam,
                           c->u));
  PF_HIP(c, lift_dirichlet(c->stream, c->g.N, c->nflag, NF_D | (NF_D << 4), c->g.N, c->d_fix, 1.0,
                           c->d));
  if (c->at1)
    PF_HIP(c, lift_dirichlet(c->stream, c->g.N, c->nflag, NF_D | (NF_D << 4), c->g.N, c->d_fix,
                             1.0, c->d_prev));
  double R0 = 0.0;
  PF_TRY(residual_u(c, c->u, c->Ru, &R0));
  c->R_ref = R0 > 0.0 ? R0 : 1.0;
  c->step_open = true;
  c->step_load = lam;
  bool ok = true;
  const auto t_u = std::chrono::steady_clock::now();
  PF_TRY(newton(c, &c->acc, &ok));   // ends on a synchronising residual read
  c->acc.time_u_ms +=
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_u).count();
  c->acc.n_stag = 1;
  if (!ok) c->acc.converged = 0;
  double r = 0.0;
  PF_TRY(qp_and_residual(c, &r));
  c->acc.r_stag = r;
  return PF_OK;
}

pf_status iterate_once(pf_ctx *c) {
  const double *Hs = c->at1 ? c->psi_p : c->H;
  bool updated = false;
  // wall time of the phase part (trial, predictor, evolution solve) and of
  // the displacement solve, split at a stream synchronisation
  const auto t_d = std::chrono::steady_clock::now();
  if (c->opts.scheme != PF_ST) {
    c->acc.gated_max = std::max<int64_t>(c->acc.gated_max, c->gated_last);
    if (c->gated_last > 0) {
      PF_TRY(trial(c, &c->acc));
      // trial-only: d already holds d + increment
      if (c->opts.trial_update == PF_TRIAL_ONLY) updated = true;
      else Hs = c->Hhat;
    }
  }
  if (!updated) PF_TRY(phase_solve(c, Hs, &c->acc));
  PF_TRY(sync(c));
  const auto t_u = std::chrono::steady_clock::now();
  bool ok = true;
  PF_TRY(newton(c, &c->acc, &ok));   // ends on a synchronising residual read
  const auto t_e = std::chrono::steady_clock::now();
  c->acc.time_d_ms += std::chrono::duration<double, std::milli>(t_u - t_d).count();
  c->acc.time_u_ms += std::chrono::duration<double, std::milli>(t_e - t_u).count();
  if (!ok) c->acc.converged = 0;
  c->acc.n_stag += 1;
  double r = 0.0;
  PF_TRY(qp_and_residual(c, &r));
  c->acc.r_stag = r;
  return PF_OK;
}

void finish_stats(pf_ctx *c, pf_step_stats *st) {
  auto t = std::chrono::steady_clock::now();
  c->acc.time_ms = std::chrono::duration<double, std::milli>(t - c->t_open).count();
  if (st) *st = c->acc;
}

pf_status commit(pf_ctx *c) {
  std::swap(c->H_prev, c->H);
  if (c->at1)
    PF_HIP(c, hipMemcpyAsync(c->d_prev, c->d, c->g.N * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
  c->step_open = false;
  double f[2];
  PF_TRY(reaction(c, load_group_of(c), f));
  c->acc.force[0] = f[0];
  c->acc.force[1] = f[1];
  return PF_OK;
}

pf_status check_opts(const pf_solver_opts *o, std::string *msg) {
  if (o->scheme < 0 || o->scheme > 3) {
    *msg = "scheme";
    return PF_E_INVALID_ARG;
  }
  if (o->precision < 0 || o->precision > 1) {
    *msg = "precision";
    return PF_E_INVALID_ARG;
  }
  if (o->precond != PF_PC_JACOBI && o->precond != PF_PC_JACOBI_CHEBYSHEV) {
    *msg = "precond";
    return PF_E_INVALID_ARG;
  }
  if (o->precond == PF_PC_JACOBI_CHEBYSHEV && (o->cheb_degree < 1 || o->cheb_degree > 16)) {
    *msg = "cheb_degree must be in 1..16";
    return PF_E_INVALID_ARG;
  }
  if (!(o->tol_stag > 0) || !(o->tol_pcg > 0) || !(o->tol_newton > 0) || !(o->tol_inner > 0)) {
    *msg = "tolerances must be > 0";
    return PF_E_INVALID_ARG;
  }
  if (o->max_stag < 1 || o->max_newton < 1 || o->max_cg < 1) {
    *msg = "iteration limits";
    return PF_E_INVALID_ARG;
  }
  if (!(o->trial_floor > 0) || o->trial_floor > 1) {
    *msg = "trial_floor must be in (0,1]";
    return PF_E_INVALID_ARG;
  }
  if (!(o->cheb_ratio >= 0) || (o->cheb_ratio > 0 && o->cheb_ratio <= 1)) {
    *msg = "cheb_ratio must be 0 or > 1";
    return PF_E_INVALID_ARG;
  }
  if (o->phase_model < 0 || o->phase_model > 1 ||
      (o->phase_model == PF_AT1_PENALTY && !(o->tol_ir > 0))) {
    *msg = "phase_model must be 0 or 1, with tol_ir > 0 for AT1";
    return PF_E_INVALID_ARG;
  }
  if (o->trial_operator < 0 || o->trial_operator > 1 || o->trial_update < 0 ||
      o->trial_update > 1) {
    *msg = "trial_operator and trial_update must be 0 or 1";
    return PF_E_INVALID_ARG;
  }
  if (o->guess_vectors < 0 || o->guess_vectors > kGuessMax) {
    *msg = "guess_vectors must be in 0..4";
    return PF_E_INVALID_ARG;
  }
  if (o->cg_kernels < 0 || o->cg_kernels > 2) {
    *msg = "cg_kernels must be 0, 1 or 2";
    return PF_E_INVALID_ARG;
  }
  if (o->march_rows < 0 || o->march_rows > 8 || (o->march_rows > 2 && o->march_rows != 4 &&
                                                  o->march_rows != 8)) {
    *msg = "march_rows must be 0, 1, 2, 4 or 8";
    return PF_E_INVALID_ARG;
  }
  return PF_OK;
}

}  // namespace

// =================================================================== C ABI

namespace {

// Average time of `reps` launches of the context's two-kernel CG apply
// (idempotent: it rewrites p_new, q and its partials from inputs it does not
// modify) in precision T with the current work decomposition.  u_try holds
// the right-hand side's source state (see pf_autotune).
template <class T>
pf_status time_cg_apply(pf_ctx *c, int reps, float *ms) {
  CgBuf<T> &b = buf<T>(c);
  const int n2 = 2 * c->g.N;
  if (std::is_same<T, float>::value) {
    PF_HIP(c, convert<float, double>(c->stream, c->g.N, c->bf.d, c->d));
    PF_HIP(c, convert<float, double>(c->stream, n2, c->bf.R[0], c->Ru));
    if (c->mt.split == 1) PF_HIP(c, convert<float, double>(c->stream, n2, c->bf.ulin, c->u));
  } else {
    PF_HIP(c, hipMemcpyAsync(c->bd.R[0], c->Ru, n2 * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    if (c->mt.split == 1)
      PF_HIP(c, hipMemcpyAsync(c->bd.ulin, c->u, n2 * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
  }
  PF_HIP(c, tangent_diag<T>(c->stream, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d, c->tflag,
                            c->eact, c->nflag, b.Dinv));
  CgArgs ca = cg_args(c->g, c->ms, n2, c->cgs2, c->rs, 0.0, 1 << 30);
  PF_HIP(c, cg_init<T>(c->stream, n2, b.X[0], b.R[0], b.W[0], b.P[0], b.Dinv, ca));
  auto apply = [&]() {
    return tangent_cg_apply<T>(c->stream, c->g, c->ms, c->ec, c->mt.split, b.ulin, b.d, c->tflag,
                               c->eact, c->nflag, b.W[0], b.P[0], b.P[1], b.S[0], ca);
  };
  PF_HIP(c, apply());   // warm
  PF_HIP(c, hipEventRecord(c->ev[0], c->stream));
  for (int r = 0; r < reps; ++r) PF_HIP(c, apply());
  PF_HIP(c, hipEventRecord(c->ev[1], c->stream));
  PF_TRY(sync(c));
  PF_HIP(c, hipEventElapsedTime(ms, c->ev[0], c->ev[1]));
  return PF_OK;
}

}  // namespace

extern "C" {

void pf_default_opts(pf_solver_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->scheme = PF_ST;
  o->precision = PF_FP64;
  o->precond = PF_PC_JACOBI;
  o->cheb_degree = 3;
  o->tol_stag = 1e-5;
  o->tol_pcg = 1e-10;
  o->tol_newton = 1e-9;
  o->tol_inner = 1e-5;
  o->max_stag = 500;
  o->max_newton = 25;
  o->max_cg = 200000;
  o->cg_check = 32;
  o->psi_crit = -1.0;
  o->d_gate = 0.95;
  o->trial_floor = 0.1;
  o->tol_ir = 0.01;
}

const char *pf_status_string(pf_status s) {
  switch (s) {
    case PF_OK: return "ok";
    case PF_E_INVALID_ARG: return "invalid argument";
    case PF_E_OOM: return "out of device memory";
    case PF_E_HIP: return "HIP runtime error";
    case PF_E_STATE: return "invalid state";
    case PF_E_NOT_CONVERGED: return "not converged";
    case PF_E_BREAKDOWN: return "CG breakdown";
    case PF_E_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

const char *pf_last_error(const pf_ctx *c) { return c ? c->err.c_str() : "null context"; }

pf_status pf_create(const pf_mesh_desc *mesh, const pf_material *mat, const pf_solver_opts *opts,
                    void *hip_stream, pf_ctx **out) {
  if (!mesh || !mat || !out) return PF_E_INVALID_ARG;
  *out = nullptr;
  if (mesh->nx < 1 || mesh->ny < 1 || !(mesh->lx > 0) || !(mesh->ly > 0)) return PF_E_INVALID_ARG;
  // the kernels index displacement DOFs (2N) and quadrature points (4E) with
  // 32-bit ints, and round those counts up to whole blocks
  // (each side is below 2^31, so N < 2^62 fits; compare without multiplying)
  const long long N = ((long long)mesh->nx + 1) * ((long long)mesh->ny + 1);
  const long long E = (long long)mesh->nx * mesh->ny;
  if (N > kMaxIndexCount / 2 || E > kMaxIndexCount / 4) return PF_E_INVALID_ARG;
  if (!(mat->E > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->Gc > 0) || !(mat->l > 0) ||
      !(mat->eta >= 0) || (mat->split != PF_SPLIT_VD && mat->split != PF_SPLIT_SPECTRAL))
    return PF_E_INVALID_ARG;
  pf_solver_opts o;
  if (opts) o = *opts; else pf_default_opts(&o);
  std::string msg;
  if (check_opts(&o, &msg) != PF_OK) return PF_E_INVALID_ARG;

  pf_ctx *c = new pf_ctx();
  c->opts = o;
  c->stream = static_cast<hipStream_t>(hip_stream);
  (void)hipGetDevice(&c->device);
  Grid &g = c->g;
  g.nx = mesh->nx; g.ny = mesh->ny;
  g.N = (int)N; g.E = mesh->nx * mesh->ny;
  g.hx = mesh->lx / mesh->nx; g.hy = mesh->ly / mesh->ny;
  Mat &mt = c->mt;
  mt.mu = mat->E / (2.0 * (1.0 + mat->nu));
  mt.lam = mat->E * mat->nu / ((1.0 + mat->nu) * (1.0 - 2.0 * mat->nu));
  mt.K = mt.lam + 2.0 * mt.mu / 3.0;
  mt.Gc = mat->Gc; mt.l = mat->l; mt.eta = mat->eta; mt.split = mat->split;
  c->ec = ElasCoef{2.0 * mt.mu, mt.K, mt.lam, mt.mu, mt.eta, 1.0 / g.hx, 1.0 / g.hy,
                   g.hy / 4.0, g.hx / 4.0};
  c->pc = PhaseCoef{mt.Gc * mt.l, mt.Gc / mt.l, g.hx * g.hy / 4.0, 1.0 / g.hx, 1.0 / g.hy,
                    g.hy / 4.0, g.hx / 4.0};
  c->at1 = o.phase_model == PF_AT1_PENALTY;
  if (c->at1) {
    // F_d with w = d: Laplacian factor 2 Gc l / c_w, source Gc / (c_w l)
    c->pc.Gcl = 2.0 * mt.Gc * mt.l / kAt1Cw;
    c->pc.Gc_l = mt.Gc / (kAt1Cw * mt.l);
    c->gamma = 27.0 * mt.Gc / (64.0 * mt.l * o.tol_ir * o.tol_ir);
  }
  c->ms = march_shape(g, o.march_rows);
  // the spectral tangent's 8-row marching item does not fit the register
  // file (it spills); its default is at most 4 rows
  if (o.march_rows == 0 && mat->split == PF_SPLIT_SPECTRAL && c->ms.ch == 8)
    c->ms = march_shape(g, 4);

  pf_status s = PF_OK;
  auto A = [&](auto **p, size_t n) {
    if (s == PF_OK) s = dalloc(c, p, n);
  };
  const size_t n2 = 2 * (size_t)g.N, E4 = 4 * (size_t)g.E;
  A(&c->u, n2); A(&c->u_try, n2); A(&c->d, g.N);
  A(&c->H_prev, E4); A(&c->H, E4); A(&c->Hhat, E4); A(&c->psi_s, E4);
  A(&c->Ru, n2); A(&c->Ru_try, n2); A(&c->Rd, g.N); A(&c->Rfull, n2);
  A(&c->u_unit, n2); A(&c->d_fix, g.N);
  A(&c->nflag, g.N); A(&c->qflag, g.E); A(&c->tflag, g.E);
  for (int k = 0; k < 2; ++k) {
    A(&c->bd.R[k], n2); A(&c->bd.W[k], n2); A(&c->bd.S[k], n2); A(&c->bd.X[k], n2);
    A(&c->bd.P[k], n2);
  }
  A(&c->bd.Dinv, n2); A(&c->bd.coef, E4); A(&c->bd.zc, n2); A(&c->bd.rc, n2); A(&c->bd.dc, n2);
  A(&c->bd.pv[0], n2); A(&c->bd.pv[1], n2);
  if (mat->split == PF_SPLIT_SPECTRAL) A(&c->bd.ulin, n2);
  c->bd.d = c->d;
  if (o.precision == PF_MIXED) {
    for (int k = 0; k < 2; ++k) {
      A(&c->bf.R[k], n2); A(&c->bf.W[k], n2); A(&c->bf.S[k], n2); A(&c->bf.X[k], n2);
      A(&c->bf.P[k], n2);
    }
    A(&c->bf.Dinv, n2); A(&c->bf.coef, E4); A(&c->bf.d, g.N); A(&c->bf.zc, n2); A(&c->bf.rc, n2); A(&c->bf.dc, n2);
    A(&c->bf.pv[0], n2); A(&c->bf.pv[1], n2);
    if (mat->split == PF_SPLIT_SPECTRAL) A(&c->bf.ulin, n2);
  }
  if (o.guess_vectors > 0) {
    for (int j = 0; j < o.guess_vectors; ++j) {
      if (o.precision == PF_MIXED) {
        A(&c->bf.gv[j], n2); A(&c->bf.gw[j], n2);
      } else {
        A(&c->bd.gv[j], n2); A(&c->bd.gw[j], n2);
      }
    }
    A(&c->guess_part, kGuessDots * (size_t)kPMax);
    A(&c->guess_out, kGuessDots);
  }
  A(&c->cheb_dev, 4 * (size_t)kChebCoefs);
  A(&c->mrs, 1);
  if (c->at1) {
    A(&c->psi_p, E4);
    A(&c->d_prev, g.N);
    A(&c->chi, E4);
  }
  A(&c->cgs, 2);
  A(&c->cgs2, 1);
  A(&c->cgpart, 6 * (size_t)kPMax);
  A(&c->rs.partR, 4 * (size_t)kPMax);
  A(&c->rs.icount, kICounters);
  A(&c->rs.scal, kScal);
  if (mesh->elem_active) {
    c->eact_h.assign(mesh->elem_active, mesh->elem_active + g.E);
    A(&c->eact, g.E);
    if (s == PF_OK &&
        hipMemcpyAsync(c->eact, c->eact_h.data(), g.E, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      s = PF_E_HIP;
  }
  if (s == PF_OK) {
    if (hipHostMalloc((void **)&c->cgs_h, 2 * sizeof(Cg1State)) != hipSuccess ||
        hipHostMalloc((void **)&c->cgs2_h, 2 * sizeof(CgState)) != hipSuccess ||
        hipEventCreateWithFlags(&c->poll_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->poll_ev[1], hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&c->scal_h, kScal * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&c->icount_h, kICounters * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void **)&c->cheb_h, 4 * kChebCoefs * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&c->mrs_h, sizeof(MrState)) != hipSuccess ||
        hipHostMalloc((void **)&c->guess_h, kGuessDots * sizeof(double)) != hipSuccess)
      s = PF_E_OOM;
  }
  if (s == PF_OK) s = upload_constraints(c);
  if (s != PF_OK) {
    pf_destroy(c);
    return s;
  }
  *out = c;
  return PF_OK;
}

pf_status pf_destroy(pf_ctx *c) {
  if (!c) return PF_OK;
  (void)hipStreamSynchronize(c->stream);
  for (auto &b : c->bufs) raw_free(c->al, *b.field);
  for (auto &gr : c->groups) {
    raw_free(c->al, gr.d_dof);
    raw_free(c->al, gr.d_comp);
  }
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->ready_ev) (void)hipEventDestroy(c->ready_ev);
  for (auto &e : c->poll_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &gr : c->graphs) (void)hipGraphExecDestroy(gr.exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->cgs_h) (void)hipHostFree(c->cgs_h);
  if (c->cgs2_h) (void)hipHostFree(c->cgs2_h);
  if (c->scal_h) (void)hipHostFree(c->scal_h);
  if (c->icount_h) (void)hipHostFree(c->icount_h);
  if (c->cheb_h) (void)hipHostFree(c->cheb_h);
  if (c->mrs_h) (void)hipHostFree(c->mrs_h);
  if (c->guess_h) (void)hipHostFree(c->guess_h);
  delete c;
  return PF_OK;
}

pf_status pf_set_allocator(pf_ctx *c, pf_alloc_fn alloc, pf_release_fn release, void *user) {
  if (!c) return PF_E_INVALID_ARG;
  if ((alloc == nullptr) != (release == nullptr))
    return fail(c, PF_E_INVALID_ARG, "allocator needs both callbacks or neither");
  if (c->step_open) return fail(c, PF_E_STATE, "cannot move buffers inside a step");
  PF_TRY(sync(c));
  // every buffer to move: the registered ones, then the group DOF lists
  std::vector<std::pair<void **, size_t>> moves;
  for (auto &b : c->bufs) moves.push_back({b.field, b.bytes});
  for (auto &gr : c->groups) {
    if (gr.d_dof) moves.push_back({reinterpret_cast<void **>(&gr.d_dof), gr.n * sizeof(int64_t)});
    if (gr.d_comp) moves.push_back({reinterpret_cast<void **>(&gr.d_comp),
                                    (size_t)std::max(gr.n, 16)});
  }
  const Allocator nal{alloc, release, user};
  std::vector<void *> fresh(moves.size(), nullptr);
  for (size_t k = 0; k < moves.size(); ++k) {
    if (raw_alloc(nal, &fresh[k], moves[k].second) != hipSuccess) {
      for (size_t j = 0; j < k; ++j) raw_free(nal, fresh[j]);
      return fail(c, PF_E_OOM, "allocator returned no (or misaligned) memory");
    }
  }
  for (size_t k = 0; k < moves.size(); ++k) {
    hipError_t e = hipMemcpyAsync(fresh[k], *moves[k].first, moves[k].second,
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && k + 1 == moves.size()) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(c->stream);
      for (void *v : fresh) raw_free(nal, v);
      return fail(c, PF_E_HIP, std::string("buffer copy: ") + hipGetErrorString(e));
    }
  }
  // captured graphs hold the old addresses
  for (auto &gr : c->graphs) (void)hipGraphExecDestroy(gr.exec);
  c->graphs.clear();
  for (size_t k = 0; k < moves.size(); ++k) {
    raw_free(c->al, *moves[k].first);
    *moves[k].first = fresh[k];
  }
  c->bd.d = c->d;
  c->al = nal;
  return PF_OK;
}

pf_status pf_set_dirichlet_u(pf_ctx *c, int32_t group, int64_t n, const int64_t *node,
                             const int8_t *comp, const double *val) {
  if (!c) return PF_E_INVALID_ARG;
  if (c->step_open) return fail(c, PF_E_STATE, "cannot change constraints inside a step");
  if (group < 0 || group >= kGroups || n < 0 || (n > 0 && (!node || !comp || !val)))
    return fail(c, PF_E_INVALID_ARG, "bad Dirichlet group arguments");
  Group &gr = c->groups[group];
  for (int64_t k = 0; k < n; ++k) {
    if (node[k] < 0 || node[k] >= c->g.N) return fail(c, PF_E_INVALID_ARG, "node out of range");
    if (comp[k] != 0 && comp[k] != 1) return fail(c, PF_E_INVALID_ARG, "component must be 0 or 1");
    if (!is_finite(val[k])) return fail(c, PF_E_NONFINITE, "non-finite Dirichlet value");
  }
  gr.node.assign(node, node + n);
  gr.comp.assign(comp, comp + n);
  gr.val.assign(val, val + n);
  return upload_constraints(c);
}

pf_status pf_set_dirichlet_d(pf_ctx *c, int64_t n, const int64_t *node, const double *value) {
  if (!c) return PF_E_INVALID_ARG;
  if (c->step_open) return fail(c, PF_E_STATE, "cannot change constraints inside a step");
  if (n < 0 || (n > 0 && (!node || !value))) return fail(c, PF_E_INVALID_ARG, "bad arguments");
  for (int64_t k = 0; k < n; ++k) {
    if (node[k] < 0 || node[k] >= c->g.N) return fail(c, PF_E_INVALID_ARG, "node out of range");
    if (!is_finite(value[k])) return fail(c, PF_E_NONFINITE, "non-finite Dirichlet value");
  }
  c->dnode.assign(node, node + n);
  c->dval.assign(value, value + n);
  PF_TRY(upload_constraints(c));
  // impose on the committed state right away
  PF_HIP(c, lift_dirichlet(c->stream, c->g.N, c->nflag, NF_D | (NF_D << 4), c->g.N, c->d_fix,
                           1.0, c->d));
  return sync(c);
}

pf_status pf_free_dofs(pf_ctx *c, int64_t *nu, int64_t *nd) {
  if (!c) return PF_E_INVALID_ARG;
  if (nu) *nu = c->n_free_u;
  if (nd) *nd = c->n_free_d;
  return PF_OK;
}

pf_status pf_staggered_iterate(pf_ctx *c, double lam, pf_step_stats *st) {
  if (!c) return PF_E_INVALID_ARG;
  if (!is_finite(lam)) return fail(c, PF_E_INVALID_ARG, "non-finite load factor");
  pf_status s;
  if (!c->step_open) {
    s = open_step(c, lam);
  } else {
    if (lam != c->step_load) return fail(c, PF_E_STATE, "load factor differs from the open step");
    s = iterate_once(c);
  }
  finish_stats(c, st);
  return s;
}

pf_status pf_commit_step(pf_ctx *c) {
  if (!c) return PF_E_INVALID_ARG;
  if (!c->step_open) return fail(c, PF_E_STATE, "no open step");
  return commit(c);
}

pf_status pf_load_step(pf_ctx *c, double lam, pf_step_stats *st) {
  if (!c) return PF_E_INVALID_ARG;
  if (c->step_open) return fail(c, PF_E_STATE, "a step is already open");
  if (!is_finite(lam)) return fail(c, PF_E_INVALID_ARG, "non-finite load factor");
  pf_status s = open_step(c, lam);
  if (s != PF_OK) { c->step_open = false; finish_stats(c, st); return s; }
  while (c->acc.r_stag > c->opts.tol_stag && c->acc.n_stag < c->opts.max_stag) {
    s = iterate_once(c);
    if (s != PF_OK) { c->step_open = false; finish_stats(c, st); return s; }
  }
  const bool conv = c->acc.r_stag <= c->opts.tol_stag;
  s = commit(c);
  if (!conv) c->acc.converged = 0;
  finish_stats(c, st);
  if (s != PF_OK) return s;
  return c->acc.converged ? PF_OK : PF_E_NOT_CONVERGED;
}

pf_status pf_reaction_force(pf_ctx *c, int32_t group, double force[2]) {
  if (!c || !force || group < 0 || group >= kGroups) return PF_E_INVALID_ARG;
  return reaction(c, group, force);
}

pf_status pf_get_state(pf_ctx *c, double *u, double *d, double *H) {
  if (!c) return PF_E_INVALID_ARG;
  PF_TRY(sync(c));
  if (u) PF_HIP(c, hipMemcpy(u, c->u, 2 * (size_t)c->g.N * sizeof(double), hipMemcpyDeviceToHost));
  if (d) PF_HIP(c, hipMemcpy(d, c->d, (size_t)c->g.N * sizeof(double), hipMemcpyDeviceToHost));
  if (H) {
    const double *src = c->step_open ? c->H : c->H_prev;
    PF_HIP(c, hipMemcpy(H, src, 4 * (size_t)c->g.E * sizeof(double), hipMemcpyDeviceToHost));
  }
  return PF_OK;
}

pf_status pf_set_state(pf_ctx *c, const double *u, const double *d, const double *H) {
  if (!c) return PF_E_INVALID_ARG;
  if (c->step_open) return fail(c, PF_E_STATE, "cannot set state inside a step");
  const size_t n2 = 2 * (size_t)c->g.N, n = c->g.N, e4 = 4 * (size_t)c->g.E;
  if (u) for (size_t k = 0; k < n2; ++k) if (!is_finite(u[k])) return fail(c, PF_E_NONFINITE, "u has NaN/Inf");
  if (d) for (size_t k = 0; k < n; ++k) if (!is_finite(d[k])) return fail(c, PF_E_NONFINITE, "d has NaN/Inf");
  if (H) for (size_t k = 0; k < e4; ++k) if (!is_finite(H[k])) return fail(c, PF_E_NONFINITE, "H has NaN/Inf");
  PF_TRY(sync(c));
  if (u) PF_HIP(c, hipMemcpy(c->u, u, n2 * sizeof(double), hipMemcpyHostToDevice));
  if (d) PF_HIP(c, hipMemcpy(c->d, d, n * sizeof(double), hipMemcpyHostToDevice));
  if (d && c->at1) PF_HIP(c, hipMemcpy(c->d_prev, d, n * sizeof(double), hipMemcpyHostToDevice));
  if (H) PF_HIP(c, hipMemcpy(c->H_prev, H, e4 * sizeof(double), hipMemcpyHostToDevice));
  return PF_OK;
}

pf_status pf_set_profiling(pf_ctx *c, int32_t enable) {
  if (!c) return PF_E_INVALID_ARG;
  if (enable && !c->ev[0]) {
    for (auto &e : c->ev) PF_HIP(c, hipEventCreate(&e));
  }
  c->profiling = enable != 0;
  c->prof_tick[0] = c->prof_tick[1] = 0;
  for (int k = 0; k < 4; ++k) {
    c->prof_launches[k] = 0;
    c->prof_ms[k] = 0.0;
  }
  return PF_OK;
}

pf_status pf_kernel_time(pf_ctx *c, int32_t kernel, int64_t *launches, double *total_ms,
                         int64_t *nodes_per_launch) {
  if (!c || kernel < 0 || kernel > 3) return PF_E_INVALID_ARG;
  if (launches) *launches = c->prof_launches[kernel];
  if (total_ms) *total_ms = c->prof_ms[kernel];
  if (nodes_per_launch) *nodes_per_launch = c->g.N;
  return PF_OK;
}

// ---------------------------------------------------------------- batch

struct pf_batch {
  std::vector<pf_ctx *> members;
  int workers = 4;
  bool shared = true;
  std::unique_ptr<BatchSvc> svc;
};

pf_status pf_batch_create(int32_t n, pf_ctx *const *members, pf_batch **out) {
  if (!out || n < 1 || !members) return PF_E_INVALID_ARG;
  *out = nullptr;
  std::vector<pf_ctx *> m(members, members + n);
  for (int i = 0; i < n; ++i) {
    if (!m[i]) return PF_E_INVALID_ARG;
    for (int j = 0; j < i; ++j)
      if (m[j] == m[i]) return PF_E_INVALID_ARG;
  }
  pf_batch *b = new pf_batch();
  b->members = std::move(m);
  b->workers = 4;
  *out = b;
  return PF_OK;
}

pf_status pf_batch_set_workers(pf_batch *b, int32_t workers) {
  if (!b || workers < 1) return PF_E_INVALID_ARG;
  b->workers = workers;
  return PF_OK;
}

pf_status pf_batch_set_shared_launches(pf_batch *b, int32_t enable) {
  if (!b) return PF_E_INVALID_ARG;
  b->shared = enable != 0;
  return PF_OK;
}

pf_status pf_batch_load_step(pf_batch *b, const double *lam, pf_step_stats *stats) {
  if (!b || !lam) return PF_E_INVALID_ARG;
  const int n = (int)b->members.size();
  std::vector<pf_status> st(n, PF_OK);
  std::vector<pf_step_stats> ss(n);
  if (b->shared) {
    // one host thread per member; FP32 Jacobi CG solves go to the service
    if (!b->svc) {
      auto svc = std::make_unique<BatchSvc>();
      if (hipStreamCreateWithFlags(&svc->stream, hipStreamNonBlocking) != hipSuccess)
        return PF_E_HIP;
      b->svc = std::move(svc);
    }
    BatchSvc *svc = b->svc.get();
    int check = std::max(4, b->members[0]->opts.cg_check);
    svc->check = check + (check & 1);
    svc->stop = false;
    for (pf_ctx *c : b->members) c->svc = svc;
    std::thread service(service_loop, svc);
    auto work = [&](int i) { st[i] = pf_load_step(b->members[i], lam[i], &ss[i]); };
    std::vector<std::thread> th;
    for (int i = 1; i < n; ++i) th.emplace_back(work, i);
    work(0);
    for (auto &t : th) t.join();
    {
      std::lock_guard<std::mutex> lk(svc->mu);
      svc->stop = true;
    }
    svc->work_cv.notify_all();
    service.join();
    for (pf_ctx *c : b->members) c->svc = nullptr;
  } else {
    std::atomic<int> next(0);
    auto work = [&]() {
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= n) return;
        st[i] = pf_load_step(b->members[i], lam[i], &ss[i]);
      }
    };
    const int nw = std::min(b->workers, n);
    std::vector<std::thread> th;
    for (int w = 1; w < nw; ++w) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
  }
  if (stats)
    for (int i = 0; i < n; ++i) stats[i] = ss[i];
  pf_status worst = PF_OK;
  for (int i = 0; i < n; ++i) {
    if (st[i] != PF_OK && st[i] != PF_E_NOT_CONVERGED) return st[i];
    if (st[i] == PF_E_NOT_CONVERGED) worst = PF_E_NOT_CONVERGED;
  }
  return worst;
}

pf_status pf_batch_destroy(pf_batch *b) {
  delete b;
  return PF_OK;
}

// ------------------------------------------------------------- autotune

pf_status pf_autotune(pf_ctx *c, int32_t reps, int32_t *chosen) {
  if (!c || reps < 1) return PF_E_INVALID_ARG;
  if (c->step_open) return fail(c, PF_E_STATE, "cannot autotune inside a step");
  if (!c->ev[0]) {
    for (auto &e : c->ev) PF_HIP(c, hipEventCreate(&e));
  }
  // operator data for the timed kernel: tangent bits and diagonal at the
  // committed state; right-hand side: the residual after lifting the
  // Dirichlet data to load factor 1 (nonzero, so no kernel exits early)
  const int n2 = 2 * c->g.N;
  PF_HIP(c, hipMemcpyAsync(c->u_try, c->u, n2 * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  PF_HIP(c, lift_dirichlet(c->stream, n2, c->nflag, NF_UX | (NF_UY << 4), c->g.N, c->u_unit, 1.0,
                           c->u_try));
  double nr = 0.0;
  PF_TRY(residual_u(c, c->u_try, c->Ru, &nr));
  PF_HIP(c, tangent_flags(c->stream, c->g, c->u, c->eact, c->tflag));
  const March keep = c->ms;
  float best = 0.f;
  int best_ch = keep.ch;
  // the displacement solves use the single-kernel CG (column marching only)
  // in FP64 with Jacobi unless two kernels are asked for
  const bool fp32 = c->opts.precision == PF_MIXED;
  const bool cg1 = !fp32 && c->opts.precond == PF_PC_JACOBI && c->opts.cg_kernels != 2;
  const std::vector<int> cands = cg1 ? std::vector<int>{2, 4, 8} : std::vector<int>{1, 2, 4, 8};
  for (int ch : cands) {
    c->ms = march_shape(c->g, ch);
    float ms = 0.f;
    if (cg1) {
      if (c->mt.split == 1)
        PF_HIP(c, hipMemcpyAsync(c->bd.ulin, c->u, n2 * sizeof(double), hipMemcpyDeviceToDevice,
                                 c->stream));
      PF_HIP(c, tangent_diag<double>(c->stream, c->g, c->ms, c->ec, c->mt.split, c->bd.ulin,
                                     c->d, c->tflag, c->eact, c->nflag, c->bd.Dinv));
      PF_HIP(c, hipMemcpyAsync(c->bd.R[0], c->Ru, n2 * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
      Cg1Args a;
      a.st = c->cgs;
      a.part = c->cgpart;
      a.np = cg1_blocks(c->ms);
      a.tol2 = 0.0;
      a.maxit = 1 << 30;
      a.parity = 0;
      a.init = 1;
      PF_TRY(launch_k<double>(c, c->stream, K_ELASTIC, a));
      a.init = 0;
      a.parity = 1;
      PF_TRY(launch_k<double>(c, c->stream, K_ELASTIC, a));   // warm
      PF_HIP(c, hipEventRecord(c->ev[0], c->stream));
      for (int r = 0; r < reps; ++r) PF_TRY(launch_k<double>(c, c->stream, K_ELASTIC, a));
      PF_HIP(c, hipEventRecord(c->ev[1], c->stream));
      PF_TRY(sync(c));
      PF_HIP(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    } else if (fp32) {
      PF_TRY(time_cg_apply<float>(c, reps, &ms));
    } else {
      PF_TRY(time_cg_apply<double>(c, reps, &ms));
    }
    if (best == 0.f || ms < best) {
      best = ms;
      best_ch = ch;
    }
  }
  c->ms = march_shape(c->g, best_ch);
  // graphs captured with another work decomposition are stale
  for (auto &gr : c->graphs) (void)hipGraphExecDestroy(gr.exec);
  c->graphs.clear();
  if (chosen) *chosen = best_ch;
  return PF_OK;
}

// ------------------------------------------------------------- op entry

pf_status pf_op_internal_force(pf_ctx *c, const double *u, const double *d, double *R) {
  if (!c || !u || !d || !R) return PF_E_INVALID_ARG;
  PF_HIP(c, internal_force(c->stream, c->g, c->ms, c->ec, c->mt.split, u, d, c->eact, nullptr,
                           false, R, c->rs));
  return PF_OK;
}

pf_status pf_op_tangent_apply(pf_ctx *c, const double *u, const double *d, const double *p,
                              double *q) {
  if (!c || !u || !d || !p || !q) return PF_E_INVALID_ARG;
  PF_HIP(c, tangent_flags(c->stream, c->g, u, c->eact, c->tflag));
  PF_HIP(c, tangent_apply_plain(c->stream, c->g, c->ms, c->ec, c->mt.split, u, d, c->tflag,
                                c->eact, p, q));
  return PF_OK;
}

pf_status pf_op_phase_apply(pf_ctx *c, const double *coef, const double *p, double *q) {
  if (!c || !coef || !p || !q) return PF_E_INVALID_ARG;
  PF_HIP(c, phase_apply_plain(c->stream, c->g, c->ms, c->pc, coef, c->eact, p, q));
  return PF_OK;
}

pf_status pf_op_qp_update(pf_ctx *c, int32_t scheme, const double *u, const double *d,
                          const double *H_prev, double *H, double *psi_s, uint8_t *flags,
                          int64_t *n_gated) {
  if (!c || !u || !d || !H_prev || !H || !psi_s || !flags) return PF_E_INVALID_ARG;
  if (scheme < 0 || scheme > 3) return fail(c, PF_E_INVALID_ARG, "scheme");
  PF_TRY(zero_icount(c));
  QpParams qp{scheme, psi_crit_of(c), c->opts.d_gate};
  PF_HIP(c, qp_update(c->stream, c->g, c->mt, qp, u, d, c->eact, H_prev, H, psi_s, flags, nullptr,
                      c->rs));
  if (n_gated) {
    PF_TRY(read_scal(c));
    *n_gated = (int64_t)c->icount_h[IC_GATED];
  }
  return PF_OK;
}

pf_status pf_op_predictor(pf_ctx *c, const double *d, const double *dd, const double *H,
                          const double *psi_s, const uint8_t *flags, double *Hhat) {
  if (!c || !d || !dd || !H || !psi_s || !flags || !Hhat) return PF_E_INVALID_ARG;
  PF_HIP(c, predictor<double>(c->stream, c->g, c->mt, d, dd, H, psi_s, flags, c->eact, Hhat));
  return PF_OK;
}

}  // extern "C"
