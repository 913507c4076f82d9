// 3-D operator kernels (trilinear hexahedra) and their C ABI.
//
// The tangent apply, and the internal force on meshes with enough tiles,
// evaluate each element once, in tiles of node columns marching in z
// (t3_block); the phase apply, diagonals and right-hand side run one thread
// per node, which gathers the contributions of its up to eight elements, and
// the quadrature-point updates one thread per element.  Every output is written by one thread
// in a fixed order (deterministic, no atomics).  The arithmetic lives in
// pf3d_ops.h.

#include "../../include/phasefield3d.h"
#include "pf3d_ops.h"
#include "pf3d_solver.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

using namespace pf3d;

namespace {

struct T3DevSync {
  __device__ void operator()() const { __syncthreads(); }
};

// Element-once operator (t3_block) with the element operator Op; a non-null
// done that is set skips the launch (a CG solve that has already ended).
// MINB blocks per CU are asked for: two for the VD tangent and force, which
// without the spectral split's registers fit them.
template <class Op, int MINB>
__global__ void __launch_bounds__(kTpb3, MINB) k3_tiled(Op op, Grid3 g, Mat3 m, const int *done) {
  if (done != nullptr && *done) return;
  __shared__ T3LdsT<typename Op::Node, Op::NC> sm;
  double out[1][8 * Op::NC], carry[1][Op::NC];
  t3_block<Op, 1>(op, g, m, blockIdx.x, threadIdx.x, sm, out, carry, T3DevSync{});
}

template <class Op, int MINB>
void launch_tiled(hipStream_t s, const Op &op, const Grid3 &g, const Mat3 &m, const int *done) {
  hipLaunchKernelGGL((k3_tiled<Op, MINB>), dim3(t3_blocks(g)), dim3(kTpb3), 0, s, op, g, m, done);
}

// q = K_t(u; d) p
void launch_tangent_tiled(hipStream_t s, const Grid3 &g, const Mat3 &m, const double *u,
                          const double *d, const double *p, double *q, const int *done) {
  if (m.split == 1) launch_tiled<T3TangentOp<1>, 1>(s, T3TangentOp<1>{u, d, p, q}, g, m, done);
  else launch_tiled<T3TangentOp<0>, 2>(s, T3TangentOp<0>{u, d, p, q}, g, m, done);
}

__global__ void __launch_bounds__(kTpb3) k3_internal_force(Grid3 g, Mat3 m, const double *u,
                                                           const double *d, double *R) {
  const int n = grid_index(blockIdx.x, threadIdx.x);
  if (n < g.N) node_internal_force(g, m, n, u, d, R);
}

// R = internal force at (u, d): element-once tiles where they fill the GPU
// (t3_force_tiled), else the node gather
void launch_force(hipStream_t s, const Grid3 &g, const Mat3 &m, const double *u,
                  const double *d, double *R) {
  if (!t3_force_tiled(g))
    hipLaunchKernelGGL(k3_internal_force, dim3(grid_blocks(g.N)), dim3(kTpb3), 0, s, g, m, u, d,
                       R);
  else if (m.split == 1)
    launch_tiled<T3ForceOp<1>, 1>(s, T3ForceOp<1>{u, d, R}, g, m, nullptr);
  else
    launch_tiled<T3ForceOp<0>, 2>(s, T3ForceOp<0>{u, d, R}, g, m, nullptr);
}

// Phase operator by node gather: its element is cheap, and one thread per
// node keeps many more waves in flight than the tiles' march through the
// layers (the tiled form measured 1.3-6x slower on 32^3-96^3 cubes).  A
// non-null done that is set skips the launch.
__global__ void __launch_bounds__(kTpb3) k3_phase_apply(Grid3 g, Mat3 m, const double *coef,
                                                        const double *p, double *q,
                                                        const int *done) {
  if (done != nullptr && *done) return;
  const int n = grid_index(blockIdx.x, threadIdx.x);
  if (n < g.N) node_phase_apply(g, m, n, coef, p, q);
}

void launch_phase_apply(hipStream_t s, const Grid3 &g, const Mat3 &m, const double *coef,
                        const double *p, double *q, const int *done) {
  hipLaunchKernelGGL(k3_phase_apply, dim3(grid_blocks(g.N)), dim3(kTpb3), 0, s, g, m, coef, p,
                     q, done);
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

// ---- the load step's device backend

template <class F>
__global__ void __launch_bounds__(kTpb3) k3_each(F f, int count) {
  const int i = grid_index(blockIdx.x, threadIdx.x);
  if (i < count) f(i);
}

// Per-block sum of f over the block's indices by a fixed binary tree in LDS
// (the order the host replay reproduces); one partial per block.
template <class F>
__global__ void __launch_bounds__(kTpb3) k3_sum(F f, int count, double *part) {
  __shared__ double v[kTpb3];
  const int i = grid_index(blockIdx.x, threadIdx.x);
  v[threadIdx.x] = i < count ? f(i) : 0.0;
  __syncthreads();
  for (int h = kTpb3 / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) v[threadIdx.x] += v[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Both sums of a Sum2 functor, by the same tree; partials a, b of block k
// at part[2k], part[2k + 1].
template <class F>
__global__ void __launch_bounds__(kTpb3) k3_sum2(F f, int count, double *part) {
  __shared__ double va[kTpb3], vb[kTpb3];
  const int i = grid_index(blockIdx.x, threadIdx.x);
  Sum2 x{0.0, 0.0};
  if (i < count) x = f(i);
  va[threadIdx.x] = x.a;
  vb[threadIdx.x] = x.b;
  __syncthreads();
  for (int h = kTpb3 / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      va[threadIdx.x] += va[threadIdx.x + h];
      vb[threadIdx.x] += vb[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = va[0];
    part[2 * blockIdx.x + 1] = vb[0];
  }
}

// The two sums in block order, left at sa and sb, then post(0) (one thread).
template <class P>
__global__ void k3_finish2(const double *part, int nb, double *sa, double *sb, P post) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nb; ++k) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  *sa = a;
  *sb = b;
  post(0);
}

// The block partials added in block order, left at slot (one thread: the
// order of the host's sum).
__global__ void k3_finish(const double *part, int nb, double *slot) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += part[b];
  *slot = t;
}

// Runs the solver's per-index functors as kernels on one stream.  Block
// partials of a sum come back through a pinned buffer and are added on the
// host in block order.  The first failing HIP call is kept in err; later
// calls still run but the context reports PF_E_HIP.
struct DeviceBackend {
  hipStream_t s = nullptr;
  double *part = nullptr, *part_h = nullptr;
  int part_cap = 0;
  int part_gen = 0;   // bumped whenever part is reallocated (recorded graphs hold it)
  hipError_t err = hipSuccess;
  struct Graph {
    int key, gen;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  hipStream_t cap = nullptr;   // recording stream (created on first use)
  bool capturing = false;
  // the stream launches go to: the recording stream while a batch is
  // recorded, else the context's stream
  hipStream_t st() const { return capturing ? cap : s; }

  void note(hipError_t e) {
    if (err == hipSuccess && e != hipSuccess) err = e;
  }
  bool reserve(int blocks) {
    if (blocks <= part_cap) return true;
    if (part) note(hipFree(part));
    if (part_h) note(hipHostFree(part_h));
    part = part_h = nullptr;
    part_cap = 0;
    if (hipMalloc((void **)&part, blocks * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&part_h, blocks * sizeof(double)) != hipSuccess) {
      note(hipErrorOutOfMemory);
      return false;
    }
    part_cap = blocks;
    ++part_gen;
    return true;
  }
  // A CG batch recorded under key, replayed while the partials buffer it
  // reduces into is the same one.
  bool replay(int key) {
    for (const Graph &g : graphs)
      if (g.key == key && g.gen == part_gen) {
        note(hipGraphLaunch(g.exec, s));
        return true;
      }
    return false;
  }
  // The batch is recorded on a stream of the backend's own and replayed on
  // the context's stream (which may be the null stream).
  bool capture_begin(int blocks) {
    if (err != hipSuccess || !reserve(blocks)) return false;
    if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
      cap = nullptr;
      (void)hipGetLastError();
      return false;
    }
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    capturing = true;
    return true;
  }
  // Ends the recording, keeps the graph under key (replacing an older one)
  // and launches it once.
  void capture_end(int key) {
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &graph);
    capturing = false;
    note(e);
    if (e != hipSuccess) return;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    note(e);
    if (e != hipSuccess) return;
    for (size_t k = 0; k < graphs.size();)
      if (graphs[k].key == key) {
        (void)hipGraphExecDestroy(graphs[k].exec);
        graphs.erase(graphs.begin() + k);
      } else {
        ++k;
      }
    graphs.push_back({key, part_gen, ex});
    note(hipGraphLaunch(ex, s));
  }
  void *alloc(size_t bytes) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    note(hipMemsetAsync(p, 0, bytes, s));
    return p;
  }
  void release(void *p) {
    if (p) note(hipFree(p));
  }
  void upload(void *dst, const void *src, size_t n) {
    note(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s));
    note(hipStreamSynchronize(s));
  }
  void download(void *dst, const void *src, size_t n) {
    note(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s));
    note(hipStreamSynchronize(s));
  }
  template <class F>
  void each(int count, const F &f) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k3_each<F>, dim3(grid_blocks(count)), dim3(kTpb3), 0, st(), f, count);
    note(hipGetLastError());
  }
  // the element-once operators; the applies are skipped while *done is set
  void tangent_apply(const Grid3 &g, const Mat3 &m, const double *u, const double *d,
                     const double *p, double *q, const int *done) {
    launch_tangent_tiled(st(), g, m, u, d, p, q, done);
    note(hipGetLastError());
  }
  void internal_force(const Grid3 &g, const Mat3 &m, const double *u, const double *d,
                      double *R) {
    launch_force(st(), g, m, u, d, R);
    note(hipGetLastError());
  }
  void phase_apply(const Grid3 &g, const Mat3 &m, const double *coef, const double *p,
                   double *q, const int *done) {
    launch_phase_apply(st(), g, m, coef, p, q, done);
    note(hipGetLastError());
  }
  bool ok() const { return err == hipSuccess; }
  template <class F>
  void sum_into(int count, const F &f, double *slot) {
    const int nb = grid_blocks(count);
    if (count <= 0) {
      hipLaunchKernelGGL(k3_finish, dim3(1), dim3(1), 0, st(), part, 0, slot);
      note(hipGetLastError());
      return;
    }
    if (!reserve(nb)) return;
    hipLaunchKernelGGL(k3_sum<F>, dim3(nb), dim3(kTpb3), 0, st(), f, count, part);
    note(hipGetLastError());
    hipLaunchKernelGGL(k3_finish, dim3(1), dim3(1), 0, st(), part, nb, slot);
    note(hipGetLastError());
  }
  template <class F, class P>
  void sum2_into(int count, const F &f, double *sa, double *sb, const P &post) {
    const int nb = count > 0 ? grid_blocks(count) : 0;
    if (nb > 0) {
      if (!reserve(2 * nb)) return;
      hipLaunchKernelGGL(k3_sum2<F>, dim3(nb), dim3(kTpb3), 0, st(), f, count, part);
      note(hipGetLastError());
    }
    hipLaunchKernelGGL(k3_finish2<P>, dim3(1), dim3(1), 0, st(), part, nb, sa, sb, post);
    note(hipGetLastError());
  }
  template <class F>
  double sum(int count, const F &f) {
    const int nb = grid_blocks(count);
    if (count <= 0 || !reserve(nb)) return 0.0;
    hipLaunchKernelGGL(k3_sum<F>, dim3(nb), dim3(kTpb3), 0, st(), f, count, part);
    note(hipGetLastError());
    note(hipMemcpyAsync(part_h, part, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    note(hipStreamSynchronize(s));
    if (err != hipSuccess) return 0.0;
    double total = 0.0;
    for (int b = 0; b < nb; ++b) total += part_h[b];
    return total;
  }
  ~DeviceBackend() {
    (void)hipStreamSynchronize(s);
    for (const Graph &g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (cap) (void)hipStreamDestroy(cap);
    if (part) (void)hipFree(part);
    if (part_h) (void)hipHostFree(part_h);
  }
};

}  // namespace

struct pf3d_ctx {
  pf3d::Grid3 g{};
  DeviceBackend be;
  std::unique_ptr<pf3d::Solver3<DeviceBackend>> sol;
  int load_group = 1;
  int gsize[pf3d::kGroups3] = {};
};

extern "C" {

pf_status pf3d_op_internal_force(const pf3d_mesh *mesh, const pf_material *mat,
                                 const double *u, const double *d, double *R,
                                 void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!u || !d || !R || make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  launch_force(static_cast<hipStream_t>(hip_stream), g, m, u, d, R);
  return launched();
}

pf_status pf3d_op_tangent_apply(const pf3d_mesh *mesh, const pf_material *mat,
                                const double *u, const double *d, const double *p,
                                double *q, void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!u || !d || !p || !q || make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  launch_tangent_tiled(static_cast<hipStream_t>(hip_stream), g, m, u, d, p, q, nullptr);
  return launched();
}

pf_status pf3d_op_phase_apply(const pf3d_mesh *mesh, const pf_material *mat,
                              const double *coef, const double *p, double *q,
                              void *hip_stream) {
  Grid3 g;
  Mat3 m;
  if (!coef || !p || !q || make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK)
    return PF_E_INVALID_ARG;
  launch_phase_apply(static_cast<hipStream_t>(hip_stream), g, m, coef, p, q, nullptr);
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

pf_status pf3d_create(const pf3d_mesh *mesh, const pf_material *mat,
                      const pf_solver_opts *opts, void *hip_stream, pf3d_ctx **out) {
  if (!out) return PF_E_INVALID_ARG;
  *out = nullptr;
  Grid3 g;
  Mat3 m;
  pf_solver_opts o;
  if (opts) o = *opts;
  else pf_default_opts(&o);
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK || check_opts3(&o) != PF_OK)
    return PF_E_INVALID_ARG;
  auto *c = new pf3d_ctx();
  c->g = g;
  c->be.s = static_cast<hipStream_t>(hip_stream);
  c->sol.reset(new Solver3<DeviceBackend>(c->be, g, m, o));
  const bool ok = c->sol->init() &&
                  c->be.reserve(std::max(2 * grid_blocks(3 * g.N), grid_blocks(8 * g.E)));
  if (!ok || c->be.err != hipSuccess) {
    const pf_status s = c->be.err == hipErrorOutOfMemory || !ok ? PF_E_OOM : PF_E_HIP;
    pf3d_destroy(c);
    return s;
  }
  *out = c;
  return PF_OK;
}

pf_status pf3d_destroy(pf3d_ctx *c) {
  delete c;
  return PF_OK;
}

pf_status pf3d_set_dirichlet_u(pf3d_ctx *c, int32_t group, int64_t n, const int64_t *node,
                               const int8_t *comp, const double *value_per_unit_load) {
  if (!c || group < 0 || group >= kGroups3 || n < 0 ||
      (n > 0 && (!node || !comp || !value_per_unit_load)))
    return PF_E_INVALID_ARG;
  for (int64_t k = 0; k < n; ++k) {
    if (node[k] < 0 || node[k] >= c->g.N || comp[k] < 0 || comp[k] > 2) return PF_E_INVALID_ARG;
    if (!std::isfinite(value_per_unit_load[k])) return PF_E_NONFINITE;
  }
  if (!c->sol->set_dirichlet_u(group, n, node, comp, value_per_unit_load)) return PF_E_OOM;
  c->gsize[group] = (int)n;
  return c->be.err == hipSuccess ? PF_OK : PF_E_HIP;
}

pf_status pf3d_set_dirichlet_d(pf3d_ctx *c, int64_t n, const int64_t *node, const double *value) {
  if (!c || n < 0 || (n > 0 && (!node || !value))) return PF_E_INVALID_ARG;
  for (int64_t k = 0; k < n; ++k) {
    if (node[k] < 0 || node[k] >= c->g.N) return PF_E_INVALID_ARG;
    if (!std::isfinite(value[k])) return PF_E_NONFINITE;
  }
  if (!c->sol->set_dirichlet_d(n, node, value)) return PF_E_OOM;
  return c->be.err == hipSuccess ? PF_OK : PF_E_HIP;
}

pf_status pf3d_load_step(pf3d_ctx *c, double load_factor, pf_step_stats *stats) {
  if (!c) return PF_E_INVALID_ARG;
  if (!std::isfinite(load_factor)) return PF_E_INVALID_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  Counts3 st;
  c->sol->load_step(load_factor, &st);
  double f[3] = {0.0, 0.0, 0.0};
  const int grp = c->gsize[1] > 0 ? 1 : 0;
  c->sol->reaction(grp, f);
  if (c->be.err != hipSuccess) return PF_E_HIP;
  if (!std::isfinite(st.r_stag)) return PF_E_NONFINITE;
  if (stats) {
    *stats = pf_step_stats{};
    stats->n_stag = st.n_stag;
    stats->n_newton = st.n_newton;
    stats->n_trial = st.n_trial;
    stats->n_dsolve = st.n_dsolve;
    stats->n_cg_u = st.n_cg_u;
    stats->n_cg_d = st.n_cg_d;
    stats->n_cg_trial = st.n_cg_trial;
    stats->gated_max = st.gated_max;
    stats->floor_hits = st.floor_hits;
    stats->r_stag = st.r_stag;
    stats->force[0] = f[0];
    stats->force[1] = f[1];
    stats->time_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->dof_updates = st.dof_updates;
    stats->converged = st.converged ? 1 : 0;
    stats->cg_not_converged = (int32_t)st.cg_not_converged;
  }
  return st.converged ? PF_OK : PF_E_NOT_CONVERGED;
}

pf_status pf3d_reaction_force(pf3d_ctx *c, int32_t group, double force[3]) {
  if (!c || !force || group < 0 || group >= kGroups3) return PF_E_INVALID_ARG;
  c->sol->reaction(group, force);
  return c->be.err == hipSuccess ? PF_OK : PF_E_HIP;
}

pf_status pf3d_set_state(pf3d_ctx *c, const double *u, const double *d, const double *H) {
  if (!c) return PF_E_INVALID_ARG;
  const size_t n3 = 3 * (size_t)c->g.N, n = c->g.N, e8 = 8 * (size_t)c->g.E;
  if (u)
    for (size_t k = 0; k < n3; ++k)
      if (!std::isfinite(u[k])) return PF_E_NONFINITE;
  if (d)
    for (size_t k = 0; k < n; ++k)
      if (!std::isfinite(d[k])) return PF_E_NONFINITE;
  if (H)
    for (size_t k = 0; k < e8; ++k)
      if (!std::isfinite(H[k])) return PF_E_NONFINITE;
  c->sol->set_state(u, d, H);
  return c->be.err == hipSuccess ? PF_OK : PF_E_HIP;
}

pf_status pf3d_get_state(pf3d_ctx *c, double *u, double *d, double *H) {
  if (!c) return PF_E_INVALID_ARG;
  c->sol->get_state(u, d, H);
  return c->be.err == hipSuccess ? PF_OK : PF_E_HIP;
}

}  // extern "C"
