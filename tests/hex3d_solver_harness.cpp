// Host replay of the 3-D load step, for the tests only: the solver of
// pf3d_solver.h runs on a backend that replays every launch's grid on the
// host, block by block and thread by thread, and every reduction with the
// device kernel's per-block tree and block order.  Built host-only (no
// device code, no HIP calls), so it runs without a GPU.
#include "../paper_2209_07969_amd/csrc/pf3d_solver.h"

#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

using namespace pf3d;

namespace {

struct HostBackend {
  void *alloc(size_t bytes) {
    void *p = std::malloc(bytes);
    if (p) std::memset(p, 0, bytes);
    return p;
  }
  void release(void *p) { std::free(p); }
  void upload(void *dst, const void *src, size_t n) { std::memcpy(dst, src, n); }
  void download(void *dst, const void *src, size_t n) { std::memcpy(dst, src, n); }
  template <class F>
  void each(int count, const F &f) {
    for (int b = 0; b < grid_blocks(count); ++b)
      for (int t = 0; t < kTpb3; ++t) {
        const int i = grid_index(b, t);
        if (i < count) f(i);
      }
  }
  // the operators of the device's kernels, replayed block by block
  void tangent_apply(const Grid3 &g, const Mat3 &m, const double *u, const double *d,
                     const double *p, double *q, const int *done) {
    if (!*done) t3_tangent_host(g, m, u, d, p, q);
  }
  void internal_force(const Grid3 &g, const Mat3 &m, const double *u, const double *d,
                      double *R) {
    if (t3_force_tiled(g)) t3_force_host(g, m, u, d, R);
    else each(g.N, [&](int n) { node_internal_force(g, m, n, u, d, R); });
  }
  void phase_apply(const Grid3 &g, const Mat3 &m, const double *coef, const double *p,
                   double *q, const int *done) {
    if (done == nullptr || !*done)
      each(g.N, [&](int n) { node_phase_apply(g, m, n, coef, p, q); });
  }
  bool ok() const { return true; }
  // no recording on the host: a batch runs as it is enqueued
  bool replay(int) { return false; }
  bool capture_begin(int) { return false; }
  void capture_end(int) {}
  template <class F>
  void sum_into(int count, const F &f, double *slot) {
    *slot = sum(count, f);
  }
  template <class F, class P>
  void sum2_into(int count, const F &f, double *sa, double *sb, const P &post) {
    double ta = 0.0, tb = 0.0;
    double va[kTpb3], vb[kTpb3];
    for (int b = 0; b < grid_blocks(count); ++b) {
      for (int t = 0; t < kTpb3; ++t) {
        const int i = grid_index(b, t);
        Sum2 x{0.0, 0.0};
        if (i < count) x = f(i);
        va[t] = x.a;
        vb[t] = x.b;
      }
      for (int h = kTpb3 / 2; h > 0; h >>= 1)
        for (int t = 0; t < h; ++t) {
          va[t] += va[t + h];
          vb[t] += vb[t + h];
        }
      ta += va[0];
      tb += vb[0];
    }
    *sa = ta;
    *sb = tb;
    post(0);
  }
  template <class F>
  double sum(int count, const F &f) {
    double total = 0.0;
    double v[kTpb3];
    for (int b = 0; b < grid_blocks(count); ++b) {
      for (int t = 0; t < kTpb3; ++t) {
        const int i = grid_index(b, t);
        v[t] = i < count ? f(i) : 0.0;
      }
      for (int h = kTpb3 / 2; h > 0; h >>= 1)
        for (int t = 0; t < h; ++t) v[t] += v[t + h];
      total += v[0];
    }
    return total;
  }
};

struct HostCtx {
  HostBackend be;
  std::unique_ptr<Solver3<HostBackend>> sol;
};

}  // namespace

extern "C" {

void *h3s_create(const pf3d_mesh *mesh, const pf_material *mat, const pf_solver_opts *opts) {
  Grid3 g;
  Mat3 m;
  if (make_grid(mesh, &g) != PF_OK || make_mat(mat, &m) != PF_OK || check_opts3(opts) != PF_OK)
    return nullptr;
  auto *c = new HostCtx();
  c->sol.reset(new Solver3<HostBackend>(c->be, g, m, *opts));
  if (!c->sol->init()) {
    delete c;
    return nullptr;
  }
  return c;
}

int h3s_set_dirichlet_u(void *h, int grp, long long n, const int64_t *node, const int8_t *comp,
                        const double *val) {
  return static_cast<HostCtx *>(h)->sol->set_dirichlet_u(grp, n, node, comp, val) ? 0 : 1;
}

int h3s_set_dirichlet_d(void *h, long long n, const int64_t *node, const double *val) {
  return static_cast<HostCtx *>(h)->sol->set_dirichlet_d(n, node, val) ? 0 : 1;
}

// stats: n_stag, n_newton, n_trial, n_dsolve, n_cg_u, n_cg_d, n_cg_trial,
// gated_max, floor_hits, converged
int h3s_load_step(void *h, double lam, long long stats[10], double *r_stag) {
  Counts3 st;
  static_cast<HostCtx *>(h)->sol->load_step(lam, &st);
  const long long v[10] = {st.n_stag, st.n_newton, st.n_trial, st.n_dsolve, st.n_cg_u,
                           st.n_cg_d, st.n_cg_trial, st.gated_max, st.floor_hits,
                           st.converged ? 1 : 0};
  for (int k = 0; k < 10; ++k) stats[k] = v[k];
  *r_stag = st.r_stag;
  return 0;
}

void h3s_reaction(void *h, int grp, double f[3]) {
  static_cast<HostCtx *>(h)->sol->reaction(grp, f);
}

void h3s_get_state(void *h, double *u, double *d, double *H) {
  static_cast<HostCtx *>(h)->sol->get_state(u, d, H);
}

void h3s_set_state(void *h, const double *u, const double *d, const double *H) {
  static_cast<HostCtx *>(h)->sol->set_state(u, d, H);
}

void h3s_destroy(void *h) { delete static_cast<HostCtx *>(h); }

}  // extern "C"
