// Device-free paths of the C ABI, for a build of the library whose host code
// carries AddressSanitizer / UndefinedBehaviorSanitizer: option validation,
// status strings, argument checks on null handles.  Every call here returns
// before any device work.  Exit status 0 when every call behaves as the
// header documents.
#include <cstdio>
#include <cstring>

#include "../include/phasefield.h"
#include "../include/phasefield3d.h"

static int failures = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

static pf_status create_with(void (*edit)(pf_solver_opts *)) {
  pf_mesh_desc mesh{4, 4, 1.0, 1.0, nullptr};
  pf_material mat{2.1e5, 0.3, 2.7, 0.03, 1e-6, 0};
  pf_solver_opts o;
  pf_default_opts(&o);
  o.precond = 1;
  edit(&o);
  pf_ctx *ctx = nullptr;
  pf_status s = pf_create(&mesh, &mat, &o, nullptr, &ctx);
  CHECK(ctx == nullptr);
  return s;
}

int main() {
  pf_solver_opts o;
  std::memset(&o, 0xab, sizeof(o));
  pf_default_opts(&o);
  CHECK(o.max_stag == 500 && o.trial_floor == 0.1 && o.tol_ir == 0.01 && o.phase_model == 0);
  for (int s = PF_OK; s <= PF_E_NONFINITE; ++s) CHECK(pf_status_string((pf_status)s) != nullptr);

  CHECK(create_with([](pf_solver_opts *p) { p->scheme = 7; }) == PF_E_INVALID_ARG);
  CHECK(create_with([](pf_solver_opts *p) { p->precision = 2; }) == PF_E_INVALID_ARG);
  CHECK(create_with([](pf_solver_opts *p) { p->cheb_degree = 0; }) == PF_E_INVALID_ARG);
  CHECK(create_with([](pf_solver_opts *p) { p->cheb_ratio = 0.5; }) == PF_E_INVALID_ARG);
  CHECK(create_with([](pf_solver_opts *p) { p->march_rows = 3; }) == PF_E_INVALID_ARG);
  CHECK(create_with([](pf_solver_opts *p) { p->trial_floor = 0.0; }) == PF_E_INVALID_ARG);
  CHECK(create_with([](pf_solver_opts *p) { p->trial_operator = 2; }) == PF_E_INVALID_ARG);
  CHECK(create_with([](pf_solver_opts *p) { p->phase_model = 1; p->tol_ir = 0.0; }) ==
        PF_E_INVALID_ARG);
  CHECK(create_with([](pf_solver_opts *p) { p->max_cg = 0; }) == PF_E_INVALID_ARG);

  pf_mesh_desc bad{0, 4, 1.0, 1.0, nullptr};
  pf_material mat{2.1e5, 0.3, 2.7, 0.03, 1e-6, 0};
  pf_default_opts(&o);
  pf_ctx *ctx = nullptr;
  CHECK(pf_create(&bad, &mat, &o, nullptr, &ctx) == PF_E_INVALID_ARG && ctx == nullptr);
  CHECK(pf_create(nullptr, &mat, &o, nullptr, &ctx) == PF_E_INVALID_ARG);
  // meshes whose 2N or 4E overflow 32-bit kernel indices, and the largest nx
  const int32_t big[][2] = {{23200, 23200}, {1, 1 << 29}, {2147483647, 1}, {2147483647, 2147483647}};
  for (const auto &s : big) {
    pf_mesh_desc m{s[0], s[1], 1.0, 1.0, nullptr};
    CHECK(pf_create(&m, &mat, &o, nullptr, &ctx) == PF_E_INVALID_ARG && ctx == nullptr);
  }

  // 3-D operators: refused before any launch
  double x[24] = {0};
  uint16_t fl[1] = {0};
  const pf3d_mesh m3{1, 1, 1, 1.0, 1.0, 1.0};
  const pf3d_mesh m3bad[] = {{0, 1, 1, 1.0, 1.0, 1.0}, {1, 1, 1, 1.0, 0.0, 1.0},
                             {1024, 1024, 1024, 1.0, 1.0, 1.0},
                             {2147483647, 2147483647, 2147483647, 1.0, 1.0, 1.0}};
  for (const auto &mb : m3bad)
    CHECK(pf3d_op_internal_force(&mb, &mat, x, x, x, nullptr) == PF_E_INVALID_ARG);
  pf_material no_split = mat;
  no_split.split = 2;
  CHECK(pf3d_op_tangent_apply(&m3, &no_split, x, x, x, x, nullptr) == PF_E_INVALID_ARG);
  CHECK(pf3d_op_phase_apply(&m3, &mat, nullptr, x, x, nullptr) == PF_E_INVALID_ARG);
  CHECK(pf3d_op_qp_update(&m3, &mat, 9, -1.0, 0.95, x, x, x, x, x, fl, nullptr) ==
        PF_E_INVALID_ARG);
  // 3-D load steps: options outside the path and null handles are refused
  pf3d_ctx *c3 = nullptr;
  pf_solver_opts o3;
  pf_default_opts(&o3);
  o3.precision = PF_MIXED;
  CHECK(pf3d_create(&m3, &mat, &o3, nullptr, &c3) == PF_E_INVALID_ARG && c3 == nullptr);
  pf_default_opts(&o3);
  o3.phase_model = PF_AT1_PENALTY;
  CHECK(pf3d_create(&m3, &mat, &o3, nullptr, &c3) == PF_E_INVALID_ARG && c3 == nullptr);
  CHECK(pf3d_create(&m3bad[0], &mat, nullptr, nullptr, &c3) == PF_E_INVALID_ARG);
  CHECK(pf3d_load_step(nullptr, 1.0, nullptr) == PF_E_INVALID_ARG);
  CHECK(pf3d_reaction_force(nullptr, 1, x) == PF_E_INVALID_ARG);
  CHECK(pf3d_get_state(nullptr, x, x, x) == PF_E_INVALID_ARG);
  CHECK(pf3d_set_state(nullptr, x, x, x) == PF_E_INVALID_ARG);
  CHECK(pf3d_set_dirichlet_d(nullptr, 0, nullptr, nullptr) == PF_E_INVALID_ARG);
  CHECK(pf3d_destroy(nullptr) == PF_OK);

  CHECK(pf_load_step(nullptr, 1.0, nullptr) == PF_E_INVALID_ARG);
  CHECK(pf_staggered_iterate(nullptr, 1.0, nullptr) == PF_E_INVALID_ARG);
  CHECK(pf_commit_step(nullptr) == PF_E_INVALID_ARG);
  CHECK(pf_destroy(nullptr) == PF_E_INVALID_ARG || pf_destroy(nullptr) == PF_OK);
  CHECK(pf_set_allocator(nullptr, nullptr, nullptr, nullptr) == PF_E_INVALID_ARG);
  pf_batch *b = nullptr;
  CHECK(pf_batch_create(0, nullptr, &b) == PF_E_INVALID_ARG && b == nullptr);
  CHECK(pf_batch_set_workers(nullptr, 4) == PF_E_INVALID_ARG);
  CHECK(pf_batch_set_shared_launches(nullptr, 1) == PF_E_INVALID_ARG);
  std::printf(failures ? "host checks: %d failures\n" : "host checks: ok\n", failures);
  return failures ? 1 : 0;
}
