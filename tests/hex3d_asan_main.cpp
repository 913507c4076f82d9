// The 3-D kernels' host replay under AddressSanitizer and
// UndefinedBehaviorSanitizer: every operator and a few load steps on meshes
// of one and of several ragged blocks, with each array in a heap buffer of
// exactly its documented size, so that any index outside a buffer, as the
// device grid would compute it, is reported.  Exit status 0 and
// "hex3d asan: ok" when nothing is.
#include "hex3d_host_harness.cpp"
#include "hex3d_solver_harness.cpp"

#include <cmath>
#include <cstdio>
#include <vector>

namespace {

uint64_t lcg = 2209;
double rnd() {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return double(lcg >> 11) / double(1ull << 53);
}

std::vector<double> field(size_t n, double scale, double shift = 0.0) {
  std::vector<double> v(n);
  for (auto &x : v) x = shift + scale * rnd();
  return v;
}

void run_ops(const pf3d_mesh &mesh, const pf_material &mat) {
  const size_t N = size_t(mesh.nx + 1) * (mesh.ny + 1) * (mesh.nz + 1);
  const size_t E = size_t(mesh.nx) * mesh.ny * mesh.nz;
  auto u = field(3 * N, 2e-3, -1e-3), d = field(N, 0.9), p = field(3 * N, 1.0, -0.5);
  auto coef = field(8 * E, 50.0, 0.1), Hprev = field(8 * E, 30.0), dd = field(N, 0.1, -0.05);
  std::vector<double> R(3 * N), q(3 * N), Dt(3 * N), qd(N), Dp(N), b(N), H(8 * E), ps(8 * E),
      Hh(8 * E), ct(8 * E);
  std::vector<uint16_t> fl(E);
  long long ng = 0, below = 0;
  h3_internal_force(&mesh, &mat, u.data(), d.data(), R.data());
  h3_tangent_apply(&mesh, &mat, u.data(), d.data(), p.data(), q.data());
  h3_phase_apply(&mesh, &mat, coef.data(), d.data(), qd.data());
  // the element-once grids against the node gathers: the same per-element
  // arithmetic summed in another order
  std::vector<double> Rg(3 * N), qg(3 * N);
  // (the ABI's force takes the gather on small meshes: compare the tiles)
  h3_internal_force_tiled(&mesh, &mat, u.data(), d.data(), R.data());
  h3_internal_force_gather(&mesh, &mat, u.data(), d.data(), Rg.data());
  h3_tangent_apply_gather(&mesh, &mat, u.data(), d.data(), p.data(), qg.data());
  const std::vector<double> *pairs[2][2] = {{&R, &Rg}, {&q, &qg}};
  const char *names[2] = {"internal force", "tangent apply"};
  for (int k = 0; k < 2; ++k) {
    const std::vector<double> &a = *pairs[k][0], &b = *pairs[k][1];
    double dmax = 0.0, bmax = 0.0;
    for (size_t i = 0; i < a.size(); ++i) {
      dmax = std::fmax(dmax, std::fabs(a[i] - b[i]));
      bmax = std::fmax(bmax, std::fabs(b[i]));
    }
    if (!(dmax <= 1e-12 * bmax)) {
      std::printf("tiled %s differs from the gather: %g of %g\n", names[k], dmax, bmax);
      std::exit(1);
    }
  }
  h3_tangent_diag(&mesh, &mat, u.data(), d.data(), Dt.data());
  h3_phase_diag(&mesh, &mat, coef.data(), Dp.data());
  h3_phase_rhs(&mesh, Hprev.data(), b.data());
  for (int scheme = 0; scheme < 4; ++scheme) {
    h3_qp_update(&mesh, &mat, scheme, 0.0, 0.95, u.data(), d.data(), Hprev.data(), H.data(),
                 ps.data(), fl.data(), &ng);
    h3_predictor(&mesh, &mat, d.data(), dd.data(), H.data(), ps.data(), fl.data(), Hh.data());
    h3_phase_coef(&mesh, &mat, 1, 0.1, 1, H.data(), ps.data(), fl.data(), d.data(), ct.data(),
                  &below);
  }
}

void run_steps(const pf3d_mesh &mesh, const pf_material &mat, int scheme) {
  // the library's defaults (pf_default_opts), capped so that the steps
  // reach every path (gated trial, predictor, phase solve, Newton) quickly;
  // they need not converge, only touch every index
  pf_solver_opts o;
  std::memset(&o, 0, sizeof(o));
  o.scheme = scheme;
  o.cheb_degree = 3;
  o.tol_stag = 1e-5;
  o.tol_pcg = 1e-10;
  o.tol_newton = 1e-9;
  o.tol_inner = 1e-5;
  o.max_stag = 3;
  o.max_newton = 2;
  o.max_cg = 20;
  o.cg_check = 32;
  o.psi_crit = 0.0;
  o.d_gate = 0.95;
  o.trial_floor = 0.1;
  o.tol_ir = 0.01;
  void *h = h3s_create(&mesh, &mat, &o);
  if (!h) {
    std::printf("create failed\n");
    std::exit(1);
  }
  // bottom face fixed, top face pulled in y, a line of d = 1 at mid height
  std::vector<int64_t> bot, top, notch;
  std::vector<int8_t> cb, ctop;
  std::vector<double> vb, vt, vn;
  for (int k = 0; k <= mesh.nz; ++k)
    for (int i = 0; i <= mesh.nx; ++i) {
      const int64_t nb = i + int64_t(k) * (mesh.nx + 1) * (mesh.ny + 1);
      const int64_t nt = nb + int64_t(mesh.ny) * (mesh.nx + 1);
      for (int c = 0; c < 3; ++c) {
        bot.push_back(nb);
        cb.push_back(int8_t(c));
        vb.push_back(0.0);
      }
      top.push_back(nt);
      ctop.push_back(1);
      vt.push_back(1.0);
      if (2 * i <= mesh.nx) {
        notch.push_back(nb + int64_t(mesh.ny / 2) * (mesh.nx + 1));
        vn.push_back(1.0);
      }
    }
  h3s_set_dirichlet_u(h, 0, (long long)bot.size(), bot.data(), cb.data(), vb.data());
  h3s_set_dirichlet_u(h, 1, (long long)top.size(), top.data(), ctop.data(), vt.data());
  h3s_set_dirichlet_d(h, (long long)notch.size(), notch.data(), vn.data());
  long long st[10];
  double r = 0.0, f[3];
  int trials = 0;
  for (double lam : {4e-3, 2e-3}) {
    h3s_load_step(h, lam, st, &r);
    trials += int(st[2]);
  }
  if (scheme != 0 && trials == 0) {
    std::printf("no trial solve ran\n");
    std::exit(1);
  }
  h3s_reaction(h, 1, f);
  const size_t N = size_t(mesh.nx + 1) * (mesh.ny + 1) * (mesh.nz + 1);
  const size_t E = size_t(mesh.nx) * mesh.ny * mesh.nz;
  std::vector<double> u(3 * N), d(N), H(8 * E);
  h3s_get_state(h, u.data(), d.data(), H.data());
  h3s_destroy(h);
}

}  // namespace

int main() {
  // the last spans two tiles of node columns in x and y and two chunks of
  // node planes in z of the element-once apply
  const pf3d_mesh meshes[] = {{1, 1, 1, 1.0, 1.0, 1.0}, {5, 4, 3, 1.3, 0.7, 0.45},
                              {9, 7, 5, 1.3, 0.7, 0.45}, {17, 16, 9, 1.1, 0.9, 0.6}};
  for (int split = 0; split < 2; ++split) {
    const pf_material mat{2.1e5, 0.3, 2.7, 0.2, 1e-6, split};
    for (const auto &m : meshes) run_ops(m, mat);
    run_steps(meshes[1], mat, 1);
    run_steps(meshes[2], mat, 3);
  }
  std::printf("hex3d asan: ok\n");
  return 0;
}
