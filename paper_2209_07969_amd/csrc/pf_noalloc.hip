// Allocation-free tangent apply (pf_tangent_apply_noalloc).
//
// The same operation and kernels as pf_op_tangent_apply: the split tangent
// K_t(u; d) (Section 2, eq_sigma and the active indicators of
// eq_definition_+) applied to p.  pf_op_tangent_apply keeps the per-element
// indicator bytes in a buffer of its context; this entry point needs no
// context and allocates nothing: the indicator bytes go to a file-scope
// device array of the library, one copy per device, whose address is looked
// up once per device on the first call there.

#include "../../include/phasefield.h"
#include "pf_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

using namespace pf;

// One byte per element: the tr(eps) > 0 bits of its four quadrature points.
// Every call rewrites the nx*ny bytes it uses before reading them.
static __device__ __align__(256) uint8_t scratch[PF_NOALLOC_MAX_ELEMENTS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};   // device address of scratch, per device

// Device address of this device's scratch array (hipGetSymbolAddress once
// per device, with that device current).  Host code never passes the array's
// own name to a kernel: on the host it is only a stand-in for the symbol.
pf_status scratch_for_current_device(uint8_t **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PF_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PF_E_HIP;
    g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
  }
  *out = g_scratch_ptr[dev];
  return PF_OK;
}

}  // namespace

extern "C" pf_status pf_tangent_apply_noalloc(const pf_mesh_desc *mesh, const pf_material *mat,
                                              const double *u, const double *d, const double *p,
                                              double *q, void *hip_stream) {
  if (!mesh || !mat || !u || !d || !p || !q) return PF_E_INVALID_ARG;
  if (mesh->nx < 1 || mesh->ny < 1 || !(mesh->lx > 0) || !(mesh->ly > 0)) return PF_E_INVALID_ARG;
  // one scratch byte per element; compare without multiplying past 64 bits
  if ((long long)mesh->nx > PF_NOALLOC_MAX_ELEMENTS / (long long)mesh->ny)
    return PF_E_INVALID_ARG;
  if (!(mat->E > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->eta >= 0) ||
      (mat->split != PF_SPLIT_VD && mat->split != PF_SPLIT_SPECTRAL))
    return PF_E_INVALID_ARG;
  uint8_t *flags = nullptr;
  pf_status s = scratch_for_current_device(&flags);
  if (s != PF_OK) return s;
  Grid g;
  g.nx = mesh->nx;
  g.ny = mesh->ny;
  g.N = (mesh->nx + 1) * (mesh->ny + 1);
  g.E = mesh->nx * mesh->ny;
  g.hx = mesh->lx / mesh->nx;
  g.hy = mesh->ly / mesh->ny;
  const double mu = mat->E / (2.0 * (1.0 + mat->nu));
  const double lam = mat->E * mat->nu / ((1.0 + mat->nu) * (1.0 - 2.0 * mat->nu));
  const double K = lam + 2.0 * mu / 3.0;
  const ElasCoef ec{2.0 * mu, K, lam, mu, mat->eta, 1.0 / g.hx, 1.0 / g.hy, g.hy / 4.0,
                    g.hx / 4.0};
  // the work decomposition a context with default options chooses
  March m = march_shape(g, 0);
  if (mat->split == PF_SPLIT_SPECTRAL && m.ch == 8) m = march_shape(g, 4);
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const uint8_t *eact = mesh->elem_active;   // a device pointer here, or null
  if (tangent_flags(st, g, u, eact, flags) != hipSuccess) return PF_E_HIP;
  if (tangent_apply_plain(st, g, m, ec, mat->split, u, d, flags, eact, p, q) != hipSuccess)
    return PF_E_HIP;
  return PF_OK;
}
