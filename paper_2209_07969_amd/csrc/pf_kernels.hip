// HIP kernels (gfx950) for AT2 phase-field fracture with fixed-stress
// staggering on a structured Q1 plane-strain mesh.
//
// Operator applies (elasticity tangent, internal force, AT2 phase operator,
// their diagonals) use one column-marching kernel: a wavefront covers 64
// consecutive element columns and walks up a chunk of element rows.  Lane L
// computes element (ie, je), ie = 63*strip - 1 + L, keeps the contributions
// of its element row to the row above in registers, and takes the
// contribution of its left neighbour column with one lane shuffle.  Every
// node value is therefore summed exactly once, in registers, with no atomics
// and no LDS round trip; the only redundant work is one element column per
// 63 and one element row per chunk.
//
// Element geometry on the uniform grid: with edge differences
// Db = u1-u0, Dt = u2-u3, Dl = u3-u0, Dr = u2-u1 and the Gauss weights
// a = (1+1/sqrt3)/2, b = (1-1/sqrt3)/2, the derivatives at QP q are
//   du/dx = (wB Db + wT Dt)/hx,  du/dy = (wL Dl + wR Dr)/hy,
// (wB,wT) = (a,b) for q = 0,1 and (b,a) for q = 2,3; (wL,wR) = (a,b) for
// q = 0,3 and (b,a) for q = 1,2.  The transpose maps edge duals back to the
// corners: f0 = -Eb - El, f1 = Eb - Er, f2 = Et + Er, f3 = El - Et.
//
// Reductions are deterministic and need no communication between blocks of
// one kernel: wave shuffles and a fixed-order LDS sum give one partial per
// block, stored with a plain vector store; the next kernel in the stream
// (every one of its blocks, or a one-block finaliser) sums the partials in a
// fixed order.  Device-scope fences are avoided on purpose: on a GPU whose
// L2 is split across dies they write back the local L2.

#include "pf_internal.h"

#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>
#include <utility>

namespace pf {
namespace {

constexpr double GA = 0.78867513459481288225;   // (1 + 1/sqrt(3)) / 2
constexpr double GB = 0.21132486540518711775;   // (1 - 1/sqrt(3)) / 2
constexpr int WPB = 4;                            // waves per block (march)
constexpr int TPB = 256;
static_assert(kPMax % (2 * TPB) == 0, "block_sum reads pairs of partials, kPMax / (2 TPB) per thread");

// ------------------------------------------------------- lane shifts

// Lane L receives lane L-1's value (lane 0 receives 0).  One DPP
// whole-wavefront shift per 32-bit word: a plain VALU move, with no LDS
// crossbar round trip as a general shuffle would need.  bound_ctrl makes
// the hardware write 0 where the source lane does not exist, so no old value
// has to be set up first.
constexpr int kDppWaveShr1 = 0x138;
__device__ inline int lane_up_bits(int x) {
  return __builtin_amdgcn_update_dpp(0, x, kDppWaveShr1, 0xf, 0xf, true);
}
__device__ inline float lane_up(float x) {
  return __int_as_float(lane_up_bits(__float_as_int(x)));
}
__device__ inline double lane_up(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = lane_up_bits(static_cast<int>(b));
  const int hi = lane_up_bits(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
}

// Load at a 32-bit byte offset from a uniform base: the scalar-base form of
// the global load, with no 64-bit address arithmetic per lane.
template <class T>
__device__ inline T ldo(const T *base, unsigned byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// ------------------------------------------------------------ reductions

// DPP move of a double: lanes whose source lies outside the row (or whose
// row is masked off by ROWS) receive 0.
template <int CTRL, int ROWS>
__device__ inline double dpp_take(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWS, 0xf,
                                             false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
}

// Sum over the wavefront, complete in lane 63: a shift-and-add scan within
// each 16-lane row (shifts 1, 2, 4, 8), then row 0's total into row 1 and
// row 2's into row 3 (row_bcast:15), then row 1's into rows 2-3
// (row_bcast:31).  Fixed order, so every launch gives the same bits.
__device__ inline double wave_sum_last(double x) {
  x += dpp_take<0x111, 0xf>(x);
  x += dpp_take<0x112, 0xf>(x);
  x += dpp_take<0x114, 0xf>(x);
  x += dpp_take<0x118, 0xf>(x);
  x += dpp_take<0x142, 0xa>(x);
  x += dpp_take<0x143, 0xc>(x);
  return x;
}

// Block partial of NV sums: wave sums, then a fixed-order LDS sum by
// thread 0, stored to part[k * kPMax + bid].  All threads call it.
template <int NV>
__device__ inline void block_partial_at(double (&v)[NV], double *part, int bid) {
  __shared__ double sh[NV][TPB / 64];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_last(v[k]);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < TPB / 64; ++w) s += sh[k][w];
      part[k * kPMax + bid] = s;
    }
  }
}

template <int NV>
__device__ inline void block_partial(double (&v)[NV], double *part) {
  block_partial_at<NV>(v, part, blockIdx.x);
}

// Fixed-order sum of np <= kPMax partials written by an earlier kernel,
// returned in every thread of the block (bit-identical in every block).
// Thread t reads the pair of partials (2t, 2t+1) + 2 TPB r for the rounds
// r < nr = ceil(np / (2 TPB)), one 16-byte load each, and adds them in round
// order; in the last round the partials at np or beyond count 0.  The round
// count is a template argument (block_sum dispatches on nr, which is
// uniform), so every load is issued before the first add, the prologue of a
// kernel costs one memory round trip, and only the last round is masked.
// The pointer is 16-byte aligned (buffers are 256-byte aligned and every
// partial array starts at an even index).
template <int NV, int NR>
__device__ inline void block_sum_rounds(const double *part, int np, double (&s)[NV]) {
  const unsigned off = 16u * threadIdx.x;   // byte offset of the thread's pair in round 0
  double2 v[NV][NR];
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < NR; ++r)
      v[k][r] = ldo(reinterpret_cast<const double2 *>(part + k * kPMax + r * 2 * TPB), off);
  const int b = 2 * static_cast<int>(threadIdx.x) + (NR - 1) * 2 * TPB;   // last round's pair
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    v[k][NR - 1].x = b < np ? v[k][NR - 1].x : 0.0;
    v[k][NR - 1].y = b + 1 < np ? v[k][NR - 1].y : 0.0;
    // the first pair starts the sum (an add of 0.0 there would be placed
    // with its load and wait for it)
    double t = v[k][0].x + v[k][0].y;
#pragma unroll
    for (int r = 1; r < NR; ++r) t = t + v[k][r].x + v[k][r].y;
    s[k] = t;
  }
}

template <int NV>
__device__ inline void block_sum(const double *part, int np, double (&out)[NV]) {
  static_assert(kPMax == 8 * TPB, "block_sum dispatches on up to four rounds of pairs");
  __shared__ double sh[NV][TPB / 64];
  double s[NV];
  switch ((np + 2 * TPB - 1) / (2 * TPB)) {
    case 1: block_sum_rounds<NV, 1>(part, np, s); break;
    case 2: block_sum_rounds<NV, 2>(part, np, s); break;
    case 3: block_sum_rounds<NV, 3>(part, np, s); break;
    case 4: block_sum_rounds<NV, 4>(part, np, s); break;
    default:
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double w = wave_sum_last(s[k]);
    if ((threadIdx.x & 63) == 63) sh[k][threadIdx.x >> 6] = w;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) t += sh[k][w];
    out[k] = t;
  }
  __syncthreads();
}

// ---------------------------------------------------------- QP geometry

template <int q> struct QW {
  static constexpr double wB = (q < 2) ? GA : GB;
  static constexpr double wT = (q < 2) ? GB : GA;
  static constexpr double wL = (q == 0 || q == 3) ? GA : GB;
  static constexpr double wR = (q == 0 || q == 3) ? GB : GA;
};

// N_a at QP q: a^2 at the nearest corner, b^2 at the opposite one, ab else.
template <int q, int a> struct NW {
  static constexpr double v = (a == q) ? GA * GA : (a == ((q + 2) & 3)) ? GB * GB : GA * GB;
};

template <class T, int q>
__device__ inline T interp4(T v0, T v1, T v2, T v3) {
  return T(NW<q, 0>::v) * v0 + T(NW<q, 1>::v) * v1 + T(NW<q, 2>::v) * v2 + T(NW<q, 3>::v) * v3;
}

__device__ inline bool elem_exists(const Grid &g, int ie, int je, const uint8_t *eact) {
  if (ie < 0 || ie >= g.nx || je < 0 || je >= g.ny) return false;
  if (eact != nullptr && eact[ie + je * g.nx] == 0) return false;
  return true;
}

__device__ inline bool node_exists(const Grid &g, int i, int j) {
  return i >= 0 && i <= g.nx && j >= 0 && j <= g.ny;
}

// Unchecked loads for work items that lie inside the mesh (ldo, above):
// every array an op reads this way is split into planes of at most N
// values, so the offsets fit in 32 bits while N * 8 bytes does.
__device__ inline bool offsets32(const Grid &g) { return g.N < (1 << 29); }

// True when the box of nodes [i0, i0 + n) x [j0, j0 + n) and the elements
// between them lie inside the mesh and the 32-bit offsets apply.
__device__ inline bool box_inside(const Grid &g, int i0, int j0, int n) {
  return offsets32(g) && i0 >= 0 && j0 >= 0 && i0 + n - 1 <= g.nx && j0 + n - 1 <= g.ny;
}

// Ops with unchecked loads (load_fast, load_aux_fast, eload_fast,
// load_own_fast, by node and element index) take that path in the LDS-tile
// kernels for tiles inside the mesh.
template <class Op, class = void>
struct HasFast : std::false_type {};
template <class Op>
struct HasFast<Op, std::void_t<decltype(std::declval<const Op &>().load_fast(0u))>>
    : std::true_type {};

// Data an operator needs only at the nodes a work item stores: fetched with
// the item's first loads (load_own) instead of after the element maths, so
// no dependent memory round trip remains at the end of a kernel.
struct OwnFlag { uint8_t nf; };
__device__ inline OwnFlag load_flag(const uint8_t *nflag, const Grid &g, int i, int j) {
  OwnFlag o{0};
  if (nflag != nullptr && node_exists(g, i, j)) o.nf = nflag[i + j * (g.nx + 1)];
  return o;
}

// --------------------------------------------------------- element maths

// Elasticity, volumetric-deviatoric split.  sigma = A2 eps + (kap - A2/3) t I
// (in-plane), sxy = A2/2 gamma with A2 = 2 mu g; kap = g K if the QP is
// active (t > 0, strict) else K.  NONLIN: active bit from the current strain
// (residual); otherwise from `bits` (tangent frozen at the Newton point).
template <class T, bool NONLIN>
__device__ inline void elastic_element(const T (&ux)[4], const T (&uy)[4], const T (&dn)[4],
                                       unsigned bits, const ElasCoef &c, T (&fx)[4],
                                       T (&fy)[4]) {
  const T Dbx = ux[1] - ux[0], Dtx = ux[2] - ux[3], Dlx = ux[3] - ux[0], Drx = ux[2] - ux[1];
  const T Dby = uy[1] - uy[0], Dty = uy[2] - uy[3], Dly = uy[3] - uy[0], Dry = uy[2] - uy[1];
  const T ihx = T(c.ihx), ihy = T(c.ihy), twomu = T(c.two_mu), K = T(c.K), eta = T(c.eta);
  const T a = T(GA), b = T(GB);
  // x-derivatives take one value on the bottom QP pair (0, 1) and one on the
  // top pair (2, 3); y-derivatives one on the left pair (0, 3) and one on
  // the right pair (1, 2)
  const T exB = (a * Dbx + b * Dtx) * ihx, exT = (b * Dbx + a * Dtx) * ihx;
  const T vxB = (a * Dby + b * Dty) * ihx, vxT = (b * Dby + a * Dty) * ihx;
  const T eyL = (a * Dly + b * Dry) * ihy, eyR = (b * Dly + a * Dry) * ihy;
  const T uyL = (a * Dlx + b * Drx) * ihy, uyR = (b * Dlx + a * Drx) * ihy;
  T sxx[4], syy[4], sxy[4];
#define PF_QP(q)                                                                         \
  {                                                                                      \
    const T exx = (q < 2) ? exB : exT;                                                   \
    const T uyx = (q < 2) ? vxB : vxT;                                                   \
    const T eyy = (q == 0 || q == 3) ? eyL : eyR;                                        \
    const T uxy = (q == 0 || q == 3) ? uyL : uyR;                                        \
    const T dq = interp4<T, q>(dn[0], dn[1], dn[2], dn[3]);                              \
    const T om = T(1) - dq;                                                              \
    const T gq = om * om + eta;                                                          \
    const T A2 = twomu * gq;                                                             \
    const T t = exx + eyy;                                                               \
    bool act = NONLIN ? (t > T(0)) : (((bits >> q) & 1u) != 0u);                        \
    const T kap = act ? gq * K : K;                                                      \
    const T lq = kap - A2 * T(1.0 / 3.0);                                                \
    sxx[q] = A2 * exx + lq * t;                                                          \
    syy[q] = A2 * eyy + lq * t;                                                          \
    sxy[q] = T(0.5) * A2 * (uxy + uyx);                                                  \
  }
  PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
  // edge duals: each is a weighted sum over a QP pair, with the quadrature
  // scale folded into the weights
  const T sa = T(c.sx) * a, sb = T(c.sx) * b, ta = T(c.sy) * a, tb = T(c.sy) * b;
  const T xB = sxx[0] + sxx[1], xT = sxx[2] + sxx[3];
  const T yL = syy[0] + syy[3], yR = syy[1] + syy[2];
  const T sB = sxy[0] + sxy[1], sT = sxy[2] + sxy[3];
  const T sL = sxy[0] + sxy[3], sR = sxy[1] + sxy[2];
  const T Ebx = sa * xB + sb * xT, Etx = sb * xB + sa * xT;
  const T Elx = ta * sL + tb * sR, Erx = tb * sL + ta * sR;
  const T Eby = sa * sB + sb * sT, Ety = sb * sB + sa * sT;
  const T Ely = ta * yL + tb * yR, Ery = tb * yL + ta * yR;
  fx[0] = -Ebx - Elx; fx[1] = Ebx - Erx; fx[2] = Etx + Erx; fx[3] = Elx - Etx;
  fy[0] = -Eby - Ely; fy[1] = Eby - Ery; fy[2] = Ety + Ery; fy[3] = Ely - Ety;
}

// Diagonal of the elasticity tangent: for corner a and component x the
// strain of a unit nodal value is (dNa/dx, 0, dNa/dy), giving
// C00 Nx^2 + C22 Ny^2 (y: C11 Ny^2 + C22 Nx^2), C22 = A2/2.
template <class T>
__device__ inline void elastic_diag_element(const T (&dn)[4], unsigned bits, const ElasCoef &c,
                                            T (&fx)[4], T (&fy)[4]) {
  const T wdet = T(c.sx) / T(c.ihx);     // hx hy / 4
  const T ihx2 = T(c.ihx) * T(c.ihx), ihy2 = T(c.ihy) * T(c.ihy);
#pragma unroll
  for (int a = 0; a < 4; ++a) { fx[a] = 0; fy[a] = 0; }
#define PF_QP(q)                                                                         \
  {                                                                                      \
    const T wB = T(QW<q>::wB), wT = T(QW<q>::wT), wL = T(QW<q>::wL), wR = T(QW<q>::wR);  \
    const T dq = interp4<T, q>(dn[0], dn[1], dn[2], dn[3]);                              \
    const T om = T(1) - dq;                                                              \
    const T gq = om * om + T(c.eta);                                                     \
    const T A2 = T(c.two_mu) * gq;                                                       \
    const bool act = ((bits >> q) & 1u) != 0u;                                           \
    const T kap = act ? gq * T(c.K) : T(c.K);                                            \
    const T C00 = A2 * T(2.0 / 3.0) + kap;                                               \
    const T C22 = T(0.5) * A2;                                                           \
    const T nx2[4] = {wB * wB * ihx2, wB * wB * ihx2, wT * wT * ihx2, wT * wT * ihx2};    \
    const T ny2[4] = {wL * wL * ihy2, wR * wR * ihy2, wR * wR * ihy2, wL * wL * ihy2};    \
    for (int a = 0; a < 4; ++a) {                                                        \
      fx[a] += wdet * (C00 * nx2[a] + C22 * ny2[a]);                                     \
      fy[a] += wdet * (C00 * ny2[a] + C22 * nx2[a]);                                     \
    }                                                                                    \
  }
  PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
}

// Spectral split (Miehe), plane strain with the out-of-plane eigenvalue 0.
// In-plane eigenvalues e1 >= e2 of eps; with P1 = (eps - e2 I)/(e1 - e2) the
// active strain is eps+ = eps (e2 > 0), 0 (e1 <= 0) or e1 P1 (mixed signs),
// and its derivative along an increment de is de, 0 or
//   (1 - 2 th)(P1:de) P1 + th (P1 de + de P1),  th = e1/(e1 - e2).
// In the mixed case e1 - e2 >= max(e1, -e2) > 0, so no division degenerates.
// Stress: sigma = lam kap t I + 2 mu (g - 1) eps+ + 2 mu eps, kap = g if
// t > 0 else 1 (the same for the tangent with eps+ -> d eps+).
template <class T>
struct SpecLin {
  T a, b, cc, th, e1;
  int cs;   // 0: no eigenvalue active, 1: both active, 2: only e1 active
};

template <class T>
__device__ inline void spec_lin(T exx, T eyy, T exy, SpecLin<T> &s) {
  const T t = exx + eyy;
  const T dd = T(0.5) * (exx - eyy);
  const T r = sqrt(dd * dd + exy * exy);
  const T e1 = T(0.5) * t + r, e2 = T(0.5) * t - r;
  s.e1 = e1;
  s.a = s.b = s.cc = s.th = T(0);
  if (e2 > T(0)) {
    s.cs = 1;
  } else if (!(e1 > T(0))) {
    s.cs = 0;
  } else {
    s.cs = 2;
    const T D = e1 - e2;
    s.a = (exx - e2) / D;
    s.b = exy / D;
    s.cc = (eyy - e2) / D;
    s.th = e1 / D;
  }
}

template <class T>
__device__ inline void spec_dplus(const SpecLin<T> &s, T dxx, T dyy, T dxy, T &oxx, T &oyy,
                                  T &oxy) {
  if (s.cs == 1) {
    oxx = dxx; oyy = dyy; oxy = dxy;
  } else if (s.cs == 0) {
    oxx = T(0); oyy = T(0); oxy = T(0);
  } else {
    const T sp = s.a * dxx + T(2) * s.b * dxy + s.cc * dyy;
    const T k1 = (T(1) - T(2) * s.th) * sp;
    oxx = k1 * s.a + T(2) * s.th * (s.a * dxx + s.b * dxy);
    oyy = k1 * s.cc + T(2) * s.th * (s.b * dxy + s.cc * dyy);
    oxy = k1 * s.b + s.th * (s.b * (dxx + dyy) + dxy);
  }
}

// Spectral-split element: NONLIN = internal force at (ux, uy); otherwise the
// tangent at the linearisation point (lx, ly) applied to (ux, uy).
template <class T, bool NONLIN>
__device__ inline void spectral_element(const T (&ux)[4], const T (&uy)[4], const T (&dn)[4],
                                        const T (&lx)[4], const T (&ly)[4], const ElasCoef &c,
                                        T (&fx)[4], T (&fy)[4]) {
  const T Dbx = ux[1] - ux[0], Dtx = ux[2] - ux[3], Dlx = ux[3] - ux[0], Drx = ux[2] - ux[1];
  const T Dby = uy[1] - uy[0], Dty = uy[2] - uy[3], Dly = uy[3] - uy[0], Dry = uy[2] - uy[1];
  const T Lbx = lx[1] - lx[0], Ltx = lx[2] - lx[3], Llx = lx[3] - lx[0], Lrx = lx[2] - lx[1];
  const T Lby = ly[1] - ly[0], Lty = ly[2] - ly[3], Lly = ly[3] - ly[0], Lry = ly[2] - ly[1];
  const T ihx = T(c.ihx), ihy = T(c.ihy), twomu = T(c.two_mu), lam = T(c.lam), eta = T(c.eta);
  T Ebx = 0, Etx = 0, Elx = 0, Erx = 0, Eby = 0, Ety = 0, Ely = 0, Ery = 0;
#define PF_QP(q)                                                                         \
  {                                                                                      \
    const T wB = T(QW<q>::wB), wT = T(QW<q>::wT), wL = T(QW<q>::wL), wR = T(QW<q>::wR);  \
    const T exx = (wB * Dbx + wT * Dtx) * ihx;                                           \
    const T eyy = (wL * Dly + wR * Dry) * ihy;                                           \
    const T exy = T(0.5) * ((wL * Dlx + wR * Drx) * ihy + (wB * Dby + wT * Dty) * ihx);  \
    T pxx, pyy, pxy, tl;                                                                 \
    if (NONLIN) {                                                                        \
      SpecLin<T> sl;                                                                     \
      spec_lin(exx, eyy, exy, sl);                                                       \
      if (sl.cs == 1) { pxx = exx; pyy = eyy; pxy = exy; }                               \
      else if (sl.cs == 0) { pxx = T(0); pyy = T(0); pxy = T(0); }                       \
      else { pxx = sl.e1 * sl.a; pyy = sl.e1 * sl.cc; pxy = sl.e1 * sl.b; }              \
      tl = exx + eyy;                                                                    \
    } else {                                                                             \
      const T lxx = (wB * Lbx + wT * Ltx) * ihx;                                         \
      const T lyy = (wL * Lly + wR * Lry) * ihy;                                         \
      const T lxy = T(0.5) * ((wL * Llx + wR * Lrx) * ihy + (wB * Lby + wT * Lty) * ihx);\
      SpecLin<T> sl;                                                                     \
      spec_lin(lxx, lyy, lxy, sl);                                                       \
      spec_dplus(sl, exx, eyy, exy, pxx, pyy, pxy);                                      \
      tl = lxx + lyy;                                                                    \
    }                                                                                    \
    const T dq = interp4<T, q>(dn[0], dn[1], dn[2], dn[3]);                              \
    const T om = T(1) - dq;                                                              \
    const T gq = om * om + eta;                                                          \
    const T kv = lam * ((tl > T(0)) ? gq : T(1)) * (exx + eyy);                          \
    const T m2 = twomu * (gq - T(1));                                                    \
    const T sxx = kv + m2 * pxx + twomu * exx;                                           \
    const T syy = kv + m2 * pyy + twomu * eyy;                                           \
    const T sxy = m2 * pxy + twomu * exy;                                                \
    Ebx += wB * sxx; Etx += wT * sxx; Elx += wL * sxy; Erx += wR * sxy;                  \
    Eby += wB * sxy; Ety += wT * sxy; Ely += wL * syy; Ery += wR * syy;                  \
  }
  PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
  const T sx = T(c.sx), sy = T(c.sy);
  Ebx *= sx; Etx *= sx; Elx *= sy; Erx *= sy;
  Eby *= sx; Ety *= sx; Ely *= sy; Ery *= sy;
  fx[0] = -Ebx - Elx; fx[1] = Ebx - Erx; fx[2] = Etx + Erx; fx[3] = Elx - Etx;
  fy[0] = -Eby - Ely; fy[1] = Eby - Ery; fy[2] = Ety + Ery; fy[3] = Ely - Ety;
}

// Diagonal of the spectral tangent at (lx, ly): the unit nodal value of
// corner a, component x, has strain (Nx, 0, Ny/2) and contributes
// sxx Nx + sxy Ny (component y: (0, Ny, Nx/2) -> syy Ny + sxy Nx).
template <class T>
__device__ inline void spectral_diag_element(const T (&dn)[4], const T (&lx)[4], const T (&ly)[4],
                                             const ElasCoef &c, T (&fx)[4], T (&fy)[4]) {
  const T Lbx = lx[1] - lx[0], Ltx = lx[2] - lx[3], Llx = lx[3] - lx[0], Lrx = lx[2] - lx[1];
  const T Lby = ly[1] - ly[0], Lty = ly[2] - ly[3], Lly = ly[3] - ly[0], Lry = ly[2] - ly[1];
  const T ihx = T(c.ihx), ihy = T(c.ihy), twomu = T(c.two_mu), lam = T(c.lam);
  const T wdet = T(c.sx) / T(c.ihx);
#pragma unroll
  for (int a = 0; a < 4; ++a) { fx[a] = 0; fy[a] = 0; }
#define PF_QP(q)                                                                         \
  {                                                                                      \
    const T wB = T(QW<q>::wB), wT = T(QW<q>::wT), wL = T(QW<q>::wL), wR = T(QW<q>::wR);  \
    const T lxx = (wB * Lbx + wT * Ltx) * ihx;                                           \
    const T lyy = (wL * Lly + wR * Lry) * ihy;                                           \
    const T lxy = T(0.5) * ((wL * Llx + wR * Lrx) * ihy + (wB * Lby + wT * Lty) * ihx);  \
    SpecLin<T> sl;                                                                       \
    spec_lin(lxx, lyy, lxy, sl);                                                         \
    const T dq = interp4<T, q>(dn[0], dn[1], dn[2], dn[3]);                              \
    const T om = T(1) - dq;                                                              \
    const T gq = om * om + T(c.eta);                                                     \
    const T kap = lam * ((lxx + lyy > T(0)) ? gq : T(1));                                \
    const T m2 = twomu * (gq - T(1));                                                    \
    const T Nx[4] = {-wB * ihx, wB * ihx, wT * ihx, -wT * ihx};                          \
    const T Ny[4] = {-wL * ihy, -wR * ihy, wR * ihy, wL * ihy};                          \
    for (int a = 0; a < 4; ++a) {                                                        \
      T pxx, pyy, pxy;                                                                   \
      spec_dplus(sl, Nx[a], T(0), T(0.5) * Ny[a], pxx, pyy, pxy);                        \
      const T sxx = kap * Nx[a] + m2 * pxx + twomu * Nx[a];                              \
      const T sxy = m2 * pxy + twomu * T(0.5) * Ny[a];                                   \
      fx[a] += wdet * (sxx * Nx[a] + sxy * Ny[a]);                                       \
      spec_dplus(sl, T(0), Ny[a], T(0.5) * Nx[a], pxx, pyy, pxy);                        \
      const T syy = kap * Ny[a] + m2 * pyy + twomu * Ny[a];                              \
      const T sxy2 = m2 * pxy + twomu * T(0.5) * Nx[a];                                  \
      fy[a] += wdet * (syy * Ny[a] + sxy2 * Nx[a]);                                      \
    }                                                                                    \
  }
  PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
}

// Phase operator sum [c_q N N^T + Gc l grad N grad N^T] w detJ applied to p.
template <class T>
__device__ inline void phase_element(const T (&p)[4], const T (&cq)[4], const PhaseCoef &c,
                                     T (&f)[4]) {
  const T Db = p[1] - p[0], Dt = p[2] - p[3], Dl = p[3] - p[0], Dr = p[2] - p[1];
  const T ihx = T(c.ihx), ihy = T(c.ihy), wdet = T(c.wdet), Gcl = T(c.Gcl);
  T Eb = 0, Et = 0, El = 0, Er = 0;
  f[0] = 0; f[1] = 0; f[2] = 0; f[3] = 0;
#define PF_QP(q)                                                                         \
  {                                                                                      \
    const T wB = T(QW<q>::wB), wT = T(QW<q>::wT), wL = T(QW<q>::wL), wR = T(QW<q>::wR);  \
    const T gx = (wB * Db + wT * Dt) * ihx;                                              \
    const T gy = (wL * Dl + wR * Dr) * ihy;                                              \
    Eb += wB * gx; Et += wT * gx; El += wL * gy; Er += wR * gy;                          \
    const T m = cq[q] * wdet * interp4<T, q>(p[0], p[1], p[2], p[3]);                    \
    f[0] += m * T(NW<q, 0>::v); f[1] += m * T(NW<q, 1>::v);                              \
    f[2] += m * T(NW<q, 2>::v); f[3] += m * T(NW<q, 3>::v);                              \
  }
  PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
  const T sx = T(c.sx) * Gcl, sy = T(c.sy) * Gcl;
  Eb *= sx; Et *= sx; El *= sy; Er *= sy;
  f[0] += -Eb - El; f[1] += Eb - Er; f[2] += Et + Er; f[3] += El - Et;
}

template <class T>
__device__ inline void phase_diag_element(const T (&cq)[4], const PhaseCoef &c, T (&f)[4]) {
  const T ihx2 = T(c.ihx * c.ihx), ihy2 = T(c.ihy * c.ihy), wdet = T(c.wdet), Gcl = T(c.Gcl);
  f[0] = 0; f[1] = 0; f[2] = 0; f[3] = 0;
#define PF_QP(q)                                                                         \
  {                                                                                      \
    const T wB = T(QW<q>::wB), wT = T(QW<q>::wT), wL = T(QW<q>::wL), wR = T(QW<q>::wR);  \
    const T nx2[4] = {wB * wB * ihx2, wB * wB * ihx2, wT * wT * ihx2, wT * wT * ihx2};    \
    const T ny2[4] = {wL * wL * ihy2, wR * wR * ihy2, wR * wR * ihy2, wL * wL * ihy2};    \
    const T n2[4] = {T(NW<q, 0>::v * NW<q, 0>::v), T(NW<q, 1>::v * NW<q, 1>::v),          \
                     T(NW<q, 2>::v * NW<q, 2>::v), T(NW<q, 3>::v * NW<q, 3>::v)};          \
    for (int a = 0; a < 4; ++a) f[a] += wdet * (cq[q] * n2[a] + Gcl * (nx2[a] + ny2[a])); \
  }
  PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
}

// ------------------------------------------------------- marching kernel
//
// Work item = (strip, chunk).  Lane L of a wave holds node column
// c = 62*strip - 1 + L and computes element column c - 1 (lane 0 computes
// none), so the wave owns node columns 62*strip .. 62*strip + 61 and each
// node is summed once: corner 0 of its own element plus, by one lane
// shuffle, corner 1 of the left neighbour's.  The chunk owns CH node rows;
// all CH + 2 node rows and CH + 1 element rows of a work item are loaded
// into registers before any element is computed, so a wave has its whole
// item in flight at once.
//
// An Op provides:
//   T, Node, Elem, NF (accumulated components), NR (reduction values)
//   Node load(i, j)          raw node values, zero outside the grid
//   void fin(Node &)         turn raw values into operand values (CG: p = z + beta p_old)
//   Elem eload(ie, je)       element data (flags, coefficients); .active = 0 if none
//   void element(bl, br, tr, tl, const Elem&, T f[NF][4])
//   void store(i, j, const T v[NF], const Node &n, double red[NR])
//   static Node shfl_up(const Node&)   lane L receives lane L-1's value

constexpr int CSTRIP = 62;

template <int CH, class Op>
struct Item {
  typename Op::Node R[CH + 2];
  typename Op::Elem El[CH + 1];
  typename Op::Own O[CH];   // the lane's stored column, rows j0 .. j0+CH-1
};

template <int CH, class Op>
__device__ inline void item_load(const Op &op, const Grid &g, const March &ms, int w, int lane,
                                 Item<CH, Op> &it) {
  const int strip = w % ms.nstrips;
  const int chunk = w / ms.nstrips;
  const int c = strip * CSTRIP - 1 + lane;
  const int j0 = chunk * CH;
#pragma unroll
  for (int r = 0; r < CH + 2; ++r) it.R[r] = op.load(c, j0 - 1 + r);
#pragma unroll
  for (int r = 0; r < CH + 1; ++r)
    it.El[r] = (lane > 0) ? op.eload(c - 1, j0 - 1 + r) : typename Op::Elem{};
#pragma unroll
  for (int r = 0; r < CH; ++r) it.O[r] = op.load_own(c - 1, j0 + r);
}

template <int CH, class Op>
__device__ inline void item_compute(const Op &op, const Grid &g, const March &ms, int w,
                                    int lane, Item<CH, Op> &it, double *red) {
  using T = typename Op::T;
  using Node = typename Op::Node;
  constexpr int NF = Op::NF;
  const int strip = w % ms.nstrips;
  const int chunk = w / ms.nstrips;
  const int n = strip * CSTRIP - 2 + lane;          // node column this lane stores
  const int j0 = chunk * CH;
  const bool own_col = lane >= 2 && n >= 0 && n <= g.nx;
#pragma unroll
  for (int r = 0; r < CH + 2; ++r) op.fin(it.R[r]);
  Node br = it.R[0];
  Node bl = Op::shfl_up(br);
  T c2[NF], c3[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) { c2[k] = T(0); c3[k] = T(0); }
#pragma unroll
  for (int r = 0; r < CH + 1; ++r) {
    const int je = j0 - 1 + r;
    const Node tr = it.R[r + 1];
    const Node tl = Op::shfl_up(tr);
    T f[NF][4];
    op.element(bl, br, tr, tl, it.El[r], f);
    T out[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const T A = f[k][1] + c2[k];
      const T Al = lane_up(A);
      out[k] = f[k][0] + c3[k] + Al;
      c3[k] = f[k][3];
      c2[k] = f[k][2];
    }
    if (r >= 1 && own_col && je <= g.ny) op.store(n, je, out, bl, it.O[r - 1], red);
    bl = tl;
    br = tr;
  }
}

// XCD-aware block order: workgroups are dispatched to the 8 dies round
// robin, so block b runs on die b % 8.  Renumbering the blocks so that each
// die owns a contiguous range makes the work items of one die a horizontal
// band of the mesh, and the node rows shared by vertically adjacent chunks
// are then re-read from that die's own L2.  The map is a bijection of
// [0, nb).
constexpr int kXcd = 8;
__device__ inline int xcd_block(int b, int nb) {
  const int x = b % kXcd, k = b / kXcd;
  const int per = nb / kXcd, rem = nb % kXcd;
  return x * per + min(x, rem) + k;
}

// ------------------------------------------------------------ LDS tiles
//
// One block per tile of kTile x kTile owned nodes.  The block stages the
// (kTile+2)^2 nodes around the tile in LDS (after fin), each of its 256
// threads computes one of the (kTile+1)^2 elements touching the tile and
// writes the element's corner values to LDS, and each owned node sums the
// four corner values of its elements.  Compared with column marching the
// dependency chain of a wave is one element instead of a column of them,
// at the price of computing the ring of elements around the tile in both
// neighbouring tiles.

constexpr int kTile = 15;
constexpr int kTileN = kTile + 2;   // staged nodes per side
constexpr int kTileE = kTile + 1;   // elements per side (kTileE^2 == TPB)
constexpr int kTileLoads = (kTileN * kTileN + TPB - 1) / TPB;

template <class Op>
struct TileLds {
  typename Op::Node node[kTileN * kTileN];
  typename Op::T f[Op::NF][4][kTileE * kTileE];
};

template <class Op>
struct TileRegs {
  typename Op::Node n[kTileLoads];
  typename Op::Elem e;
  typename Op::Own o;   // the thread's owned node
};

template <class Op>
__device__ inline void tile_load(const Op &op, const March &ms, int tile, TileRegs<Op> &tr) {
  static_assert(kTileE * kTileE == TPB, "one element per thread");
  const int i0 = (tile % ms.nstrips) * kTile - 1, j0 = (tile / ms.nstrips) * kTile - 1;
  if constexpr (HasFast<Op>::value) {
    const Grid &g = op.g;
    if (box_inside(g, i0, j0, kTileN)) {
      const unsigned row = unsigned(g.nx) + 1u, base = unsigned(j0) * row + unsigned(i0);
#pragma unroll
      for (int r = 0; r < kTileLoads; ++r) {
        const unsigned k = threadIdx.x + r * TPB;
        if (k < kTileN * kTileN) tr.n[r] = op.load_fast(base + (k / kTileN) * row + k % kTileN);
      }
      tr.e = op.eload_fast(unsigned(j0) * unsigned(g.nx) + unsigned(i0) +
                           (threadIdx.x / kTileE) * unsigned(g.nx) + threadIdx.x % kTileE);
      if (threadIdx.x < kTile * kTile)
        tr.o = op.load_own_fast(base + row + 1u + (threadIdx.x / kTile) * row +
                                threadIdx.x % kTile);
      return;
    }
  }
#pragma unroll
  for (int r = 0; r < kTileLoads; ++r) {
    const int k = threadIdx.x + r * TPB;
    if (k < kTileN * kTileN) tr.n[r] = op.load(i0 + k % kTileN, j0 + k / kTileN);
  }
  tr.e = op.eload(i0 + threadIdx.x % kTileE, j0 + threadIdx.x / kTileE);
  if (threadIdx.x < kTile * kTile)
    tr.o = op.load_own(i0 + 1 + threadIdx.x % kTile, j0 + 1 + threadIdx.x / kTile);
}

template <class Op>
__device__ inline void tile_compute(const Op &op, const Grid &g, const March &ms, int tile,
                                    TileRegs<Op> &tr, TileLds<Op> &sm, double *red) {
  using T = typename Op::T;
  constexpr int NF = Op::NF;
#pragma unroll
  for (int r = 0; r < kTileLoads; ++r) {
    const int k = threadIdx.x + r * TPB;
    if (k < kTileN * kTileN) {
      op.fin(tr.n[r]);
      sm.node[k] = tr.n[r];
    }
  }
  __syncthreads();
  {
    // element (el, ej) of the tile: corner 0 is staged node (el, ej)
    const int el = threadIdx.x % kTileE, ej = threadIdx.x / kTileE;
    const int b = ej * kTileN + el;
    T f[NF][4];
    op.element(sm.node[b], sm.node[b + 1], sm.node[b + kTileN + 1], sm.node[b + kTileN], tr.e, f);
#pragma unroll
    for (int q = 0; q < NF; ++q)
#pragma unroll
      for (int a = 0; a < 4; ++a) sm.f[q][a][threadIdx.x] = f[q][a];
  }
  __syncthreads();
  if (threadIdx.x < kTile * kTile) {
    // owned node (li, lj) is staged node (li+1, lj+1): corner 2 of element
    // (li, lj), 3 of (li+1, lj), 1 of (li, lj+1), 0 of (li+1, lj+1)
    const int li = threadIdx.x % kTile, lj = threadIdx.x / kTile;
    const int i = (tile % ms.nstrips) * kTile + li, j = (tile / ms.nstrips) * kTile + lj;
    if (i <= g.nx && j <= g.ny) {
      const int e = lj * kTileE + li;
      T out[NF];
#pragma unroll
      for (int q = 0; q < NF; ++q)
        out[q] = sm.f[q][2][e] + sm.f[q][3][e + 1] + sm.f[q][1][e + kTileE] +
                 sm.f[q][0][e + kTileE + 1];
      op.store(i, j, out, sm.node[(lj + 1) * kTileN + li + 1], tr.o, red);
    }
  }
  __syncthreads();   // the LDS is reused by the block's next tile
}

template <int CH, class Op>
__device__ inline void march_items(const Op &op, const Grid &g, const March &ms, int wfirst,
                                   int wstride, double *red) {
  const int lane = threadIdx.x & 63;
  const int nw = ms.nstrips * ms.nchunks;
  for (int w = wfirst; w < nw; w += wstride) {
    Item<CH, Op> it;
    item_load<CH>(op, g, ms, w, lane, it);
    item_compute<CH>(op, g, ms, w, lane, it, red);
  }
}

// Generic marching kernel; an op with NR > 0 writes block partials to `part`.
template <int CH, class Op>
__global__ void __launch_bounds__(TPB) k_march(Op op, Grid g, March ms, double *part) {
  constexpr int NRR = Op::NR > 0 ? Op::NR : 1;
  double red[NRR];
#pragma unroll
  for (int k = 0; k < NRR; ++k) red[k] = 0.0;
  if constexpr (CH == 1) {
    __shared__ TileLds<Op> sm;
    const int nt = ms.nstrips * ms.nchunks;
    for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
      TileRegs<Op> tr;
      tile_load(op, ms, t, tr);
      tile_compute(op, g, ms, t, tr, sm, red);
    }
  } else {
    march_items<CH>(op, g, ms, xcd_block(blockIdx.x, gridDim.x) * WPB + (threadIdx.x >> 6),
                    gridDim.x * WPB, red);
  }
  if (Op::NR > 0) block_partial<NRR>(red, part);
}

int march_blocks(const March &m) {
  const int nw = m.nstrips * m.nchunks;
  int b = m.ch == 1 ? nw : (nw + WPB - 1) / WPB;
  return b > kPMax ? kPMax : b;
}

// Element data: flags byte for the tangent, 4 QP coefficients for the phase.
struct ElemFlags { uint8_t bits; uint8_t active; };
template <class T> struct ElemCoef { T c[4]; uint8_t active; };
struct ElemH { double H[4]; uint8_t active; };
struct ElemNone { uint8_t active; };

// ---- elasticity tangent (optionally fused with the CG direction update
//      p = z + beta p_old; the fused op also accumulates p.q)
//
// Node record: the input vector (px, py) and the damage d, plus only what
// the variant reads besides: the old direction ox, oy (fused CG apply) and
// the linearisation point lx, ly (spectral split).  The records are staged
// in LDS, so unused fields would cost LDS and occupancy.
template <class T, bool FUSED, int SPL> struct TanNode { T px, py, d; };
template <class T> struct TanNode<T, true, 0> { T px, py, d, ox, oy; };
template <class T> struct TanNode<T, false, 1> { T px, py, d, lx, ly; };
template <class T> struct TanNode<T, true, 1> { T px, py, d, ox, oy, lx, ly; };

template <class TT, bool FUSED, bool MASK, int SPL = 0>
struct OpTangent {
  using T = TT;
  using Elem = ElemFlags;
  static constexpr int NF = 2;
  static constexpr int NR = FUSED ? 1 : 0;
  // raw: px, py = z; ox, oy = p_old (fused only); fin: p = z + beta p_old;
  // lx, ly = linearisation point (spectral split only)
  using Node = TanNode<T, FUSED, SPL>;
  Grid g; ElasCoef c;
  const T *d; const uint8_t *qflag; const uint8_t *eact; const uint8_t *nflag;
  const T *z; const T *pold; T *pnew; T *q;
  T beta;
  const T *ulin;

  __device__ Node load(int i, int j) const {
    Node n{};
    if (node_exists(g, i, j)) {
      const int k = i + j * (g.nx + 1);
      n.px = z[k];
      n.py = z[k + g.N];
      if constexpr (FUSED) {
        n.ox = pold[k];
        n.oy = pold[k + g.N];
      }
      if constexpr (SPL == 1) {
        n.lx = ulin[k];
        n.ly = ulin[k + g.N];
      }
      n.d = d[k];
    }
    return n;
  }
  __device__ void fin(Node &n) const {
    if constexpr (FUSED) {
      n.px += beta * n.ox;
      n.py += beta * n.oy;
    }
  }
  // operator data only (no CG vectors): d and, for the spectral split, the
  // linearisation point
  __device__ Node load_aux(int i, int j) const {
    Node n{};
    if (node_exists(g, i, j)) {
      const int k = i + j * (g.nx + 1);
      n.d = d[k];
      if constexpr (SPL == 1) {
        n.lx = ulin[k];
        n.ly = ulin[k + g.N];
      }
    }
    return n;
  }
  __device__ Node load_fast(unsigned k) const {
    Node n;
    const unsigned o = k * unsigned(sizeof(T));
    n.px = ldo(z, o);
    n.py = ldo(z + g.N, o);
    if constexpr (FUSED) {
      n.ox = ldo(pold, o);
      n.oy = ldo(pold + g.N, o);
    }
    if constexpr (SPL == 1) {
      n.lx = ldo(ulin, o);
      n.ly = ldo(ulin + g.N, o);
    }
    n.d = ldo(d, o);
    return n;
  }
  __device__ Node load_aux_fast(unsigned k) const {
    Node n{};
    const unsigned o = k * unsigned(sizeof(T));
    n.d = ldo(d, o);
    if constexpr (SPL == 1) {
      n.lx = ldo(ulin, o);
      n.ly = ldo(ulin + g.N, o);
    }
    return n;
  }
  // both bytes are loaded before either is used (no dependent round trip)
  __device__ Elem eload_fast(unsigned e) const {
    Elem el;
    el.bits = ldo(qflag, e);
    el.active = eact == nullptr ? uint8_t(1) : ldo(eact, e);   // nonzero = active
    return el;
  }
  __device__ OwnFlag load_own_fast(unsigned k) const {
    return OwnFlag{nflag == nullptr ? uint8_t(0) : ldo(nflag, k)};
  }
  __device__ void set_u(Node &n, const T (&u)[2]) const {
    n.px = u[0];
    n.py = u[1];
  }
  __device__ void get_u(const Node &n, T (&u)[2]) const {
    u[0] = n.px;
    u[1] = n.py;
  }
  __device__ bool masked(int k, int comp) const {
    return (nflag[k] & (comp == 0 ? NF_UX : NF_UY)) != 0;
  }
  using Own = OwnFlag;
  __device__ Own load_own(int i, int j) const { return load_flag(nflag, g, i, j); }
  static __device__ bool masked_own(const Own &o, int q) {
    return (o.nf & (q == 0 ? NF_UX : NF_UY)) != 0;
  }
  __device__ Elem eload(int ie, int je) const {
    Elem e{0, 0};
    if (elem_exists(g, ie, je, eact)) {
      e.bits = qflag[ie + je * g.nx];
      e.active = 1;
    }
    return e;
  }
  static __device__ Node shfl_up(const Node &n) {
    Node m{};   // the old direction is not passed on: fin has been applied
    m.px = lane_up(n.px);
    m.py = lane_up(n.py);
    m.d = lane_up(n.d);
    if constexpr (SPL == 1) {
      m.lx = lane_up(n.lx);
      m.ly = lane_up(n.ly);
    }
    return m;
  }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, T (&f)[2][4]) const {
    if (!e.active) {
#pragma unroll
      for (int a = 0; a < 4; ++a) { f[0][a] = 0; f[1][a] = 0; }
      return;
    }
    const T ux[4] = {n0.px, n1.px, n2.px, n3.px};
    const T uy[4] = {n0.py, n1.py, n2.py, n3.py};
    const T dn[4] = {n0.d, n1.d, n2.d, n3.d};
    if constexpr (SPL == 1) {
      const T lx[4] = {n0.lx, n1.lx, n2.lx, n3.lx};
      const T ly[4] = {n0.ly, n1.ly, n2.ly, n3.ly};
      spectral_element<T, false>(ux, uy, dn, lx, ly, c, f[0], f[1]);
    } else {
      elastic_element<T, false>(ux, uy, dn, e.bits, c, f[0], f[1]);
    }
  }
  __device__ void store(int i, int j, const T (&v)[2], const Node &n, const Own &o,
                        double *red) const {
    const int k = i + j * (g.nx + 1);
    T qx = v[0], qy = v[1];
    if (MASK) {
      if (o.nf & NF_UX) qx = T(0);
      if (o.nf & NF_UY) qy = T(0);
    }
    q[k] = qx;
    q[k + g.N] = qy;
    if (FUSED) {
      pnew[k] = n.px;
      pnew[k + g.N] = n.py;
      red[0] += double(n.px) * double(qx) + double(n.py) * double(qy);
    }
  }
};

// ---- phase operator (K_dd, augmented block), optionally fused
template <class TT, bool FUSED, bool MASK>
struct OpPhase {
  using T = TT;
  using Elem = ElemCoef<TT>;
  static constexpr int NF = 1;
  static constexpr int NR = FUSED ? 1 : 0;
  struct Node { T p, o; };
  Grid g; PhaseCoef c;
  const T *coef; const uint8_t *eact; const uint8_t *nflag;
  const T *z; const T *pold; T *pnew; T *q;
  T beta;

  __device__ Node load(int i, int j) const {
    Node n{T(0), T(0)};
    if (node_exists(g, i, j)) {
      const int k = i + j * (g.nx + 1);
      n.p = z[k];
      if (FUSED) n.o = pold[k];
    }
    return n;
  }
  __device__ void fin(Node &n) const {
    if (FUSED) n.p += beta * n.o;
  }
  __device__ Node load_aux(int, int) const { return Node{T(0), T(0)}; }
  __device__ Node load_fast(unsigned k) const {
    const unsigned o = k * unsigned(sizeof(T));
    Node n{ldo(z, o), T(0)};
    if (FUSED) n.o = ldo(pold, o);
    return n;
  }
  __device__ Node load_aux_fast(unsigned) const { return Node{T(0), T(0)}; }
  __device__ Elem eload_fast(unsigned e) const {
    Elem el;
    const unsigned o = e * unsigned(sizeof(T));
#pragma unroll
    for (int q = 0; q < 4; ++q) el.c[q] = ldo(coef + q * g.E, o);
    el.active = eact == nullptr ? uint8_t(1) : ldo(eact, e);   // nonzero = active
    return el;
  }
  __device__ OwnFlag load_own_fast(unsigned k) const {
    return OwnFlag{nflag == nullptr ? uint8_t(0) : ldo(nflag, k)};
  }
  __device__ void set_u(Node &n, const T (&u)[1]) const { n.p = u[0]; }
  __device__ void get_u(const Node &n, T (&u)[1]) const { u[0] = n.p; }
  __device__ bool masked(int k, int) const { return (nflag[k] & NF_D) != 0; }
  using Own = OwnFlag;
  __device__ Own load_own(int i, int j) const { return load_flag(nflag, g, i, j); }
  static __device__ bool masked_own(const Own &o, int) { return (o.nf & NF_D) != 0; }
  __device__ Elem eload(int ie, int je) const {
    Elem e{};
    if (elem_exists(g, ie, je, eact)) {
      const int el = ie + je * g.nx;
      e.c[0] = coef[el];
      e.c[1] = coef[el + g.E];
      e.c[2] = coef[el + 2 * g.E];
      e.c[3] = coef[el + 3 * g.E];
      e.active = 1;
    }
    return e;
  }
  static __device__ Node shfl_up(const Node &n) { return Node{lane_up(n.p), T(0)}; }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, T (&f)[1][4]) const {
    if (!e.active) {
      f[0][0] = f[0][1] = f[0][2] = f[0][3] = T(0);
      return;
    }
    const T p[4] = {n0.p, n1.p, n2.p, n3.p};
    const T cq[4] = {e.c[0], e.c[1], e.c[2], e.c[3]};
    phase_element<T>(p, cq, c, f[0]);
  }
  __device__ void store(int i, int j, const T (&v)[1], const Node &n, const Own &o,
                        double *red) const {
    const int k = i + j * (g.nx + 1);
    T qv = v[0];
    if (MASK && (o.nf & NF_D)) qv = T(0);
    q[k] = qv;
    if (FUSED) {
      pnew[k] = n.p;
      red[0] += double(n.p) * double(qv);
    }
  }
};

// ---- internal force (FP64, nonlinear split stress); reduces ||R||^2 over
//      free DOFs when a node-flag array is given
template <int SPL>
struct OpForce {
  using T = double;
  using Elem = ElemNone;
  static constexpr int NF = 2;
  static constexpr int NR = 1;
  struct Node { double ux, uy, d; };
  Grid g; ElasCoef c;
  const double *u; const double *dd; const uint8_t *eact; const uint8_t *nflag;
  double *R; double sign;

  __device__ Node load(int i, int j) const {
    Node n{0.0, 0.0, 0.0};
    if (node_exists(g, i, j)) {
      const int k = i + j * (g.nx + 1);
      n.ux = u[k]; n.uy = u[k + g.N]; n.d = dd[k];
    }
    return n;
  }
  __device__ void fin(Node &) const {}
  __device__ Elem eload(int ie, int je) const {
    return Elem{uint8_t(elem_exists(g, ie, je, eact) ? 1 : 0)};
  }
  static __device__ Node shfl_up(const Node &n) {
    return Node{lane_up(n.ux), lane_up(n.uy), lane_up(n.d)};
  }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, double (&f)[2][4]) const {
    if (!e.active) {
#pragma unroll
      for (int a = 0; a < 4; ++a) { f[0][a] = 0; f[1][a] = 0; }
      return;
    }
    const double ux[4] = {n0.ux, n1.ux, n2.ux, n3.ux};
    const double uy[4] = {n0.uy, n1.uy, n2.uy, n3.uy};
    const double dn[4] = {n0.d, n1.d, n2.d, n3.d};
    if (SPL == 1) spectral_element<double, true>(ux, uy, dn, ux, uy, c, f[0], f[1]);
    else elastic_element<double, true>(ux, uy, dn, 0u, c, f[0], f[1]);
  }
  using Own = OwnFlag;
  __device__ Own load_own(int i, int j) const { return load_flag(nflag, g, i, j); }
  __device__ void store(int i, int j, const double (&v)[2], const Node &, const Own &o,
                        double *red) const {
    const int k = i + j * (g.nx + 1);
    double rx = v[0], ry = v[1];
    if (o.nf & NF_UX) rx = 0.0;
    if (o.nf & NF_UY) ry = 0.0;
    R[k] = sign * rx;
    R[k + g.N] = sign * ry;
    red[0] += rx * rx + ry * ry;
  }
};

// ---- phase residual R_d = K_dd(H) d - b(H) (FP64); reduces ||R_d||^2 and
//      ||b||^2 over free nodes
struct OpPhaseRes {
  using T = double;
  using Elem = ElemH;
  static constexpr int NF = 2;   // [0] = K_dd d - b, [1] = b
  static constexpr int NR = 2;
  struct Node { double d; };
  Grid g; PhaseCoef c;
  const double *H; const double *dd; const uint8_t *eact; const uint8_t *nflag;
  double *R; double sign;

  __device__ Node load(int i, int j) const {
    Node n{0.0};
    if (node_exists(g, i, j)) n.d = dd[i + j * (g.nx + 1)];
    return n;
  }
  __device__ void fin(Node &) const {}
  __device__ Elem eload(int ie, int je) const {
    Elem e{};
    if (elem_exists(g, ie, je, eact)) {
      const int el = ie + je * g.nx;
      e.H[0] = H[el];
      e.H[1] = H[el + g.E];
      e.H[2] = H[el + 2 * g.E];
      e.H[3] = H[el + 3 * g.E];
      e.active = 1;
    }
    return e;
  }
  static __device__ Node shfl_up(const Node &n) { return Node{lane_up(n.d)}; }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, double (&f)[2][4]) const {
    if (!e.active) {
#pragma unroll
      for (int a = 0; a < 4; ++a) { f[0][a] = 0; f[1][a] = 0; }
      return;
    }
    const double *Hq = e.H;
    const double cq[4] = {c.Gc_l + 2.0 * Hq[0], c.Gc_l + 2.0 * Hq[1], c.Gc_l + 2.0 * Hq[2],
                          c.Gc_l + 2.0 * Hq[3]};
    const double p[4] = {n0.d, n1.d, n2.d, n3.d};
    phase_element<double>(p, cq, c, f[0]);
    // b_a = sum_q 2 H_q N_a(q) w detJ
    const double w2 = 2.0 * c.wdet;
    f[1][0] = w2 * (NW<0, 0>::v * Hq[0] + NW<1, 0>::v * Hq[1] + NW<2, 0>::v * Hq[2] + NW<3, 0>::v * Hq[3]);
    f[1][1] = w2 * (NW<0, 1>::v * Hq[0] + NW<1, 1>::v * Hq[1] + NW<2, 1>::v * Hq[2] + NW<3, 1>::v * Hq[3]);
    f[1][2] = w2 * (NW<0, 2>::v * Hq[0] + NW<1, 2>::v * Hq[1] + NW<2, 2>::v * Hq[2] + NW<3, 2>::v * Hq[3]);
    f[1][3] = w2 * (NW<0, 3>::v * Hq[0] + NW<1, 3>::v * Hq[1] + NW<2, 3>::v * Hq[2] + NW<3, 3>::v * Hq[3]);
#pragma unroll
    for (int a = 0; a < 4; ++a) f[0][a] -= f[1][a];
  }
  using Own = OwnFlag;
  __device__ Own load_own(int i, int j) const { return load_flag(nflag, g, i, j); }
  __device__ void store(int i, int j, const double (&v)[2], const Node &, const Own &o,
                        double *red) const {
    const int k = i + j * (g.nx + 1);
    double r = v[0], b = v[1];
    if (o.nf & NF_D) { r = 0.0; b = 0.0; }
    R[k] = sign * r;
    red[0] += r * r;
    red[1] += b * b;
  }
};

// ---- AT1 residual with the penalty (Section 2, eq_evolution_equation;
//      F_d of Section 3.2 with w = d): per quadrature point
//      N [2 Psi+ d - 2 Psi+ + Gc/(c_w l) + gamma <d - d_{n-1}>_-]
//      + (2 Gc l / c_w) grad N . grad d.  c.Gc_l holds Gc/(c_w l) and c.Gcl
//      2 Gc l / c_w in an AT1 context.  [0] = F_d, [1] = sum 2 Psi+ N.
struct OpPhaseResAT1 {
  using T = double;
  using Elem = ElemH;
  static constexpr int NF = 2;
  static constexpr int NR = 2;
  struct Node { double d, dp; };
  Grid g; PhaseCoef c;
  const double *psi; const double *dd; const double *dprev; const uint8_t *eact;
  const uint8_t *nflag;
  double *R; double sign; double gamma;

  __device__ Node load(int i, int j) const {
    Node n{0.0, 0.0};
    if (node_exists(g, i, j)) {
      const int k = i + j * (g.nx + 1);
      n.d = dd[k];
      n.dp = dprev[k];
    }
    return n;
  }
  __device__ void fin(Node &) const {}
  __device__ Elem eload(int ie, int je) const {
    Elem e{};
    if (elem_exists(g, ie, je, eact)) {
      const int el = ie + je * g.nx;
      e.H[0] = psi[el];
      e.H[1] = psi[el + g.E];
      e.H[2] = psi[el + 2 * g.E];
      e.H[3] = psi[el + 3 * g.E];
      e.active = 1;
    }
    return e;
  }
  static __device__ Node shfl_up(const Node &n) { return Node{lane_up(n.d), lane_up(n.dp)}; }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, double (&f)[2][4]) const {
    if (!e.active) {
#pragma unroll
      for (int a = 0; a < 4; ++a) { f[0][a] = 0; f[1][a] = 0; }
      return;
    }
    const double *Pq = e.H;
    const double cq[4] = {2.0 * Pq[0], 2.0 * Pq[1], 2.0 * Pq[2], 2.0 * Pq[3]};
    const double p[4] = {n0.d, n1.d, n2.d, n3.d};
    phase_element<double>(p, cq, c, f[0]);
    // QP source Gc/(c_w l) + gamma min(d_q - d_{n-1,q}, 0) - 2 Psi+_q
    const double pp[4] = {n0.dp, n1.dp, n2.dp, n3.dp};
    double sq[4];
    sq[0] = interp4<double, 0>(p[0], p[1], p[2], p[3]) - interp4<double, 0>(pp[0], pp[1], pp[2], pp[3]);
    sq[1] = interp4<double, 1>(p[0], p[1], p[2], p[3]) - interp4<double, 1>(pp[0], pp[1], pp[2], pp[3]);
    sq[2] = interp4<double, 2>(p[0], p[1], p[2], p[3]) - interp4<double, 2>(pp[0], pp[1], pp[2], pp[3]);
    sq[3] = interp4<double, 3>(p[0], p[1], p[2], p[3]) - interp4<double, 3>(pp[0], pp[1], pp[2], pp[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      sq[q] = c.Gc_l + gamma * (sq[q] < 0.0 ? sq[q] : 0.0) - 2.0 * Pq[q];
    const double w = c.wdet, w2 = 2.0 * c.wdet;
#define PF_NA(a)                                                                              \
  f[0][a] += w * (NW<0, a>::v * sq[0] + NW<1, a>::v * sq[1] + NW<2, a>::v * sq[2] +          \
                  NW<3, a>::v * sq[3]);                                                       \
  f[1][a] = w2 * (NW<0, a>::v * Pq[0] + NW<1, a>::v * Pq[1] + NW<2, a>::v * Pq[2] +          \
                  NW<3, a>::v * Pq[3]);
    PF_NA(0) PF_NA(1) PF_NA(2) PF_NA(3)
#undef PF_NA
  }
  using Own = OwnFlag;
  __device__ Own load_own(int i, int j) const { return load_flag(nflag, g, i, j); }
  __device__ void store(int i, int j, const double (&v)[2], const Node &, const Own &o,
                        double *red) const {
    const int k = i + j * (g.nx + 1);
    double r = v[0], b = v[1];
    if (o.nf & NF_D) { r = 0.0; b = 0.0; }
    R[k] = sign * r;
    red[0] += r * r;
    red[1] += b * b;
  }
};

// ---- Jacobi diagonals (inverse, 0 on fixed DOFs)
template <class TT, int SPL = 0>
struct OpTangentDiag {
  using T = TT;
  using Elem = ElemFlags;
  static constexpr int NF = 2;
  static constexpr int NR = 0;
  struct Node { T d, lx, ly; };
  Grid g; ElasCoef c;
  const T *d; const uint8_t *qflag; const uint8_t *eact; const uint8_t *nflag; T *Dinv;
  const T *ulin;
  __device__ Node load(int i, int j) const {
    Node n{T(0), T(0), T(0)};
    if (node_exists(g, i, j)) {
      const int k = i + j * (g.nx + 1);
      n.d = d[k];
      if (SPL == 1) {
        n.lx = ulin[k];
        n.ly = ulin[k + g.N];
      }
    }
    return n;
  }
  __device__ void fin(Node &) const {}
  __device__ Elem eload(int ie, int je) const {
    Elem e{0, 0};
    if (elem_exists(g, ie, je, eact)) {
      e.bits = qflag[ie + je * g.nx];
      e.active = 1;
    }
    return e;
  }
  static __device__ Node shfl_up(const Node &n) {
    return Node{lane_up(n.d), SPL == 1 ? lane_up(n.lx) : T(0),
                SPL == 1 ? lane_up(n.ly) : T(0)};
  }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, T (&f)[2][4]) const {
    if (!e.active) {
#pragma unroll
      for (int a = 0; a < 4; ++a) { f[0][a] = 0; f[1][a] = 0; }
      return;
    }
    const T dn[4] = {n0.d, n1.d, n2.d, n3.d};
    if (SPL == 1) {
      const T lx[4] = {n0.lx, n1.lx, n2.lx, n3.lx};
      const T ly[4] = {n0.ly, n1.ly, n2.ly, n3.ly};
      spectral_diag_element<T>(dn, lx, ly, c, f[0], f[1]);
    } else {
      elastic_diag_element<T>(dn, e.bits, c, f[0], f[1]);
    }
  }
  using Own = OwnFlag;
  __device__ Own load_own(int i, int j) const { return load_flag(nflag, g, i, j); }
  __device__ void store(int i, int j, const T (&v)[2], const Node &, const Own &o,
                        double *) const {
    const int k = i + j * (g.nx + 1);
    Dinv[k] = ((o.nf & NF_UX) || !(v[0] > T(0))) ? T(0) : T(1) / v[0];
    Dinv[k + g.N] = ((o.nf & NF_UY) || !(v[1] > T(0))) ? T(0) : T(1) / v[1];
  }
};

template <class TT>
struct OpPhaseDiag {
  using T = TT;
  using Elem = ElemCoef<TT>;
  static constexpr int NF = 1;
  static constexpr int NR = 0;
  struct Node { T dummy; };
  Grid g; PhaseCoef c;
  const T *coef; const uint8_t *eact; const uint8_t *nflag; T *Dinv;
  int absdiag;   // 1: D = |diag| (SPD for an indefinite operator), 1 where it is 0
  __device__ Node load(int, int) const { return Node{T(0)}; }
  __device__ void fin(Node &) const {}
  __device__ Elem eload(int ie, int je) const {
    Elem e{};
    if (elem_exists(g, ie, je, eact)) {
      const int el = ie + je * g.nx;
      e.c[0] = coef[el];
      e.c[1] = coef[el + g.E];
      e.c[2] = coef[el + 2 * g.E];
      e.c[3] = coef[el + 3 * g.E];
      e.active = 1;
    }
    return e;
  }
  static __device__ Node shfl_up(const Node &n) { return n; }
  __device__ void element(const Node &, const Node &, const Node &, const Node &,
                          const Elem &e, T (&f)[1][4]) const {
    if (!e.active) {
      f[0][0] = f[0][1] = f[0][2] = f[0][3] = T(0);
      return;
    }
    const T cq[4] = {e.c[0], e.c[1], e.c[2], e.c[3]};
    phase_diag_element<T>(cq, c, f[0]);
  }
  using Own = OwnFlag;
  __device__ Own load_own(int i, int j) const { return load_flag(nflag, g, i, j); }
  __device__ void store(int i, int j, const T (&v)[1], const Node &, const Own &o,
                        double *) const {
    const int k = i + j * (g.nx + 1);
    if (absdiag) {
      const T a = v[0] < T(0) ? -v[0] : v[0];
      Dinv[k] = (o.nf & NF_D) ? T(0) : (a > T(0) ? T(1) / a : T(1));
    } else {
      Dinv[k] = ((o.nf & NF_D) || !(v[0] > T(0))) ? T(0) : T(1) / v[0];
    }
  }
};

template <class Op>
hipError_t launch_march(hipStream_t s, const Op &op, const Grid &g, const March &m,
                        double *part) {
  const dim3 grid(march_blocks(m)), block(TPB);
  switch (m.ch) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_march<1, Op>), grid, block, 0, s, op, g, m, part); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_march<2, Op>), grid, block, 0, s, op, g, m, part); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_march<4, Op>), grid, block, 0, s, op, g, m, part); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_march<8, Op>), grid, block, 0, s, op, g, m, part); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Finalise NV block partials into scal[slot..slot+NV) (one block).
template <int NV>
__global__ void __launch_bounds__(TPB) k_finalize(const double *part, int np, double *scal,
                                                  int slot) {
  double s[NV];
  block_sum<NV>(part, np, s);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) scal[slot + k] = s[k];
  }
}

template <class Op, int NV>
hipError_t launch_march_reduce(hipStream_t s, const Op &op, const Grid &g, const March &m,
                               RedScratch rs, int slot) {
  const int nb = march_blocks(m);
  hipError_t e = launch_march(s, op, g, m, rs.partR);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_finalize<NV>), dim3(1), dim3(TPB), 0, s, rs.partR, nb,
                     rs.scal, slot);
  return hipGetLastError();
}

// ------------------------------------------------- two-kernel CG (FP32)
//
// Standard PCG with two kernels per iteration, used for the FP32 inner
// solves (its recurrences keep their convergence rate at FP32 rounding,
// where the single-reduction form below loses about a fifth).
// Iteration k = apply kernel A_k then vector kernel B_k.
//   A_k: reduce B_{k-1}'s partials -> rz_k, rr_k; decide done; beta =
//        rz_k / rz_{k-1}; p = z + beta p_old; q = A p; partials p.q.
//   B_k: reduce A_k's partials -> pq; alpha = rz_k / pq; x += alpha p;
//        r -= alpha q; z = D^-1 r; partials r.z, r.r.
// Block 0 of each kernel records its scalars in its own half of CgState.

template <class T>
__global__ void __launch_bounds__(TPB) k_cg_init(int n, T *x, T *r, T *z, T *pold,
                                                 const T *Dinv, CgArgs ca) {
  double v[2] = {0.0, 0.0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (!ca.warm) x[i] = T(0);
    pold[i] = T(0);
    if (!ca.ext) {
      const T ri = r[i];
      const T zi = Dinv[i] * ri;
      z[i] = zi;
      v[0] += double(ri) * double(zi);
      v[1] += double(ri) * double(ri);
    }
  }
  if (!ca.ext) block_partial<2>(v, ca.partB);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ca.st->b.rz_prev = 0.0;
    ca.st->b.rr0 = 0.0;
    ca.st->b.tol2 = ca.tol2;
    ca.st->b.rr_abs = ca.rr_abs;
    ca.st->b.done = 0;
    ca.st->b.iters = 0;
    ca.st->b.first = 1;
  }
}

// Prologue of the apply kernels: returns done (uniform) and beta.
__device__ inline int cg_apply_prologue(const CgArgs &ca, double *beta, int bid) {
  double s[2];
  block_sum<2>(ca.partB, ca.npb, s);
  const double rz = s[0], rr = s[1];
  const int first = ca.st->b.first;
  const int iters = ca.st->b.iters;
  int done = ca.st->b.done;
  const double rr0 = first ? rr : ca.st->b.rr0;
  if (!done) {
    if (!(rr == rr) || !(rz == rz)) done = 2;
    else if (rr <= (ca.st->b.rr_abs > 0.0 ? ca.st->b.rr_abs : ca.st->b.tol2 * rr0)) done = 1;
    else if (iters >= ca.maxit) done = 3;
  }
  if (bid == 0 && threadIdx.x == 0) {
    ca.st->a.rz = rz;
    ca.st->a.rr = rr;
    ca.st->a.rr0 = rr0;
    ca.st->a.done = done;
    ca.st->a.iters = iters;
  }
  *beta = first ? 0.0 : rz / ca.st->b.rz_prev;
  return done;
}

// Block bid of nb of the apply A_k (one CG system).
template <int CH, class Op>
__device__ inline void cg_apply_run(Op op, const Grid &g, const March &ms, const CgArgs &ca,
                                    int bid, int nb) {
  double red[1] = {0.0};
  if constexpr (CH == 1) {
    __shared__ TileLds<Op> sm;
    const int nt = ms.nstrips * ms.nchunks;
    int t = xcd_block(bid, nb);
    // the first tile's loads are in flight during the prologue's reduction
    TileRegs<Op> tr;
    if (t < nt) tile_load(op, ms, t, tr);
    double beta = 0.0;
    if (cg_apply_prologue(ca, &beta, bid) != 0) return;
    op.beta = typename Op::T(beta);
    for (; t < nt; t += nb) {
      tile_compute(op, g, ms, t, tr, sm, red);
      if (t + nb < nt) tile_load(op, ms, t + nb, tr);
    }
  } else {
    const int lane = threadIdx.x & 63;
    const int w0 = xcd_block(bid, nb) * WPB + (threadIdx.x >> 6);
    const int nw = ms.nstrips * ms.nchunks;
    // issue the first work item's loads before the prologue's reduction
    Item<CH, Op> it;
    if (w0 < nw) item_load<CH>(op, g, ms, w0, lane, it);
    double beta = 0.0;
    if (cg_apply_prologue(ca, &beta, bid) != 0) return;
    op.beta = typename Op::T(beta);
    if (w0 < nw) item_compute<CH>(op, g, ms, w0, lane, it, red);
    march_items<CH>(op, g, ms, w0 + nb * WPB, nb * WPB, red);
  }
  block_partial_at<1>(red, ca.partA, bid);
}

template <int CH, class Op>
__global__ void __launch_bounds__(TPB) k_cg_apply(Op op, Grid g, March ms, CgArgs ca) {
  cg_apply_run<CH>(op, g, ms, ca, blockIdx.x, gridDim.x);
}

// Prologue of the fused update: the CG state, p.q from the apply's
// partials and alpha.  Records the exit in the state (bid 0) and returns
// whether the iteration is active (uniform).
__device__ inline bool cg_update_prologue(const CgArgs &ca, double *alpha, int bid) {
  const int done = ca.st->a.done;
  const double rz = ca.st->a.rz;
  const double rr0 = ca.st->a.rr0;
  const int iters = ca.st->a.iters;
  int exitc = done;
  double pq = 0.0;
  if (exitc == 0) {
    double pqs[1];
    block_sum<1>(ca.partA, ca.ga, pqs);
    pq = pqs[0];
    if (!(pq > 0.0)) exitc = 2;
  }
  if (exitc != 0 && bid == 0 && threadIdx.x == 0) {
    ca.st->b.done = exitc;
    ca.st->b.iters = iters;
    ca.st->b.rr0 = rr0;
    ca.st->b.first = 0;
  }
  *alpha = exitc == 0 ? rz / pq : 0.0;
  return exitc == 0;
}

// Block bid of nb of the fused update + first Chebyshev step.  Unlike the
// apply it never exits early: after convergence the step still runs on the
// unchanged r, as the separate kernels did.
template <int CH, class Op>
__device__ inline void cg_updcheb_run(Op op, const Grid &g, const March &ms, const CgArgs &ca,
                                      int bid, int nb) {
  double red[2] = {0.0, 0.0};
  double alpha = 0.0;
  if constexpr (CH == 1) {
    __shared__ TileLds<Op> sm;
    const int nt = ms.nstrips * ms.nchunks;
    int t = xcd_block(bid, nb);
    TileRegs<Op> tr;
    if (t < nt) tile_load(op, ms, t, tr);
    op.act = cg_update_prologue(ca, &alpha, bid) ? 1 : 0;
    op.alpha = typename Op::T(alpha);
    for (; t < nt; t += nb) {
      tile_compute(op, g, ms, t, tr, sm, red);
      if (t + nb < nt) tile_load(op, ms, t + nb, tr);
    }
  } else {
    const int lane = threadIdx.x & 63;
    const int w0 = xcd_block(bid, nb) * WPB + (threadIdx.x >> 6);
    const int nw = ms.nstrips * ms.nchunks;
    Item<CH, Op> it;
    if (w0 < nw) item_load<CH>(op, g, ms, w0, lane, it);
    op.act = cg_update_prologue(ca, &alpha, bid) ? 1 : 0;
    op.alpha = typename Op::T(alpha);
    if (w0 < nw) item_compute<CH>(op, g, ms, w0, lane, it, red);
    march_items<CH>(op, g, ms, w0 + nb * WPB, nb * WPB, red);
  }
  if (op.last) block_partial_at<2>(red, ca.partB, bid);
  if (op.act && bid == 0 && threadIdx.x == 0) {
    ca.st->b.rz_prev = ca.st->a.rz;
    ca.st->b.rr0 = ca.st->a.rr0;
    ca.st->b.done = 0;
    ca.st->b.iters = ca.st->a.iters + 1;
    ca.st->b.first = 0;
  }
}

template <int CH, class Op>
__global__ void __launch_bounds__(TPB) k_cg_updcheb(Op op, Grid g, March ms, CgArgs ca) {
  cg_updcheb_run<CH>(op, g, ms, ca, blockIdx.x, gridDim.x);
}

// ---- CG update fused with the first two Jacobi-Chebyshev steps (LDS tiles)
//
// The block of a tile of kTile x kTile owned nodes stages the (kTile+4)^2
// nodes around it, a ring of two.  Pass 1: every staged node takes
// r_new = r - alpha q (while the CG is active) and d0 = D^-1 r_new / theta;
// the (kTile+3)^2 elements among them apply the operator to d0, and the
// (kTile+2)^2 nodes of the tile and its first ring form res1 = r_new - A d0,
// d1 = c1 d0 + c2 D^-1 res1 and z1 = d0 + d1.  Pass 2: the (kTile+1)^2
// elements touching the tile apply the operator to d1, and the owned nodes
// form res2 = res1 - A d1, d2 = c3 d1 + c4 D^-1 res2 and z2 = z1 + d2.
// Owned nodes write x + alpha p and r_new to the other buffer of each pair,
// z2 and, when more steps follow, d2 and res2; when the polynomial ends
// here they write the partials of r.z and r.r instead.  Node for node this
// is the arithmetic of the fused update and one further Chebyshev step
// (OpUpdCheb, OpCheb), without the second launch and without writing and
// re-reading d1, z1 and res1.  Both neighbouring tiles compute the first
// ring.  Nothing it reads is written, so a launch may be repeated.
constexpr int kU2N = kTile + 4;   // staged nodes per side
constexpr int kU2E = kTile + 3;   // pass-1 elements per side
constexpr int kU2M = kTile + 2;   // pass-1 nodes per side (tile and first ring)

template <class Base>
struct UpdCheb2 {
  using T = typename Base::T;
  Base base;
  const T *x; const T *r; T *xo; T *ro; const T *p; const T *q; const T *Dinv;
  T *dnext; T *zo; T *reso;
  int N;
  const double *cf;   // cf[0] = 1/theta; cf[1], cf[2]: step 1; cf[3], cf[4]: step 2
  int last;           // step 2 is the polynomial's last
};

template <class Base>
struct UpdCheb2Lds {
  using T = typename Base::T;
  static constexpr int NF = Base::NF;
  typename Base::Node a[kU2N * kU2N];   // operator input d0, staged nodes
  typename Base::Node b[kU2M * kU2M];   // operator input d1, tile and first ring
  typename Base::Own own[kU2N * kU2N];
  typename Base::Elem el[kU2E * kU2E];
  T rn[NF][kU2N * kU2N];                // r_new
  T di[NF][kU2N * kU2N];                // D^-1
  T rs1[NF][kU2M * kU2M];
  T z1[NF][kU2M * kU2M];
  T f[NF][4][kU2E * kU2E];              // element corner values, both passes
};

template <class Base>
struct UpdCheb2Regs {
  using T = typename Base::T;
  static constexpr int NF = Base::NF;
  static constexpr int NSL = (kU2N * kU2N + TPB - 1) / TPB;
  static constexpr int NEL = (kU2E * kU2E + TPB - 1) / TPB;
  typename Base::Node n[NSL];
  typename Base::Own o[NSL];
  T r[NSL][NF], q[NSL][NF], di[NSL][NF];
  typename Base::Elem e[NEL];
};

template <class Base>
__device__ inline void updcheb2_load(const UpdCheb2<Base> &op, const Grid &g, const March &ms,
                                     int tile, UpdCheb2Regs<Base> &tr) {
  using T = typename Base::T;
  constexpr int NF = Base::NF;
  const int i0 = (tile % ms.nstrips) * kTile - 2, j0 = (tile / ms.nstrips) * kTile - 2;
  if constexpr (HasFast<Base>::value) {
    if (box_inside(g, i0, j0, kU2N)) {
      const unsigned row = unsigned(g.nx) + 1u, base = unsigned(j0) * row + unsigned(i0);
#pragma unroll
      for (int r = 0; r < UpdCheb2Regs<Base>::NSL; ++r) {
        const unsigned k = threadIdx.x + r * TPB;
        if (k < kU2N * kU2N) {
          const unsigned idx = base + (k / kU2N) * row + k % kU2N;
          const unsigned o = idx * unsigned(sizeof(T));
          tr.n[r] = op.base.load_aux_fast(idx);
          tr.o[r] = op.base.load_own_fast(idx);
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            tr.r[r][f] = ldo(op.r + f * op.N, o);
            tr.q[r][f] = ldo(op.q + f * op.N, o);
            tr.di[r][f] = ldo(op.Dinv + f * op.N, o);
          }
        }
      }
      const unsigned ebase = unsigned(j0) * unsigned(g.nx) + unsigned(i0);
#pragma unroll
      for (int r = 0; r < UpdCheb2Regs<Base>::NEL; ++r) {
        const unsigned e = threadIdx.x + r * TPB;
        if (e < kU2E * kU2E)
          tr.e[r] = op.base.eload_fast(ebase + (e / kU2E) * unsigned(g.nx) + e % kU2E);
      }
      return;
    }
  }
  // the thread index is opaque here, so that the compiler does not hoist
  // this path's per-thread address arithmetic out of the kernel's tile loop
  // (where it would hold registers through the computation of every tile)
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int r = 0; r < UpdCheb2Regs<Base>::NSL; ++r) {
    const int k = tid + r * TPB;
#pragma unroll
    for (int f = 0; f < NF; ++f) tr.r[r][f] = tr.q[r][f] = tr.di[r][f] = T(0);
    if (k < kU2N * kU2N) {
      const int i = i0 + k % kU2N, j = j0 + k / kU2N;
      tr.n[r] = op.base.load_aux(i, j);
      tr.o[r] = op.base.load_own(i, j);
      if (node_exists(g, i, j)) {
        const int idx = i + j * (g.nx + 1);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          tr.r[r][f] = op.r[idx + f * op.N];
          tr.q[r][f] = op.q[idx + f * op.N];
          tr.di[r][f] = op.Dinv[idx + f * op.N];
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < UpdCheb2Regs<Base>::NEL; ++r) {
    const int e = tid + r * TPB;
    if (e < kU2E * kU2E) tr.e[r] = op.base.eload(i0 + e % kU2E, j0 + e / kU2E);
  }
}

template <class Base>
__device__ inline void updcheb2_compute(const UpdCheb2<Base> &op, const Grid &g, const March &ms,
                                        int tile, const UpdCheb2Regs<Base> &tr,
                                        UpdCheb2Lds<Base> &sm, bool act, typename Base::T alpha,
                                        double (&red)[2]) {
  using T = typename Base::T;
  constexpr int NF = Base::NF;
  const Base &B = op.base;
  const T c0 = T(op.cf[0]), c1 = T(op.cf[1]), c2 = T(op.cf[2]), c3 = T(op.cf[3]),
          c4 = T(op.cf[4]);
  // stage: r_new and d0 on every staged node
#pragma unroll
  for (int r = 0; r < UpdCheb2Regs<Base>::NSL; ++r) {
    const int k = threadIdx.x + r * TPB;
    if (k < kU2N * kU2N) {
      T d0[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        T rn = tr.r[r][f];
        if (act) rn = rn - alpha * tr.q[r][f];
        sm.rn[f][k] = rn;
        sm.di[f][k] = tr.di[r][f];
        d0[f] = tr.di[r][f] * rn * c0;
      }
      typename Base::Node n = tr.n[r];
      B.set_u(n, d0);
      sm.a[k] = n;
      sm.own[k] = tr.o[r];
    }
  }
#pragma unroll
  for (int r = 0; r < UpdCheb2Regs<Base>::NEL; ++r) {
    const int e = threadIdx.x + r * TPB;
    if (e < kU2E * kU2E) sm.el[e] = tr.e[r];
  }
  __syncthreads();
  // pass 1: A d0 on the (kTile+3)^2 elements of the staged nodes
#pragma unroll
  for (int r = 0; r < UpdCheb2Regs<Base>::NEL; ++r) {
    const int e = threadIdx.x + r * TPB;
    if (e < kU2E * kU2E) {
      const int b = (e / kU2E) * kU2N + e % kU2E;
      T fe[NF][4];
      B.element(sm.a[b], sm.a[b + 1], sm.a[b + kU2N + 1], sm.a[b + kU2N], sm.el[e], fe);
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 0; c < 4; ++c) sm.f[f][c][e] = fe[f][c];
    }
  }
  __syncthreads();
  // pass 1 nodes: staged node (a, b), 1 <= a, b <= kTile + 2, is corner 2 of
  // element (a-1, b-1), 3 of (a, b-1), 1 of (a-1, b) and 0 of (a, b)
  for (int m = threadIdx.x; m < kU2M * kU2M; m += TPB) {
    const int a = 1 + m % kU2M, b = 1 + m / kU2M;
    const int k = b * kU2N + a, e = (b - 1) * kU2E + (a - 1);
    T d0[NF], d1[NF];
    B.get_u(sm.a[k], d0);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      T Ad = sm.f[f][2][e] + sm.f[f][3][e + 1] + sm.f[f][1][e + kU2E] + sm.f[f][0][e + kU2E + 1];
      if (Base::masked_own(sm.own[k], f)) Ad = T(0);
      const T rs = sm.rn[f][k] - Ad;
      const T dk = c1 * d0[f] + c2 * sm.di[f][k] * rs;
      sm.rs1[f][m] = rs;
      sm.z1[f][m] = d0[f] + dk;
      d1[f] = dk;
    }
    typename Base::Node n = sm.a[k];
    B.set_u(n, d1);
    sm.b[m] = n;
  }
  __syncthreads();
  // x and p of the owned node are needed only at the end: their loads are
  // issued here, in flight during pass 2, instead of with the staged loads
  // (where they would hold registers through pass 1)
  T xv[NF], pv[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) xv[f] = pv[f] = T(0);
  if (act && threadIdx.x < kTile * kTile) {
    const int i = (tile % ms.nstrips) * kTile + threadIdx.x % kTile;
    const int j = (tile / ms.nstrips) * kTile + threadIdx.x / kTile;
    if (i <= g.nx && j <= g.ny) {
      const int idx = i + j * (g.nx + 1);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        xv[f] = op.x[idx + f * op.N];
        pv[f] = op.p[idx + f * op.N];
      }
    }
  }
  // pass 2: A d1 on the (kTile+1)^2 elements touching the tile; element
  // (a, b), 1 <= a, b <= kTile + 1, has corner 0 at pass-1 node (a, b)
  {
    static_assert(kTileE * kTileE == TPB, "one pass-2 element per thread");
    const int a = 1 + threadIdx.x % kTileE, b = 1 + threadIdx.x / kTileE;
    const int m0 = (b - 1) * kU2M + (a - 1);
    T fe[NF][4];
    B.element(sm.b[m0], sm.b[m0 + 1], sm.b[m0 + kU2M + 1], sm.b[m0 + kU2M],
              sm.el[b * kU2E + a], fe);
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int c = 0; c < 4; ++c) sm.f[f][c][threadIdx.x] = fe[f][c];
  }
  __syncthreads();
  // owned nodes: staged node (2 + li, 2 + lj)
  if (threadIdx.x < kTile * kTile) {
    const int li = threadIdx.x % kTile, lj = threadIdx.x / kTile;
    const int i = (tile % ms.nstrips) * kTile + li, j = (tile / ms.nstrips) * kTile + lj;
    if (i <= g.nx && j <= g.ny) {
      const int e = lj * kTileE + li;
      const int m = (lj + 1) * kU2M + (li + 1), k = (lj + 2) * kU2N + (li + 2);
      const int gk = i + j * (g.nx + 1);
      T d1[NF];
      B.get_u(sm.b[m], d1);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        T Ad = sm.f[f][2][e] + sm.f[f][3][e + 1] + sm.f[f][1][e + kTileE] +
               sm.f[f][0][e + kTileE + 1];
        if (Base::masked_own(sm.own[k], f)) Ad = T(0);
        const T rs = sm.rs1[f][m] - Ad;
        const T dk = c3 * d1[f] + c4 * sm.di[f][k] * rs;
        const T z = sm.z1[f][m] + dk;
        const T rn = sm.rn[f][k];
        const int idx = gk + f * op.N;
        op.zo[idx] = z;
        if (op.last) {
          red[0] += double(rn) * double(z);
          red[1] += double(rn) * double(rn);
        } else {
          op.dnext[idx] = dk;
          op.reso[idx] = rs;
        }
        if (act) {
          op.xo[idx] = xv[f] + alpha * pv[f];
          op.ro[idx] = rn;
        }
      }
    }
  }
  __syncthreads();   // the LDS is reused by the block's next tile
}

// FP32 with compact node records (VD tangent, phase operator): ask for five
// blocks per CU, so that one launch at 512^2 (1225 tiles) holds every tile
// at once; the others take what their registers allow.
template <class Base>
constexpr int updcheb2_min_blocks() {
  using T = typename Base::T;
  return (sizeof(T) == 4 && sizeof(typename Base::Node) <= 3 * sizeof(T)) ? 5 : 1;
}

template <class Base>
__global__ void __launch_bounds__(TPB, updcheb2_min_blocks<Base>())
    k_cg_updcheb2(UpdCheb2<Base> op, Grid g, March ms, CgArgs ca) {
  using T = typename Base::T;
  __shared__ UpdCheb2Lds<Base> sm;
  const int bid = blockIdx.x, nb = gridDim.x;
  const int nt = ms.nstrips * ms.nchunks;
  double red[2] = {0.0, 0.0};
  double alpha = 0.0;
  const int t0 = xcd_block(bid, nb);
  // the first tile's loads are in flight during the prologue's reduction;
  // a later tile of the block is loaded after the previous one is done (a
  // prefetch would hold its registers through the whole computation)
  UpdCheb2Regs<Base> tr;
  if (t0 < nt) updcheb2_load(op, g, ms, t0, tr);
  const bool act = cg_update_prologue(ca, &alpha, bid);
  for (int t = t0; t < nt; t += nb) {
    if (t != t0) updcheb2_load(op, g, ms, t, tr);
    updcheb2_compute(op, g, ms, t, tr, sm, act, T(alpha), red);
  }
  if (op.last) block_partial_at<2>(red, ca.partB, bid);
  if (act && bid == 0 && threadIdx.x == 0) {
    ca.st->b.rz_prev = ca.st->a.rz;
    ca.st->b.rr0 = ca.st->a.rr0;
    ca.st->b.done = 0;
    ca.st->b.iters = ca.st->a.iters + 1;
    ca.st->b.first = 0;
  }
}

// Elements per thread whose operands are loaded before the scalars.
constexpr int kUpd = 4;

template <class T>
__device__ inline void upd_load(int n, int i0, int stride, const T *__restrict__ x,
                                const T *__restrict__ p, const T *__restrict__ q,
                                const T *__restrict__ r, const T *__restrict__ Dinv, bool ext,
                                T (&xv)[kUpd], T (&pv)[kUpd], T (&qv)[kUpd], T (&rv)[kUpd],
                                T (&dv)[kUpd]) {
#pragma unroll
  for (int k = 0; k < kUpd; ++k) {
    const int i = i0 + k * stride;
    xv[k] = pv[k] = qv[k] = rv[k] = dv[k] = T(0);
    if (i < n) {
      xv[k] = x[i];
      pv[k] = p[i];
      qv[k] = q[i];
      rv[k] = r[i];
      if (!ext) dv[k] = Dinv[i];
    }
  }
}

// Block bid of nb of the update B_k (one CG system).
template <class T>
__device__ inline void cg_update_run(int n, T *__restrict__ x, T *__restrict__ r,
                                     T *__restrict__ z, const T *__restrict__ p,
                                     const T *__restrict__ q, const T *__restrict__ Dinv,
                                     const CgArgs &ca, const ChebFuse<T> &cf, int bid, int nb) {
  const int stride = nb * blockDim.x;
  int i0 = bid * blockDim.x + threadIdx.x;
  // ext: the preconditioner runs elsewhere; fused: its first step is here
  const bool fused = cf.d0 != nullptr;
  const bool ext = ca.ext != 0 && !fused;
  const bool parts = !ext && (!fused || cf.last);
  const T it = fused ? T(cf.coef[0]) : T(0);
  // the first group's operands are in flight while the scalars are reduced
  T xv[kUpd], pv[kUpd], qv[kUpd], rv[kUpd], dv[kUpd];
  upd_load(n, i0, stride, x, p, q, r, Dinv, ext, xv, pv, qv, rv, dv);
  const int done = ca.st->a.done;
  const double rz = ca.st->a.rz;
  const double rr0 = ca.st->a.rr0;
  const int iters = ca.st->a.iters;
  int exitc = done;
  double pq = 0.0;
  if (exitc == 0) {
    double pqs[1];
    block_sum<1>(ca.partA, ca.ga, pqs);
    pq = pqs[0];
    if (!(pq > 0.0)) exitc = 2;
  }
  if (exitc != 0) {
    if (bid == 0 && threadIdx.x == 0) {
      ca.st->b.done = exitc;
      ca.st->b.iters = iters;
      ca.st->b.rr0 = rr0;
      ca.st->b.first = 0;
    }
    // a fused Chebyshev step still runs on the unchanged r, as it would
    // in a kernel of its own
    if (!fused) return;
  }
  const bool act = exitc == 0;
  const T alpha = act ? T(rz / pq) : T(0);
  double v[2] = {0.0, 0.0};
  for (;;) {
#pragma unroll
    for (int k = 0; k < kUpd; ++k) {
      const int i = i0 + k * stride;
      if (i < n) {
        T ri = rv[k];
        if (act) {
          const T xi = xv[k] + alpha * pv[k];
          ri = rv[k] - alpha * qv[k];
          x[i] = xi;
          r[i] = ri;
        }
        if (fused) {
          const T zi = dv[k] * ri * it;
          cf.d0[i] = zi;
          z[i] = zi;
          cf.res[i] = ri;
          v[0] += double(ri) * double(zi);
          v[1] += double(ri) * double(ri);
        } else if (!ext) {
          const T zi = dv[k] * ri;
          z[i] = zi;
          v[0] += double(ri) * double(zi);
          v[1] += double(ri) * double(ri);
        }
      }
    }
    i0 += kUpd * stride;
    if (i0 >= n) break;
    upd_load(n, i0, stride, x, p, q, r, Dinv, ext, xv, pv, qv, rv, dv);
  }
  if (parts) block_partial_at<2>(v, ca.partB, bid);
  if (act && bid == 0 && threadIdx.x == 0) {
    ca.st->b.rz_prev = rz;
    ca.st->b.rr0 = rr0;
    ca.st->b.done = 0;
    ca.st->b.iters = iters + 1;
    ca.st->b.first = 0;
  }
}

template <class T>
__global__ void __launch_bounds__(TPB) k_cg_update(int n, T *x, T *r, T *z, const T *p,
                                                   const T *q, const T *Dinv, CgArgs ca,
                                                   ChebFuse<T> cf) {
  cg_update_run<T>(n, x, r, z, p, q, Dinv, ca, cf, blockIdx.x, gridDim.x);
}

// Shared launches of many CG systems (see BatchUpdateEntry).
template <class Op>
struct BatchApplyEntry {
  Op op;
  Grid g;
  March ms;
  CgArgs ca;
  int b0, nb;
};

template <int CH, class Op>
__global__ void __launch_bounds__(TPB) k_cg_apply_batch(const char *tab, const int *bmap) {
  const BatchApplyEntry<Op> &e =
      *reinterpret_cast<const BatchApplyEntry<Op> *>(tab + size_t(bmap[blockIdx.x]) *
                                                               kBatchEntryBytes);
  cg_apply_run<CH>(e.op, e.g, e.ms, e.ca, blockIdx.x - e.b0, e.nb);
}

template <class T>
__global__ void __launch_bounds__(TPB) k_cg_update_batch(const BatchUpdateEntry<T> *tab,
                                                         const int *bmap) {
  const BatchUpdateEntry<T> &e = tab[bmap[blockIdx.x]];
  const int bid = blockIdx.x - e.b0;
  const ChebFuse<T> none{nullptr, nullptr, nullptr, 0};
  cg_update_run<T>(e.n, e.x, e.r, e.z, e.p, e.q, e.Dinv, e.ca, none, bid, e.nb);
  // the thread that wrote this system's CG state also publishes it
  if (bid == 0 && threadIdx.x == 0) {
    e.status[0] = e.ca.st->b.done;
    e.status[1] = e.ca.st->b.iters;
  }
}

int vec_blocks(int n) {
  int b = (n + 4 * TPB - 1) / (4 * TPB);
  if (b > kPMax) b = kPMax;
  if (b < 1) b = 1;
  return b;
}

// ------------------------------------------ Jacobi-Chebyshev and power

template <class T>
__global__ void __launch_bounds__(TPB) k_cheb_init(int n, const T *r, const T *Dinv, T *d0, T *z,
                                                   T *res, CgArgs ca, ChebStep cs) {
  double v[2] = {0.0, 0.0};
  const T it = T(cs.coef[0]);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const T ri = r[i];
    const T di = Dinv[i] * ri * it;
    d0[i] = di;
    z[i] = di;
    res[i] = ri;
    v[0] += double(ri) * double(di);
    v[1] += double(ri) * double(ri);
  }
  if (cs.last) block_partial<2>(v, ca.partB);
}

// Chebyshev step on top of an operator op (its input vector is d_{k-1}):
// d_k = c1 d_{k-1} + c2 D^-1 (res - A d_{k-1}), z += d_k, res -= A d_{k-1}.
// z and res are read from one buffer and written to another, so a launch
// leaves its inputs intact and may be repeated (timing samples).
template <class Base>
struct OpCheb {
  using T = typename Base::T;
  using Elem = typename Base::Elem;
  using Node = typename Base::Node;
  static constexpr int NF = Base::NF;
  static constexpr int NR = 2;
  Base base;
  const T *r; const T *Dinv; T *dnext;
  const T *zi; const T *resi; T *zo; T *reso;
  int N;
  const double *cf;   // device coefficients
  int step;           // this is step `step` >= 1 of the polynomial
  int last;
  __device__ Node load(int i, int j) const { return base.load(i, j); }
  __device__ void fin(Node &n) const { base.fin(n); }
  __device__ Elem eload(int ie, int je) const { return base.eload(ie, je); }
  static __device__ Node shfl_up(const Node &n) { return Base::shfl_up(n); }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, T (&f)[NF][4]) const {
    base.element(n0, n1, n2, n3, e, f);
  }
  struct Own {
    typename Base::Own b;
    T res[NF], z[NF], di[NF], r[NF];
  };
  __device__ Own load_own(int i, int j) const {
    Own o;
    o.b = base.load_own(i, j);
#pragma unroll
    for (int q = 0; q < NF; ++q) o.res[q] = o.z[q] = o.di[q] = o.r[q] = T(0);
    if (node_exists(base.g, i, j)) {
      const int k = i + j * (base.g.nx + 1);
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const int idx = k + q * N;
        o.res[q] = resi[idx];
        o.z[q] = zi[idx];
        o.di[q] = Dinv[idx];
        if (last) o.r[q] = r[idx];
      }
    }
    return o;
  }
  __device__ void store(int i, int j, const T (&v)[NF], const Node &n, const Own &o,
                        double *red) const {
    const int k = i + j * (base.g.nx + 1);
    const T c1 = T(cf[2 * step - 1]), c2 = T(cf[2 * step]);
    T dp[NF];
    base.get_u(n, dp);
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const int idx = k + q * N;
      const T Ad = Base::masked_own(o.b, q) ? T(0) : v[q];
      const T rs = o.res[q] - Ad;
      const T dk = c1 * dp[q] + c2 * o.di[q] * rs;
      const T y = o.z[q] + dk;
      reso[idx] = rs;
      dnext[idx] = dk;
      zo[idx] = y;
      if (last) {
        red[0] += double(o.r[q]) * double(y);
        red[1] += double(o.r[q]) * double(o.r[q]);
      }
    }
  }
};

// CG vector update fused with the first Chebyshev step (degree >= 2):
// staged nodes (halo included) take r_new = r - alpha q (when the CG is
// still active) and d0 = D^-1 r_new / theta; the operator is applied to d0;
// owned nodes then write x + alpha p and r_new (to the other buffer of the
// x and r pairs) and the step's outputs res1 = r_new - A d0,
// d1 = c1 d0 + c2 D^-1 res1, z1 = d0 + d1.  Nothing it reads is written, so
// a launch may be repeated (timing samples).
template <class Base>
struct OpUpdCheb {
  using T = typename Base::T;
  using Elem = typename Base::Elem;
  static constexpr int NF = Base::NF;
  static constexpr int NR = 2;
  struct Node {
    typename Base::Node b;
    T r[NF], q[NF], di[NF], x[NF], p[NF];
  };
  Base base;
  const T *x; const T *r; T *xo; T *ro; const T *p; const T *q; const T *Dinv;
  T *dnext; T *zo; T *reso;
  int N;
  const double *cf;   // device coefficients: cf[0] = 1/theta, cf[1], cf[2] = step 1
  T alpha;
  int act, last;
  __device__ Node load(int i, int j) const {
    Node n;
    n.b = base.load_aux(i, j);
#pragma unroll
    for (int f = 0; f < NF; ++f) n.r[f] = n.q[f] = n.di[f] = n.x[f] = n.p[f] = T(0);
    if (node_exists(base.g, i, j)) {
      const int k = i + j * (base.g.nx + 1);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int idx = k + f * N;
        n.r[f] = r[idx];
        n.q[f] = q[idx];
        n.di[f] = Dinv[idx];
        n.x[f] = x[idx];
        n.p[f] = p[idx];
      }
    }
    return n;
  }
  __device__ void fin(Node &n) const {
    T d0[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (act) n.r[f] = n.r[f] - alpha * n.q[f];
      d0[f] = n.di[f] * n.r[f] * T(cf[0]);
    }
    base.set_u(n.b, d0);
  }
  __device__ Elem eload(int ie, int je) const { return base.eload(ie, je); }
  static __device__ Node shfl_up(const Node &n) {
    Node m;
    m.b = Base::shfl_up(n.b);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      m.r[f] = lane_up(n.r[f]);
      m.q[f] = T(0);
      m.di[f] = lane_up(n.di[f]);
      m.x[f] = lane_up(n.x[f]);
      m.p[f] = lane_up(n.p[f]);
    }
    return m;
  }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, T (&f)[NF][4]) const {
    base.element(n0.b, n1.b, n2.b, n3.b, e, f);
  }
  using Own = typename Base::Own;
  __device__ Own load_own(int i, int j) const { return base.load_own(i, j); }
  __device__ void store(int i, int j, const T (&v)[NF], const Node &n, const Own &o,
                        double *red) const {
    const int k = i + j * (base.g.nx + 1);
    T d0[NF];
    base.get_u(n.b, d0);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int idx = k + f * N;
      const T Ad = Base::masked_own(o, f) ? T(0) : v[f];
      const T rs = n.r[f] - Ad;
      const T dk = T(cf[1]) * d0[f] + T(cf[2]) * n.di[f] * rs;
      const T y = d0[f] + dk;
      reso[idx] = rs;
      dnext[idx] = dk;
      zo[idx] = y;
      if (act) {
        xo[idx] = n.x[f] + alpha * n.p[f];
        ro[idx] = n.r[f];
      }
      if (last) {
        red[0] += double(n.r[f]) * double(y);
        red[1] += double(n.r[f]) * double(n.r[f]);
      }
    }
  }
};

// Power-iteration step on D^-1 A: the input vector is scaled by `scale`.
template <class Base>
struct OpPower {
  using T = typename Base::T;
  using Elem = typename Base::Elem;
  using Node = typename Base::Node;
  static constexpr int NF = Base::NF;
  static constexpr int NR = 2;
  Base base;
  const T *Dinv; T *vnext;
  int N;
  T scale;
  __device__ Node load(int i, int j) const { return base.load(i, j); }
  __device__ void fin(Node &n) const {
    T u[NF];
    base.get_u(n, u);
#pragma unroll
    for (int q = 0; q < NF; ++q) u[q] *= scale;
    base.set_u(n, u);
  }
  __device__ Elem eload(int ie, int je) const { return base.eload(ie, je); }
  static __device__ Node shfl_up(const Node &n) { return Base::shfl_up(n); }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, T (&f)[NF][4]) const {
    base.element(n0, n1, n2, n3, e, f);
  }
  struct Own {
    typename Base::Own b;
    T di[NF];
  };
  __device__ Own load_own(int i, int j) const {
    Own o;
    o.b = base.load_own(i, j);
#pragma unroll
    for (int q = 0; q < NF; ++q) o.di[q] = T(0);
    if (node_exists(base.g, i, j)) {
      const int k = i + j * (base.g.nx + 1);
#pragma unroll
      for (int q = 0; q < NF; ++q) o.di[q] = Dinv[k + q * N];
    }
    return o;
  }
  __device__ void store(int i, int j, const T (&v)[NF], const Node &n, const Own &o,
                        double *red) const {
    const int k = i + j * (base.g.nx + 1);
    T vv[NF];
    base.get_u(n, vv);
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const int idx = k + q * N;
      const T di = o.di[q];
      const T Av = Base::masked_own(o.b, q) ? T(0) : v[q];
      vnext[idx] = di * Av;
      red[0] += double(vv[q]) * double(Av);
      if (di > T(0)) red[1] += double(vv[q]) * double(vv[q]) / double(di);
    }
  }
};

template <class T>
__global__ void k_power_start(int n, const T *Dinv, T *v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // deterministic start with components along every eigenvector
  const unsigned h = (unsigned)i * 2654435761u;
  const T w = T(0.5) + T((h >> 8) & 0xffff) * T(1.0 / 65536.0);
  v[i] = Dinv[i] > T(0) ? w : T(0);
}

// --------------------------------------------------- single-kernel CG
//
// Chronopoulos-Gear CG with one reduction and one kernel per iteration.
// Iteration i (kernel K_i, i >= 1) with alpha = alpha_{i-1}, beta = beta_{i-1}
// from the prologue:
//   s_{i-1} = w_{i-1} + beta s_{i-2}         (every node of the work item)
//   r_i     = r_{i-1} - alpha s_{i-1}
//   u_i     = D^-1 r_i
//   p_{i-1} = u_{i-1} + beta p_{i-2},  x_i = x_{i-1} + alpha p_{i-1}   (owned)
//   w_i     = A u_i;  partials gamma_i = r_i.u_i, delta_i = w_i.u_i, r_i.r_i
// with beta_{i-1} = gamma_{i-1}/gamma_{i-2} and
// alpha_{i-1} = gamma_{i-1} / (delta_{i-1} - beta_{i-1} gamma_{i-1}/alpha_{i-2}).
// K_0 forms u_0 = D^-1 r_0, w_0 = A u_0 and zeroes x_0, p_{-1}, s_{-1}.
// The halo rows of a work item recompute s, r, u from the parity-(i-1)
// vectors they read, so no block needs another block's output of the same
// kernel.

__device__ inline int cg1_prologue(const Cg1Args &a, double *alpha, double *beta) {
  const int cur = a.parity, prv = cur ^ 1;
  double s3[3];
  block_sum<3>(a.part + prv * 3 * kPMax, a.np, s3);
  const double gam = s3[0], del = s3[1], rr = s3[2];
  const Cg1State S = a.st[prv];
  int done = S.done;
  const double rr0 = S.first ? rr : S.rr0;
  double al = 0.0, be = 0.0;
  if (!done) {
    if (!(rr == rr) || !(gam == gam) || !(del == del)) done = 2;
    else if (rr <= a.tol2 * rr0) done = 1;
    else if (S.iters >= a.maxit) done = 3;
  }
  if (!done) {
    if (S.first) {
      be = 0.0;
      const double den = del;
      if (!(den > 0.0)) done = 2;
      else al = gam / den;
    } else {
      be = gam / S.gamma_prev;
      const double den = del - be * gam / S.alpha_prev;
      if (!(den > 0.0)) done = 2;
      else al = gam / den;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Cg1State o;
    o.alpha_prev = al;
    o.gamma_prev = gam;
    o.rr0 = rr0;
    o.rr = rr;
    o.done = done;
    o.iters = done ? S.iters : S.iters + 1;
    o.first = 0;
    o.pad = 0;
    a.st[cur] = o;
  }
  *alpha = al;
  *beta = be;
  return done;
}

template <int CH, class Op>
struct Cg1Item {
  using T = typename Op::T;
  static constexpr int NC = Op::NF;
  T r[CH + 2][NC], w[CH + 2][NC], s[CH + 2][NC], di[CH + 2][NC];
  T po[CH][NC], xo[CH][NC];
  typename Op::Node aux[CH + 2];
  typename Op::Elem El[CH + 1];
};

template <int CH, class Op>
__device__ inline void cg1_load(const Op &op, const Grid &g, const March &ms, int w, int lane,
                                const CgVecs<typename Op::T> &v, const Cg1Args &a,
                                Cg1Item<CH, Op> &it) {
  using T = typename Op::T;
  constexpr int NC = Op::NF;
  const int cur = a.parity, prv = cur ^ 1;
  const int strip = w % ms.nstrips, chunk = w / ms.nstrips;
  const int c = strip * CSTRIP - 1 + lane;
  const int j0 = chunk * CH;
  const T *Rin = a.init ? v.R[cur] : v.R[prv];
#pragma unroll
  for (int r = 0; r < CH + 2; ++r) {
    const int j = j0 - 1 + r;
    it.aux[r] = op.load_aux(c, j);
    const bool ex = node_exists(g, c, j);
    const int k = c + j * (g.nx + 1);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      it.r[r][q] = ex ? Rin[k + q * g.N] : T(0);
      it.di[r][q] = ex ? v.Dinv[k + q * g.N] : T(0);
      it.w[r][q] = (ex && !a.init) ? v.W[prv][k + q * g.N] : T(0);
      it.s[r][q] = (ex && !a.init) ? v.S[cur][k + q * g.N] : T(0);
    }
  }
  // owned rows j0 .. j0+CH-1 also need p and x (owned column only)
  const int n = c - 1;
  const bool own_col = lane >= 2 && n >= 0 && n <= g.nx;
#pragma unroll
  for (int r = 0; r < CH; ++r) {
    const int j = j0 + r;
    const bool ok = own_col && j <= g.ny && !a.init;
    const int k = n + j * (g.nx + 1);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      it.po[r][q] = ok ? v.P[prv][k + q * g.N] : T(0);
      it.xo[r][q] = ok ? v.X[prv][k + q * g.N] : T(0);
    }
  }
#pragma unroll
  for (int r = 0; r < CH + 1; ++r)
    it.El[r] = (lane > 0) ? op.eload(c - 1, j0 - 1 + r) : typename Op::Elem{};
}

template <int CH, class Op>
__device__ inline void cg1_compute(const Op &op, const Grid &g, const March &ms, int w, int lane,
                                   const CgVecs<typename Op::T> &v, const Cg1Args &a,
                                   typename Op::T alpha, typename Op::T beta,
                                   Cg1Item<CH, Op> &it, double (&red)[3]) {
  using T = typename Op::T;
  using Node = typename Op::Node;
  constexpr int NC = Op::NF;
  const int cur = a.parity, prv = cur ^ 1;
  const int strip = w % ms.nstrips, chunk = w / ms.nstrips;
  const int c = strip * CSTRIP - 1 + lane;
  const int n = c - 1;                          // node column this lane stores
  const int j0 = chunk * CH;
  const bool own_col = lane >= 2 && n >= 0 && n <= g.nx;
  // recurrences at every node of the item (lane holds column c)
  T u[CH + 2][NC], rn[CH + 2][NC], sn[CH + 2][NC];
#pragma unroll
  for (int r = 0; r < CH + 2; ++r) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if (a.init) {
        sn[r][q] = T(0);
        rn[r][q] = it.r[r][q];
      } else {
        sn[r][q] = it.w[r][q] + beta * it.s[r][q];
        rn[r][q] = it.r[r][q] - alpha * sn[r][q];
      }
      u[r][q] = it.di[r][q] * rn[r][q];
    }
  }
  // owned updates: the lane storing column n = c - 1 takes the values of the
  // left neighbour lane (column c - 1) by one shuffle
#pragma unroll
  for (int r = 1; r <= CH; ++r) {
    T rl[NC], sl[NC], ul[NC], rol[NC], dil[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      rl[q] = lane_up(rn[r][q]);
      sl[q] = lane_up(sn[r][q]);
      ul[q] = lane_up(u[r][q]);
      rol[q] = lane_up(it.r[r][q]);
      dil[q] = lane_up(it.di[r][q]);
    }
    const int j = j0 - 1 + r;
    if (own_col && j <= g.ny) {
      const int k = n + j * (g.nx + 1);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        T pn, xn;
        if (a.init) {
          pn = T(0);
          xn = T(0);
        } else {
          pn = dil[q] * rol[q] + beta * it.po[r - 1][q];   // p_{i-1} = u_{i-1} + beta p_{i-2}
          xn = it.xo[r - 1][q] + alpha * pn;
        }
        v.P[cur][k + q * g.N] = pn;
        v.X[cur][k + q * g.N] = xn;
        if (!a.init) v.R[cur][k + q * g.N] = rl[q];
        v.S[prv][k + q * g.N] = sl[q];
        red[0] += double(rl[q]) * double(ul[q]);
        red[2] += double(rl[q]) * double(rl[q]);
      }
    }
  }
  // w = A u over the item's element rows
  Node nodes[CH + 2];
#pragma unroll
  for (int r = 0; r < CH + 2; ++r) {
    nodes[r] = it.aux[r];
    op.set_u(nodes[r], u[r]);
  }
  Node br = nodes[0];
  Node bl = Op::shfl_up(br);
  T c2[NC], c3[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) { c2[q] = T(0); c3[q] = T(0); }
#pragma unroll
  for (int r = 0; r < CH + 1; ++r) {
    const int je = j0 - 1 + r;
    const Node tr = nodes[r + 1];
    const Node tl = Op::shfl_up(tr);
    T f[NC][4];
    op.element(bl, br, tr, tl, it.El[r], f);
    T out[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const T A = f[q][1] + c2[q];
      const T Al = lane_up(A);
      out[q] = f[q][0] + c3[q] + Al;
      c3[q] = f[q][3];
      c2[q] = f[q][2];
    }
    if (r >= 1 && own_col && je <= g.ny) {
      const int k = n + je * (g.nx + 1);
      T uo[NC];
      op.get_u(bl, uo);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const T wv = op.masked(k, q) ? T(0) : out[q];
        v.W[cur][k + q * g.N] = wv;
        red[1] += double(wv) * double(uo[q]);
      }
    }
    bl = tl;
    br = tr;
  }
}

template <int CH, class Op>
__global__ void __launch_bounds__(TPB) k_cg1(Op op, Grid g, March ms,
                                             CgVecs<typename Op::T> v, Cg1Args a) {
  using T = typename Op::T;
  const int lane = threadIdx.x & 63;
  const int w0 = xcd_block(blockIdx.x, gridDim.x) * WPB + (threadIdx.x >> 6);
  const int nw = ms.nstrips * ms.nchunks;
  Cg1Item<CH, Op> it;
  if (w0 < nw) cg1_load<CH>(op, g, ms, w0, lane, v, a, it);
  double alpha = 0.0, beta = 0.0;
  if (!a.init) {
    if (cg1_prologue(a, &alpha, &beta) != 0) return;
  } else if (blockIdx.x == 0 && threadIdx.x == 0) {
    Cg1State o{};
    o.first = 1;
    a.st[0] = o;
  }
  double red[3] = {0.0, 0.0, 0.0};
  if (w0 < nw) cg1_compute<CH>(op, g, ms, w0, lane, v, a, T(alpha), T(beta), it, red);
  for (int w = w0 + gridDim.x * WPB; w < nw; w += gridDim.x * WPB) {
    Cg1Item<CH, Op> it2;
    cg1_load<CH>(op, g, ms, w, lane, v, a, it2);
    cg1_compute<CH>(op, g, ms, w, lane, v, a, T(alpha), T(beta), it2, red);
  }
  block_partial<3>(red, a.part + a.parity * 3 * kPMax);
}


// ------------------------------------------------------ element kernels

// Quadrature-point update (one thread per element): strain, split energies,
// history max, tangent indicator bits and the softening gate (Section 3.5).
__global__ void __launch_bounds__(TPB) k_qp_update(Grid g, Mat mt, QpParams qp,
                                                   const double *u, const double *d,
                                                   const uint8_t *eact, const double *Hprev,
                                                   double *H, double *psi_s, uint8_t *qflag,
                                                   double *psi_out, RedScratch rs) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long ng = 0;
  if (e < g.E) {
    const int ie = e % g.nx, je = e / g.nx;
    const bool act = (eact == nullptr) || eact[e] != 0;
    uint8_t fl = 0;
    if (!act) {
      for (int q = 0; q < 4; ++q) {
        H[e + q * g.E] = Hprev[e + q * g.E];
        psi_s[e + q * g.E] = 0.0;
        if (psi_out) psi_out[e + q * g.E] = 0.0;
      }
    } else {
      const int n0 = ie + je * (g.nx + 1);
      const int nn[4] = {n0, n0 + 1, n0 + 1 + (g.nx + 1), n0 + (g.nx + 1)};
      double ux[4], uy[4], dn[4];
      for (int a = 0; a < 4; ++a) {
        ux[a] = u[nn[a]];
        uy[a] = u[nn[a] + g.N];
        dn[a] = d[nn[a]];
      }
      const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy;
      const double Dbx = ux[1] - ux[0], Dtx = ux[2] - ux[3], Dlx = ux[3] - ux[0], Drx = ux[2] - ux[1];
      const double Dby = uy[1] - uy[0], Dty = uy[2] - uy[3], Dly = uy[3] - uy[0], Dry = uy[2] - uy[1];
#define PF_QP(q)                                                                         \
  {                                                                                      \
    const double wB = QW<q>::wB, wT = QW<q>::wT, wL = QW<q>::wL, wR = QW<q>::wR;         \
    const double exx = (wB * Dbx + wT * Dtx) * ihx;                                      \
    const double uxy = (wL * Dlx + wR * Drx) * ihy;                                      \
    const double uyx = (wB * Dby + wT * Dty) * ihx;                                      \
    const double eyy = (wL * Dly + wR * Dry) * ihy;                                      \
    const double exy = 0.5 * (uxy + uyx);                                                \
    const double t = exx + eyy;                                                          \
    const double m3 = t * (1.0 / 3.0);                                                   \
    const double devdev = (exx - m3) * (exx - m3) + (eyy - m3) * (eyy - m3) + m3 * m3 + 2.0 * exy * exy; \
    const double tp = t > 0.0 ? t : 0.0;                                                 \
    double pvol, pdev;                                                                   \
    if (mt.split == 1) {                                                                 \
      const double hd = 0.5 * (exx - eyy);                                               \
      const double rr = sqrt(hd * hd + exy * exy);                                       \
      const double e1 = 0.5 * t + rr, e2 = 0.5 * t - rr;                                 \
      const double p1 = e1 > 0.0 ? e1 : 0.0, p2 = e2 > 0.0 ? e2 : 0.0;                   \
      pvol = 0.5 * mt.lam * tp * tp;                                                     \
      pdev = mt.mu * (p1 * p1 + p2 * p2);                                                \
    } else {                                                                             \
      pvol = 0.5 * mt.K * tp * tp;                                                       \
      pdev = mt.mu * devdev;                                                             \
    }                                                                                    \
    const double pplus = pvol + pdev;                                                    \
    if (psi_out) psi_out[e + q * g.E] = pplus;                                           \
    const double hp = Hprev[e + q * g.E];                                                \
    H[e + q * g.E] = pplus > hp ? pplus : hp;                                            \
    double ps = 0.0;                                                                     \
    if (qp.scheme == 1) ps = pvol;                                                       \
    else if (qp.scheme == 2) ps = pdev;                                                  \
    else if (qp.scheme == 3) ps = pplus;                                                 \
    psi_s[e + q * g.E] = ps;                                                             \
    if (t > 0.0) fl |= uint8_t(1u << q);                                                 \
    const double dq = interp4<double, q>(dn[0], dn[1], dn[2], dn[3]);                    \
    if (qp.scheme != 0 && pplus > qp.psi_crit && pplus > hp && dq < qp.d_gate) {          \
      fl |= uint8_t(1u << (q + 4));                                                      \
      ng += 1;                                                                           \
    }                                                                                    \
  }
      PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
    }
    qflag[e] = fl;
  }
  // block count of gated points (integer, order-independent)
  __shared__ unsigned long long shc[TPB / 64];
  for (int off = 32; off > 0; off >>= 1) ng += __shfl_down(ng, off, 64);
  if ((threadIdx.x & 63) == 0) shc[threadIdx.x >> 6] = ng;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += shc[w];
    if (s) atomicAdd(rs.icount + IC_GATED, s);
  }
}

// Tangent indicator bits only (tr eps > 0 at each QP), for the Newton tangent.
__global__ void __launch_bounds__(TPB) k_tangent_flags(Grid g, const double *u,
                                                       const uint8_t *eact, uint8_t *qflag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.E) return;
  const int ie = e % g.nx, je = e / g.nx;
  uint8_t fl = 0;
  if (eact == nullptr || eact[e] != 0) {
    const int n0 = ie + je * (g.nx + 1);
    const int nn[4] = {n0, n0 + 1, n0 + 1 + (g.nx + 1), n0 + (g.nx + 1)};
    double ux[4], uy[4];
    for (int a = 0; a < 4; ++a) {
      ux[a] = u[nn[a]];
      uy[a] = u[nn[a] + g.N];
    }
    const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy;
    const double Dbx = ux[1] - ux[0], Dtx = ux[2] - ux[3];
    const double Dly = uy[3] - uy[0], Dry = uy[2] - uy[1];
#define PF_QP(q)                                                                 \
  {                                                                              \
    const double exx = (QW<q>::wB * Dbx + QW<q>::wT * Dtx) * ihx;                \
    const double eyy = (QW<q>::wL * Dly + QW<q>::wR * Dry) * ihy;                \
    if (exx + eyy > 0.0) fl |= uint8_t(1u << q);                                 \
  }
    PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
  }
  qflag[e] = fl;
}

// Mass coefficient of the augmented block K_dd + K~ (Section 3.4): on gated
// points c - c_S floored at theta*c, c = Gc/l + 2H, c_S = 8(1-d)^2/g psi_S.
template <class T>
__global__ void __launch_bounds__(TPB) k_trial_coef(Grid g, Mat mt, double theta, int floor,
                                                    const double *H, const double *psi_s,
                                                    const uint8_t *qflag, const double *d,
                                                    const uint8_t *eact, const T *cbase, T *coef,
                                                    RedScratch rs) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long hits = 0;
  if (e < g.E) {
    const int ie = e % g.nx, je = e / g.nx;
    const bool act = (eact == nullptr) || eact[e] != 0;
    const uint8_t fl = qflag[e];
    double dn[4] = {0, 0, 0, 0};
    if (act && (fl >> 4)) {
      const int n0 = ie + je * (g.nx + 1);
      dn[0] = d[n0];
      dn[1] = d[n0 + 1];
      dn[2] = d[n0 + 1 + (g.nx + 1)];
      dn[3] = d[n0 + (g.nx + 1)];
    }
    const double Gc_l = mt.Gc / mt.l;
#define PF_QP(q)                                                                 \
  {                                                                              \
    const double c = cbase ? double(cbase[e + q * g.E])                          \
                           : Gc_l + 2.0 * H[e + q * g.E];                        \
    double ct = act ? c : 0.0;                                                   \
    if (act && ((fl >> (q + 4)) & 1u)) {                                         \
      const double dq = interp4<double, q>(dn[0], dn[1], dn[2], dn[3]);          \
      const double om = 1.0 - dq;                                                \
      const double cS = 8.0 * om * om / (om * om + mt.eta) * psi_s[e + q * g.E]; \
      ct = c - cS;                                                               \
      if (ct < theta * c) {                                                      \
        if (floor) ct = theta * c;                                               \
        hits += 1;                                                               \
      }                                                                          \
    }                                                                            \
    coef[e + q * g.E] = T(ct);                                                   \
  }
    PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
  }
  __shared__ unsigned long long shc[TPB / 64];
  for (int off = 32; off > 0; off >>= 1) hits += __shfl_down(hits, off, 64);
  if ((threadIdx.x & 63) == 0) shc[threadIdx.x >> 6] = hits;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += shc[w];
    if (s) atomicAdd(rs.icount + IC_FLOOR, s);
  }
}

template <class T>
__global__ void __launch_bounds__(TPB) k_at2_coef(Grid g, Mat mt, const double *H,
                                                  const uint8_t *eact, T *coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * g.E) return;
  const int e = i % g.E;
  const bool act = (eact == nullptr) || eact[e] != 0;
  coef[i] = act ? T(mt.Gc / mt.l + 2.0 * H[i]) : T(0);
}

// AT1 with the penalty: mass coefficient of the semismooth Newton matrix,
// 2 Psi+_q + gamma chi_q with chi_q = [d_q < d_{n-1,q}] at the quadrature
// point (Section 2, eq_evolution_equation).  With at_kink, points with
// d_q = d_{n-1,q} count as active too (the other generalised derivative at
// the kink).  chi is kept per point; the points whose chi changed since
// the last call are counted (IC_CHI).
template <class T>
__global__ void __launch_bounds__(TPB) k_at1_coef(Grid g, double gamma, const double *psi,
                                                  const double *d, const double *dprev,
                                                  const uint8_t *eact, T *coef, uint8_t *chi,
                                                  int at_kink, RedScratch rs) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long nc = 0;
  if (e < g.E) {
    const int ie = e % g.nx, je = e / g.nx;
    const bool act = (eact == nullptr) || eact[e] != 0;
    const int n0 = ie + je * (g.nx + 1);
    const int nn[4] = {n0, n0 + 1, n0 + 1 + (g.nx + 1), n0 + (g.nx + 1)};
    double dn[4], pn[4];
    for (int a = 0; a < 4; ++a) {
      dn[a] = d[nn[a]];
      pn[a] = dprev[nn[a]];
    }
#define PF_QP(q)                                                                 \
  {                                                                              \
    const int iq = e + q * g.E;                                                  \
    const double dq = interp4<double, q>(dn[0], dn[1], dn[2], dn[3]);            \
    const double pq = interp4<double, q>(pn[0], pn[1], pn[2], pn[3]);            \
    const uint8_t x = (act && (dq < pq || (at_kink && dq == pq))) ? 1 : 0;      \
    if (x != chi[iq]) nc += 1;                                                   \
    chi[iq] = x;                                                                 \
    coef[iq] = act ? T(2.0 * psi[iq] + (x ? gamma : 0.0)) : T(0);                \
  }
    PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
  }
  __shared__ unsigned long long shc[TPB / 64];
  for (int off = 32; off > 0; off >>= 1) nc += __shfl_down(nc, off, 64);
  if ((threadIdx.x & 63) == 0) shc[threadIdx.x >> 6] = nc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += shc[w];
    if (t) atomicAdd(rs.icount + IC_CHI, t);
  }
}

// Fixed-stress predictor: on gated points with Dd_q > 0 the active energy is
// advanced to the half step, psi+ (1 + a Dd)^2 on the scheme's part, a =
// 2(1-d)/g (eq:epn1, e_dev_1/2); elsewhere H is kept.
template <class TD>
__global__ void __launch_bounds__(TPB) k_predictor(Grid g, Mat mt, const double *d,
                                                   const TD *dd, const double *H,
                                                   const double *psi_s, const uint8_t *qflag,
                                                   const uint8_t *eact, double *Hhat) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.E) return;
  const int ie = e % g.nx, je = e / g.nx;
  const uint8_t fl = qflag[e];
  const bool act = (eact == nullptr) || eact[e] != 0;
  if (!act || (fl >> 4) == 0) {
    for (int q = 0; q < 4; ++q) Hhat[e + q * g.E] = H[e + q * g.E];
    return;
  }
  const int n0 = ie + je * (g.nx + 1);
  const int nn[4] = {n0, n0 + 1, n0 + 1 + (g.nx + 1), n0 + (g.nx + 1)};
  double dn[4], ddn[4];
  for (int a = 0; a < 4; ++a) {
    dn[a] = d[nn[a]];
    ddn[a] = double(dd[nn[a]]);
  }
#define PF_QP(q)                                                                 \
  {                                                                              \
    const double h = H[e + q * g.E];                                             \
    double out = h;                                                              \
    const double ddq = interp4<double, q>(ddn[0], ddn[1], ddn[2], ddn[3]);       \
    if (((fl >> (q + 4)) & 1u) && ddq > 0.0) {                                   \
      const double dq = interp4<double, q>(dn[0], dn[1], dn[2], dn[3]);          \
      const double om = 1.0 - dq;                                                \
      const double a = 2.0 * om / (om * om + mt.eta);                            \
      const double sc = 1.0 + a * ddq;                                           \
      const double ph = h + (sc * sc - 1.0) * psi_s[e + q * g.E];                \
      out = ph > h ? ph : h;                                                     \
    }                                                                            \
    Hhat[e + q * g.E] = out;                                                     \
  }
  PF_QP(0) PF_QP(1) PF_QP(2) PF_QP(3)
#undef PF_QP
}

// --------------------------------------------------------- small vectors

__global__ void k_lift(int n, const uint8_t *mask, uint8_t bits, int nmask,
                       const double *unit, double lam, double *u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t b = (i < nmask) ? (bits & 0x0f) : (bits >> 4);
  if (mask[i % nmask] & b) u[i] = lam * unit[i];
}

template <class TS>
__global__ void k_axpy_into(int n, double *out, const double *x, double alpha, const TS *y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i] + alpha * double(y[i]);
}

template <class TO, class TI>
__global__ void k_convert(int n, TO *out, const TI *in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = TO(in[i]);
}

__global__ void k_fill_zero(size_t nwords, uint32_t *p) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

__global__ void k_fill_zero_bytes(size_t n, uint8_t *p) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Reaction force of a Dirichlet group: fixed-order sum of R over its entries,
// split by component (single block, deterministic).
__global__ void __launch_bounds__(TPB) k_group_sum(int n, const int64_t *dof,
                                                   const int8_t *comp, const double *R,
                                                   RedScratch rs) {
  double v[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double r = R[dof[i]];
    if (comp[i] == 0) v[0] += r; else v[1] += r;
  }
  block_partial<2>(v, rs.partR);
  __syncthreads();
  if (threadIdx.x == 0) {
    rs.scal[SC_SUM_X] = rs.partR[0];
    rs.scal[SC_SUM_Y] = rs.partR[kPMax];
  }
}

// ---- starting guess of a displacement solve from earlier solutions

// Per thread over a grid stride: v_j . w_k (j <= k), v_j . b and b . b in
// FP64, then block partials (unused pairs add 0).
template <class T>
__global__ void __launch_bounds__(TPB) k_guess_dots(GuessArgs<T> a, const T *b, double *part) {
  double acc[kGuessDots];
#pragma unroll
  for (int k = 0; k < kGuessDots; ++k) acc[k] = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    double v[kGuessMax], w[kGuessMax];
#pragma unroll
    for (int j = 0; j < kGuessMax; ++j) {
      v[j] = j < a.m ? double(a.v[j][i]) : 0.0;
      w[j] = j < a.m ? double(a.w[j][i]) : 0.0;
    }
    const double bi = double(b[i]);
    int k = 0;
#pragma unroll
    for (int j = 0; j < kGuessMax; ++j)
#pragma unroll
      for (int l = j; l < kGuessMax; ++l) acc[k++] += v[j] * w[l];
#pragma unroll
    for (int j = 0; j < kGuessMax; ++j) acc[k++] += v[j] * bi;
    acc[k] += bi * bi;
  }
  block_partial<kGuessDots>(acc, part);
}

// One block: each of nv partial arrays (stride kPMax) summed in the fixed
// order of block_sum, to out[k].
__global__ void __launch_bounds__(TPB) k_finalize_each(const double *part, int np, int nv,
                                                       double *out) {
  for (int k = 0; k < nv; ++k) {
    double s[1];
    block_sum<1>(part + k * kPMax, np, s);
    if (threadIdx.x == 0) out[k] = s[0];
  }
}

template <class T>
__global__ void __launch_bounds__(TPB) k_guess_combine(GuessArgs<T> a, GuessCoef c, T *x,
                                                       T *rb) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    double xi = 0.0, ri = double(rb[i]);
#pragma unroll
    for (int j = 0; j < kGuessMax; ++j)
      if (j < a.m) {
        xi += c.c[j] * double(a.v[j][i]);
        ri -= c.c[j] * double(a.w[j][i]);
      }
    x[i] = T(xi);
    rb[i] = T(ri);
  }
}

// ------------------------------------------------------------- MINRES
//
// Preconditioned MINRES for the unfloored trial block of the evolution
// equation, which is symmetric but may be indefinite (FP64).  Lanczos with
// M = |diag A| builds v_j; a Givens QR of the tridiagonal matrix gives the
// minimum-residual iterate x_j = x_{j-1} + phi_j w_j with
// w_j = (v_j - eps_j w_{j-2} - delta_j w_{j-1}) / gamma_j.

// Scalars of step j's apply, the same in every block.
struct MrStep {
  double s;       // 1 / beta_j  (v_j = s y_{j-1})
  double sprev;   // 1 / beta_{j-1}
  double oldeps, delta, igamma, phi;   // rotation of step j - 1
  int upd;        // 1: update w and x of step j - 1
  int done;       // -1 finished before this launch, else MrHalf::done
};

// Reduce beta_j, rotate for step j - 1 and test convergence; block 0
// records the state in half a.
__device__ inline MrStep mr_apply_prologue(const MrArgs &a, int bid) {
  MrStep m{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0, 0};
  MrHalf h = a.st->b;
  if (h.done != 0) {
    m.done = -1;
    return m;
  }
  double s2[1];
  block_sum<1>(a.partB, a.gb, s2);
  int done = 0;
  if (!(s2[0] >= 0.0) || !isfinite(s2[0])) done = 2;   // M must be SPD
  const double beta = done ? 0.0 : sqrt(s2[0]);
  if (h.first) {
    h.beta1 = beta;
    h.phibar = beta;
    h.cs = -1.0;
    h.sn = 0.0;
    h.dbar = 0.0;
    h.epsln = 0.0;
    if (done == 0 && beta == 0.0) done = 1;   // b = 0: x = 0
  } else if (done == 0) {
    const double oldeps = h.epsln;
    const double delta = h.cs * h.dbar + h.sn * h.alfa;
    const double gbar = h.sn * h.dbar - h.cs * h.alfa;
    h.epsln = h.sn * beta;
    h.dbar = -h.cs * beta;
    const double gamma = sqrt(gbar * gbar + beta * beta);
    if (!(gamma > 0.0) || !isfinite(gamma)) {
      done = 2;   // singular tridiagonal: no minimum-residual step
    } else {
      h.cs = gbar / gamma;
      h.sn = beta / gamma;
      m.phi = h.cs * h.phibar;
      h.phibar = h.sn * h.phibar;
      m.oldeps = oldeps;
      m.delta = delta;
      m.igamma = 1.0 / gamma;
      m.sprev = 1.0 / h.beta;
      m.upd = 1;
      h.iters += 1;
      // beta = 0 ends the Lanczos process with sn = 0, phibar = 0
      if (h.phibar <= a.tol * h.beta1) done = 1;
      else if (h.iters >= a.maxit) done = 3;
    }
  }
  h.oldb = h.first ? 0.0 : h.beta;
  h.beta = beta;
  h.first = 0;
  h.done = done;
  if (bid == 0 && threadIdx.x == 0) a.st->a = h;
  m.s = beta > 0.0 ? 1.0 / beta : 0.0;
  m.done = done;
  return m;
}

// Apply of Lanczos step j on top of a phase operator whose input vector is
// y_{j-1}: q = A v_j with v_j = y_{j-1} / beta_j; the stored nodes also take
// w_{j-1} = (v_{j-1} - eps w_{j-3} - delta w_{j-2}) / gamma into wo (which
// holds w_{j-3}) and x += phi w_{j-1}.  Partials: v_j . q.
template <class Base>
struct OpMrApply {
  using T = typename Base::T;
  using Elem = typename Base::Elem;
  using Node = typename Base::Node;
  static constexpr int NF = 1;
  static constexpr int NR = 1;
  Base base;
  const T *yprev;   // y_{j-2}
  T *wo;            // w_{j-3} in, w_{j-1} out
  const T *wb;      // w_{j-2}
  T *x; T *q;
  T s, sprev, oldeps, delta, igamma, phi;
  int upd;
  __device__ Node load(int i, int j) const { return base.load(i, j); }
  __device__ void fin(Node &n) const {
    T u[1];
    base.get_u(n, u);
    u[0] *= s;
    base.set_u(n, u);
  }
  __device__ Elem eload(int ie, int je) const { return base.eload(ie, je); }
  static __device__ Node shfl_up(const Node &n) { return Base::shfl_up(n); }
  __device__ void element(const Node &n0, const Node &n1, const Node &n2, const Node &n3,
                          const Elem &e, T (&f)[1][4]) const {
    base.element(n0, n1, n2, n3, e, f);
  }
  struct Own {
    typename Base::Own b;
    T yp, wa, wbv, xv;
  };
  __device__ Own load_own(int i, int j) const {
    Own o;
    o.b = base.load_own(i, j);
    o.yp = o.wa = o.wbv = o.xv = T(0);
    if (node_exists(base.g, i, j)) {
      const int k = i + j * (base.g.nx + 1);
      o.yp = yprev[k];
      o.wa = wo[k];
      o.wbv = wb[k];
      o.xv = x[k];
    }
    return o;
  }
  __device__ void store(int i, int j, const T (&v)[1], const Node &n, const Own &o,
                        double *red) const {
    const int k = i + j * (base.g.nx + 1);
    T vv[1];
    base.get_u(n, vv);
    const T qv = Base::masked_own(o.b, 0) ? T(0) : v[0];
    q[k] = qv;
    red[0] += double(vv[0]) * double(qv);
    if (upd) {
      const T wn = (o.yp * sprev - oldeps * o.wa - delta * o.wbv) * igamma;
      wo[k] = wn;
      x[k] = o.xv + phi * wn;
    }
  }
};

template <int CH, class Op>
__global__ void __launch_bounds__(TPB) k_mr_apply(Op op, Grid g, March ms, MrArgs a, int n) {
  const int bid = blockIdx.x, nb = gridDim.x;
  const int lane = threadIdx.x & 63;
  const int w0 = xcd_block(bid, nb) * WPB + (threadIdx.x >> 6);
  const int nw = ms.nstrips * ms.nchunks;
  // the first work item's loads are in flight during the prologue
  Item<CH, Op> it;
  if (w0 < nw) item_load<CH>(op, g, ms, w0, lane, it);
  const MrStep m = mr_apply_prologue(a, bid);
  if (m.done < 0 || m.done == 2) return;
  if (m.done != 0) {
    // converged or capped: only the last step's w and x update remains
    if (m.upd) {
      for (int k = bid * TPB + threadIdx.x; k < n; k += nb * TPB) {
        const double wn = (op.yprev[k] * m.sprev - m.oldeps * op.wo[k] - m.delta * op.wb[k]) *
                          m.igamma;
        op.wo[k] = wn;
        op.x[k] += m.phi * wn;
      }
    }
    return;
  }
  op.s = m.s;
  op.sprev = m.sprev;
  op.oldeps = m.oldeps;
  op.delta = m.delta;
  op.igamma = m.igamma;
  op.phi = m.phi;
  op.upd = m.upd;
  double red[1] = {0.0};
  if (w0 < nw) item_compute<CH>(op, g, ms, w0, lane, it, red);
  march_items<CH>(op, g, ms, w0 + nb * WPB, nb * WPB, red);
  block_partial_at<1>(red, a.partA, bid);
}

__global__ void __launch_bounds__(TPB) k_mr_init(int n, const double *rhs, MrVecs v, MrArgs a) {
  double acc[1] = {0.0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double b = rhs[i];
    v.r[0][i] = 0.0;
    v.r[1][i] = b;
    v.x[i] = 0.0;
    v.w[0][i] = 0.0;
    v.w[1][i] = 0.0;
    const double y = v.Dinv[i] * b;
    v.y[0][i] = y;
    acc[0] += b * y;
  }
  block_partial<1>(acc, a.partB);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    MrHalf h{};
    h.first = 1;
    a.st->a = h;
    a.st->b = h;
  }
}

// Vector kernel of step j: r_{j+1} (into the slot of r_{j-1}), y_j and the
// partials of beta_{j+1}^2; block 0 publishes the state in half b.
__global__ void __launch_bounds__(TPB) k_mr_update(int n, MrVecs v, MrArgs a, int j) {
  MrHalf h = a.st->a;
  if (h.done != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a.st->b = h;
    return;
  }
  double al[1];
  block_sum<1>(a.partA, a.ga, al);
  const double alfa = al[0];
  if (!isfinite(alfa)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      h.done = 2;
      a.st->b = h;
    }
    return;
  }
  const double c1 = alfa / h.beta;
  const double c2 = h.oldb > 0.0 ? h.beta / h.oldb : 0.0;
  const double *rj = v.r[j & 1];
  double *rm = v.r[(j + 1) & 1];
  double *y = v.y[j & 1];
  double acc[1] = {0.0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double rn = v.q[i] - c1 * rj[i] - c2 * rm[i];
    rm[i] = rn;
    const double yi = v.Dinv[i] * rn;
    y[i] = yi;
    acc[0] += rn * yi;
  }
  block_partial<1>(acc, a.partB);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h.alfa = alfa;
    a.st->b = h;
  }
}

}  // namespace

// ======================================================== host launchers

March march_shape(const Grid &g, int ch_override) {
  March m;
  if (ch_override == 1) {
    m.ch = 1;
    m.nstrips = (g.nx + 1 + kTile - 1) / kTile;
    m.nchunks = (g.ny + 1 + kTile - 1) / kTile;
    return m;
  }
  m.nstrips = (g.nx + 1 + CSTRIP - 1) / CSTRIP;
  int ch = ch_override;
  if (ch != 2 && ch != 4 && ch != 8) {
    // smallest chunk that gives at most two work items per SIMD
    const long long waves = 2LL * 4 * 256;
    ch = 8;
    for (int c : {2, 4}) {
      if ((long long)m.nstrips * ((g.ny + 1 + c - 1) / c) <= waves) {
        ch = c;
        break;
      }
    }
  }
  m.ch = ch;
  m.nchunks = (g.ny + 1 + ch - 1) / ch;
  return m;
}







template <class T>
hipError_t cg_init(hipStream_t s, int n, T *x, T *r, T *z, T *p_old, const T *Dinv,
                   const CgArgs &ca) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_init<T>), dim3(ca.gb), dim3(TPB), 0, s, n, x, r, z,
                     p_old, Dinv, ca);
  return hipGetLastError();
}

template <class T>
hipError_t cg_update(hipStream_t s, int n, T *x, T *r, T *z, const T *p, const T *q,
                     const T *Dinv, const CgArgs &ca, const ChebFuse<T> &cf) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_update<T>), dim3(ca.gb), dim3(TPB), 0, s, n, x, r, z,
                     p, q, Dinv, ca, cf);
  return hipGetLastError();
}

template <class Op>
hipError_t launch_cg_apply(hipStream_t s, const Op &op, const Grid &g, const March &m,
                           const CgArgs &ca) {
  const dim3 grid(ca.ga), block(TPB);
  switch (m.ch) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_apply<1, Op>), grid, block, 0, s, op, g, m, ca); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_apply<2, Op>), grid, block, 0, s, op, g, m, ca); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_apply<4, Op>), grid, block, 0, s, op, g, m, ca); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_apply<8, Op>), grid, block, 0, s, op, g, m, ca); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t tangent_cg_apply(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                            int split, const T *ulin, const T *d, const uint8_t *qflag,
                            const uint8_t *eact, const uint8_t *nflag, const T *z,
                            const T *p_old, T *p_new, T *q, const CgArgs &ca) {
  if (split == 1) {
    using Op = OpTangent<T, true, true, 1>;
    Op op{g, c, d, qflag, eact, nflag, z, p_old, p_new, q, T(0), ulin};
    return launch_cg_apply(s, op, g, m, ca);
  }
  using Op = OpTangent<T, true, true, 0>;
  Op op{g, c, d, qflag, eact, nflag, z, p_old, p_new, q, T(0), nullptr};
  return launch_cg_apply(s, op, g, m, ca);
}

template <class T>
hipError_t phase_cg_apply(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const T *coef, const uint8_t *eact, const uint8_t *nflag, const T *z,
                          const T *p_old, T *p_new, T *q, const CgArgs &ca) {
  using Op = OpPhase<T, true, true>;
  Op op{g, c, coef, eact, nflag, z, p_old, p_new, q, T(0)};
  return launch_cg_apply(s, op, g, m, ca);
}

template <class Op>
void write_batch_entry(void *dst, const Op &op, const Grid &g, const March &m, const CgArgs &ca,
                       int b0, int nb) {
  static_assert(sizeof(BatchApplyEntry<Op>) <= kBatchEntryBytes, "batch entry too large");
  BatchApplyEntry<Op> e{op, g, m, ca, b0, nb};
  std::memcpy(dst, &e, sizeof(e));
}

template <class T>
void tangent_batch_entry(void *dst, const Grid &g, const March &m, const ElasCoef &c, int split,
                         const T *ulin, const T *d, const uint8_t *qflag, const uint8_t *eact,
                         const uint8_t *nflag, const T *z, const T *p_old, T *p_new, T *q,
                         const CgArgs &ca, int b0, int nb) {
  if (split == 1) {
    using Op = OpTangent<T, true, true, 1>;
    write_batch_entry(dst, Op{g, c, d, qflag, eact, nflag, z, p_old, p_new, q, T(0), ulin}, g, m,
                      ca, b0, nb);
  } else {
    using Op = OpTangent<T, true, true, 0>;
    write_batch_entry(dst, Op{g, c, d, qflag, eact, nflag, z, p_old, p_new, q, T(0), nullptr}, g,
                      m, ca, b0, nb);
  }
}

template <class T>
void phase_batch_entry(void *dst, const Grid &g, const March &m, const PhaseCoef &c,
                       const T *coef, const uint8_t *eact, const uint8_t *nflag, const T *z,
                       const T *p_old, T *p_new, T *q, const CgArgs &ca, int b0, int nb) {
  using Op = OpPhase<T, true, true>;
  write_batch_entry(dst, Op{g, c, coef, eact, nflag, z, p_old, p_new, q, T(0)}, g, m, ca, b0, nb);
}

template <class Op>
hipError_t launch_apply_batch(hipStream_t s, int ch, const void *tab, const int *bmap,
                              int nblocks) {
  const dim3 grid(nblocks), block(TPB);
  const char *t = static_cast<const char *>(tab);
  switch (ch) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_apply_batch<1, Op>), grid, block, 0, s, t, bmap); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_apply_batch<2, Op>), grid, block, 0, s, t, bmap); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_apply_batch<4, Op>), grid, block, 0, s, t, bmap); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_apply_batch<8, Op>), grid, block, 0, s, t, bmap); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t tangent_cg_apply_batch(hipStream_t s, int split, int ch, const void *tab,
                                  const int *bmap, int nblocks) {
  if (split == 1) return launch_apply_batch<OpTangent<T, true, true, 1>>(s, ch, tab, bmap, nblocks);
  return launch_apply_batch<OpTangent<T, true, true, 0>>(s, ch, tab, bmap, nblocks);
}

template <class T>
hipError_t phase_cg_apply_batch(hipStream_t s, int ch, const void *tab, const int *bmap,
                                int nblocks) {
  return launch_apply_batch<OpPhase<T, true, true>>(s, ch, tab, bmap, nblocks);
}

template <class T>
hipError_t cg_update_batch(hipStream_t s, const BatchUpdateEntry<T> *tab, const int *bmap,
                           int nblocks) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_update_batch<T>), dim3(nblocks), dim3(TPB), 0, s, tab,
                     bmap);
  return hipGetLastError();
}

CgArgs cg_args(const Grid &, const March &m, int n, CgState *st, RedScratch rs, double tol,
               int maxit) {
  CgArgs ca;
  ca.st = st;
  ca.partA = rs.partR;
  ca.partB = rs.partR + 2 * kPMax;
  ca.ga = march_blocks(m);
  ca.gb = vec_blocks(n);
  ca.tol2 = tol * tol;
  ca.maxit = maxit;
  ca.ext = 0;
  ca.npb = ca.gb;
  ca.warm = 0;
  ca.rr_abs = 0.0;
  return ca;
}

template <class Op>
hipError_t launch_updcheb(hipStream_t s, const Op &op, const Grid &g, const March &m,
                          const CgArgs &ca) {
  const dim3 grid(march_blocks(m)), block(TPB);
  switch (m.ch) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_updcheb<1, Op>), grid, block, 0, s, op, g, m, ca); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_updcheb<2, Op>), grid, block, 0, s, op, g, m, ca); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_updcheb<4, Op>), grid, block, 0, s, op, g, m, ca); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_updcheb<8, Op>), grid, block, 0, s, op, g, m, ca); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t tangent_updcheb(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                           int split, const T *ulin, const T *d, const uint8_t *qflag,
                           const uint8_t *eact, const uint8_t *nflag, const T *x_in, T *x_out,
                           const T *r_in, T *r_out, const T *p, const T *q, const T *Dinv,
                           T *dnext, T *z_out, T *res_out, const CgArgs &ca, const ChebStep &s0,
                           const ChebStep &s1) {
  if (split == 1) {
    using B = OpTangent<T, false, true, 1>;
    OpUpdCheb<B> op{B{g, c, d, qflag, eact, nflag, nullptr, nullptr, nullptr, nullptr, T(0), ulin},
                    x_in, r_in, x_out, r_out, p, q, Dinv, dnext, z_out, res_out, g.N, s1.coef,
                    T(0), 0, s1.last};
    return launch_updcheb(s, op, g, m, ca);
  }
  using B = OpTangent<T, false, true, 0>;
  OpUpdCheb<B> op{B{g, c, d, qflag, eact, nflag, nullptr, nullptr, nullptr, nullptr, T(0), nullptr},
                  x_in, r_in, x_out, r_out, p, q, Dinv, dnext, z_out, res_out, g.N, s1.coef,
                  T(0), 0, s1.last};
  return launch_updcheb(s, op, g, m, ca);
}

template <class T>
hipError_t phase_updcheb(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                         const T *coef, const uint8_t *eact, const uint8_t *nflag,
                         const T *x_in, T *x_out, const T *r_in, T *r_out, const T *p,
                         const T *q, const T *Dinv, T *dnext, T *z_out, T *res_out,
                         const CgArgs &ca, const ChebStep &s0, const ChebStep &s1) {
  using B = OpPhase<T, false, true>;
  OpUpdCheb<B> op{B{g, c, coef, eact, nflag, nullptr, nullptr, nullptr, nullptr, T(0)}, x_in,
                  r_in, x_out, r_out, p, q, Dinv, dnext, z_out, res_out, g.N, s1.coef, T(0), 0,
                  s1.last};
  return launch_updcheb(s, op, g, m, ca);
}

template <class Base>
hipError_t launch_updcheb2(hipStream_t s, const UpdCheb2<Base> &op, const Grid &g,
                           const March &m, const CgArgs &ca) {
  if (m.ch != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_updcheb2<Base>), dim3(march_blocks(m)), dim3(TPB), 0, s,
                     op, g, m, ca);
  return hipGetLastError();
}

template <class T>
hipError_t tangent_updcheb2(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                            int split, const T *ulin, const T *d, const uint8_t *qflag,
                            const uint8_t *eact, const uint8_t *nflag, const T *x_in, T *x_out,
                            const T *r_in, T *r_out, const T *p, const T *q, const T *Dinv,
                            T *dnext, T *z_out, T *res_out, const CgArgs &ca,
                            const ChebStep &s2) {
  if (split == 1) {
    using B = OpTangent<T, false, true, 1>;
    UpdCheb2<B> op{B{g, c, d, qflag, eact, nflag, nullptr, nullptr, nullptr, nullptr, T(0), ulin},
                   x_in, r_in, x_out, r_out, p, q, Dinv, dnext, z_out, res_out, g.N, s2.coef,
                   s2.last};
    return launch_updcheb2(s, op, g, m, ca);
  }
  using B = OpTangent<T, false, true, 0>;
  UpdCheb2<B> op{B{g, c, d, qflag, eact, nflag, nullptr, nullptr, nullptr, nullptr, T(0), nullptr},
                 x_in, r_in, x_out, r_out, p, q, Dinv, dnext, z_out, res_out, g.N, s2.coef,
                 s2.last};
  return launch_updcheb2(s, op, g, m, ca);
}

template <class T>
hipError_t phase_updcheb2(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const T *coef, const uint8_t *eact, const uint8_t *nflag,
                          const T *x_in, T *x_out, const T *r_in, T *r_out, const T *p,
                          const T *q, const T *Dinv, T *dnext, T *z_out, T *res_out,
                          const CgArgs &ca, const ChebStep &s2) {
  using B = OpPhase<T, false, true>;
  UpdCheb2<B> op{B{g, c, coef, eact, nflag, nullptr, nullptr, nullptr, nullptr, T(0)}, x_in, r_in,
                 x_out, r_out, p, q, Dinv, dnext, z_out, res_out, g.N, s2.coef, s2.last};
  return launch_updcheb2(s, op, g, m, ca);
}

template <class T>
hipError_t cheb_init(hipStream_t s, int n, const T *r, const T *Dinv, T *d0, T *z, T *res,
                     const CgArgs &ca, const ChebStep &cs) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cheb_init<T>), dim3(ca.gb), dim3(TPB), 0, s, n, r, Dinv,
                     d0, z, res, ca, cs);
  return hipGetLastError();
}

template <class T>
hipError_t tangent_cheb_step(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                             int split, const T *ulin, const T *d, const uint8_t *qflag,
                             const uint8_t *eact, const uint8_t *nflag, const T *dprev, T *dnext,
                             const T *z_in, T *z_out, const T *res_in, T *res_out, const T *r,
                             const T *Dinv, const CgArgs &ca, const ChebStep &cs) {
  if (split == 1) {
    using B = OpTangent<T, false, true, 1>;
    OpCheb<B> op{B{g, c, d, qflag, eact, nflag, dprev, nullptr, nullptr, nullptr, T(0), ulin},
                 r, Dinv, dnext, z_in, res_in, z_out, res_out, g.N, cs.coef, cs.k, cs.last};
    return launch_march(s, op, g, m, ca.partB);
  }
  using B = OpTangent<T, false, true, 0>;
  OpCheb<B> op{B{g, c, d, qflag, eact, nflag, dprev, nullptr, nullptr, nullptr, T(0), nullptr},
               r, Dinv, dnext, z_in, res_in, z_out, res_out, g.N, cs.coef, cs.k, cs.last};
  return launch_march(s, op, g, m, ca.partB);
}

template <class T>
hipError_t phase_cheb_step(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                           const T *coef, const uint8_t *eact, const uint8_t *nflag,
                           const T *dprev, T *dnext, const T *z_in, T *z_out, const T *res_in,
                           T *res_out, const T *r, const T *Dinv, const CgArgs &ca,
                           const ChebStep &cs) {
  using B = OpPhase<T, false, true>;
  OpCheb<B> op{B{g, c, coef, eact, nflag, dprev, nullptr, nullptr, nullptr, T(0)}, r, Dinv,
               dnext, z_in, res_in, z_out, res_out, g.N, cs.coef, cs.k, cs.last};
  return launch_march(s, op, g, m, ca.partB);
}

template <class T>
hipError_t tangent_power_step(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                              int split, const T *ulin, const T *d, const uint8_t *qflag,
                              const uint8_t *eact, const uint8_t *nflag, const T *v, T *vnext,
                              const T *Dinv, double scale, RedScratch rs) {
  if (split == 1) {
    using B = OpTangent<T, false, true, 1>;
    OpPower<B> op{B{g, c, d, qflag, eact, nflag, v, nullptr, nullptr, nullptr, T(0), ulin}, Dinv,
                  vnext, g.N, T(scale)};
    return launch_march_reduce<OpPower<B>, 2>(s, op, g, m, rs, SC_NORM_A);
  }
  using B = OpTangent<T, false, true, 0>;
  OpPower<B> op{B{g, c, d, qflag, eact, nflag, v, nullptr, nullptr, nullptr, T(0), nullptr}, Dinv,
                vnext, g.N, T(scale)};
  return launch_march_reduce<OpPower<B>, 2>(s, op, g, m, rs, SC_NORM_A);
}

template <class T>
hipError_t phase_power_step(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                            const T *coef, const uint8_t *eact, const uint8_t *nflag, const T *v,
                            T *vnext, const T *Dinv, double scale, RedScratch rs) {
  using B = OpPhase<T, false, true>;
  OpPower<B> op{B{g, c, coef, eact, nflag, v, nullptr, nullptr, nullptr, T(0)}, Dinv, vnext, g.N,
                T(scale)};
  return launch_march_reduce<OpPower<B>, 2>(s, op, g, m, rs, SC_NORM_A);
}

template <class T>
hipError_t power_start(hipStream_t s, int n, const T *Dinv, T *v) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_power_start<T>), dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s,
                     n, Dinv, v);
  return hipGetLastError();
}

int cg1_blocks(const March &m) { return march_blocks(m); }

template <class Op>
hipError_t launch_cg1(hipStream_t s, const Op &op, const Grid &g, const March &m,
                      const CgVecs<typename Op::T> &v, const Cg1Args &a) {
  const dim3 grid(a.np), block(TPB);
  switch (m.ch) {
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg1<2, Op>), grid, block, 0, s, op, g, m, v, a); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg1<4, Op>), grid, block, 0, s, op, g, m, v, a); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg1<8, Op>), grid, block, 0, s, op, g, m, v, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t tangent_cg1(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                       int split, const T *ulin, const T *d, const uint8_t *qflag,
                       const uint8_t *eact, const uint8_t *nflag, const CgVecs<T> &v,
                       const Cg1Args &a) {
  if (split == 1) {
    OpTangent<T, false, true, 1> op{g, c, d, qflag, eact, nflag, nullptr, nullptr, nullptr,
                                    nullptr, T(0), ulin};
    return launch_cg1(s, op, g, m, v, a);
  }
  OpTangent<T, false, true, 0> op{g, c, d, qflag, eact, nflag, nullptr, nullptr, nullptr,
                                  nullptr, T(0), nullptr};
  return launch_cg1(s, op, g, m, v, a);
}

template <class T>
hipError_t phase_cg1(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                     const T *coef, const uint8_t *eact, const uint8_t *nflag,
                     const CgVecs<T> &v, const Cg1Args &a) {
  OpPhase<T, false, true> op{g, c, coef, eact, nflag, nullptr, nullptr, nullptr, nullptr, T(0)};
  return launch_cg1(s, op, g, m, v, a);
}

template <class T>
hipError_t tangent_diag(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                        int split, const T *ulin, const T *d, const uint8_t *qflag,
                        const uint8_t *eact, const uint8_t *nflag, T *Dinv) {
  if (split == 1) {
    OpTangentDiag<T, 1> op{g, c, d, qflag, eact, nflag, Dinv, ulin};
    return launch_march(s, op, g, m, nullptr);
  }
  OpTangentDiag<T, 0> op{g, c, d, qflag, eact, nflag, Dinv, nullptr};
  return launch_march(s, op, g, m, nullptr);
}

template <class T>
hipError_t phase_diag(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                      const T *coef, const uint8_t *eact, const uint8_t *nflag, T *Dinv,
                      int absdiag) {
  OpPhaseDiag<T> op{g, c, coef, eact, nflag, Dinv, absdiag};
  return launch_march(s, op, g, m, nullptr);
}

int vec_block_count(int n) { return vec_blocks(n); }

hipError_t mr_init(hipStream_t s, int n, const double *rhs, const MrVecs &v, const MrArgs &a) {
  if (a.gb != vec_blocks(n)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mr_init, dim3(a.gb), dim3(TPB), 0, s, n, rhs, v, a);
  return hipGetLastError();
}

hipError_t phase_mr_apply(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const double *coef, const uint8_t *eact, const uint8_t *nflag,
                          const MrVecs &v, const MrArgs &a, int j) {
  if (j < 1 || a.ga != march_blocks(m)) return hipErrorInvalidValue;
  using B = OpPhase<double, false, true>;
  using Op = OpMrApply<B>;
  Op op{B{g, c, coef, eact, nflag, v.y[(j - 1) & 1], nullptr, nullptr, nullptr, 0.0},
        v.y[j & 1], v.w[(j - 1) & 1], v.w[j & 1], v.x, v.q, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0};
  const dim3 grid(a.ga), block(TPB);
  switch (m.ch) {
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mr_apply<2, Op>), grid, block, 0, s, op, g, m, a, g.N); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mr_apply<4, Op>), grid, block, 0, s, op, g, m, a, g.N); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mr_apply<8, Op>), grid, block, 0, s, op, g, m, a, g.N); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mr_update(hipStream_t s, int n, const MrVecs &v, const MrArgs &a, int j) {
  if (j < 1 || a.gb != vec_blocks(n)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mr_update, dim3(a.gb), dim3(TPB), 0, s, n, v, a, j);
  return hipGetLastError();
}

hipError_t tangent_apply_plain(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                               int split, const double *ulin, const double *d,
                               const uint8_t *qflag, const uint8_t *eact, const double *p,
                               double *q) {
  if (split == 1) {
    OpTangent<double, false, false, 1> op{g, c, d, qflag, eact, nullptr, p, nullptr, nullptr, q,
                                          0.0, ulin};
    return launch_march(s, op, g, m, nullptr);
  }
  OpTangent<double, false, false, 0> op{g, c, d, qflag, eact, nullptr, p, nullptr, nullptr, q,
                                        0.0, nullptr};
  return launch_march(s, op, g, m, nullptr);
}

template <class T>
hipError_t tangent_apply_masked(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                                int split, const T *ulin, const T *d, const uint8_t *qflag,
                                const uint8_t *eact, const uint8_t *nflag, const T *p, T *q) {
  if (split == 1) {
    OpTangent<T, false, true, 1> op{g, c, d, qflag, eact, nflag, p, nullptr, nullptr, q, T(0),
                                    ulin};
    return launch_march(s, op, g, m, nullptr);
  }
  OpTangent<T, false, true, 0> op{g, c, d, qflag, eact, nflag, p, nullptr, nullptr, q, T(0),
                                  nullptr};
  return launch_march(s, op, g, m, nullptr);
}

template <class T>
hipError_t guess_dots(hipStream_t s, const GuessArgs<T> &a, const T *b, double *part,
                      double *out) {
  const int nb = vec_blocks(a.n);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_guess_dots<T>), dim3(nb), dim3(TPB), 0, s, a, b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize_each, dim3(1), dim3(TPB), 0, s, part, nb, kGuessDots, out);
  return hipGetLastError();
}

template <class T>
hipError_t guess_combine(hipStream_t s, const GuessArgs<T> &a, const GuessCoef &c, T *x, T *rb) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_guess_combine<T>), dim3(vec_blocks(a.n)), dim3(TPB), 0, s,
                     a, c, x, rb);
  return hipGetLastError();
}

hipError_t phase_apply_plain(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                             const double *coef, const uint8_t *eact, const double *p,
                             double *q) {
  OpPhase<double, false, false> op{g, c, coef, eact, nullptr, p, nullptr, nullptr, q, 0.0};
  return launch_march(s, op, g, m, nullptr);
}

hipError_t internal_force(hipStream_t s, const Grid &g, const March &m, const ElasCoef &c,
                          int split, const double *u, const double *d, const uint8_t *eact,
                          const uint8_t *nflag, bool neg, double *R, RedScratch rs) {
  if (split == 1) {
    OpForce<1> op{g, c, u, d, eact, nflag, R, neg ? -1.0 : 1.0};
    return launch_march_reduce<OpForce<1>, 1>(s, op, g, m, rs, SC_NORM_A);
  }
  OpForce<0> op{g, c, u, d, eact, nflag, R, neg ? -1.0 : 1.0};
  return launch_march_reduce<OpForce<0>, 1>(s, op, g, m, rs, SC_NORM_A);
}

hipError_t phase_residual(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                          const double *H, const double *d, const uint8_t *eact,
                          const uint8_t *nflag, bool neg, double *R, RedScratch rs) {
  OpPhaseRes op{g, c, H, d, eact, nflag, R, neg ? -1.0 : 1.0};
  return launch_march_reduce<OpPhaseRes, 2>(s, op, g, m, rs, SC_NORM_A);
}

hipError_t phase_residual_at1(hipStream_t s, const Grid &g, const March &m, const PhaseCoef &c,
                              const double *psi, const double *d, const double *dprev,
                              double gamma, const uint8_t *eact, const uint8_t *nflag, bool neg,
                              double *R, RedScratch rs) {
  OpPhaseResAT1 op{g, c, psi, d, dprev, eact, nflag, R, neg ? -1.0 : 1.0, gamma};
  return launch_march_reduce<OpPhaseResAT1, 2>(s, op, g, m, rs, SC_NORM_A);
}

hipError_t at1_coef(hipStream_t s, const Grid &g, double gamma, const double *psi,
                    const double *d, const double *dprev, const uint8_t *eact, double *coef,
                    uint8_t *chi, int at_kink, RedScratch rs) {
  const int blocks = (g.E + TPB - 1) / TPB;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_at1_coef<double>), dim3(blocks), dim3(TPB), 0, s, g, gamma,
                     psi, d, dprev, eact, coef, chi, at_kink, rs);
  return hipGetLastError();
}

hipError_t qp_update(hipStream_t s, const Grid &g, const Mat &mt, const QpParams &qp,
                     const double *u, const double *d, const uint8_t *eact,
                     const double *H_prev, double *H, double *psi_s, uint8_t *qflag,
                     double *psi_out, RedScratch rs) {
  const int blocks = (g.E + TPB - 1) / TPB;
  hipLaunchKernelGGL(k_qp_update, dim3(blocks), dim3(TPB), 0, s, g, mt, qp, u, d, eact, H_prev,
                     H, psi_s, qflag, psi_out, rs);
  return hipGetLastError();
}

hipError_t tangent_flags(hipStream_t s, const Grid &g, const double *u, const uint8_t *eact,
                         uint8_t *qflag) {
  const int blocks = (g.E + TPB - 1) / TPB;
  hipLaunchKernelGGL(k_tangent_flags, dim3(blocks), dim3(TPB), 0, s, g, u, eact, qflag);
  return hipGetLastError();
}

template <class T>
hipError_t trial_coef(hipStream_t s, const Grid &g, const Mat &mt, double theta, int floor,
                      const double *H, const double *psi_s, const uint8_t *qflag,
                      const double *d, const uint8_t *eact, const T *cbase, T *coef,
                      RedScratch rs) {
  const int blocks = (g.E + TPB - 1) / TPB;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trial_coef<T>), dim3(blocks), dim3(TPB), 0, s, g, mt,
                     theta, floor, H, psi_s, qflag, d, eact, cbase, coef, rs);
  return hipGetLastError();
}

template <class T>
hipError_t at2_coef(hipStream_t s, const Grid &g, const Mat &mt, const double *H,
                    const uint8_t *eact, T *coef) {
  const int blocks = (4 * g.E + TPB - 1) / TPB;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_at2_coef<T>), dim3(blocks), dim3(TPB), 0, s, g, mt, H,
                     eact, coef);
  return hipGetLastError();
}

template <class TD>
hipError_t predictor(hipStream_t s, const Grid &g, const Mat &mt, const double *d, const TD *dd,
                     const double *H, const double *psi_s, const uint8_t *qflag,
                     const uint8_t *eact, double *Hhat) {
  const int blocks = (g.E + TPB - 1) / TPB;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_predictor<TD>), dim3(blocks), dim3(TPB), 0, s, g, mt, d,
                     dd, H, psi_s, qflag, eact, Hhat);
  return hipGetLastError();
}

hipError_t lift_dirichlet(hipStream_t s, int n, const uint8_t *fixedmask, uint8_t bits,
                          int nmask, const double *unit, double lam, double *u) {
  hipLaunchKernelGGL(k_lift, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, n, fixedmask, bits,
                     nmask, unit, lam, u);
  return hipGetLastError();
}

template <class TS>
hipError_t axpy_into(hipStream_t s, int n, double *out, const double *x, double alpha,
                     const TS *y) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_axpy_into<TS>), dim3((n + TPB - 1) / TPB), dim3(TPB), 0,
                     s, n, out, x, alpha, y);
  return hipGetLastError();
}

template <class TO, class TI>
hipError_t convert(hipStream_t s, int n, TO *out, const TI *in) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_convert<TO, TI>), dim3((n + TPB - 1) / TPB), dim3(TPB), 0,
                     s, n, out, in);
  return hipGetLastError();
}

hipError_t group_sum(hipStream_t s, int n, const int64_t *dof, const int8_t *comp,
                     const double *R, RedScratch rs) {
  hipLaunchKernelGGL(k_group_sum, dim3(1), dim3(TPB), 0, s, n, dof, comp, R, rs);
  return hipGetLastError();
}

hipError_t fill_zero_bytes(hipStream_t s, void *p, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(p) & 3) == 0 && (bytes & 3) == 0) {
    const size_t nw = bytes / 4;
    size_t blocks = (nw + TPB - 1) / TPB;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(TPB), 0, s, nw,
                       reinterpret_cast<uint32_t *>(p));
  } else {
    hipLaunchKernelGGL(k_fill_zero_bytes, dim3((unsigned)((bytes + TPB - 1) / TPB)), dim3(TPB), 0,
                       s, bytes, reinterpret_cast<uint8_t *>(p));
  }
  return hipGetLastError();
}

// -------------------------------------------------- explicit instantiation
#define PF_INST(T)                                                                              \
  template hipError_t tangent_diag<T>(hipStream_t, const Grid &, const March &,                \
                                      const ElasCoef &, int, const T *, const T *,             \
                                      const uint8_t *, const uint8_t *, const uint8_t *, T *); \
  template hipError_t phase_diag<T>(hipStream_t, const Grid &, const March &,                  \
                                    const PhaseCoef &, const T *, const uint8_t *,             \
                                    const uint8_t *, T *, int);                                \
  template hipError_t trial_coef<T>(hipStream_t, const Grid &, const Mat &, double, int,       \
                                    const double *, const double *, const uint8_t *,           \
                                    const double *, const uint8_t *, const T *, T *,           \
                                    RedScratch);                                               \
  template hipError_t at2_coef<T>(hipStream_t, const Grid &, const Mat &, const double *,      \
                                  const uint8_t *, T *);                                       \
  template hipError_t predictor<T>(hipStream_t, const Grid &, const Mat &, const double *,     \
                                   const T *, const double *, const double *,                  \
                                   const uint8_t *, const uint8_t *, double *);                \
  template hipError_t axpy_into<T>(hipStream_t, int, double *, const double *, double,         \
                                   const T *);                                                 \
  template hipError_t cg_init<T>(hipStream_t, int, T *, T *, T *, T *, const T *,             \
                                 const CgArgs &);                                              \
  template hipError_t tangent_apply_masked<T>(hipStream_t, const Grid &, const March &,        \
                                              const ElasCoef &, int, const T *, const T *,     \
                                              const uint8_t *, const uint8_t *,                \
                                              const uint8_t *, const T *, T *);                \
  template hipError_t guess_dots<T>(hipStream_t, const GuessArgs<T> &, const T *, double *,    \
                                    double *);                                                 \
  template hipError_t guess_combine<T>(hipStream_t, const GuessArgs<T> &, const GuessCoef &,   \
                                       T *, T *);                                              \
  template hipError_t cg_update<T>(hipStream_t, int, T *, T *, T *, const T *, const T *,      \
                                   const T *, const CgArgs &, const ChebFuse<T> &);            \
  template hipError_t tangent_cg_apply<T>(hipStream_t, const Grid &, const March &,            \
                                          const ElasCoef &, int, const T *, const T *,         \
                                          const uint8_t *, const uint8_t *, const uint8_t *,   \
                                          const T *, const T *, T *, T *, const CgArgs &);     \
  template hipError_t phase_cg_apply<T>(hipStream_t, const Grid &, const March &,              \
                                        const PhaseCoef &, const T *, const uint8_t *,         \
                                        const uint8_t *, const T *, const T *, T *, T *,       \
                                        const CgArgs &);                                       \
  template hipError_t cheb_init<T>(hipStream_t, int, const T *, const T *, T *, T *, T *,     \
                                   const CgArgs &, const ChebStep &);                          \
  template hipError_t tangent_cheb_step<T>(hipStream_t, const Grid &, const March &,           \
                                           const ElasCoef &, int, const T *, const T *,        \
                                           const uint8_t *, const uint8_t *, const uint8_t *,  \
                                           const T *, T *, const T *, T *, const T *, T *,     \
                                           const T *, const T *, const CgArgs &,               \
                                           const ChebStep &);                                  \
  template hipError_t phase_cheb_step<T>(hipStream_t, const Grid &, const March &,             \
                                         const PhaseCoef &, const T *, const uint8_t *,        \
                                         const uint8_t *, const T *, T *, const T *, T *,      \
                                         const T *, T *, const T *, const T *,                 \
                                         const CgArgs &, const ChebStep &);                    \
  template hipError_t tangent_updcheb<T>(hipStream_t, const Grid &, const March &,             \
                                         const ElasCoef &, int, const T *, const T *,          \
                                         const uint8_t *, const uint8_t *, const uint8_t *,    \
                                         const T *, T *, const T *, T *, const T *, const T *, \
                                         const T *, T *, T *, T *, const CgArgs &,             \
                                         const ChebStep &, const ChebStep &);                  \
  template hipError_t phase_updcheb<T>(hipStream_t, const Grid &, const March &,               \
                                       const PhaseCoef &, const T *, const uint8_t *,          \
                                       const uint8_t *, const T *, T *, const T *, T *,        \
                                       const T *, const T *, const T *, T *, T *, T *,         \
                                       const CgArgs &, const ChebStep &, const ChebStep &);    \
  template hipError_t tangent_updcheb2<T>(hipStream_t, const Grid &, const March &,            \
                                          const ElasCoef &, int, const T *, const T *,         \
                                          const uint8_t *, const uint8_t *, const uint8_t *,   \
                                          const T *, T *, const T *, T *, const T *,           \
                                          const T *, const T *, T *, T *, T *,                 \
                                          const CgArgs &, const ChebStep &);                   \
  template hipError_t phase_updcheb2<T>(hipStream_t, const Grid &, const March &,              \
                                        const PhaseCoef &, const T *, const uint8_t *,         \
                                        const uint8_t *, const T *, T *, const T *, T *,       \
                                        const T *, const T *, const T *, T *, T *, T *,        \
                                        const CgArgs &, const ChebStep &);                     \
  template hipError_t tangent_power_step<T>(hipStream_t, const Grid &, const March &,          \
                                            const ElasCoef &, int, const T *, const T *,       \
                                            const uint8_t *, const uint8_t *, const uint8_t *, \
                                            const T *, T *, const T *, double, RedScratch);    \
  template hipError_t phase_power_step<T>(hipStream_t, const Grid &, const March &,            \
                                          const PhaseCoef &, const T *, const uint8_t *,       \
                                          const uint8_t *, const T *, T *, const T *, double,  \
                                          RedScratch);                                         \
  template hipError_t power_start<T>(hipStream_t, int, const T *, T *);                        \
  template hipError_t tangent_cg1<T>(hipStream_t, const Grid &, const March &, const ElasCoef &, \
                                     int, const T *, const T *, const uint8_t *,               \
                                     const uint8_t *, const uint8_t *, const CgVecs<T> &,      \
                                     const Cg1Args &);                                         \
  template hipError_t phase_cg1<T>(hipStream_t, const Grid &, const March &, const PhaseCoef &, \
                                   const T *, const uint8_t *, const uint8_t *,                \
                                   const CgVecs<T> &, const Cg1Args &);

PF_INST(double)
PF_INST(float)
#undef PF_INST

template void tangent_batch_entry<float>(void *, const Grid &, const March &, const ElasCoef &,
                                         int, const float *, const float *, const uint8_t *,
                                         const uint8_t *, const uint8_t *, const float *,
                                         const float *, float *, float *, const CgArgs &, int,
                                         int);
template void phase_batch_entry<float>(void *, const Grid &, const March &, const PhaseCoef &,
                                       const float *, const uint8_t *, const uint8_t *,
                                       const float *, const float *, float *, float *,
                                       const CgArgs &, int, int);
template hipError_t tangent_cg_apply_batch<float>(hipStream_t, int, int, const void *,
                                                  const int *, int);
template hipError_t phase_cg_apply_batch<float>(hipStream_t, int, const void *, const int *, int);
template hipError_t cg_update_batch<float>(hipStream_t, const BatchUpdateEntry<float> *,
                                           const int *, int);

template hipError_t convert<float, double>(hipStream_t, int, float *, const double *);
template hipError_t convert<double, float>(hipStream_t, int, double *, const float *);

}  // namespace pf
