// Device helpers shared by the cell-operator kernels: node indexing of the tensor-product cell,
// the terrain-following map and its metric, and the XCD-aware block order.
#pragma once

#include "dg_internal.hpp"

namespace dg {
namespace dev {

constexpr int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}
constexpr int p2ceil(int x) {
  int r = 1;
  while (r < x) r <<= 1;
  return r;
}

template <int D, int NP>
struct Cfg {
  static constexpr int NL = ipow(NP, D);
  static constexpr int NFP = ipow(NP, D - 1);
  static constexpr int MS = 1 << (D - 1);
  static constexpr int TPC = p2ceil(NL);
  static constexpr int NT = TPC > 256 ? TPC : 256;
  static constexpr int CPB = NT / TPC;
};

// ------------------------------------------------------------------------------- node indexing
template <int D, int NP>
__device__ __forceinline__ int along(int node, int k) {
  if (k == 0) return node % NP;
  if (D == 3 && k == 1) return (node / NP) % NP;
  return node / ipow(NP, D - 1);
}
// tangential (face-point) index of a node w.r.t. axis k: tangential axes ascending, first fastest
template <int D, int NP>
__device__ __forceinline__ int tang(int node, int k) {
  if (D == 2) return k == 0 ? node / NP : node % NP;
  if (k == 0) return node / NP;
  if (k == 1) return (node % NP) + NP * (node / (NP * NP));
  return node % (NP * NP);
}
// The NP values of a contiguous line (the x-normal line of a cell: nodes x fastest) in 16-byte
// vector loads plus a scalar tail: gfx950 global loads need only the element alignment, and
// across a wavefront one such line per lane reads ~20 cache lines per instruction, so fewer,
// wider instructions cut the address-processing work.
template <int NP, class T>
__device__ __forceinline__ void load_line(const T* p, T (&v)[NP]) {
  constexpr int W = 16 / (int)sizeof(T);
  typedef T V __attribute__((ext_vector_type(W), aligned(sizeof(T))));
#pragma unroll
  for (int j = 0; j < NP / W; ++j) {
    const V x = *(const V*)(p + j * W);
#pragma unroll
    for (int i = 0; i < W; ++i) v[j * W + i] = x[i];
  }
#pragma unroll
  for (int q = NP / W * W; q < NP; ++q) v[q] = p[q];
}

template <int D, int NP>
__device__ __forceinline__ int compose(int k, int q, int a) {
  if (D == 2) return k == 0 ? q + NP * a : a + NP * q;
  if (k == 0) return q + NP * a;
  if (k == 1) return (a % NP) + NP * (q + NP * (a / NP));
  return a + NP * NP * q;
}

// ---------------------------------------------------------------------------------- geometry
template <class T>
__device__ __forceinline__ void terrain(const Terrain& t, int dim, T x, T y, T& h, T& hx, T& hy) {
  const T dx = x - (T)t.xc;
  const T dy = (dim == 3) ? y - (T)t.yc : T(0);
  const T h0 = (T)t.h0, ia2 = (T)t.ia2;
  h = hx = hy = T(0);
  switch (t.kind) {
    case 1: {  // Witch of Agnesi: h0 a^2 / (a^2 + dx^2)
      const T iq = T(1) / (T(1) + dx * dx * ia2);
      h = h0 * iq;
      hx = T(-2) * dx * ia2 * h * iq;
      break;
    }
    case 2: {  // bell (Section 3.1, Eq. (3)): h0 / (1 + (dx^2 + dy^2)/a^2)^(3/2)
      const T tt = T(1) + (dx * dx + dy * dy) * ia2;
      const T it = T(1) / tt;
      h = h0 * it * sqrt(it);
      const T c = T(-3) * h * it * ia2;
      hx = c * dx;
      hy = c * dy;
      break;
    }
    case 3: {  // Gaussian hill: h0 exp(-(dx^2 + dy^2) / (2 sigma^2))
      h = h0 * exp(-(dx * dx + dy * dy) * (T(0.5) * ia2));
      hx = -dx * ia2 * h;
      hy = -dy * ia2 * h;
      break;
    }
    case 4: {  // Gaussian ridge along y: h0 exp(-((x - xc)/a)^2)
      h = h0 * exp(-(dx * dx) * ia2);
      hx = T(-2) * dx * ia2 * h;
      break;
    }
    default:
      break;
  }
}

// Metric of the cell map at level lev composed with z = zeta + h (1 - zeta / H), given the
// terrain height and slopes at the point's horizontal position and its logical height zeta:
// Gam[k][l] = det(J) (J^{-1})_{kl} (row k = area-weighted normal of a face of constant xi_k).
template <int D, class T>
__device__ __forceinline__ void metric_h(const MeshDev& m, int lev, T h, T hx, T hy, T zeta,
                                         T (&Gam)[D][D], T& J) {
  const T invH = (T)m.invH;
  const T Jt = T(1) - h * invH;
  const T om = T(1) - zeta * invH;
  if constexpr (D == 3) {
    const T a = T(0.5) * (T)m.dxl[lev][0], b = T(0.5) * (T)m.dxl[lev][1];
    const T f = T(0.5) * (T)m.dxl[lev][2] * Jt;
    Gam[0][0] = b * f; Gam[0][1] = 0; Gam[0][2] = 0;
    Gam[1][0] = 0; Gam[1][1] = a * f; Gam[1][2] = 0;
    Gam[2][0] = -a * b * (hx * om); Gam[2][1] = -a * b * (hy * om); Gam[2][2] = a * b;
    J = a * b * f;
  } else {
    const T a = T(0.5) * (T)m.dxl[lev][0];
    const T f = T(0.5) * (T)m.dxl[lev][1] * Jt;
    Gam[0][0] = f; Gam[0][1] = 0;
    Gam[1][0] = -a * (hx * om); Gam[1][1] = a;
    J = a * f;
  }
}

// Metric at a logical point X (terrain evaluated there).
template <int D, class T>
__device__ __forceinline__ void metric(const MeshDev& m, int lev, const T* X, T (&Gam)[D][D], T& J) {
  T h, hx, hy;
  terrain<T>(m.ter, D, X[0], D == 3 ? X[1] : T(0), h, hx, hy);
  metric_h<D, T>(m, lev, h, hx, hy, X[D - 1], Gam, J);
}

// XCD-aware block order: the hardware hands consecutive workgroups to the 8 XCDs in turn; remap
// so that each XCD walks a contiguous range of Morton-ordered cells and neighbour reads hit its L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  constexpr int X = 8;
  const int q = nblocks / X, r = nblocks % X;
  const int x = b % X, i = b / X;
  return x * q + (x < r ? x : r) + i;
}

// ----------------------------------------------------------------------------------- fluxes
template <int D>
__device__ __forceinline__ void adv_flux_n(const double* U, const double* N, double* F) {
  double mn = 0.0, m2 = 0.0;
#pragma unroll
  for (int l = 0; l < D; ++l) { mn += U[1 + l] * N[l]; m2 += U[1 + l] * U[1 + l]; }
  const double un = mn / U[0];
  F[0] = mn;
#pragma unroll
  for (int l = 0; l < D; ++l) F[1 + l] = U[1 + l] * un;
  F[1 + D] = 0.5 * m2 / U[0] * un;
}

// Rusanov flux with the advective speed (acoustics are treated implicitly).
template <int D>
__device__ __forceinline__ void rusanov(const double* UL, const double* UR, const double* N, double* F) {
  double FL[D + 2], FR[D + 2];
  adv_flux_n<D>(UL, N, FL);
  adv_flux_n<D>(UR, N, FR);
  double vl = 0.0, vr = 0.0;
#pragma unroll
  for (int l = 0; l < D; ++l) { vl += UL[1 + l] * N[l]; vr += UR[1 + l] * N[l]; }
  const double lam = fmax(fabs(vl / UL[0]), fabs(vr / UR[0]));
#pragma unroll
  for (int f = 0; f < D + 2; ++f) F[f] = 0.5 * (FL[f] + FR[f]) - 0.5 * lam * (UR[f] - UL[f]);
}

// Slip wall: Rusanov against the mirror state, simplified: no mass and energy flux, momentum
// (m.N)(v + |v|) N / |N|^2 with v = (m.N)/rho, N the outward area-weighted normal.
template <int D>
__device__ __forceinline__ void wall_flux(const double* U, const double* N, double* F) {
  double mn = 0.0, nn = 0.0;
#pragma unroll
  for (int l = 0; l < D; ++l) { mn += U[1 + l] * N[l]; nn += N[l] * N[l]; }
  const double v = mn / U[0];
  F[0] = 0.0;
#pragma unroll
  for (int l = 0; l < D; ++l) F[1 + l] = mn * (v + fabs(v)) * N[l] / nn;
  F[1 + D] = 0.0;
}

}  // namespace dev
}  // namespace dg
