// Matrix-free DG cell operators for gfx950.
//
// One kernel template serves the three operators of the IMEX-DG step (arXiv 2408.08129,
// Section 2 and Section 3.2): the explicit advective residual, the weak gradient B and the weak
// divergence C with the pressure-jump penalty P.  A workgroup owns CPB cells; one thread owns one
// node of one cell.  The cell's data is staged in LDS, the volume term is a sum-factorised 1D
// contraction along each axis, and the face terms are evaluated face by face:
//   (a) traces of the own cell (from LDS) and of the neighbour (gathered along its normal lines
//       from HBM / L2; no trace buffer, no atomics: every cell writes only its own outputs),
//   (b) numerical flux at the face quadrature points; on a 2:1 hanging face the flux lives on
//       the fine sub-face points, the coarse trace is interpolated there with 1D matrices,
//   (c) on the coarse side the sub-face fluxes are restricted back with the transposed matrices,
//   (d) lift along the normal lines with l(+-1)/w.
// The face geometry is evaluated from the integer description of the (sub)face so that both
// sides of a face see the same normal.
#include "dg_internal.hpp"

namespace dg {
namespace {

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
  const T a = (T)t.a, h0 = (T)t.h0;
  h = hx = hy = T(0);
  switch (t.kind) {
    case 1: {  // Witch of Agnesi
      const T q = a * a + dx * dx;
      h = h0 * a * a / q;
      hx = T(-2) * dx * h / q;
      break;
    }
    case 2: {  // bell (Section 3.1, Eq. (3))
      const T tt = T(1) + (dx * dx + dy * dy) / (a * a);
      h = h0 / (tt * sqrt(tt));
      const T c = T(-3) * h / (tt * a * a);
      hx = c * dx;
      hy = c * dy;
      break;
    }
    case 3: {  // Gaussian hill
      h = h0 * exp(-(dx * dx + dy * dy) / (T(2) * a * a));
      hx = -dx / (a * a) * h;
      hy = -dy / (a * a) * h;
      break;
    }
    case 4: {  // Gaussian ridge along y
      h = h0 * exp(-(dx * dx) / (a * a));
      hx = T(-2) * dx / (a * a) * h;
      break;
    }
    default:
      break;
  }
}

// Metric of the affine cell map at level lev composed with z = zeta + h (1 - zeta / H) at the
// logical point X: Gam[k][l] = det(J) (J^{-1})_{kl} (row k = area-weighted normal of a face of
// constant xi_k), J = det(J).
template <int D, class T>
__device__ __forceinline__ void metric(const MeshDev& m, int lev, const T* X, T (&Gam)[D][D], T& J) {
  const T H = (T)m.L[D - 1];
  T half[D];
#pragma unroll
  for (int a = 0; a < D; ++a) half[a] = (T)(0.5 * m.L[a] / (double)(m.nb[a] << lev));
  T h, hx, hy;
  terrain<T>(m.ter, D, X[0], D == 3 ? X[1] : T(0), h, hx, hy);
  const T Jt = T(1) - h / H;
  const T om = T(1) - X[D - 1] / H;
  if constexpr (D == 3) {
    const T a = half[0], b = half[1], e = half[2], f = e * Jt;
    Gam[0][0] = b * f; Gam[0][1] = 0; Gam[0][2] = 0;
    Gam[1][0] = 0; Gam[1][1] = a * f; Gam[1][2] = 0;
    Gam[2][0] = -a * b * (hx * om); Gam[2][1] = -a * b * (hy * om); Gam[2][2] = a * b;
    J = a * b * f;
  } else {
    const T a = half[0], e = half[1], f = e * Jt;
    Gam[0][0] = f; Gam[0][1] = 0;
    Gam[1][0] = -a * (hx * om); Gam[1][1] = a;
    J = a * f;
  }
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

// ------------------------------------------------------------------------------------- ops
template <int D>
struct OpExplicit {
  using T = double;
  static constexpr int NIN = D + 2, NTR = D + 2, NOUT = D + 2;
  const double* __restrict__ U;
  double* __restrict__ R;
  long N;
  __device__ __forceinline__ void load(long idx, T* in) const {
#pragma unroll
    for (int g = 0; g < NIN; ++g) in[g] = U[g * N + idx];
  }
  __device__ __forceinline__ void transform(const T* in, T* tr) const {
#pragma unroll
    for (int g = 0; g < NTR; ++g) tr[g] = in[g];
  }
  __device__ __forceinline__ void vol(const T* tr, const T (&Gam)[D][D], T (&G)[NOUT][D]) const {
    const double rho = tr[0];
    double u[D], m2 = 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) { u[l] = tr[1 + l] / rho; m2 += tr[1 + l] * tr[1 + l]; }
    const double rk = 0.5 * m2 / rho;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double Gu = 0.0;
#pragma unroll
      for (int l = 0; l < D; ++l) Gu += Gam[k][l] * u[l];
      G[0][k] = rho * Gu;
#pragma unroll
      for (int l = 0; l < D; ++l) G[1 + l][k] = tr[1 + l] * Gu;
      G[1 + D][k] = rk * Gu;
    }
  }
  __device__ __forceinline__ void face(int kind, int left, const T* tm, const T* tn, const T* Nv,
                                       T, T, T* phi) const {
    double F[D + 2];
    const double sign = left ? 1.0 : -1.0;
    if (kind == kWall) {
      double No[D];
#pragma unroll
      for (int a = 0; a < D; ++a) No[a] = sign * Nv[a];
      wall_flux<D>(tm, No, F);
#pragma unroll
      for (int o = 0; o < NOUT; ++o) phi[o] = -F[o];
    } else {
      if (left) rusanov<D>(tm, tn, Nv, F);
      else rusanov<D>(tn, tm, Nv, F);
#pragma unroll
      for (int o = 0; o < NOUT; ++o) phi[o] = -sign * F[o];
    }
  }
  __device__ __forceinline__ void finalize(long idx, const T* acc, T, T J, const T* tr) const {
#pragma unroll
    for (int o = 0; o < NOUT; ++o) R[o * N + idx] = acc[o] / J;
    R[(1 + D) * N + idx] = acc[1 + D] / J - kG * tr[D];
  }
};

template <int D, class TT>
struct OpGrad {
  using T = TT;
  static constexpr int NIN = 2, NTR = 1, NOUT = D;
  GradArgs<T> a;
  long N;
  __device__ __forceinline__ void load(long idx, T* in) const {
    in[0] = a.p[idx];
    in[1] = a.dinv ? a.dinv[idx] : T(1);
  }
  __device__ __forceinline__ void transform(const T* in, T* tr) const {
    tr[0] = a.dinv ? a.scale * in[1] * in[0] : in[0];
  }
  __device__ __forceinline__ void vol(const T* tr, const T (&Gam)[D][D], T (&G)[NOUT][D]) const {
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
      for (int k = 0; k < D; ++k) G[l][k] = -Gam[k][l] * tr[0];
  }
  __device__ __forceinline__ void face(int kind, int left, const T* tm, const T* tn, const T* Nv,
                                       T, T, T* phi) const {
    const T sign = left ? T(1) : T(-1);
    T ph = tm[0];
    if (kind != kWall) ph = left ? T(0.5) * (tm[0] + tn[0]) : T(0.5) * (tn[0] + tm[0]);
#pragma unroll
    for (int l = 0; l < D; ++l) phi[l] = sign * ph * Nv[l];
  }
  __device__ __forceinline__ void finalize(long idx, const T* acc, T, T J, const T*) const {
#pragma unroll
    for (int l = 0; l < D; ++l) a.q[l * N + idx] = acc[l] / J;
  }
};

template <int D, class TT>
struct OpDiv {
  using T = TT;
  static constexpr int NIN = D + 3, NTR = D + 1, NOUT = 1;
  DivArgs<T> a;
  long N;
  __device__ __forceinline__ void load(long idx, T* in) const {
#pragma unroll
    for (int l = 0; l < D; ++l) in[l] = a.qv[l * N + idx];
    in[D] = a.h ? a.h[idx] : T(1);
    in[D + 1] = a.p ? a.p[idx] : T(0);
    in[D + 2] = a.dinv ? a.dinv[idx] : T(1);
  }
  __device__ __forceinline__ void transform(const T* in, T* tr) const {
#pragma unroll
    for (int l = 0; l < D; ++l) tr[l] = in[D] * in[l];
    tr[D] = a.dinv ? a.scale * in[D + 2] * in[D + 1] : in[D + 1];
  }
  __device__ __forceinline__ void vol(const T* tr, const T (&Gam)[D][D], T (&G)[NOUT][D]) const {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T Gk = 0;
#pragma unroll
      for (int l = 0; l < D; ++l) Gk += Gam[k][l] * tr[l];
      G[0][k] = -a.adiv * Gk;
    }
  }
  __device__ __forceinline__ void face(int kind, int left, const T* tm, const T* tn, const T* Nv,
                                       T lm, T ln, T* phi) const {
    if (kind == kWall) { phi[0] = 0; return; }
    const T sign = left ? T(1) : T(-1);
    T wm = 0, wn = 0, nn = 0;
#pragma unroll
    for (int l = 0; l < D; ++l) { wm += Nv[l] * tm[l]; wn += Nv[l] * tn[l]; nn += Nv[l] * Nv[l]; }
    const T wh = left ? T(0.5) * (wm + wn) : T(0.5) * (wn + wm);
    T v = a.adiv * sign * wh;
    if (a.apen != T(0)) {
      const T lf = lm > ln ? lm : ln;
      v += a.apen * (lf * sqrt(nn) * (tm[D] - tn[D]));
    }
    phi[0] = v;
  }
  __device__ __forceinline__ void finalize(long idx, const T* acc, T w, T J, const T* tr) const {
    if (a.weak) a.out[idx] = w * (acc[0] + a.amass * J * tr[D]);
    else a.out[idx] = acc[0] / J;
  }
  __device__ __forceinline__ T lam(int cell) const { return a.lam ? a.lam[cell] : T(0); }
};

template <class Op> struct HasLam { static constexpr bool value = false; };
template <int D, class T> struct HasLam<OpDiv<D, T>> { static constexpr bool value = true; };

// --------------------------------------------------------------------------------- the kernel
template <int D, int NP, class Op>
__global__ void __launch_bounds__((Cfg<D, NP>::NT)) k_cell(const Op op, const MeshDev m) {
  using C = Cfg<D, NP>;
  using T = typename Op::T;
  constexpr int NL = C::NL, NFP = C::NFP, MS = C::MS, TPC = C::TPC, CPB = C::CPB, NT = C::NT;
  constexpr int NTR = Op::NTR, NOUT = Op::NOUT, NIN = Op::NIN;
  constexpr TabLayout TL{NP};
  constexpr int VOLSZ = CPB * NOUT * D * NL;
  constexpr int O_TOWN = 0;
  constexpr int O_NB = O_TOWN + CPB * NTR * NFP;
  constexpr int O_FL = O_NB + CPB * MS * NTR * NFP;
  constexpr int O_FR = O_FL + CPB * MS * NOUT * NFP;
  constexpr int FACESZ = O_FR + CPB * NOUT * NFP;
  constexpr int SCR = VOLSZ > FACESZ ? VOLSZ : FACESZ;

  __shared__ T sTab[TL.size()];
  __shared__ T sT[CPB * NTR * NL];
  __shared__ T sScr[SCR];
  __shared__ int4 sCell[CPB];
  __shared__ int sKind[CPB][2 * D];
  __shared__ int4 sNbr[CPB][2 * D];
  __shared__ T sLam[CPB];

  const int tid = threadIdx.x;
  const int lc = tid / TPC;
  const int node = tid % TPC;
  const int cell0 = blockIdx.x * CPB;
  const int cell = cell0 + lc;
  const bool active = (node < NL) && (cell < m.ncell);

  const T* gtab;
  if constexpr (sizeof(T) == 8) gtab = (const T*)m.tab;
  else gtab = (const T*)m.tabf;
  for (int t = tid; t < TL.size(); t += NT) sTab[t] = gtab[t];
  if (tid < CPB * 2 * D) {
    const int c = tid / (2 * D), f = tid % (2 * D);
    const int cc = cell0 + c;
    if (cc < m.ncell) {
      sKind[c][f] = m.fkind[cc * 2 * D + f];
      sNbr[c][f] = m.fnbr[cc * 2 * D + f];
    } else {
      sKind[c][f] = kWall;
      sNbr[c][f] = make_int4(-1, -1, -1, -1);
    }
  }
  if (tid < CPB) {
    const int cc = cell0 + tid;
    sCell[tid] = cc < m.ncell ? m.cell[cc] : make_int4(0, 0, 0, 0);
    if constexpr (HasLam<Op>::value) sLam[tid] = cc < m.ncell ? op.lam(cc) : T(0);
  }
  // own inputs -> trace fields at the nodes
  T trn[NTR];
  if (active) {
    T in[NIN];
    op.load((long)cell * NL + node, in);
    op.transform(in, trn);
#pragma unroll
    for (int g = 0; g < NTR; ++g) sT[(lc * NTR + g) * NL + node] = trn[g];
  }
  __syncthreads();

  const T* Xi = &sTab[TL.xi()];
  const T* Wt = &sTab[TL.w()];
  const T* Dt = &sTab[TL.dt()];
  const T* Lb = &sTab[TL.lb()];
  const T* Lbw = &sTab[TL.lbw()];
  const T* Pi = &sTab[TL.pi()];
  const T* Rw = &sTab[TL.rw()];

  // ---------------------------------------------------------------- volume term
  T acc[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) acc[o] = 0;
  T Jn = 1, wn = 1;
  const int4 ci = sCell[lc];
  const int lev = ci.x;
  const int cidx[3] = {ci.y, ci.z, ci.w};
  if (active) {
    T X[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int ia = along<D, NP>(node, a);
      const T dx = (T)(m.L[a] / (double)(m.nb[a] << lev));
      X[a] = dx * ((T)cidx[a] + T(0.5) * (T(1) + Xi[ia]));
      wn *= Wt[ia];
    }
    T Gam[D][D];
    metric<D, T>(m, lev, X, Gam, Jn);
    T G[NOUT][D];
    op.vol(trn, Gam, G);
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int k = 0; k < D; ++k) sScr[((lc * NOUT + o) * D + k) * NL + node] = G[o][k];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int ik = along<D, NP>(node, k);
      const int ak = tang<D, NP>(node, k);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const T dq = Dt[ik * NP + q];
        const int nq = compose<D, NP>(k, q, ak);
#pragma unroll
        for (int o = 0; o < NOUT; ++o) acc[o] += dq * sScr[((lc * NOUT + o) * D + k) * NL + nq];
      }
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- face terms
  T* sTown = &sScr[O_TOWN];
  T* sNb = &sScr[O_NB];
  T* sFl = &sScr[O_FL];
  T* sFr = &sScr[O_FR];
  for (int f = 0; f < 2 * D; ++f) {
    const int k = f >> 1, s = f & 1;
    // (a) own traces and neighbour traces
    for (int t = tid; t < CPB * NFP; t += NT) {
      const int c = t / NFP, j = t % NFP;
      if (cell0 + c >= m.ncell) continue;
#pragma unroll
      for (int g = 0; g < NTR; ++g) {
        T v = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) v += Lb[s * NP + q] * sT[(c * NTR + g) * NL + compose<D, NP>(k, q, j)];
        sTown[(c * NTR + g) * NFP + j] = v;
      }
    }
    for (int t = tid; t < CPB * MS * NFP; t += NT) {
      const int c = t / (MS * NFP), sub = (t / NFP) % MS, j = t % NFP;
      if (cell0 + c >= m.ncell) continue;
      const int kind = sKind[c][f];
      if (kind == kWall) continue;
      if (kind != kCoarse && sub > 0) continue;
      const int4 nb4 = sNbr[c][f];
      const int nb = sub == 0 ? nb4.x : sub == 1 ? nb4.y : sub == 2 ? nb4.z : nb4.w;
      T v[NTR];
#pragma unroll
      for (int g = 0; g < NTR; ++g) v[g] = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        T in[NIN], tr[NTR];
        op.load((long)nb * NL + compose<D, NP>(k, q, j), in);
        op.transform(in, tr);
        const T lq = Lb[(1 - s) * NP + q];
#pragma unroll
        for (int g = 0; g < NTR; ++g) v[g] += lq * tr[g];
      }
#pragma unroll
      for (int g = 0; g < NTR; ++g) sNb[((c * MS + sub) * NTR + g) * NFP + j] = v[g];
    }
    __syncthreads();
    // (b) fluxes at the (sub)face points
    for (int t = tid; t < CPB * MS * NFP; t += NT) {
      const int c = t / (MS * NFP), sub = (t / NFP) % MS, j = t % NFP;
      if (cell0 + c >= m.ncell) continue;
      const int kind = sKind[c][f];
      if (kind != kCoarse && sub > 0) continue;
      const int4 cc = sCell[c];
      const int cl = cc.x;
      const int cid[3] = {cc.y, cc.z, cc.w};
      T tm[NTR], tn[NTR];
      const int j0 = j % NP, j1 = j / NP;
      if (kind == kCoarse) {
        // own (coarse) trace interpolated to the fine sub-face point
        const int c0 = sub & 1, c1 = sub >> 1;
#pragma unroll
        for (int g = 0; g < NTR; ++g) {
          const T* Tc = &sTown[(c * NTR + g) * NFP];
          T v = 0;
          if constexpr (D == 3) {
#pragma unroll
            for (int a1 = 0; a1 < NP; ++a1) {
              T u = 0;
#pragma unroll
              for (int a0 = 0; a0 < NP; ++a0) u += Pi[(c0 * NP + j0) * NP + a0] * Tc[a0 + NP * a1];
              v += Pi[(c1 * NP + j1) * NP + a1] * u;
            }
          } else {
#pragma unroll
            for (int a0 = 0; a0 < NP; ++a0) v += Pi[(c0 * NP + j) * NP + a0] * Tc[a0];
          }
          tm[g] = v;
          tn[g] = sNb[((c * MS + sub) * NTR + g) * NFP + j];
        }
      } else {
#pragma unroll
        for (int g = 0; g < NTR; ++g) tm[g] = sTown[(c * NTR + g) * NFP + j];
        if (kind == kConf) {
#pragma unroll
          for (int g = 0; g < NTR; ++g) tn[g] = sNb[((c * MS) * NTR + g) * NFP + j];
        } else if (kind == kFine) {
          // neighbour (coarse) trace interpolated to my point; my position in its face
          int cs[2] = {0, 0};
          int tt = 0;
#pragma unroll
          for (int ax = 0; ax < D; ++ax)
            if (ax != k) cs[tt++] = cid[ax] & 1;
#pragma unroll
          for (int g = 0; g < NTR; ++g) {
            const T* Tc = &sNb[((c * MS) * NTR + g) * NFP];
            T v = 0;
            if constexpr (D == 3) {
#pragma unroll
              for (int a1 = 0; a1 < NP; ++a1) {
                T u = 0;
#pragma unroll
                for (int a0 = 0; a0 < NP; ++a0) u += Pi[(cs[0] * NP + j0) * NP + a0] * Tc[a0 + NP * a1];
                v += Pi[(cs[1] * NP + j1) * NP + a1] * u;
              }
            } else {
#pragma unroll
              for (int a0 = 0; a0 < NP; ++a0) v += Pi[(cs[0] * NP + j) * NP + a0] * Tc[a0];
            }
            tn[g] = v;
          }
        } else {
#pragma unroll
          for (int g = 0; g < NTR; ++g) tn[g] = tm[g];
        }
      }
      // face geometry from the integer description of the (sub)face
      int lf;
      long P;
      long Tt[3] = {0, 0, 0};
      if (kind == kCoarse) {
        lf = cl + 1;
        P = s ? 2L * (cid[k] + 1) : 2L * cid[k];
        int tt = 0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax)
          if (ax != k) { Tt[ax] = 2L * cid[ax] + ((sub >> tt) & 1); ++tt; }
      } else {
        lf = cl;
        P = s ? (long)cid[k] + 1 : (long)cid[k];
#pragma unroll
        for (int ax = 0; ax < D; ++ax)
          if (ax != k) Tt[ax] = cid[ax];
      }
      const long nk = (long)m.nb[k] << lf;
      if (m.per[k] && P >= nk) P -= nk;
      T X[D];
      {
        int tt = 0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
          const T dx = (T)(m.L[ax] / (double)(m.nb[ax] << lf));
          if (ax == k) {
            X[ax] = dx * (T)P;
          } else {
            const int jj = tt == 0 ? j0 : j1;
            X[ax] = dx * ((T)Tt[ax] + T(0.5) * (T(1) + Xi[jj]));
            ++tt;
          }
        }
      }
      T Gam[D][D], Jf;
      metric<D, T>(m, lf, X, Gam, Jf);
      T Nv[D];
#pragma unroll
      for (int a = 0; a < D; ++a) Nv[a] = Gam[k][a];
      T lm = 0, ln = 0;
      if constexpr (HasLam<Op>::value) {
        lm = sLam[c];
        if (kind != kWall) {
          const int4 nb4 = sNbr[c][f];
          const int nb = sub == 0 ? nb4.x : sub == 1 ? nb4.y : sub == 2 ? nb4.z : nb4.w;
          ln = op.lam(nb);
        }
      }
      T phi[NOUT];
      op.face(kind, s, tm, tn, Nv, lm, ln, phi);
#pragma unroll
      for (int o = 0; o < NOUT; ++o) sFl[((c * MS + sub) * NOUT + o) * NFP + j] = phi[o];
    }
    __syncthreads();
    // (c) collect; restrict the sub-face fluxes of a coarse face
    for (int t = tid; t < CPB * NFP; t += NT) {
      const int c = t / NFP, a = t % NFP;
      if (cell0 + c >= m.ncell) continue;
      const int kind = sKind[c][f];
      const int a0 = a % NP, a1 = a / NP;
#pragma unroll
      for (int o = 0; o < NOUT; ++o) {
        T v;
        if (kind == kCoarse) {
          v = 0;
#pragma unroll
          for (int sub = 0; sub < MS; ++sub) {
            const int c0 = sub & 1, c1 = sub >> 1;
            const T* Fs = &sFl[((c * MS + sub) * NOUT + o) * NFP];
            if constexpr (D == 3) {
#pragma unroll
              for (int j1 = 0; j1 < NP; ++j1) {
                T u = 0;
#pragma unroll
                for (int j0 = 0; j0 < NP; ++j0) u += Rw[(c0 * NP + a0) * NP + j0] * Fs[j0 + NP * j1];
                v += Rw[(c1 * NP + a1) * NP + j1] * u;
              }
            } else {
#pragma unroll
              for (int j0 = 0; j0 < NP; ++j0) v += Rw[(c0 * NP + a) * NP + j0] * Fs[j0];
            }
          }
        } else {
          v = sFl[((c * MS) * NOUT + o) * NFP + a];
        }
        sFr[(c * NOUT + o) * NFP + a] = v;
      }
    }
    __syncthreads();
    // (d) lift along the normal lines
    if (active) {
      const int ik = along<D, NP>(node, k);
      const int a = tang<D, NP>(node, k);
      const T lw = Lbw[s * NP + ik];
#pragma unroll
      for (int o = 0; o < NOUT; ++o) acc[o] += lw * sFr[(lc * NOUT + o) * NFP + a];
    }
    __syncthreads();
  }

  if (active) op.finalize((long)cell * NL + node, acc, wn, Jn, trn);
}

template <int D, int NP, class Op>
int run(const Op& op, const MeshDev& m, hipStream_t s) {
  using C = Cfg<D, NP>;
  if (m.ncell == 0) return 0;
  const int grid = (m.ncell + C::CPB - 1) / C::CPB;
  hipLaunchKernelGGL((k_cell<D, NP, Op>), dim3(grid), dim3(C::NT), 0, s, op, m);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace

#define DG_DISPATCH(D_, DEG_, EXPR)            \
  switch (DEG_) {                              \
    case 1: { constexpr int NP = 2; EXPR; }    \
    case 2: { constexpr int NP = 3; EXPR; }    \
    case 3: { constexpr int NP = 4; EXPR; }    \
    case 4: { constexpr int NP = 5; EXPR; }    \
    case 5: { constexpr int NP = 6; EXPR; }    \
    default: return -6;                        \
  }

int launch_explicit(const MeshDev& m, int degree, const double* U, double* R, hipStream_t s) {
  if (m.dim == 2) {
    OpExplicit<2> op{U, R, m.N};
    DG_DISPATCH(2, degree, return (run<2, NP>(op, m, s)));
  } else {
    OpExplicit<3> op{U, R, m.N};
    DG_DISPATCH(3, degree, return (run<3, NP>(op, m, s)));
  }
}

template <class T>
static int grad_impl(const MeshDev& m, int degree, const GradArgs<T>& a, hipStream_t s) {
  if (m.dim == 2) {
    OpGrad<2, T> op{a, m.N};
    DG_DISPATCH(2, degree, return (run<2, NP>(op, m, s)));
  } else {
    OpGrad<3, T> op{a, m.N};
    DG_DISPATCH(3, degree, return (run<3, NP>(op, m, s)));
  }
}

template <class T>
static int div_impl(const MeshDev& m, int degree, const DivArgs<T>& a, hipStream_t s) {
  if (m.dim == 2) {
    OpDiv<2, T> op{a, m.N};
    DG_DISPATCH(2, degree, return (run<2, NP>(op, m, s)));
  } else {
    OpDiv<3, T> op{a, m.N};
    DG_DISPATCH(3, degree, return (run<3, NP>(op, m, s)));
  }
}

int launch_grad64(const MeshDev& m, int degree, const GradArgs<double>& a, hipStream_t s) {
  return grad_impl<double>(m, degree, a, s);
}
int launch_div64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s) {
  return div_impl<double>(m, degree, a, s);
}
int launch_grad32(const MeshDev& m, int degree, const GradArgs<float>& a, hipStream_t s) {
  return grad_impl<float>(m, degree, a, s);
}
int launch_div32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s) {
  return div_impl<float>(m, degree, a, s);
}

// ------------------------------------------------------------------------------- node geometry
namespace {

struct Atm { int kind; double a0, a1, a2; };

__device__ void background(const Atm& at, double z, double& p, double& rho) {
  if (at.kind == 0) {
    p = at.a0 * exp(-kG * z / (kR * at.a1));
    rho = p / (kR * at.a1);
  } else {
    const double pref = at.a0, Tref = at.a1, Nb = at.a2;
    const double Gm = (kGamma - 1.0) / kGamma;
    const double rhoref = pref / (kR * Tref);
    const double sz = exp(-Nb * Nb * z / kG);
    const double base = 1.0 - (kG * kG / (Nb * Nb)) * Gm * (rhoref / pref) * (1.0 - sz);
    p = pref * pow(base, 1.0 / Gm);
    rho = rhoref * pow(p / pref, 1.0 / kGamma) * sz;
  }
}

template <int D, int NP>
__global__ void k_geometry(const MeshDev m, const Atm at, double* x, double* y, double* z,
                           double* wJ, double* pbar, double* rbar) {
  constexpr int NL = ipow(NP, D);
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= m.N) return;
  const int cell = (int)(gid / NL), node = (int)(gid % NL);
  const int4 ci = m.cell[cell];
  const int cidx[3] = {ci.y, ci.z, ci.w};
  const double* Xi = m.tab;  // TabLayout::xi() == 0
  const double* Wt = m.tab + NP;
  double X[D], w = 1.0;
  for (int a = 0; a < D; ++a) {
    const int ia = along<D, NP>(node, a);
    const double dx = m.L[a] / (double)(m.nb[a] << ci.x);
    X[a] = dx * (cidx[a] + 0.5 * (1.0 + Xi[ia]));
    w *= Wt[ia];
  }
  double Gam[D][D], J;
  metric<D, double>(m, ci.x, X, Gam, J);
  double h, hx, hy;
  terrain<double>(m.ter, D, X[0], D == 3 ? X[1] : 0.0, h, hx, hy);
  const double H = m.L[D - 1];
  const double zz = X[D - 1] + h * (1.0 - X[D - 1] / H);
  if (x) x[gid] = X[0];
  if (y) y[gid] = D == 3 ? X[1] : 0.0;
  if (z) z[gid] = zz;
  if (wJ) wJ[gid] = w * J;
  if (pbar || rbar) {
    double p, r;
    background(at, zz, p, r);
    if (pbar) pbar[gid] = p;
    if (rbar) rbar[gid] = r;
  }
}

}  // namespace

int launch_geometry(const MeshDev& m, int degree, double* x, double* y, double* z, double* wJ,
                    double* pbar, double* rbar, int atm_kind, const double* atm, hipStream_t s) {
  Atm at{atm_kind, atm[0], atm[1], atm[2]};
  const int grid = (int)((m.N + 255) / 256);
  if (m.N == 0) return 0;
#define DG_GEO(D_)                                                                               \
  DG_DISPATCH(D_, degree,                                                                        \
              hipLaunchKernelGGL((k_geometry<D_, NP>), dim3(grid), dim3(256), 0, s, m, at, x, y, \
                                 z, wJ, pbar, rbar);                                             \
              return hipGetLastError() == hipSuccess ? 0 : -3)
  if (m.dim == 2) {
    DG_GEO(2);
  } else {
    DG_GEO(3);
  }
#undef DG_GEO
}

}  // namespace dg
