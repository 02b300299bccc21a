// Matrix-free DG cell operators for gfx950: the general cell kernel.
//
// One kernel template serves the three operators of the IMEX-DG step (arXiv 2408.08129,
// Section 2 and Section 3.2): the explicit advective residual, the weak gradient B and the weak
// divergence C with the pressure-jump penalty P.  The column kernels (dg_helm.hip) do the bulk
// of the work; this kernel adds the terms of the 2:1 faces for the cells that have one (its
// faces-only mode) and serves the operator variants the column kernels leave out (Jacobi-scaled
// p).  A workgroup owns CPB cells, taken from a cell list; one thread owns one node of one cell.
// The cell's data is staged in LDS, the volume term is a sum-factorised 1D
// contraction along each axis, and the face terms are evaluated face by face:
//   (a) traces of the own cell (from LDS) and of the neighbour (gathered along its normal lines
//       from HBM / L2; no trace buffer, no atomics: every cell writes only its own outputs),
//   (b) numerical flux at the face quadrature points; on a 2:1 hanging face the flux lives on
//       the fine sub-face points, the coarse trace is interpolated there with 1D matrices,
//   (c) on the coarse side the sub-face fluxes are restricted back with the transposed matrices,
//   (d) lift along the normal lines with l(+-1)/w.
// The face geometry is evaluated from the integer description of the (sub)face so that both
// sides of a face see the same normal.
#include "dg_device.hpp"

namespace dg {
namespace {
using namespace dev;

// ------------------------------------------------------------------------------------- ops
template <int D>
struct OpExplicit {
  using T = double;
  static constexpr int NIN = D + 2, NTR = D + 2, NOUT = D + 2;
  // compact index of volume flux component (o, k); all are non-zero
  static constexpr int NVOL = NOUT * D;
  static constexpr int vidx(int o, int k) { return o * D + k; }
  const double* __restrict__ U;
  double* __restrict__ R;
  unsigned N;
  __device__ __forceinline__ void load(unsigned idx, T* in) const {
#pragma unroll
    for (int g = 0; g < NIN; ++g) in[g] = U[g * N + idx];
  }
  __device__ __forceinline__ void load_face(unsigned idx, int, T* in) const { load(idx, in); }
  static constexpr bool need(int, int) { return true; }
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
  __device__ __forceinline__ void finalize(unsigned idx, const T* acc, T, T J, const T* tr) const {
    const T iJ = T(1) / J;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) R[o * N + idx] = acc[o] * iJ;
    R[(1 + D) * N + idx] = acc[1 + D] * iJ - kG * tr[D];
  }
  // adds the lifted 2:1 face terms to an output the column kernel has written
  __device__ __forceinline__ void finalize_add(unsigned idx, const T* acc, T, T J) const {
    const T iJ = T(1) / J;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) R[o * N + idx] += acc[o] * iJ;
  }
};

template <int D, class TT>
struct OpGrad {
  using T = TT;
  static constexpr int NIN = 2, NTR = 1, NOUT = D;
  // -p Gam^T: the terrain-following map makes Gam[k][l] zero for k < d-1, l != k
  static constexpr int NVOL = D == 3 ? 5 : 3;
  static constexpr int vidx(int o, int k) {
    return D == 3 ? (k == 0 ? (o == 0 ? 0 : -1) : k == 1 ? (o == 1 ? 1 : -1) : 2 + o)
                  : (k == 0 ? (o == 0 ? 0 : -1) : 1 + o);
  }
  GradArgs<T> a;
  unsigned N;
  __device__ __forceinline__ void load(unsigned idx, T* in) const {
    in[0] = a.p[idx];
    in[1] = a.dinv ? a.dinv[idx] : T(1);
  }
  __device__ __forceinline__ void load_face(unsigned idx, int, T* in) const { load(idx, in); }
  static constexpr bool need(int, int) { return true; }
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
  __device__ __forceinline__ void finalize(unsigned idx, const T* acc, T, T J, const T* tr) const {
    T iJ = T(1) / J;
    if (a.h) iJ *= a.h[idx];
#pragma unroll
    for (int l = 0; l < D; ++l) a.q[l * N + idx] = acc[l] * iJ;
    if (a.z) a.z[idx] = tr[0];
  }
  __device__ __forceinline__ void finalize_add(unsigned idx, const T* acc, T, T J) const {
    T iJ = T(1) / J;
    if (a.h) iJ *= a.h[idx];
#pragma unroll
    for (int l = 0; l < D; ++l) a.q[l * N + idx] += acc[l] * iJ;
  }
};

template <int D, class TT>
struct OpDiv {
  using T = TT;
  static constexpr int NIN = D + 3, NTR = D + 1, NOUT = 1;
  static constexpr int NVOL = D;
  static constexpr int vidx(int o, int k) { return o * D + k; }
  DivArgs<T> a;
  unsigned N;
  __device__ __forceinline__ void load(unsigned idx, T* in) const {
#pragma unroll
    for (int l = 0; l < D; ++l) in[l] = a.qv[l * N + idx];
    in[D] = a.h ? a.h[idx] : T(1);
    in[D + 1] = a.p ? a.p[idx] : T(0);
    in[D + 2] = a.dinv ? a.dinv[idx] : T(1);
  }
  // Trace field g is needed on faces normal to axis k: for k < d-1 the area-weighted normal of
  // the terrain-following map is (0..N_k..0), so only component k of the vector field enters.
  static constexpr bool need(int k, int g) { return g >= D || k == D - 1 || g == k; }
  __device__ __forceinline__ void load_face(unsigned idx, int k, T* in) const {
#pragma unroll
    for (int l = 0; l < D; ++l) in[l] = need(k, l) ? a.qv[l * N + idx] : T(0);
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
  __device__ __forceinline__ void finalize(unsigned idx, const T* acc, T w, T J, const T* tr) const {
    if (a.weak) a.out[idx] = w * (acc[0] + a.amass * J * tr[D]);
    else a.out[idx] = acc[0] / J;
  }
  __device__ __forceinline__ void finalize_add(unsigned idx, const T* acc, T w, T J) const {
    const T v = a.weak ? w * acc[0] : acc[0] / J;
    a.out[idx] += v;
  }
  __device__ __forceinline__ T lam(int cell) const { return a.lam ? a.lam[cell] : T(0); }
};

// The enthalpy-split divergence's two 2:1-face terms in one pass (a.h = h - hbar, a.hb = hbar):
// C((h - hbar) qv) with the penalty and mass terms of a (output 0), and C(qv) (output 1), whose
// lifted value the node multiplies by hbar.  Each output is the one of the corresponding OpDiv
// pass (the second with h = 1, no p, no penalty), and they are added to out in that order.
template <int D, class TT>
struct OpDivSplit {
  using T = TT;
  static constexpr int NIN = D + 2, NTR = 2 * D + 1, NOUT = 2;
  static constexpr int NVOL = 2 * D;
  static constexpr int vidx(int o, int k) { return o * D + k; }
  DivArgs<T> a;
  unsigned N;
  __device__ __forceinline__ void load(unsigned idx, T* in) const {
#pragma unroll
    for (int l = 0; l < D; ++l) in[l] = a.qv[l * N + idx];
    in[D] = a.h[idx];
    in[D + 1] = a.p ? a.p[idx] : T(0);
  }
  // as OpDiv, for both vector traces (h - hbar) qv (0..d-1) and qv (d+1..2d); p is trace d
  static constexpr bool need(int k, int g) {
    return g == D || k == D - 1 || (g < D ? g == k : g - D - 1 == k);
  }
  __device__ __forceinline__ void load_face(unsigned idx, int k, T* in) const {
#pragma unroll
    for (int l = 0; l < D; ++l) in[l] = (k == D - 1 || l == k) ? a.qv[l * N + idx] : T(0);
    in[D] = a.h[idx];
    in[D + 1] = a.p ? a.p[idx] : T(0);
  }
  __device__ __forceinline__ void transform(const T* in, T* tr) const {
#pragma unroll
    for (int l = 0; l < D; ++l) {
      tr[l] = in[D] * in[l];
      tr[D + 1 + l] = in[l];
    }
    tr[D] = in[D + 1];
  }
  __device__ __forceinline__ void vol(const T* tr, const T (&Gam)[D][D], T (&G)[NOUT][D]) const {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T G0 = 0, G1 = 0;
#pragma unroll
      for (int l = 0; l < D; ++l) {
        G0 += Gam[k][l] * tr[l];
        G1 += Gam[k][l] * tr[D + 1 + l];
      }
      G[0][k] = -a.adiv * G0;
      G[1][k] = -a.adiv * G1;
    }
  }
  __device__ __forceinline__ void face(int kind, int left, const T* tm, const T* tn, const T* Nv,
                                       T lm, T ln, T* phi) const {
    if (kind == kWall) {
      phi[0] = 0;
      phi[1] = 0;
      return;
    }
    const T sign = left ? T(1) : T(-1);
    T wm = 0, wn = 0, nn = 0, um = 0, un = 0;
#pragma unroll
    for (int l = 0; l < D; ++l) {
      wm += Nv[l] * tm[l];
      wn += Nv[l] * tn[l];
      nn += Nv[l] * Nv[l];
      um += Nv[l] * tm[D + 1 + l];
      un += Nv[l] * tn[D + 1 + l];
    }
    const T wh = left ? T(0.5) * (wm + wn) : T(0.5) * (wn + wm);
    T v = a.adiv * sign * wh;
    if (a.apen != T(0)) {
      const T lf = lm > ln ? lm : ln;
      v += a.apen * (lf * sqrt(nn) * (tm[D] - tn[D]));
    }
    phi[0] = v;
    const T uh = left ? T(0.5) * (um + un) : T(0.5) * (un + um);
    phi[1] = a.adiv * sign * uh;
  }
  __device__ __forceinline__ void finalize(unsigned idx, const T* acc, T w, T J, const T* tr) const {
    T o = a.weak ? w * (acc[0] + a.amass * J * tr[D]) : acc[0] / J;
    o += a.hb[idx] * (a.weak ? w * acc[1] : acc[1] / J);
    a.out[idx] = o;
  }
  __device__ __forceinline__ void finalize_add(unsigned idx, const T* acc, T w, T J) const {
    T o = a.out[idx];
    o += a.weak ? w * acc[0] : acc[0] / J;
    o += a.hb[idx] * (a.weak ? w * acc[1] : acc[1] / J);
    a.out[idx] = o;
  }
  __device__ __forceinline__ T lam(int cell) const { return a.lam ? a.lam[cell] : T(0); }
};

// Arguments of the general cell kernel: the operator and the cells to visit (list[0..n), or the
// cells 0..n-1 without a list).
template <class Op>
struct CellArgs {
  Op op;
  const int* list;
  int n;
};

template <class Op> struct HasLam { static constexpr bool value = false; };
template <int D, class T> struct HasLam<OpDiv<D, T>> { static constexpr bool value = true; };
template <int D, class T> struct HasLam<OpDivSplit<D, T>> { static constexpr bool value = true; };

// --------------------------------------------------------------------------------- the kernel
// Coarse-face values at a fine sub-face point (tensor interpolation along the tangential axes).
template <int D, int NP, class T>
__device__ __forceinline__ T interp_sub(const T* Pi, const T* Tc, int c0, int c1, int j) {
  T v = 0;
  if constexpr (D == 3) {
    const int j0 = j % NP, j1 = j / NP;
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
  return v;
}

// Area-weighted normal (lower -> upper side along k) at face point j of the (sub)face of cell
// (cl, cid) through face f (= 2k + s), evaluated from the integer description of the (sub)face;
// for a coarse face, sub selects the fine sub-face.  Used on 2:1 faces.
template <int D, int NP, class T>
__device__ __forceinline__ void face_normal(const MeshDev& m, const T* Xi, int cl, const int* cid,
                                            int k, int s, bool coarse, int sub, int j, T* Nv) {
  int lf;
  int P;
  int Tt[3] = {0, 0, 0};
  if (coarse) {
    lf = cl + 1;
    P = s ? 2 * (cid[k] + 1) : 2 * cid[k];
    int tt = 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax)
      if (ax != k) { Tt[ax] = 2 * cid[ax] + ((sub >> tt) & 1); ++tt; }
  } else {
    lf = cl;
    P = s ? cid[k] + 1 : cid[k];
#pragma unroll
    for (int ax = 0; ax < D; ++ax)
      if (ax != k) Tt[ax] = cid[ax];
  }
  if (m.per[k] && P >= m.nlev[lf][k]) P -= m.nlev[lf][k];
  T X[D];
  int tt = 0;
  const int j0 = j % NP, j1 = j / NP;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    const T dx = (T)m.dxl[lf][ax];
    if (ax == k) {
      X[ax] = dx * (T)P;
    } else {
      const int jj = tt == 0 ? j0 : j1;
      X[ax] = dx * ((T)Tt[ax] + T(0.5) * (T(1) + Xi[jj]));
      ++tt;
    }
  }
  T Gam[D][D], Jf;
  metric<D, T>(m, lf, X, Gam, Jf);
#pragma unroll
  for (int a = 0; a < D; ++a) Nv[a] = Gam[k][a];
}

// Terrain table of a cell: (h, h_x, h_y) at every horizontal position its nodes and its own
// conforming-face points use: NHV volume columns, then the x faces (side, y index), then (3D)
// the y faces (side, x index).  Face positions are reduced across periodic boundaries.
template <int D, int NP>
struct TerTab {
  static constexpr int NHV = D == 3 ? NP * NP : NP;
  static constexpr int NHX = D == 3 ? 2 * NP : 2;
  static constexpr int NHY = D == 3 ? 2 * NP : 0;
  static constexpr int NH = NHV + NHX + NHY;
};

// Phases of one workgroup (CPB cells, one thread per node):
//   P0 own inputs -> trace fields in LDS; terrain table per cell;
//   P1 volume fluxes and own traces of all faces;
//   P2 volume contraction, and in the same phase the numerical flux at every point of every
//      conforming or wall face (neighbour traces gathered along the neighbour's normal lines);
//   P3 only for faces with a 2:1 neighbour: neighbour traces, sub-face fluxes, restriction
//      (coarse side) / interpolation (fine side);
//   P4 lift of all faces along the normal lines, finalize.
// With HANG, only the 2:1 faces are evaluated and lifted, and their terms are added to the
// output (the column kernels have written the rest for these cells).
// The faces-only mode asks for 4 waves per SIMD up to degree 4: its 2:1-face phases are latency
// bound, and the register budget that buys (a few dwords of spill in the FP64 divergence) pays.
// S: Direct<CellArgs<Op>> (one mesh) or Shared<CellArgs<Op>> (a shared launch over members).
template <int D, int NP, class Op, bool HANG, class S = Direct<CellArgs<Op>>>
__global__ void __launch_bounds__((Cfg<D, NP>::NT)) __attribute__((amdgpu_waves_per_eu(HANG && NP <= 5 ? 4 : 1))) k_cell(const S src) {
  const int sg = src.seg();
  const Op& op = src.args(sg).op;
  const MeshDev& m = src.mesh(sg);
  const int* __restrict__ list = src.args(sg).list;
  const int n = src.args(sg).n;
  using C = Cfg<D, NP>;
  using T = typename Op::T;
  using TT = TerTab<D, NP>;
  constexpr int NL = C::NL, NFP = C::NFP, MS = C::MS, TPC = C::TPC, CPB = C::CPB, NT = C::NT;
  constexpr int NF = 2 * D;
  constexpr int NTR = Op::NTR, NOUT = Op::NOUT, NIN = Op::NIN;
  constexpr TabLayout TL{NP};
  constexpr int NVOL = Op::NVOL;
  constexpr int VOLSZ = CPB * NVOL * NL;
  constexpr int O_NB = 0;
  constexpr int O_FL = O_NB + CPB * MS * NTR * NFP;
  constexpr int SLOWSZ = O_FL + CPB * MS * NOUT * NFP;
  // the faces-only mode forms no volume fluxes: the scratch holds the 2:1 face buffers only
  constexpr int SCR = (!HANG && VOLSZ > SLOWSZ) ? VOLSZ : SLOWSZ;
  constexpr int NH = TT::NH;

  __shared__ T sTab[TL.size()];
  __shared__ T sT[CPB * NTR * NL];
  __shared__ T sScr[SCR];
  __shared__ T sTown[CPB * NF * NTR * NFP];
  __shared__ T sFr[CPB * NF * NOUT * NFP];
  __shared__ T sTer[CPB * NH * 3];
  __shared__ int4 sCell[CPB];
  __shared__ int sKind[CPB][NF];
  __shared__ int4 sNbr[CPB][NF];
  __shared__ T sLam[CPB];
  __shared__ int sHang[NF];
  __shared__ int sId[CPB];

  const int tid = threadIdx.x;
  const int lc = tid / TPC;
  const int node = tid % TPC;
  const int pos0 = xcd_block(src.blk(sg), src.nblk(sg)) * CPB;  // position in the cell list

  const T* gtab;
  if constexpr (sizeof(T) == 8) gtab = (const T*)m.tab;
  else gtab = (const T*)m.tabf;
  for (int t = tid; t < TL.size(); t += NT) sTab[t] = gtab[t];
  if (tid < NF) sHang[tid] = 0;
  if (tid < CPB) {
    const int i = pos0 + tid;
    const int id = i < n ? (list ? list[i] : i) : -1;
    sId[tid] = id;
    sCell[tid] = id >= 0 ? m.cell[id] : make_int4(0, 0, 0, 0);
  }
  __syncthreads();
  const int cell = sId[lc];
  const bool active = (node < NL) && (cell >= 0);
  if (tid < CPB * NF) {
    const int c = tid / NF, f = tid % NF;
    const int cc = sId[c];
    int kind = kWall;
    int4 nb = make_int4(-1, -1, -1, -1);
    if (cc >= 0) {
      kind = m.fkind[cc * NF + f];
      nb = m.fnbr[cc * NF + f];
    }
    sKind[c][f] = kind;
    sNbr[c][f] = nb;
    if (kind == kFine || kind == kCoarse) atomicOr(&sHang[f], 1);
  }
  if (tid < CPB) {
    if constexpr (HasLam<Op>::value) sLam[tid] = sId[tid] >= 0 ? op.lam(sId[tid]) : T(0);
  }
  // terrain table
  for (int t = tid; t < CPB * NH; t += NT) {
    const int c = t / NH, e = t % NH;
    const int4 ci = sCell[c];
    const int lev = ci.x;
    T x, y = 0;
    const T dx0 = (T)m.dxl[lev][0];
    const T dx1 = (T)m.dxl[lev][1];
    const T* xi = &sTab[TL.xi()];
    if (e < TT::NHV) {
      const int i0 = e % NP;
      x = dx0 * ((T)ci.y + T(0.5) * (T(1) + xi[i0]));
      if (D == 3) y = dx1 * ((T)ci.z + T(0.5) * (T(1) + xi[e / NP]));
    } else if (e < TT::NHV + TT::NHX) {
      const int ee = e - TT::NHV;
      const int sd = ee / (TT::NHX / 2), j = ee % (TT::NHX / 2);
      int P = sd ? ci.y + 1 : ci.y;
      if (m.per[0] && P >= m.nlev[lev][0]) P -= m.nlev[lev][0];
      x = dx0 * (T)P;
      if (D == 3) y = dx1 * ((T)ci.z + T(0.5) * (T(1) + xi[j]));
    } else {
      const int ee = e - TT::NHV - TT::NHX;
      const int sd = ee / NP, i = ee % NP;
      int P = sd ? ci.z + 1 : ci.z;
      if (m.per[1] && P >= m.nlev[lev][1]) P -= m.nlev[lev][1];
      x = dx0 * ((T)ci.y + T(0.5) * (T(1) + xi[i]));
      y = dx1 * (T)P;
    }
    T h, hx, hy;
    terrain<T>(m.ter, D, x, y, h, hx, hy);
    sTer[(c * NH + e) * 3 + 0] = h;
    sTer[(c * NH + e) * 3 + 1] = hx;
    sTer[(c * NH + e) * 3 + 2] = hy;
  }
  T trn[NTR];
  if (active) {
    T in[NIN];
    op.load((unsigned)cell * NL + node, in);
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

  // ---------------------------------------------------------------- P1
  T Jn = 1, wn = 1;
  {
    const int4 ci = sCell[lc];
    if (active) {
      const int i0 = along<D, NP>(node, 0);
      const int iz = along<D, NP>(node, D - 1);
      int col = i0;
      wn = Wt[i0] * Wt[iz];
      if constexpr (D == 3) {
        const int i1 = along<D, NP>(node, 1);
        col += NP * i1;
        wn *= Wt[i1];
      }
      const T zeta = (T)m.dxl[ci.x][D - 1] * ((T)(D == 3 ? ci.w : ci.z) + T(0.5) * (T(1) + Xi[iz]));
      const T* te = &sTer[(lc * NH + col) * 3];
      T Gam[D][D];
      metric_h<D, T>(m, ci.x, te[0], te[1], te[2], zeta, Gam, Jn);
      if constexpr (!HANG) {
        T G[NOUT][D];
        op.vol(trn, Gam, G);
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
          for (int k = 0; k < D; ++k)
            if (Op::vidx(o, k) >= 0) sScr[(lc * NVOL + Op::vidx(o, k)) * NL + node] = G[o][k];
      }
    }
  }
  for (int t = tid; t < CPB * NF * NFP; t += NT) {
    const int c = t / (NF * NFP), f = (t / NFP) % NF, j = t % NFP;
    if (sId[c] < 0) continue;
    if (HANG && sKind[c][f] != kFine && sKind[c][f] != kCoarse) continue;  // only 2:1 faces needed
    const int k = f >> 1, s = f & 1;
    const int base = compose<D, NP>(k, 0, j);
    const int str = compose<D, NP>(k, 1, 0);
#pragma unroll
    for (int g = 0; g < NTR; ++g) {
      T v = 0;
      if (Op::need(k, g)) {
        const T* src = &sT[(c * NTR + g) * NL + base];
#pragma unroll
        for (int q = 0; q < NP; ++q) v += Lb[s * NP + q] * src[q * str];
      }
      sTown[((c * NF + f) * NTR + g) * NFP + j] = v;
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- P2
  T acc[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) acc[o] = 0;
  if constexpr (!HANG) {  // the faces-only mode has no volume terms (and no volume scratch)
    if (active) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int ik = along<D, NP>(node, k);
        const int base = compose<D, NP>(k, 0, tang<D, NP>(node, k));
        const int str = k == 0 ? 1 : (k == 1 ? NP : NP * NP);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const T dq = Dt[ik * NP + q];
#pragma unroll
          for (int o = 0; o < NOUT; ++o)
            if (Op::vidx(o, k) >= 0) acc[o] += dq * sScr[(lc * NVOL + Op::vidx(o, k)) * NL + base + q * str];
        }
      }
    }
  }
  for (int t = tid; t < CPB * NF * NFP; t += NT) {
    const int c = t / (NF * NFP), f = (t / NFP) % NF, j = t % NFP;
    if (sId[c] < 0) continue;
    const int kind = sKind[c][f];
    if (kind != kConf && kind != kWall) continue;
    if constexpr (HANG) continue;  // conforming and wall faces belong to the column kernel
    const int k = f >> 1, s = f & 1;
    T tm[NTR], tn[NTR];
#pragma unroll
    for (int g = 0; g < NTR; ++g) tm[g] = sTown[((c * NF + f) * NTR + g) * NFP + j];
    T ln = 0;
    if (kind == kConf) {
      const int nb = sNbr[c][f].x;
      const unsigned base = (unsigned)nb * NL + compose<D, NP>(k, 0, j);
      const int str = compose<D, NP>(k, 1, 0);
#pragma unroll
      for (int g = 0; g < NTR; ++g) tn[g] = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        T in[NIN], tr[NTR];
        op.load_face(base + q * str, k, in);
        op.transform(in, tr);
        const T lq = Lb[(1 - s) * NP + q];
#pragma unroll
        for (int g = 0; g < NTR; ++g) tn[g] += lq * tr[g];
      }
      if constexpr (HasLam<Op>::value) ln = op.lam(nb);
    } else {
#pragma unroll
      for (int g = 0; g < NTR; ++g) tn[g] = tm[g];
    }
    // normal from the terrain table
    const int4 ci = sCell[c];
    const T* terc = &sTer[c * NH * 3];
    T Nv[D];
    const T invH = (T)m.invH;
    if constexpr (D == 3) {
      const T a = T(0.5) * (T)m.dxl[ci.x][0], b = T(0.5) * (T)m.dxl[ci.x][1];
      const T e = T(0.5) * (T)m.dxl[ci.x][2];
      if (k == 0) {
        const T h = terc[(TT::NHV + s * NP + (j % NP)) * 3];
        Nv[0] = b * e * (T(1) - h * invH); Nv[1] = 0; Nv[2] = 0;
      } else if (k == 1) {
        const T h = terc[(TT::NHV + TT::NHX + s * NP + (j % NP)) * 3];
        Nv[0] = 0; Nv[1] = a * e * (T(1) - h * invH); Nv[2] = 0;
      } else {
        const T* te = &terc[j * 3];
        const T zf = (T)m.dxl[ci.x][2] * (T)(s ? ci.w + 1 : ci.w);
        const T om = T(1) - zf * invH;
        Nv[0] = -a * b * (te[1] * om); Nv[1] = -a * b * (te[2] * om); Nv[2] = a * b;
      }
    } else {
      const T a = T(0.5) * (T)m.dxl[ci.x][0], e = T(0.5) * (T)m.dxl[ci.x][1];
      if (k == 0) {
        const T h = terc[(TT::NHV + s) * 3];
        Nv[0] = e * (T(1) - h * invH); Nv[1] = 0;
      } else {
        const T* te = &terc[j * 3];
        const T zf = (T)m.dxl[ci.x][1] * (T)(s ? ci.z + 1 : ci.z);
        const T om = T(1) - zf * invH;
        Nv[0] = -a * (te[1] * om); Nv[1] = a;
      }
    }
    T lm = 0;
    if constexpr (HasLam<Op>::value) lm = sLam[c];
    T phi[NOUT];
    op.face(kind, s, tm, tn, Nv, lm, ln, phi);
#pragma unroll
    for (int o = 0; o < NOUT; ++o) sFr[((c * NF + f) * NOUT + o) * NFP + j] = phi[o];
  }
  __syncthreads();

  // ---------------------------------------------------------------- P3 (2:1 faces only)
  T* sNb = &sScr[O_NB];
  T* sFl = &sScr[O_FL];
  for (int f = 0; f < NF; ++f) {
    if (!sHang[f]) continue;  // block-uniform
    const int k = f >> 1, s = f & 1;
    for (int t = tid; t < CPB * MS * NFP; t += NT) {
      const int c = t / (MS * NFP), sub = (t / NFP) % MS, j = t % NFP;
      if (sId[c] < 0) continue;
      const int kind = sKind[c][f];
      if (!(kind == kCoarse || (kind == kFine && sub == 0))) continue;
      const int4 nb4 = sNbr[c][f];
      const int nb = sub == 0 ? nb4.x : sub == 1 ? nb4.y : sub == 2 ? nb4.z : nb4.w;
      T v[NTR];
#pragma unroll
      for (int g = 0; g < NTR; ++g) v[g] = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        T in[NIN], tr[NTR];
        op.load((unsigned)nb * NL + compose<D, NP>(k, q, j), in);
        op.transform(in, tr);
        const T lq = Lb[(1 - s) * NP + q];
#pragma unroll
        for (int g = 0; g < NTR; ++g) v[g] += lq * tr[g];
      }
#pragma unroll
      for (int g = 0; g < NTR; ++g) sNb[((c * MS + sub) * NTR + g) * NFP + j] = v[g];
    }
    __syncthreads();
    for (int t = tid; t < CPB * MS * NFP; t += NT) {
      const int c = t / (MS * NFP), sub = (t / NFP) % MS, j = t % NFP;
      if (sId[c] < 0) continue;
      const int kind = sKind[c][f];
      if (!(kind == kCoarse || (kind == kFine && sub == 0))) continue;
      const int4 cc = sCell[c];
      const int cid[3] = {cc.y, cc.z, cc.w};
      T tm[NTR], tn[NTR];
      const T* Town = &sTown[((c * NF + f) * NTR) * NFP];
      if (kind == kCoarse) {
        const int c0 = sub & 1, c1 = sub >> 1;
#pragma unroll
        for (int g = 0; g < NTR; ++g) {
          tm[g] = interp_sub<D, NP, T>(Pi, Town + g * NFP, c0, c1, j);
          tn[g] = sNb[((c * MS + sub) * NTR + g) * NFP + j];
        }
      } else {
        int cs[2] = {0, 0};
        int tt = 0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax)
          if (ax != k) cs[tt++] = cid[ax] & 1;
#pragma unroll
        for (int g = 0; g < NTR; ++g) {
          tm[g] = Town[g * NFP + j];
          tn[g] = interp_sub<D, NP, T>(Pi, &sNb[((c * MS) * NTR + g) * NFP], cs[0], cs[1], j);
        }
      }
      T Nv[D];
      face_normal<D, NP, T>(m, Xi, cc.x, cid, k, s, kind == kCoarse, sub, j, Nv);
      T lm = 0, ln = 0;
      if constexpr (HasLam<Op>::value) {
        const int4 nb4 = sNbr[c][f];
        const int nb = sub == 0 ? nb4.x : sub == 1 ? nb4.y : sub == 2 ? nb4.z : nb4.w;
        lm = sLam[c];
        ln = op.lam(nb);
      }
      T phi[NOUT];
      op.face(kind, s, tm, tn, Nv, lm, ln, phi);
#pragma unroll
      for (int o = 0; o < NOUT; ++o) sFl[((c * MS + sub) * NOUT + o) * NFP + j] = phi[o];
    }
    __syncthreads();
    for (int t = tid; t < CPB * NFP; t += NT) {
      const int c = t / NFP, a = t % NFP;
      if (sId[c] < 0) continue;
      const int kind = sKind[c][f];
      if (kind != kCoarse && kind != kFine) continue;
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
        sFr[((c * NF + f) * NOUT + o) * NFP + a] = v;
      }
    }
    __syncthreads();
  }

  // ---------------------------------------------------------------- P4
  if (active) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (HANG && sKind[lc][f] != kFine && sKind[lc][f] != kCoarse) continue;  // lift 2:1 faces only
      const int k = f >> 1, s = f & 1;
      const int ik = along<D, NP>(node, k);
      const int a = tang<D, NP>(node, k);
      const T lw = Lbw[s * NP + ik];
#pragma unroll
      for (int o = 0; o < NOUT; ++o) acc[o] += lw * sFr[((lc * NF + f) * NOUT + o) * NFP + a];
    }
    if constexpr (HANG) op.finalize_add((unsigned)cell * NL + node, acc, wn, Jn);
    else op.finalize((unsigned)cell * NL + node, acc, wn, Jn, trn);
  }
}

template <int D, int NP, class Op, bool HANG = false>
int run(const Op& op, const MeshDev& m, const int* list, int n, hipStream_t s) {
  using C = Cfg<D, NP>;
  if (n <= 0) return 0;
  const int grid = (n + C::CPB - 1) / C::CPB;
  hipLaunchKernelGGL((k_cell<D, NP, Op, HANG>), dim3(grid), dim3(C::NT), 0, s,
                     Direct<CellArgs<Op>>{CellArgs<Op>{op, list, n}, m});
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// The faces-only 2:1 pass over the members' cells with such faces, in one shared launch.
template <int D, int NP, class Op, class MakeOp>
int run_hang_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, MakeOp make, hipStream_t s) {
  using C = Cfg<D, NP>;
  using A = CellArgs<Op>;
  return seg_launch<A>(
      n, md, [&](int k) { return (mh[k]->nirr + C::CPB - 1) / C::CPB; },
      [&](int k) { return A{make(k), mh[k]->irr, mh[k]->nirr}; },
      [&](const SegTab<A>& t, int g) {
        hipLaunchKernelGGL((k_cell<D, NP, Op, true, Shared<A>>), dim3(g), dim3(C::NT), 0, s, Shared<A>{t});
        return hipGetLastError() == hipSuccess ? 0 : -3;
      });
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

int launch_explicit_hang(const MeshDev& m, int degree, const double* U, double* R, hipStream_t s) {
  const int* list = m.irr;
  const int n = m.nirr;
  if (m.dim == 2) {
    OpExplicit<2> op{U, R, (unsigned)m.N};
    DG_DISPATCH(2, degree, return (run<2, NP, OpExplicit<2>, true>(op, m, list, n, s)));
  } else {
    OpExplicit<3> op{U, R, (unsigned)m.N};
    DG_DISPATCH(3, degree, return (run<3, NP, OpExplicit<3>, true>(op, m, list, n, s)));
  }
}

template <class T, bool HANG = false>
static int grad_impl(const MeshDev& m, int degree, const GradArgs<T>& a, const int* list, int n, hipStream_t s) {
  if (m.dim == 2) {
    OpGrad<2, T> op{a, (unsigned)m.N};
    DG_DISPATCH(2, degree, return (run<2, NP, OpGrad<2, T>, HANG>(op, m, list, n, s)));
  } else {
    OpGrad<3, T> op{a, (unsigned)m.N};
    DG_DISPATCH(3, degree, return (run<3, NP, OpGrad<3, T>, HANG>(op, m, list, n, s)));
  }
}

template <class T, bool HANG = false>
static int div_impl(const MeshDev& m, int degree, const DivArgs<T>& a, const int* list, int n, hipStream_t s) {
  if (m.dim == 2) {
    OpDiv<2, T> op{a, (unsigned)m.N};
    DG_DISPATCH(2, degree, return (run<2, NP, OpDiv<2, T>, HANG>(op, m, list, n, s)));
  } else {
    OpDiv<3, T> op{a, (unsigned)m.N};
    DG_DISPATCH(3, degree, return (run<3, NP, OpDiv<3, T>, HANG>(op, m, list, n, s)));
  }
}

int launch_grad_cells64(const MeshDev& m, int degree, const GradArgs<double>& a, const int* list, int n, hipStream_t s) {
  return grad_impl<double>(m, degree, a, list, n, s);
}
int launch_div_cells64(const MeshDev& m, int degree, const DivArgs<double>& a, const int* list, int n, hipStream_t s) {
  return div_impl<double>(m, degree, a, list, n, s);
}
int launch_grad_cells32(const MeshDev& m, int degree, const GradArgs<float>& a, const int* list, int n, hipStream_t s) {
  return grad_impl<float>(m, degree, a, list, n, s);
}
int launch_div_cells32(const MeshDev& m, int degree, const DivArgs<float>& a, const int* list, int n, hipStream_t s) {
  return div_impl<float>(m, degree, a, list, n, s);
}
template <class T>
static int div_split_hang_impl(const MeshDev& m, int degree, const DivArgs<T>& a, hipStream_t s) {
  if (!a.h || !a.hb) return -3;
  if (m.dim == 2) {
    OpDivSplit<2, T> op{a, (unsigned)m.N};
    DG_DISPATCH(2, degree, return (run<2, NP, OpDivSplit<2, T>, true>(op, m, m.irr, m.nirr, s)));
  } else {
    OpDivSplit<3, T> op{a, (unsigned)m.N};
    DG_DISPATCH(3, degree, return (run<3, NP, OpDivSplit<3, T>, true>(op, m, m.irr, m.nirr, s)));
  }
}
int launch_div_split_hang64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s) {
  return div_split_hang_impl<double>(m, degree, a, s);
}
int launch_div_split_hang32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s) {
  return div_split_hang_impl<float>(m, degree, a, s);
}

int launch_grad_hang64(const MeshDev& m, int degree, const GradArgs<double>& a, hipStream_t s) {
  return grad_impl<double, true>(m, degree, a, m.irr, m.nirr, s);
}
int launch_div_hang64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s) {
  return div_impl<double, true>(m, degree, a, m.irr, m.nirr, s);
}
int launch_grad_hang32(const MeshDev& m, int degree, const GradArgs<float>& a, hipStream_t s) {
  return grad_impl<float, true>(m, degree, a, m.irr, m.nirr, s);
}
int launch_div_hang32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s) {
  return div_impl<float, true>(m, degree, a, m.irr, m.nirr, s);
}

template <class T>
static int grad_hang_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<T>* a,
                         int degree, hipStream_t s) {
  if (n <= 0) return 0;
  if (mh[0]->dim == 2) {
    auto mk = [&](int k) { return OpGrad<2, T>{a[k], (unsigned)mh[k]->N}; };
    DG_DISPATCH(2, degree, return (run_hang_seg<2, NP, OpGrad<2, T>>(n, mh, md, mk, s)));
  } else {
    auto mk = [&](int k) { return OpGrad<3, T>{a[k], (unsigned)mh[k]->N}; };
    DG_DISPATCH(3, degree, return (run_hang_seg<3, NP, OpGrad<3, T>>(n, mh, md, mk, s)));
  }
}
template <class T>
static int div_hang_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<T>* a,
                        int degree, hipStream_t s) {
  if (n <= 0) return 0;
  if (mh[0]->dim == 2) {
    auto mk = [&](int k) { return OpDiv<2, T>{a[k], (unsigned)mh[k]->N}; };
    DG_DISPATCH(2, degree, return (run_hang_seg<2, NP, OpDiv<2, T>>(n, mh, md, mk, s)));
  } else {
    auto mk = [&](int k) { return OpDiv<3, T>{a[k], (unsigned)mh[k]->N}; };
    DG_DISPATCH(3, degree, return (run_hang_seg<3, NP, OpDiv<3, T>>(n, mh, md, mk, s)));
  }
}
int launch_grad_hang_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<double>* a, int degree, hipStream_t s) {
  return grad_hang_seg<double>(n, mh, md, a, degree, s);
}
int launch_grad_hang_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<float>* a, int degree, hipStream_t s) {
  return grad_hang_seg<float>(n, mh, md, a, degree, s);
}
int launch_div_hang_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<double>* a, int degree, hipStream_t s) {
  return div_hang_seg<double>(n, mh, md, a, degree, s);
}
int launch_div_hang_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<float>* a, int degree, hipStream_t s) {
  return div_hang_seg<float>(n, mh, md, a, degree, s);
}
template <class T>
static int div_split_hang_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<T>* a,
                              int degree, hipStream_t s) {
  if (n <= 0) return 0;
  for (int k = 0; k < n; ++k)
    if (!a[k].h || !a[k].hb) return -3;
  if (mh[0]->dim == 2) {
    auto mk = [&](int k) { return OpDivSplit<2, T>{a[k], (unsigned)mh[k]->N}; };
    DG_DISPATCH(2, degree, return (run_hang_seg<2, NP, OpDivSplit<2, T>>(n, mh, md, mk, s)));
  } else {
    auto mk = [&](int k) { return OpDivSplit<3, T>{a[k], (unsigned)mh[k]->N}; };
    DG_DISPATCH(3, degree, return (run_hang_seg<3, NP, OpDivSplit<3, T>>(n, mh, md, mk, s)));
  }
}
int launch_div_split_hang_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<double>* a, int degree, hipStream_t s) {
  return div_split_hang_seg<double>(n, mh, md, a, degree, s);
}
int launch_div_split_hang_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<float>* a, int degree, hipStream_t s) {
  return div_split_hang_seg<float>(n, mh, md, a, degree, s);
}
int launch_explicit_hang_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const ExpArgs* a, int degree, hipStream_t s) {
  if (n <= 0) return 0;
  if (mh[0]->dim == 2) {
    auto mk = [&](int k) { return OpExplicit<2>{a[k].U, a[k].R, (unsigned)mh[k]->N}; };
    DG_DISPATCH(2, degree, return (run_hang_seg<2, NP, OpExplicit<2>>(n, mh, md, mk, s)));
  } else {
    auto mk = [&](int k) { return OpExplicit<3>{a[k].U, a[k].R, (unsigned)mh[k]->N}; };
    DG_DISPATCH(3, degree, return (run_hang_seg<3, NP, OpExplicit<3>>(n, mh, md, mk, s)));
  }
}

// ------------------------------------------------------------------ per-cell coefficients
namespace {
// One wavefront per cell: lam = sqrt((gamma-1) max h); hbar, Jbar (J = wJ / w); coefficients of
// the fast-diagonalisation preconditioner alpha_k = (dt a)^2 hbar (2 / D_k)^2 with the vertical
// size scaled by the cell's mean terrain stretching.
template <int D, int NP, class S = Direct<CoefArgs>>
__global__ void k_cellcoef(const S src) {
  const int sg = src.seg();
  const MeshDev& m = src.mesh(sg);
  const CoefArgs& ca = src.args(sg);
  const double* __restrict__ h = ca.h;
  const double* __restrict__ wJ = ca.wJ;
  const double dta = ca.dta;
  double* lam = ca.lam;
  float* lam32 = ca.lam32;
  double* coef = ca.coef;
  float* coef32 = ca.coef32;
  constexpr int NL = ipow(NP, D);
  constexpr TabLayout TL{NP};
  const int c = src.blk(sg) * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= m.ncell) return;
  const double* w1 = m.tab + TL.w();
  double hmax = 0.0, hsum = 0.0, jsum = 0.0;
  for (int i = lane; i < NL; i += 64) {
    const double hv = h[(unsigned)c * NL + i];
    double wi = 1.0;
    for (int k = 0; k < D; ++k) wi *= w1[along<D, NP>(i, k)];
    hmax = fmax(hmax, hv);
    hsum += hv;
    jsum += wJ[(unsigned)c * NL + i] / wi;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    hmax = fmax(hmax, __shfl_xor(hmax, o, 64));
    hsum += __shfl_xor(hsum, o, 64);
    jsum += __shfl_xor(jsum, o, 64);
  }
  if (lane != 0) return;
  const double l = sqrt((kGamma - 1.0) * hmax);
  lam[c] = l;
  if (lam32) lam32[c] = (float)l;
  if (!coef) return;
  const int lev = m.cell[c].x;
  const double hb = hsum / NL, Jb = jsum / NL;
  double half = 1.0;
  for (int k = 0; k < D; ++k) half *= 0.5 * m.dxl[lev][k];
  const double stretch = Jb / half;  // mean (1 - h / H)
  double cf[4] = {1.0 / Jb, 0.0, 0.0, 0.0};
  for (int k = 0; k < D; ++k) {
    const double dk = m.dxl[lev][k] * (k == D - 1 ? stretch : 1.0);
    cf[1 + k] = dta * dta * hb * (2.0 / dk) * (2.0 / dk);
  }
  for (int k = 0; k < 4; ++k) {
    coef[c * 4 + k] = cf[k];
    if (coef32) coef32[c * 4 + k] = (float)cf[k];
  }
}
}  // namespace

namespace {
template <int D, int NP>
int run_cellcoef(const MeshDev& m, const double* h, const double* wJ, double dta, double* lam,
                 float* lam32, double* coef, float* coef32, hipStream_t s) {
  hipLaunchKernelGGL((k_cellcoef<D, NP>), dim3((m.ncell + 3) / 4), dim3(256), 0, s,
                     Direct<CoefArgs>{CoefArgs{h, wJ, dta, lam, lam32, coef, coef32}, m});
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
template <int D, int NP>
int run_cellcoef_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const CoefArgs* a, hipStream_t s) {
  return seg_launch<CoefArgs>(
      n, md, [&](int k) { return (mh[k]->ncell + 3) / 4; }, [&](int k) { return a[k]; },
      [&](const SegTab<CoefArgs>& t, int g) {
        hipLaunchKernelGGL((k_cellcoef<D, NP, Shared<CoefArgs>>), dim3(g), dim3(256), 0, s, Shared<CoefArgs>{t});
        return hipGetLastError() == hipSuccess ? 0 : -3;
      });
}
}  // namespace

int launch_cellcoef_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const CoefArgs* a, int degree,
                        hipStream_t s) {
  if (n <= 0) return 0;
  for (int k = 0; k < n; ++k)
    if (mh[k]->dim != mh[0]->dim) return -6;
  if (mh[0]->dim == 2) {
    DG_DISPATCH(2, degree, return (run_cellcoef_seg<2, NP>(n, mh, md, a, s)));
  } else {
    DG_DISPATCH(3, degree, return (run_cellcoef_seg<3, NP>(n, mh, md, a, s)));
  }
}

int launch_cellcoef(const MeshDev& m, int degree, const double* h, const double* wJ, double dta,
                    double* lam, float* lam32, double* coef, float* coef32, hipStream_t s) {
  if (m.ncell == 0) return 0;
  if (m.dim == 2) {
    DG_DISPATCH(2, degree, return (run_cellcoef<2, NP>(m, h, wJ, dta, lam, lam32, coef, coef32, s)));
  } else {
    DG_DISPATCH(3, degree, return (run_cellcoef<3, NP>(m, h, wJ, dta, lam, lam32, coef, coef32, s)));
  }
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
                           double* wJ, double* pbar, double* rbar, double* tau) {
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
    const double dx = m.dxl[ci.x][a];
    X[a] = dx * (cidx[a] + 0.5 * (1.0 + Xi[ia]));
    w *= Wt[ia];
  }
  double Gam[D][D], J;
  metric<D, double>(m, ci.x, X, Gam, J);
  double h, hx, hy;
  terrain<double>(m.ter, D, X[0], D == 3 ? X[1] : 0.0, h, hx, hy);
  const double zz = X[D - 1] + h * (1.0 - X[D - 1] * m.invH);
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
  if (tau) {
    // absorbing-layer rate: sin^2 ramps below the lid (physical height) and towards each lateral
    // side, walled or periodic, each scaled by its rate
    const double depth = m.sponge[0], rt = m.sponge[1], width = m.sponge[2], rl = m.sponge[3];
    double t = 0.0;
    if (rl > 0.0 && width > 0.0)
      for (int a = 0; a < D - 1; ++a) {
        const double d = fmin(X[a], m.L[a] - X[a]);
        if (d < width) {
          const double sn = sin(0.5 * kPi * (1.0 - d / width));
          t += rl * sn * sn;
        }
      }
    const double zs = m.L[D - 1] - depth;
    if (rt > 0.0 && zz > zs) {
      const double sn = sin(0.5 * kPi * ((zz - zs) / depth));
      t += rt * sn * sn;
    }
    tau[gid] = t;
  }
}

}  // namespace

int launch_geometry(const MeshDev& m, int degree, double* x, double* y, double* z, double* wJ,
                    double* pbar, double* rbar, double* tau, int atm_kind, const double* atm,
                    hipStream_t s) {
  Atm at{atm_kind, atm[0], atm[1], atm[2]};
  const int grid = (int)((m.N + 255) / 256);
  if (m.N == 0) return 0;
#define DG_GEO(D_)                                                                               \
  DG_DISPATCH(D_, degree,                                                                        \
              hipLaunchKernelGGL((k_geometry<D_, NP>), dim3(grid), dim3(256), 0, s, m, at, x, y, \
                                 z, wJ, pbar, rbar, tau);                                        \
              return hipGetLastError() == hipSuccess ? 0 : -3)
  if (m.dim == 2) {
    DG_GEO(2);
  } else {
    DG_GEO(3);
  }
#undef DG_GEO
}

}  // namespace dg
