// Column kernels of the cell operators (arXiv 2408.08129, Section 3.2): the two Helmholtz passes
// (the weak gradient M^{-1} B and the weak divergence C with the pressure-jump penalty), the
// explicit advective residual and the cell-wise preconditioner.  They cover every cell; a 2:1
// face contributes nothing here, and the general cell kernel adds the terms of those faces for
// the cells that have one (its faces-only mode).
//
// Layout: one thread owns one vertical column of a cell (NP nodes, the last, vertical axis is the
// slowest in the node order), so a cell is NP^(d-1) threads and a 256-thread workgroup holds
// 256 / NP^(d-1) cells.  The column is held in registers: the vertical contraction, the traces on
// the horizontal faces (bottom / top) and their lift never leave the thread.  The contractions
// along x (and y) and the traces on the x (and y) faces read the exchanged fields from LDS; the
// thread that owns column c also owns face point c of every x / y face, evaluates the flux there
// and passes it through LDS to the threads whose nodes it lifts onto.  Two workgroup barriers.
//
// The terrain-following map keeps the x and y face normals axis aligned (Gam[k][l] = 0 for
// k < d-1, l != k) and its metric constant along a column except for the slope terms of the
// vertical row, which is what lets the x / y passes exchange only the fields they need.
#include "dg_device.hpp"

namespace dg {
namespace {
using namespace dev;

template <int D, int NP>
struct Col {
  static constexpr int NC = ipow(NP, D - 1);  // columns per cell = points per face
  static constexpr int NL = NC * NP;
  static constexpr int NF = 2 * D;
  static constexpr int CPB = 256 / NC;         // cells per workgroup
  static constexpr int NTA = CPB * NC;         // threads that own a column
  static constexpr int NT = 256;
  static constexpr int NHC = D == 3 ? NP : 1;  // terrain samples per x / y face
};

// Input fields at node idx.  These kernels take p as given (no Jacobi scaling; the general cell
// kernel covers that form).  Divergence: w = h qv with the multiplier h when HH (then p may be
// absent), else the vector field already multiplied by h.
template <class T>
__device__ __forceinline__ T grad_in(const GradArgs<T>& a, unsigned idx) {
  return a.p[idx];
}
template <int D, class T, bool HH>
__device__ __forceinline__ void div_in(const DivArgs<T>& a, unsigned N, unsigned idx, int mask, T* w, T& p) {
  const T h = HH ? a.h[idx] : T(1);
#pragma unroll
  for (int l = 0; l < D; ++l) w[l] = ((mask >> l) & 1) ? (HH ? h * a.qv[l * N + idx] : a.qv[l * N + idx]) : T(0);
  if (HH) p = a.p ? a.p[idx] : T(0);
  else p = a.p[idx];
}

// Materialise a value at this point of the program: keeps the compiler from sinking arithmetic
// past a barrier and holding every operand it read live until the end of the kernel.
template <class T>
__device__ __forceinline__ void pin(T& v) {
  asm volatile("" : "+v"(v));
}

// node offset inside a cell of point q along the normal of face axis k at face point a
template <int D, int NP>
__device__ __forceinline__ int offs(int k, int q, int a) {
  return compose<D, NP>(k, q, a);
}

// FP32 up to degree 4: the divergence fits 5 waves per SIMD (<= 96 VGPRs) and the gradient 6
// (<= 80) without spills; the FP64 forms are limited by LDS (divergence) or would spill.
// SPLIT (with DIV and HH, a.h = h - hbar): the enthalpy-split energy flux in one pass,
// out = C((h - hbar) qv) + hbar C(qv) + adiv M (d hbar/dz) qv_z (+ penalty and mass terms): qv and
// h - hbar are exchanged separately, and a second accumulator carries C(qv).
// S: Direct<A> (one mesh) or Shared<A> (a shared launch over ensemble members).
template <int D, int NP, class T, bool DIV, class A, bool HH = false, bool SPLIT = false, class S = Direct<A>>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && NP <= 5 ? (DIV ? (HH ? 1 : 5) : 6) : 1))) k_col(const S src) {
  static_assert(!SPLIT || (DIV && HH), "the split form is a divergence with the h multiplier");
  const int sg = src.seg();
  const A& a = src.args(sg);
  const MeshDev& m = src.mesh(sg);
  using C = Col<D, NP>;
  constexpr int NC = C::NC, NL = C::NL, NF = C::NF, CPB = C::CPB, NHC = C::NHC;
  constexpr TabLayout TL{NP};
  constexpr int NX = DIV ? (SPLIT ? D + 1 : D) : 1;  // exchanged fields: grad p; div w_0 .. w_{d-2}, p
                                                     // (split: qv_0 .. qv_{d-2}, p, h - hbar)
  constexpr int NH = D - 1;        // horizontal axes

  __shared__ T sTab[TL.size()];
  __shared__ T sX[CPB][NX][NL];
  __shared__ T sFc[CPB][NC];               // e (1 - h/H) per column
  __shared__ T sHf[CPB][NH][2][NHC];       // e (1 - h/H) at the x / y face samples
  __shared__ T sPhi[CPB][2 * NH][NC];      // fluxes on the x / y faces
  __shared__ T sPhi2[SPLIT ? CPB : 1][SPLIT ? 2 * NH : 1][SPLIT ? NC : 1];  // split: those of C(qv)
  // gradient: the workgroup's cells are pieces of vertical runs, and a cell passes its p traces on
  // the bottom / top faces to the run neighbour in the same workgroup through LDS; the divergence
  // passes keep the Morton order and gather (the exchange cost them registers, the run order
  // locality)
  constexpr bool XZ = !DIV;
  __shared__ T sZ[XZ ? CPB : 1][2][XZ ? NC : 1];

  const int tid = threadIdx.x;
  const bool lane = tid < C::NTA;
  const int lc = lane ? tid / NC : CPB - 1;
  const int c = tid % NC;
  const int slot = xcd_block(src.blk(sg), src.nblk(sg)) * CPB + lc;
  int rcell = lane && slot < m.ncell ? slot : -1;
  if constexpr (XZ) rcell = lane ? m.runs[slot] : -1;  // see MeshDev::runs
  const int cell = rcell >= 0 ? rcell : 0;
  const int rflag = (XZ && rcell >= 0) ? m.rflag[slot] : 0;
  const unsigned N = (unsigned)m.N;
  const int i0 = c % NP;
  const int i1 = D == 3 ? c / NP : 0;

  const T* gtab;
  if constexpr (sizeof(T) == 8) gtab = (const T*)m.tab;
  else gtab = (const T*)m.tabf;
  for (int t = tid; t < TL.size(); t += C::NT) sTab[t] = gtab[t];

  // ---------------------------------------------------------------- loads
  const int4 ci = m.cell[cell];
  // 2:1 faces contribute nothing here: the general kernel adds their terms afterwards
  int kind[NF], nb[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    kind[f] = m.fkind[cell * NF + f];
    nb[f] = m.fnbr[cell * NF + f].x;
  }
  const bool active = rcell >= 0;
  const unsigned base = (unsigned)cell * NL + c;
  T pv[NP];            // grad: p; div: p (penalty / mass)
  T wv[D][NP];         // div: h qv (split: qv)
  T hv[SPLIT ? NP : 1];  // split: h - hbar
#pragma unroll
  for (int z = 0; z < NP; ++z) {
    if constexpr (SPLIT) {
      const unsigned idx = base + NC * z;
#pragma unroll
      for (int l = 0; l < D; ++l) wv[l][z] = a.qv[l * N + idx];
      hv[z] = a.h[idx];
      pv[z] = a.p ? a.p[idx] : T(0);
    } else if constexpr (DIV) {
      T w[D];
      div_in<D, T, HH>(a, N, base + NC * z, (1 << D) - 1, w, pv[z]);
#pragma unroll
      for (int l = 0; l < D; ++l) wv[l][z] = w[l];
    } else {
      pv[z] = grad_in<T>(a, base + NC * z);
    }
  }
  // neighbour traces at this thread's point of every face (tn[f][0..D-1] = w, tn[f][D] = p)
  T tn[NF][D + 1];
  T tn2[SPLIT ? NF : 1][SPLIT ? D : 1];  // split: traces of qv
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int k = f >> 1, s = f & 1;
#pragma unroll
    for (int g = 0; g <= D; ++g) tn[f][g] = 0;
    if constexpr (SPLIT) {
#pragma unroll
      for (int g = 0; g < D; ++g) tn2[f][g] = 0;
    }
    if (kind[f] != kConf) continue;
    if (k == D - 1 && ((rflag >> s) & 1)) continue;  // the neighbour's trace comes through LDS
    const unsigned nbase = (unsigned)nb[f] * NL;
    const int mask = k == D - 1 ? (1 << D) - 1 : (1 << k);
    if (k == 0) {
      // x faces: the normal line is contiguous in memory (w_0 and p are exchanged)
      const unsigned idx = nbase + offs<D, NP>(0, 0, c);
      T wl[NP], pl[NP];
      if constexpr (DIV) {
        load_line<NP>(a.qv + idx, wl);
        if constexpr (HH) {
          T hl[NP];
          load_line<NP>(a.h + idx, hl);
          if constexpr (SPLIT) {
#pragma unroll
            for (int q = 0; q < NP; ++q) tn2[f][0] += gtab[TL.lb() + (1 - s) * NP + q] * wl[q];
          }
#pragma unroll
          for (int q = 0; q < NP; ++q) wl[q] *= hl[q];
        }
      }
      if (!HH || a.p) {
        load_line<NP>(a.p + idx, pl);
      } else {
#pragma unroll
        for (int q = 0; q < NP; ++q) pl[q] = 0;
      }
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const T lq = gtab[TL.lb() + (1 - s) * NP + q];
        if constexpr (DIV) tn[f][0] += lq * wl[q];
        tn[f][D] += lq * pl[q];
      }
      continue;
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const T lq = gtab[TL.lb() + (1 - s) * NP + q];
      const unsigned idx = nbase + offs<D, NP>(k, q, c);
      if constexpr (SPLIT) {
        const T hh = a.h[idx];
#pragma unroll
        for (int l = 0; l < D; ++l) {
          if ((mask >> l) & 1) {
            const T qq = a.qv[l * N + idx];
            tn2[f][l] += lq * qq;
            tn[f][l] += lq * (hh * qq);
          }
        }
        tn[f][D] += lq * (a.p ? a.p[idx] : T(0));
      } else if constexpr (DIV) {
        T w[D], p;
        div_in<D, T, HH>(a, N, idx, mask, w, p);
#pragma unroll
        for (int l = 0; l < D; ++l) tn[f][l] += lq * w[l];
        tn[f][D] += lq * p;
      } else {
        tn[f][D] += lq * grad_in<T>(a, idx);
      }
    }
  }
  T lam_own = 0, lam_nb[NF];
  if constexpr (DIV) {
    lam_own = a.lam ? a.lam[cell] : T(0);
#pragma unroll
    for (int f = 0; f < NF; ++f) lam_nb[f] = (a.lam && kind[f] == kConf) ? a.lam[nb[f]] : T(0);
  }

  // ---------------------------------------------------------------- geometry
  const int lev = ci.x;
  const int iz = D == 3 ? ci.w : ci.z;
  const T dx0 = (T)m.dxl[lev][0], dx1 = (T)m.dxl[lev][1], dxz = (T)m.dxl[lev][D - 1];
  const T invH = (T)m.invH;
  const T ha = T(0.5) * dx0, hb = T(0.5) * dx1, he = T(0.5) * dxz;
  const T* xi = gtab + TL.xi();
  T h, hx, hy;
  {
    const T x = dx0 * ((T)ci.y + T(0.5) * (T(1) + xi[i0]));
    const T y = D == 3 ? dx1 * ((T)ci.z + T(0.5) * (T(1) + xi[i1])) : T(0);
    terrain<T>(m.ter, D, x, y, h, hx, hy);
  }
  const T fcol = he * (T(1) - h * invH);
  // face samples of e (1 - h/H): x faces (side, y index), then (3D) y faces (side, x index)
  for (int e = c; e < NH * 2 * NHC; e += NC) {
    const int ax = e / (2 * NHC), sd = (e / NHC) & 1, j = e % NHC;
    T x, y = 0;
    if (ax == 0) {
      int P = ci.y + sd;
      if (m.per[0] && P >= m.nlev[lev][0]) P -= m.nlev[lev][0];
      x = dx0 * (T)P;
      if (D == 3) y = dx1 * ((T)ci.z + T(0.5) * (T(1) + xi[j]));
    } else {
      int P = ci.z + sd;
      if (m.per[1] && P >= m.nlev[lev][1]) P -= m.nlev[lev][1];
      x = dx0 * ((T)ci.y + T(0.5) * (T(1) + xi[j]));
      y = dx1 * (T)P;
    }
    T hf, d1, d2;
    terrain<T>(m.ter, D, x, y, hf, d1, d2);
    if (lane) sHf[lc][ax][sd][j] = he * (T(1) - hf * invH);
  }
  // neighbour traces complete before the barrier (their loads have been in flight since the top)
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int g = 0; g <= D; ++g)
      if (DIV || g == D) pin(tn[f][g]);
  if constexpr (SPLIT) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int g = 0; g < D; ++g) pin(tn2[f][g]);
  }
  if (lane) {
    sFc[lc][c] = fcol;
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      if constexpr (DIV) {
#pragma unroll
        for (int l = 0; l < D - 1; ++l) sX[lc][l][c + NC * z] = wv[l][z];
        sX[lc][D - 1][c + NC * z] = pv[z];
        if constexpr (SPLIT) sX[lc][SPLIT ? D : 0][c + NC * z] = hv[z];
      } else {
        sX[lc][0][c + NC * z] = pv[z];
      }
    }
    // own p traces on the bottom and top faces for a run neighbour in this workgroup
    if (XZ && (rflag & 3)) {
      const T* lb0 = gtab + TL.lb();
      const T* lb1 = lb0 + NP;
      T tp0 = 0, tp1 = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) { tp0 += lb0[q] * pv[q]; tp1 += lb1[q] * pv[q]; }
      sZ[XZ ? lc : 0][0][XZ ? c : 0] = tp0;
      sZ[XZ ? lc : 0][1][XZ ? c : 0] = tp1;
    }
  }
  __syncthreads();

  // tables indexed by the thread's column (LDS) and by compile-time indices (scalar loads)
  const T* Dt = &sTab[TL.dt()];
  const T* Lbw = &sTab[TL.lbw()];
  const T* Wt = &sTab[TL.w()];
  const T* Dtu = gtab + TL.dt();
  const T* Lbu = gtab + TL.lb();
  const T* Lbwu = gtab + TL.lbw();
  const T* Wtu = gtab + TL.w();
  constexpr int NO = DIV ? 1 : D;
  T acc[NO][NP];
  T acc2[SPLIT ? NP : 1];  // split: C(qv)
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int z = 0; z < NP; ++z) acc[o][z] = 0;
  if constexpr (SPLIT) {
#pragma unroll
    for (int z = 0; z < NP; ++z) acc2[z] = 0;
  }

  // ---------------------------------------------------------------- horizontal contractions
  // Gam[0][0] = b f (3D) / f (2D) and Gam[1][1] = a f depend on the column only.
  const T g00 = D == 3 ? hb : T(1);
#pragma unroll
  for (int z = 0; z < NP; ++z) {
    T sx = 0, sx2 = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int col = q + NP * i1;
      if constexpr (SPLIT) {
        const T fq = sFc[lc][col] * sX[lc][0][col + NC * z];
        sx += Dt[i0 * NP + q] * (sX[lc][SPLIT ? D : 0][col + NC * z] * fq);
        sx2 += Dt[i0 * NP + q] * fq;
      } else {
        sx += Dt[i0 * NP + q] * (sFc[lc][col] * sX[lc][0][col + NC * z]);
      }
    }
    if constexpr (DIV) acc[0][z] += -a.adiv * g00 * sx;
    else acc[0][z] += -g00 * sx;
    if constexpr (SPLIT) acc2[z] += -a.adiv * g00 * sx2;
    if constexpr (D == 3) {
      T sy = 0, sy2 = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int col = i0 + NP * q;
        if constexpr (SPLIT) {
          const T fq = sFc[lc][col] * sX[lc][1][col + NC * z];
          sy += Dt[i1 * NP + q] * (sX[lc][SPLIT ? D : 0][col + NC * z] * fq);
          sy2 += Dt[i1 * NP + q] * fq;
        } else {
          sy += Dt[i1 * NP + q] * (sFc[lc][col] * sX[lc][DIV ? 1 : 0][col + NC * z]);
        }
      }
      if constexpr (DIV) acc[0][z] += -a.adiv * ha * sy;
      else acc[1][z] += -ha * sy;
      if constexpr (SPLIT) acc2[z] += -a.adiv * ha * sy2;
    }
    if constexpr (SPLIT) pin(acc2[z]);
#pragma unroll
    for (int o = 0; o < NO; ++o) pin(acc[o][z]);
  }
  // ---------------------------------------------------------------- vertical contraction
  // vertical row of Gam: 3D (-a b h_x om, -a b h_y om, a b), 2D (-a h_x om, a), om = 1 - zeta/H
  const T gzz = D == 3 ? ha * hb : ha;
  T gvz[NP];  // per node: the vertical flux components before the contraction
  T gvz2[SPLIT ? NP : 1];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const T zeta = dxz * ((T)iz + T(0.5) * (T(1) + xi[q]));
    const T om = T(1) - zeta * invH;
    if constexpr (DIV) {
      T gw = gzz * wv[D - 1][q] - gzz * (hx * om) * wv[0][q];
      if constexpr (D == 3) gw -= gzz * (hy * om) * wv[1][q];
      if constexpr (SPLIT) {
        gvz2[q] = -a.adiv * gw;
        gvz[q] = -a.adiv * (hv[q] * gw);
      } else {
        gvz[q] = -a.adiv * gw;
      }
    } else {
      gvz[q] = om;  // the slope terms are formed below per component
    }
  }
#pragma unroll
  for (int z = 0; z < NP; ++z) {
    if constexpr (DIV) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) s += Dtu[z * NP + q] * gvz[q];
      acc[0][z] += s;
      if constexpr (SPLIT) {
        T s2 = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) s2 += Dtu[z * NP + q] * gvz2[q];
        acc2[z] += s2;
        pin(acc2[z]);
      }
    } else {
      T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const T d = Dtu[z * NP + q] * pv[q];
        s0 += d * gvz[q];
        s2 += d;
      }
      // G[l][d-1] = -Gam[d-1][l] p
      acc[0][z] += gzz * hx * s0;
      if constexpr (D == 3) {
        s1 = s0;
        acc[1][z] += gzz * hy * s1;
      }
      acc[D - 1][z] += -gzz * s2;
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) pin(acc[o][z]);
  }

  // ---------------------------------------------------------------- vertical faces (registers)
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * (D - 1) + s;
    T tm[D + 1];
    T tm2[SPLIT ? D : 1];
#pragma unroll
    for (int g = 0; g <= D; ++g) tm[g] = 0;
    if constexpr (SPLIT) {
#pragma unroll
      for (int g = 0; g < D; ++g) tm2[g] = 0;
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const T lq = Lbu[s * NP + q];
      if constexpr (SPLIT) {
#pragma unroll
        for (int l = 0; l < D; ++l) {
          tm2[l] += lq * wv[l][q];
          tm[l] += lq * (hv[q] * wv[l][q]);
        }
      } else if constexpr (DIV) {
#pragma unroll
        for (int l = 0; l < D; ++l) tm[l] += lq * wv[l][q];
      }
      tm[D] += lq * pv[q];
    }
    const T zf = dxz * (T)(iz + s);
    const T omf = T(1) - zf * invH;
    T Nv[D];
    Nv[0] = -gzz * (hx * omf);
    if constexpr (D == 3) Nv[1] = -gzz * (hy * omf);
    Nv[D - 1] = gzz;
    const T sign = s ? T(1) : T(-1);
    const bool conf = kind[f] == kConf;
    // gradient: the run neighbour across this face in the same workgroup wrote its trace to LDS
    const bool inrun = (rflag >> s) & 1;
    const int ln = s ? lc + 1 : lc - 1;
    if constexpr (DIV) {
      T v = 0;
      if (conf) {
        T wm = 0, wn = 0, nn = 0;
#pragma unroll
        for (int l = 0; l < D; ++l) { wm += Nv[l] * tm[l]; wn += Nv[l] * tn[f][l]; nn += Nv[l] * Nv[l]; }
        const T wh = s ? T(0.5) * (wm + wn) : T(0.5) * (wn + wm);
        v = a.adiv * sign * wh;
        if (a.apen != T(0)) {
          const T lf = lam_own > lam_nb[f] ? lam_own : lam_nb[f];
          v += a.apen * (lf * sqrt(nn) * (tm[D] - tn[f][D]));
        }
        if constexpr (SPLIT) {
          T wm2 = 0, wn2 = 0;
#pragma unroll
          for (int l = 0; l < D; ++l) { wm2 += Nv[l] * tm2[l]; wn2 += Nv[l] * tn2[f][l]; }
          const T wh2 = s ? T(0.5) * (wm2 + wn2) : T(0.5) * (wn2 + wm2);
          const T v2 = a.adiv * sign * wh2;
#pragma unroll
          for (int z = 0; z < NP; ++z) acc2[z] += Lbwu[s * NP + z] * v2;
        }
      }
#pragma unroll
      for (int z = 0; z < NP; ++z) acc[0][z] += Lbwu[s * NP + z] * v;
    } else {
      T ph = kind[f] == kWall ? tm[D] : T(0);
      const T pn = inrun ? sZ[XZ ? ln : 0][1 - s][XZ ? c : 0] : tn[f][D];
      if (conf) ph = s ? T(0.5) * (tm[D] + pn) : T(0.5) * (pn + tm[D]);
#pragma unroll
      for (int l = 0; l < D; ++l) {
        const T phi = sign * ph * Nv[l];
#pragma unroll
        for (int z = 0; z < NP; ++z) acc[l][z] += Lbwu[s * NP + z] * phi;
      }
    }
  }

#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int z = 0; z < NP; ++z) pin(acc[o][z]);
  if constexpr (SPLIT) {
#pragma unroll
    for (int z = 0; z < NP; ++z) pin(acc2[z]);
  }

  // ---------------------------------------------------------------- x / y faces: flux at point c
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    // nodes of the normal line through face point c, and the terrain sample of that point
    const int jt = c % NP;  // 3D: the other horizontal index of the point; 2D: unused
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int f = 2 * k + s;
      T tmw = 0, tmp = 0, tmw2 = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int node = offs<D, NP>(k, q, c);
        const T lq = Lbu[s * NP + q];
        if constexpr (SPLIT) {
          const T qk = sX[lc][k][node];
          tmw2 += lq * qk;
          tmw += lq * (sX[lc][SPLIT ? D : 0][node] * qk);
          tmp += lq * sX[lc][D - 1][node];
        } else if constexpr (DIV) {
          tmw += lq * sX[lc][k][node];
          tmp += lq * sX[lc][D - 1][node];
        } else {
          tmp += lq * sX[lc][0][node];
        }
      }
      const T Nk = (D == 3 ? (k == 0 ? hb : ha) : T(1)) * sHf[lc][k][s][D == 3 ? jt : 0];
      const T sign = s ? T(1) : T(-1);
      const bool conf = kind[f] == kConf;
      T phi;
      if constexpr (DIV) {
        phi = 0;
        if (conf) {
          const T wm = Nk * tmw, wn = Nk * tn[f][k];
          const T wh = s ? T(0.5) * (wm + wn) : T(0.5) * (wn + wm);
          phi = a.adiv * sign * wh;
          if (a.apen != T(0)) {
            const T lf = lam_own > lam_nb[f] ? lam_own : lam_nb[f];
            phi += a.apen * (lf * sqrt(Nk * Nk) * (tmp - tn[f][D]));
          }
        }
        if constexpr (SPLIT) {
          T phi2 = 0;
          if (conf) {
            const T wm2 = Nk * tmw2, wn2 = Nk * tn2[f][k];
            const T wh2 = s ? T(0.5) * (wm2 + wn2) : T(0.5) * (wn2 + wm2);
            phi2 = a.adiv * sign * wh2;
          }
          if (lane) sPhi2[lc][f][c] = phi2;
        }
      } else {
        T ph = kind[f] == kWall ? tmp : T(0);
        if (conf) ph = s ? T(0.5) * (tmp + tn[f][D]) : T(0.5) * (tn[f][D] + tmp);
        phi = sign * ph * Nk;
      }
      if (lane) sPhi[lc][f][c] = phi;
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- lift of the x / y faces
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int ik = k == 0 ? i0 : i1;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T lw = Lbw[s * NP + ik];
#pragma unroll
      for (int z = 0; z < NP; ++z) {
        // face point of node (i0, i1, z) on an x face: (i1, z); on a y face: (i0, z)
        const int ap = D == 3 ? (k == 0 ? i1 : i0) + NP * z : z;
        acc[DIV ? 0 : k][z] += lw * sPhi[lc][2 * k + s][ap];
        if constexpr (SPLIT) acc2[z] += lw * sPhi2[lc][2 * k + s][ap];
      }
    }
  }

  // ---------------------------------------------------------------- finalize
  if (!active) return;
  const T J = (D == 3 ? ha * hb : ha) * fcol;
  if constexpr (DIV) {
    const T wc = D == 3 ? Wt[i0] * Wt[i1] : Wt[i0];
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      const unsigned idx = base + NC * z;
      if constexpr (SPLIT) {
        // + hbar C(qv) + adiv M (d hbar/dz) qv_z
        const T hbz = a.hb[idx], dhz = a.dhb[idx];
        if (a.weak) {
          a.out[idx] = (wc * Wtu[z]) * (acc[0][z] + hbz * acc2[z] + a.adiv * J * dhz * wv[D - 1][z] + a.amass * J * pv[z]);
        } else {
          a.out[idx] = (acc[0][z] + hbz * acc2[z]) / J + a.adiv * dhz * wv[D - 1][z];
        }
      } else {
        if (a.weak) a.out[idx] = (wc * Wtu[z]) * (acc[0][z] + a.amass * J * pv[z]);
        else a.out[idx] = acc[0][z] / J;
      }
    }
  } else {
    const T iJ0 = T(1) / J;
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      const unsigned idx = base + NC * z;
      T iJ = iJ0;
      if (a.h) iJ *= a.h[idx];
#pragma unroll
      for (int l = 0; l < D; ++l) a.q[l * N + idx] = acc[l][z] * iJ;
    }
  }
}

template <int D, int NP, class T, bool DIV, class A, bool HH = false, bool SPLIT = false>
int run_col(const A& a, const MeshDev& m, hipStream_t s) {
  using C = Col<D, NP>;
  if (m.ncell <= 0) return 0;
  int grid = (m.ncell + C::CPB - 1) / C::CPB;
  if (!DIV) {  // the gradient walks the vertical runs
    if (m.nrwg * C::CPB < m.ncell) return -3;  // the run lists were built for this layout
    grid = m.nrwg;
  }
  hipLaunchKernelGGL((k_col<D, NP, T, DIV, A, HH, SPLIT>), dim3(grid), dim3(C::NT), 0, s, Direct<A>{a, m});
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Explicit advective residual (the explicit part of the IMEX split, Section 3.2) in the column
// layout, for the cells whose faces are conforming or walls: volume fluxes (rho u, rho u (x) u,
// rho k u) with k = |u|^2 / 2, Rusanov fluxes with the advective speed, the slip-wall flux, and
// the gravity work -rho g w.  Fields and 1/rho go through LDS for the x / y passes; the same
// buffer then carries the x / y face fluxes.
template <int D, int NP, class S = Direct<ExpArgs>>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_col_exp(const S src) {
  const int sg = src.seg();
  const MeshDev& m = src.mesh(sg);
  const double* __restrict__ U = src.args(sg).U;
  double* __restrict__ R = src.args(sg).R;
  using C = Col<D, NP>;
  using T = double;
  constexpr int NC = C::NC, NL = C::NL, NF = C::NF, CPB = C::CPB, NHC = C::NHC;
  constexpr TabLayout TL{NP};
  constexpr int NH = D - 1;
  constexpr int NV = D + 2;  // rho, m_0 .. m_{d-1}, rho E
  constexpr int NXF = NV + 1;
  // one buffer per cell: first the fields and 1/rho, then the x / y face fluxes
  constexpr int NBUF = NXF * NL > 2 * NH * NV * NC ? NXF * NL : 2 * NH * NV * NC;

  __shared__ T sTab[TL.size()];
  __shared__ T sBuf[CPB][NBUF];
  __shared__ T sFc[CPB][NC];
  __shared__ T sHf[CPB][NH][2][NHC];
  T(*sX)[NXF][NL] = reinterpret_cast<T(*)[NXF][NL]>(&sBuf[0][0]);
  T(*sPhi)[2 * NH][NV][NC] = reinterpret_cast<T(*)[2 * NH][NV][NC]>(&sBuf[0][0]);

  const int tid = threadIdx.x;
  const bool lane = tid < C::NTA;
  const int lc = lane ? tid / NC : CPB - 1;
  const int c = tid % NC;
  const int pos = xcd_block(src.blk(sg), src.nblk(sg)) * CPB + lc;
  const int cell = lane && pos < m.ncell ? pos : 0;
  const unsigned N = (unsigned)m.N;
  const int i0 = c % NP;
  const int i1 = D == 3 ? c / NP : 0;
  const T* gtab = m.tab;
  for (int t = tid; t < TL.size(); t += C::NT) sTab[t] = gtab[t];

  // ---------------------------------------------------------------- loads
  const int4 ci = m.cell[cell];
  // 2:1 faces contribute nothing here: the general kernel adds their terms afterwards
  int kind[NF], nb[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    kind[f] = m.fkind[cell * NF + f];
    nb[f] = m.fnbr[cell * NF + f].x;
  }
  const bool active = lane && pos < m.ncell;
  const unsigned base = (unsigned)cell * NL + c;
  T u[NV][NP];
#pragma unroll
  for (int z = 0; z < NP; ++z)
#pragma unroll
    for (int g = 0; g < NV; ++g) u[g][z] = U[g * N + base + NC * z];
  T tn[NF][NV];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int k = f >> 1, s = f & 1;
#pragma unroll
    for (int g = 0; g < NV; ++g) tn[f][g] = 0;
    if (kind[f] != kConf) continue;
    const unsigned nbase = (unsigned)nb[f] * NL;
    if (k == 0) {
      // x faces: the normal line is contiguous in memory
      const unsigned idx = nbase + offs<D, NP>(0, 0, c);
#pragma unroll
      for (int g = 0; g < NV; ++g) {
        T l[NP];
        load_line<NP>(U + g * N + idx, l);
#pragma unroll
        for (int q = 0; q < NP; ++q) tn[f][g] += gtab[TL.lb() + (1 - s) * NP + q] * l[q];
      }
      continue;
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const T lq = gtab[TL.lb() + (1 - s) * NP + q];
      const unsigned idx = nbase + offs<D, NP>(k, q, c);
#pragma unroll
      for (int g = 0; g < NV; ++g) tn[f][g] += lq * U[g * N + idx];
    }
  }

  // ---------------------------------------------------------------- geometry
  const int lev = ci.x;
  const int iz = D == 3 ? ci.w : ci.z;
  const T dx0 = m.dxl[lev][0], dx1 = m.dxl[lev][1], dxz = m.dxl[lev][D - 1];
  const T invH = m.invH;
  const T ha = 0.5 * dx0, hb = 0.5 * dx1, he = 0.5 * dxz;
  const T* xi = gtab + TL.xi();
  T h, hx, hy;
  {
    const T x = dx0 * ((T)ci.y + 0.5 * (1.0 + xi[i0]));
    const T y = D == 3 ? dx1 * ((T)ci.z + 0.5 * (1.0 + xi[i1])) : 0.0;
    terrain<T>(m.ter, D, x, y, h, hx, hy);
  }
  const T fcol = he * (1.0 - h * invH);
  for (int e = c; e < NH * 2 * NHC; e += NC) {
    const int ax = e / (2 * NHC), sd = (e / NHC) & 1, j = e % NHC;
    T x, y = 0;
    if (ax == 0) {
      int P = ci.y + sd;
      if (m.per[0] && P >= m.nlev[lev][0]) P -= m.nlev[lev][0];
      x = dx0 * (T)P;
      if (D == 3) y = dx1 * ((T)ci.z + 0.5 * (1.0 + xi[j]));
    } else {
      int P = ci.z + sd;
      if (m.per[1] && P >= m.nlev[lev][1]) P -= m.nlev[lev][1];
      x = dx0 * ((T)ci.y + 0.5 * (1.0 + xi[j]));
      y = dx1 * (T)P;
    }
    T hf, d1, d2;
    terrain<T>(m.ter, D, x, y, hf, d1, d2);
    if (lane) sHf[lc][ax][sd][j] = he * (1.0 - hf * invH);
  }
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int g = 0; g < NV; ++g) pin(tn[f][g]);
  T ir[NP];
#pragma unroll
  for (int z = 0; z < NP; ++z) ir[z] = 1.0 / u[0][z];
  if (lane) {
    sFc[lc][c] = fcol;
#pragma unroll
    for (int z = 0; z < NP; ++z) {
#pragma unroll
      for (int g = 0; g < NV; ++g) sX[lc][g][c + NC * z] = u[g][z];
      sX[lc][NV][c + NC * z] = ir[z];
    }
  }

  const T* Dt = &sTab[TL.dt()];
  const T* Lbw = &sTab[TL.lbw()];
  const T* Dtu = gtab + TL.dt();
  const T* Lbu = gtab + TL.lb();
  const T* Lbwu = gtab + TL.lbw();
  T acc[NV][NP];
#pragma unroll
  for (int o = 0; o < NV; ++o)
#pragma unroll
    for (int z = 0; z < NP; ++z) acc[o][z] = 0;

  // the column's own work first (registers only), so that only the accumulators, the x / y
  // neighbour traces and the vertical momentum stay live across the barrier
  // ---------------------------------------------------------------- vertical contraction
  const T gzz = D == 3 ? ha * hb : ha;
  {
    T gm[NP];  // Gam[d-1] . m at each node of the column
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const T zeta = dxz * ((T)iz + 0.5 * (1.0 + xi[q]));
      const T om = 1.0 - zeta * invH;
      T t = gzz * u[D][q] - gzz * (hx * om) * u[1][q];
      if constexpr (D == 3) t -= gzz * (hy * om) * u[2][q];
      gm[q] = t;
    }
#pragma unroll
    for (int z = 0; z < NP; ++z) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const T d = Dtu[z * NP + q] * gm[q];
        const T dr = d * ir[q];
        T m2 = 0;
#pragma unroll
        for (int l = 0; l < D; ++l) m2 += u[1 + l][q] * u[1 + l][q];
        acc[0][z] += d;
#pragma unroll
        for (int l = 0; l < D; ++l) acc[1 + l][z] += dr * u[1 + l][q];
        acc[NV - 1][z] += dr * (0.5 * m2 * ir[q]);
      }
#pragma unroll
      for (int o = 0; o < NV; ++o) pin(acc[o][z]);
    }
  }
  // ---------------------------------------------------------------- vertical faces (registers)
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * (D - 1) + s;
    T tm[NV];
#pragma unroll
    for (int g = 0; g < NV; ++g) {
      T t = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) t += Lbu[s * NP + q] * u[g][q];
      tm[g] = t;
    }
    const T zf = dxz * (T)(iz + s);
    const T omf = 1.0 - zf * invH;
    T Nv[D];
    Nv[0] = -gzz * (hx * omf);
    if constexpr (D == 3) Nv[1] = -gzz * (hy * omf);
    Nv[D - 1] = gzz;
    const T sign = s ? 1.0 : -1.0;
    T F[NV], phi[NV];
    if (kind[f] == kConf) {
      if (s) rusanov<D>(tm, tn[f], Nv, F);
      else rusanov<D>(tn[f], tm, Nv, F);
#pragma unroll
      for (int o = 0; o < NV; ++o) phi[o] = -sign * F[o];
    } else if (kind[f] != kWall) {
#pragma unroll
      for (int o = 0; o < NV; ++o) phi[o] = 0;
    } else {
      T No[D];
#pragma unroll
      for (int l = 0; l < D; ++l) No[l] = sign * Nv[l];
      wall_flux<D>(tm, No, F);
#pragma unroll
      for (int o = 0; o < NV; ++o) phi[o] = -F[o];
    }
#pragma unroll
    for (int o = 0; o < NV; ++o)
#pragma unroll
      for (int z = 0; z < NP; ++z) acc[o][z] += Lbwu[s * NP + z] * phi[o];
  }
#pragma unroll
  for (int o = 0; o < NV; ++o)
#pragma unroll
    for (int z = 0; z < NP; ++z) pin(acc[o][z]);

  __syncthreads();

  // ---------------------------------------------------------------- horizontal contractions
  // along axis k < d-1 the flux through faces of constant xi_k is Gam[k][k] m_k (1, u, k)
  const T g00 = D == 3 ? hb : 1.0;
#pragma unroll
  for (int z = 0; z < NP; ++z) {
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int ik = k == 0 ? i0 : i1;
      const T gk = k == 0 ? g00 : ha;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int col = k == 0 ? q + NP * i1 : i0 + NP * q;
        const int node = col + NC * z;
        T mm[D];
#pragma unroll
        for (int l = 0; l < D; ++l) mm[l] = sX[lc][1 + l][node];
        const T r1 = sX[lc][NV][node];
        const T fl = Dt[ik * NP + q] * (gk * sFc[lc][col] * mm[k]);  // D~ Gam m_k
        const T flr = fl * r1;
        T m2 = 0;
#pragma unroll
        for (int l = 0; l < D; ++l) m2 += mm[l] * mm[l];
        acc[0][z] += fl;
#pragma unroll
        for (int l = 0; l < D; ++l) acc[1 + l][z] += flr * mm[l];
        acc[NV - 1][z] += flr * (0.5 * m2 * r1);
      }
#pragma unroll
      for (int o = 0; o < NV; ++o) pin(acc[o][z]);
    }
  }
  // ---------------------------------------------------------------- x / y faces: flux at point c
  T phx[NH][2][NV];
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int jt = c % NP;
    T line[NV][NP];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int g = 0; g < NV; ++g) line[g][q] = sX[lc][g][offs<D, NP>(k, q, c)];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int f = 2 * k + s;
      T tm[NV];
#pragma unroll
      for (int g = 0; g < NV; ++g) {
        T t = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) t += Lbu[s * NP + q] * line[g][q];
        tm[g] = t;
      }
      const T Nk = (D == 3 ? (k == 0 ? hb : ha) : 1.0) * sHf[lc][k][s][D == 3 ? jt : 0];
      T Nv[D];
#pragma unroll
      for (int l = 0; l < D; ++l) Nv[l] = l == k ? Nk : 0.0;
      const T sign = s ? 1.0 : -1.0;
      T F[NV];
      if (kind[f] == kConf) {
        if (s) rusanov<D>(tm, tn[f], Nv, F);
        else rusanov<D>(tn[f], tm, Nv, F);
#pragma unroll
        for (int o = 0; o < NV; ++o) phx[k][s][o] = -sign * F[o];
      } else if (kind[f] != kWall) {
#pragma unroll
        for (int o = 0; o < NV; ++o) phx[k][s][o] = 0;
      } else {
        T No[D];
#pragma unroll
        for (int l = 0; l < D; ++l) No[l] = sign * Nv[l];
        wall_flux<D>(tm, No, F);
#pragma unroll
        for (int o = 0; o < NV; ++o) phx[k][s][o] = -F[o];
      }
    }
  }
  __syncthreads();  // every read of the field buffer is done: it now takes the fluxes
  if (lane) {
#pragma unroll
    for (int k = 0; k < NH; ++k)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int o = 0; o < NV; ++o) sPhi[lc][2 * k + s][o][c] = phx[k][s][o];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int ik = k == 0 ? i0 : i1;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T lw = Lbw[s * NP + ik];
#pragma unroll
      for (int z = 0; z < NP; ++z) {
        const int ap = D == 3 ? (k == 0 ? i1 : i0) + NP * z : z;
#pragma unroll
        for (int o = 0; o < NV; ++o) acc[o][z] += lw * sPhi[lc][2 * k + s][o][ap];
      }
    }
  }

  // ---------------------------------------------------------------- finalize
  if (!active) return;
  const T iJ = 1.0 / ((D == 3 ? ha * hb : ha) * fcol);
#pragma unroll
  for (int z = 0; z < NP; ++z) {
    const unsigned idx = base + NC * z;
#pragma unroll
    for (int o = 0; o < NV - 1; ++o) R[o * N + idx] = acc[o][z] * iJ;
    R[(NV - 1) * N + idx] = acc[NV - 1][z] * iJ - kG * u[D][z];
  }
}

template <int D, int NP>
int run_col_exp(const double* U, double* R, const MeshDev& m, hipStream_t s) {
  using C = Col<D, NP>;
  if (m.ncell <= 0) return 0;
  const int grid = (m.ncell + C::CPB - 1) / C::CPB;
  hipLaunchKernelGGL((k_col_exp<D, NP>), dim3(grid), dim3(C::NT), 0, s, Direct<ExpArgs>{ExpArgs{U, R}, m});
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Cell-wise fast-diagonalisation preconditioner in the column layout:
// z = (1/Jbar) (S x S x S) diag(1 / (1/(gamma-1) + sum_k alpha_k mu_{i_k})) (S x S x S)^T (scale v).
// The vertical transforms stay in the thread's registers, the horizontal ones go through LDS.
template <int D, int NP, class T, class Src = Direct<FdmArgs<T>>>
__global__ void __launch_bounds__(256) k_fdm_col(const Src src) {
  const int sg = src.seg();
  const FdmArgs<T>& a = src.args(sg);
  const MeshDev& m = src.mesh(sg);
  using C = Col<D, NP>;
  constexpr int NC = C::NC, NL = C::NL, CPB = C::CPB;
  constexpr TabLayout TL{NP};
  __shared__ T sA[CPB][NL];
  __shared__ T sB[CPB][NL];
  __shared__ T sS[NP * NP];
  __shared__ T sMu[NP];
  const int tid = threadIdx.x;
  const bool lane = tid < C::NTA;
  const int lc = lane ? tid / NC : CPB - 1;
  const int c = tid % NC;
  const int cell0 = xcd_block(src.blk(sg), src.nblk(sg)) * CPB;
  const int cell = cell0 + lc;
  const bool active = lane && cell < m.ncell;
  const int cl = active ? cell : 0;
  const int i0 = c % NP;
  const int i1 = D == 3 ? c / NP : 0;
  const T* gtab;
  if constexpr (sizeof(T) == 8) gtab = (const T*)m.tab;
  else gtab = (const T*)m.tabf;
  for (int t = tid; t < NP * NP; t += C::NT) sS[t] = gtab[TL.fds() + t];
  if (tid < NP) sMu[tid] = gtab[TL.fdmu() + tid];
  const T* S = gtab + TL.fds();  // S[i][a]; compile-time indices below become scalar loads
  const unsigned base = (unsigned)cl * NL + c;
  T v[NP], w[NP];
#pragma unroll
  for (int z = 0; z < NP; ++z) v[z] = a.v[base + NC * z];
  const T sc = a.dscale ? (T)*a.dscale : a.scale;
#pragma unroll
  for (int z = 0; z < NP; ++z) v[z] *= sc;
  const T cf0 = a.coef[cl * 4 + 0], cfx = a.coef[cl * 4 + 1], cfy = a.coef[cl * 4 + 2];
  const T cfz = a.coef[cl * 4 + D];
  // vertical forward: w_j = sum_q S[q][j] v_q
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    T t = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) t += S[q * NP + j] * v[q];
    w[j] = t;
  }
  if (lane) {
#pragma unroll
    for (int z = 0; z < NP; ++z) sA[lc][c + NC * z] = w[z];
  }
  __syncthreads();
  // x forward
#pragma unroll
  for (int z = 0; z < NP; ++z) {
    T t = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) t += sS[q * NP + i0] * sA[lc][q + NP * i1 + NC * z];
    w[z] = t;
  }
  if constexpr (D == 3) {
    if (lane) {
#pragma unroll
      for (int z = 0; z < NP; ++z) sB[lc][c + NC * z] = w[z];
    }
    __syncthreads();
    // y forward
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      T t = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) t += sS[q * NP + i1] * sB[lc][i0 + NP * q + NC * z];
      w[z] = t;
    }
  }
  // divide by the separable eigenvalues
  T lh = T(1) / T(kGamma - 1.0) + cfx * sMu[i0];
  if constexpr (D == 3) lh += cfy * sMu[i1];
#pragma unroll
  for (int z = 0; z < NP; ++z) w[z] /= lh + cfz * sMu[z];
  if constexpr (D == 3) {
    // y backward (sA is free: its last readers passed the barrier before the y forward pass)
    if (lane) {
#pragma unroll
      for (int z = 0; z < NP; ++z) sA[lc][c + NC * z] = w[z];
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      T t = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) t += sS[i1 * NP + q] * sA[lc][i0 + NP * q + NC * z];
      w[z] = t;
    }
    // x backward through sB (its readers, the y forward pass, passed the barrier above)
    if (lane) {
#pragma unroll
      for (int z = 0; z < NP; ++z) sB[lc][c + NC * z] = w[z];
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      T t = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) t += sS[i0 * NP + q] * sB[lc][q + NP * i1 + NC * z];
      v[z] = t;
    }
  } else {
    // x backward through sB
    if (lane) {
#pragma unroll
      for (int z = 0; z < NP; ++z) sB[lc][c + NC * z] = w[z];
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      T t = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) t += sS[i0 * NP + q] * sB[lc][q + NC * z];
      v[z] = t;
    }
  }
  if (!active) return;
  // vertical backward: out_j = sum_q S[j][q] v_q, times 1/Jbar
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    T t = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) t += S[j * NP + q] * v[q];
    a.z[base + NC * j] = t * cf0;
  }
}

template <int D, int NP, class T>
int run_fdm_col(const FdmArgs<T>& a, const MeshDev& m, hipStream_t s) {
  using C = Col<D, NP>;
  if (m.ncell <= 0) return 0;
  const int grid = (m.ncell + C::CPB - 1) / C::CPB;
  hipLaunchKernelGGL((k_fdm_col<D, NP, T>), dim3(grid), dim3(C::NT), 0, s, Direct<FdmArgs<T>>{a, m});
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

#define DG_COL_DISPATCH(EXPR)                 \
  switch (degree) {                           \
    case 1: { constexpr int NP = 2; EXPR; }   \
    case 2: { constexpr int NP = 3; EXPR; }   \
    case 3: { constexpr int NP = 4; EXPR; }   \
    case 4: { constexpr int NP = 5; EXPR; }   \
    case 5: { constexpr int NP = 6; EXPR; }   \
    default: return -6;                       \
  }

template <class T>
int grad_col(const MeshDev& m, int degree, const GradArgs<T>& a, hipStream_t s) {
  if (m.dim == 2) {
    DG_COL_DISPATCH(return (run_col<2, NP, T, false>(a, m, s)));
  } else {
    DG_COL_DISPATCH(return (run_col<3, NP, T, false>(a, m, s)));
  }
}
template <class T, bool HH = false, bool SPLIT = false>
int div_col(const MeshDev& m, int degree, const DivArgs<T>& a, hipStream_t s) {
  if (m.dim == 2) {
    DG_COL_DISPATCH(return (run_col<2, NP, T, true, DivArgs<T>, HH, SPLIT>(a, m, s)));
  } else {
    DG_COL_DISPATCH(return (run_col<3, NP, T, true, DivArgs<T>, HH, SPLIT>(a, m, s)));
  }
}

template <class T>
int fdm_col(const MeshDev& m, int degree, const FdmArgs<T>& a, hipStream_t s) {
  if (m.dim == 2) {
    DG_COL_DISPATCH(return (run_fdm_col<2, NP, T>(a, m, s)));
  } else {
    DG_COL_DISPATCH(return (run_fdm_col<3, NP, T>(a, m, s)));
  }
}

int exp_col(const MeshDev& m, int degree, const double* U, double* R, hipStream_t s) {
  if (m.dim == 2) {
    DG_COL_DISPATCH(return (run_col_exp<2, NP>(U, R, m, s)));
  } else {
    DG_COL_DISPATCH(return (run_col_exp<3, NP>(U, R, m, s)));
  }
}

}  // namespace

int launch_explicit(const MeshDev& m, int degree, const double* U, double* R, hipStream_t s) {
  int r = exp_col(m, degree, U, R, s);
  if (r == 0) r = launch_explicit_hang(m, degree, U, R, s);
  return r;
}

int launch_fdm64(const MeshDev& m, int degree, const FdmArgs<double>& a, hipStream_t s) {
  return fdm_col<double>(m, degree, a, s);
}
int launch_fdm32(const MeshDev& m, int degree, const FdmArgs<float>& a, hipStream_t s) {
  return fdm_col<float>(m, degree, a, s);
}

// p given (no Jacobi scaling, no copy of p requested) and, for the divergence, h folded into the
// vector field: the column kernel on every cell, then the 2:1 face terms; otherwise the general
// cell kernel on every cell.
int launch_grad64(const MeshDev& m, int degree, const GradArgs<double>& a, hipStream_t s) {
  if (a.dinv || a.z) return launch_grad_cells64(m, degree, a, nullptr, m.ncell, s);
  int r = grad_col<double>(m, degree, a, s);
  if (r == 0) r = launch_grad_hang64(m, degree, a, s);
  return r;
}
int launch_div64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s) {
  if (a.dinv || (!a.h && !a.p)) return launch_div_cells64(m, degree, a, nullptr, m.ncell, s);
  int r = a.h ? div_col<double, true>(m, degree, a, s) : div_col<double>(m, degree, a, s);
  if (r == 0) r = launch_div_hang64(m, degree, a, s);
  return r;
}
// The enthalpy-split energy flux in one column pass (a.h = h - hbar, a.hb, a.dhb set), then the
// 2:1 face terms of C((h - hbar) qv) with the penalty and of C(qv) multiplied by hbar at the
// node, both in one faces-only pass.
template <class T>
int div_split(const MeshDev& m, int degree, const DivArgs<T>& a, hipStream_t s,
              int (*hang)(const MeshDev&, int, const DivArgs<T>&, hipStream_t)) {
  if (a.dinv || !a.h || !a.hb || !a.dhb) return -3;
  int r = div_col<T, true, true>(m, degree, a, s);
  if (r) return r;
  return hang(m, degree, a, s);
}
int launch_div_split64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s) {
  return div_split<double>(m, degree, a, s, launch_div_split_hang64);
}
int launch_div_split32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s) {
  return div_split<float>(m, degree, a, s, launch_div_split_hang32);
}

// ---------------------------------------------------------------- shared launches
namespace {

template <int D, int NP, class T, bool DIV, class A, bool HH = false, bool SPLIT = false>
int run_col_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const A* a, hipStream_t s) {
  using C = Col<D, NP>;
  for (int k = 0; k < n; ++k)
    if (!DIV && mh[k]->ncell > 0 && mh[k]->nrwg * C::CPB < mh[k]->ncell) return -3;
  return seg_launch<A>(
      n, md,
      [&](int k) { return mh[k]->ncell <= 0 ? 0 : DIV ? (mh[k]->ncell + C::CPB - 1) / C::CPB : mh[k]->nrwg; },
      [&](int k) { return a[k]; },
      [&](const SegTab<A>& t, int g) {
        hipLaunchKernelGGL((k_col<D, NP, T, DIV, A, HH, SPLIT, Shared<A>>), dim3(g), dim3(C::NT), 0, s, Shared<A>{t});
        return hipGetLastError() == hipSuccess ? 0 : -3;
      });
}

template <int D, int NP, class T>
int run_fdm_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const FdmArgs<T>* a, hipStream_t s) {
  using C = Col<D, NP>;
  using A = FdmArgs<T>;
  return seg_launch<A>(
      n, md, [&](int k) { return (mh[k]->ncell + C::CPB - 1) / C::CPB; }, [&](int k) { return a[k]; },
      [&](const SegTab<A>& t, int g) {
        hipLaunchKernelGGL((k_fdm_col<D, NP, T, Shared<A>>), dim3(g), dim3(C::NT), 0, s, Shared<A>{t});
        return hipGetLastError() == hipSuccess ? 0 : -3;
      });
}

template <int D, int NP>
int run_exp_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const ExpArgs* a, hipStream_t s) {
  using C = Col<D, NP>;
  return seg_launch<ExpArgs>(
      n, md, [&](int k) { return (mh[k]->ncell + C::CPB - 1) / C::CPB; }, [&](int k) { return a[k]; },
      [&](const SegTab<ExpArgs>& t, int g) {
        hipLaunchKernelGGL((k_col_exp<D, NP, Shared<ExpArgs>>), dim3(g), dim3(C::NT), 0, s, Shared<ExpArgs>{t});
        return hipGetLastError() == hipSuccess ? 0 : -3;
      });
}

template <class T>
int grad_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<T>* a, int degree,
             hipStream_t s, int (*hang)(int, const MeshDev* const*, const MeshDev* const*, const GradArgs<T>*, int, hipStream_t)) {
  if (n <= 0) return 0;
  for (int k = 0; k < n; ++k)
    if (a[k].dinv || a[k].z || mh[k]->dim != mh[0]->dim) return -6;
  int r;
  if (mh[0]->dim == 2) {
    DG_COL_DISPATCH(r = (run_col_seg<2, NP, T, false>(n, mh, md, a, s)); break);
  } else {
    DG_COL_DISPATCH(r = (run_col_seg<3, NP, T, false>(n, mh, md, a, s)); break);
  }
  return r ? r : hang(n, mh, md, a, degree, s);
}

template <class T, bool HH, bool SPLIT>
int div_col_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<T>* a, int degree,
                hipStream_t s) {
  if (mh[0]->dim == 2) {
    DG_COL_DISPATCH(return (run_col_seg<2, NP, T, true, DivArgs<T>, HH, SPLIT>(n, mh, md, a, s)));
  } else {
    DG_COL_DISPATCH(return (run_col_seg<3, NP, T, true, DivArgs<T>, HH, SPLIT>(n, mh, md, a, s)));
  }
}

template <class T>
int div_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<T>* a, int degree,
            hipStream_t s, int (*hang)(int, const MeshDev* const*, const MeshDev* const*, const DivArgs<T>*, int, hipStream_t)) {
  if (n <= 0) return 0;
  const bool hh = a[0].h != nullptr;
  for (int k = 0; k < n; ++k)
    if (a[k].dinv || (!a[k].h && !a[k].p) || (a[k].h != nullptr) != hh || mh[k]->dim != mh[0]->dim) return -6;
  const int r = hh ? div_col_seg<T, true, false>(n, mh, md, a, degree, s)
                   : div_col_seg<T, false, false>(n, mh, md, a, degree, s);
  return r ? r : hang(n, mh, md, a, degree, s);
}

// the enthalpy-split form (see div_split) for every member
template <class T>
int div_split_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<T>* a, int degree,
                  hipStream_t s, int (*hang)(int, const MeshDev* const*, const MeshDev* const*, const DivArgs<T>*, int, hipStream_t)) {
  if (n <= 0) return 0;
  for (int k = 0; k < n; ++k)
    if (a[k].dinv || !a[k].h || !a[k].hb || !a[k].dhb || mh[k]->dim != mh[0]->dim) return -6;
  const int r = div_col_seg<T, true, true>(n, mh, md, a, degree, s);
  return r ? r : hang(n, mh, md, a, degree, s);
}

template <class T>
int fdm_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const FdmArgs<T>* a, int degree, hipStream_t s) {
  if (n <= 0) return 0;
  for (int k = 0; k < n; ++k)
    if (mh[k]->dim != mh[0]->dim) return -6;
  if (mh[0]->dim == 2) {
    DG_COL_DISPATCH(return (run_fdm_seg<2, NP, T>(n, mh, md, a, s)));
  } else {
    DG_COL_DISPATCH(return (run_fdm_seg<3, NP, T>(n, mh, md, a, s)));
  }
}

}  // namespace

int launch_grad_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<double>* a, int degree, hipStream_t s) {
  return grad_seg<double>(n, mh, md, a, degree, s, launch_grad_hang_seg64);
}
int launch_grad_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<float>* a, int degree, hipStream_t s) {
  return grad_seg<float>(n, mh, md, a, degree, s, launch_grad_hang_seg32);
}
int launch_div_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<double>* a, int degree, hipStream_t s) {
  return div_seg<double>(n, mh, md, a, degree, s, launch_div_hang_seg64);
}
int launch_div_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<float>* a, int degree, hipStream_t s) {
  return div_seg<float>(n, mh, md, a, degree, s, launch_div_hang_seg32);
}
int launch_div_split_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<double>* a, int degree, hipStream_t s) {
  return div_split_seg<double>(n, mh, md, a, degree, s, launch_div_split_hang_seg64);
}
int launch_div_split_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<float>* a, int degree, hipStream_t s) {
  return div_split_seg<float>(n, mh, md, a, degree, s, launch_div_split_hang_seg32);
}
int launch_fdm_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const FdmArgs<double>* a, int degree, hipStream_t s) {
  return fdm_seg<double>(n, mh, md, a, degree, s);
}
int launch_fdm_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const FdmArgs<float>* a, int degree, hipStream_t s) {
  return fdm_seg<float>(n, mh, md, a, degree, s);
}
int launch_explicit_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const ExpArgs* a, int degree, hipStream_t s) {
  if (n <= 0) return 0;
  for (int k = 0; k < n; ++k)
    if (mh[k]->dim != mh[0]->dim || mh[k]->nq > 0) return -6;
  int r;
  if (mh[0]->dim == 2) {
    DG_COL_DISPATCH(r = (run_exp_seg<2, NP>(n, mh, md, a, s)); break);
  } else {
    DG_COL_DISPATCH(r = (run_exp_seg<3, NP>(n, mh, md, a, s)); break);
  }
  return r ? r : launch_explicit_hang_seg(n, mh, md, a, degree, s);
}

int launch_grad32(const MeshDev& m, int degree, const GradArgs<float>& a, hipStream_t s) {
  if (a.dinv || a.z) return launch_grad_cells32(m, degree, a, nullptr, m.ncell, s);
  int r = grad_col<float>(m, degree, a, s);
  if (r == 0) r = launch_grad_hang32(m, degree, a, s);
  return r;
}
int launch_div32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s) {
  if (a.dinv || !a.p) return launch_div_cells32(m, degree, a, nullptr, m.ncell, s);
  int r = a.h ? div_col<float, true>(m, degree, a, s) : div_col<float>(m, degree, a, s);
  if (r == 0) r = launch_div_hang32(m, degree, a, s);
  return r;
}

}  // namespace dg
