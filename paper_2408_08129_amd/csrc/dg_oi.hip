// Over-integrated explicit residual for gfx950: the explicit advective part of the IMEX split
// (arXiv 2408.08129, Section 3.2) with its volume and face flux integrals taken at NQ > NP Gauss
// points per direction, the de-aliasing form of the nonlinear flux.  The mass matrix stays the
// nodal (diagonal) one and the gravity work stays pointwise, as in the nodal kernels.
//
// One workgroup per cell.  Volume: the state is interpolated from the NP^d nodes to the NQ^d
// points by three 1D passes (LDS); at each point the weighted conserved fluxes' common factors
// (w rho, w m, w rho k) and the D contravariant velocities are stored, and for each direction k
// the weak-form contraction back onto the nodes is three 1D passes (derivative matrix along k,
// interpolation along the others) whose first pass forms the flux component on the fly.
// Faces, one axis (two opposite faces) at a time: traces on the NP^(d-1) face nodes (own from
// LDS; neighbours gathered along their normal lines), interpolated to the NQ^(d-1) face points
// (on a 2:1 face: the fine sub-face's points, the coarse polynomial evaluated there with the
// half-interval matrices), Rusanov / slip-wall flux times the face weight, contracted back onto
// the face nodes and lifted along the normal lines into the accumulator.  Working on one flux
// direction and one face axis at a time keeps the workgroup's LDS small enough for several
// workgroups per compute unit.
#include "dg_device.hpp"

namespace dg {
namespace {
using namespace dev;

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int D, int NP, int NQ>
struct Oi {
  static constexpr int NV = D + 2;
  static constexpr int NL = ipow(NP, D);
  static constexpr int NVQ = ipow(NQ, D);
  static constexpr int NPF = ipow(NP, D - 1);
  static constexpr int NFQ = ipow(NQ, D - 1);
  static constexpr int NF = 2 * D;
  static constexpr int MS = 1 << (D - 1);
  static constexpr int NT = 256;
  // interpolation passes (per field): x pass NQ NP^(d-1), (3D) y pass NQ^2 NP, then NQ^d
  static constexpr int IA = NQ * ipow(NP, D - 1);
  static constexpr int IB = D == 3 ? NQ * NQ * NP : 0;
  // contraction passes (per field, one flux direction): x pass NP NQ^(d-1), (3D) y pass NP^2 NQ
  static constexpr int CA = NP * ipow(NQ, D - 1);
  static constexpr int CB = D == 3 ? NP * NP * NQ : 0;
  // face arrays of one axis (two faces): own node traces, neighbour node traces (per sub-face),
  // point values, node sums
  static constexpr int FO = 2 * NV * NPF;
  static constexpr int FN = 2 * MS * NV * NPF;
  static constexpr int FL = 2 * MS * NV * NFQ;
  static constexpr int FG = 2 * NV * NPF;
  // state at the points (NV NVQ) and contravariant velocities (D NVQ), then the pass scratch;
  // the face arrays reuse all three
  static constexpr int SQ = NV * NVQ + D * NVQ;
  static constexpr int S1 = cmax(NV * (IA + IB), NV * (CA + CB));
  static constexpr int S2 = cmax(0, FO + FN + FL + FG - SQ);
  static constexpr int LDS = 8 * (2 * NV * NL + SQ + cmax(S1, S2) + OiLayout{NP, NQ}.size());
};

// y = M x along one axis of a tensor array: x has extent nin along the axis, y extent nout;
// `lo` and `hi` are the extents of the axes before and after it.
// With xs non-null the input is x times the field-independent factor xs (same layout as one
// field of x).
template <int NT>
__device__ __forceinline__ void pass1d(const double* __restrict__ Mt, bool transpose, int nin, int nout,
                                       int lo, int hi, int nfield, const double* x, int xstride,
                                       double* y, int ystride, bool accumulate, const double* xs = nullptr) {
  const int total = nfield * lo * nout * hi;
  for (int t = threadIdx.x; t < total; t += NT) {
    const int a = t % lo, o = (t / lo) % nout, b = (t / (lo * nout)) % hi, f = t / (lo * nout * hi);
    const double* xp = x + f * xstride + a + lo * nin * b;
    const double* sp = xs ? xs + a + lo * nin * b : nullptr;
    double v = 0.0;
    for (int i = 0; i < nin; ++i) {
      // forward: M[o][i] stored as Mt[o * nin + i]; transposed: M[i][o] stored as Mt[i * nout + o]
      const double mm = transpose ? Mt[i * nout + o] : Mt[o * nin + i];
      v += mm * (sp ? xp[lo * i] * sp[lo * i] : xp[lo * i]);
    }
    double* yp = y + f * ystride + a + lo * o + lo * nout * b;
    if (accumulate) *yp += v;
    else *yp = v;
  }
}

template <int D, int NP, int NQ>
__global__ void __launch_bounds__(256) k_exp_oi(const double* __restrict__ U, double* __restrict__ R,
                                                const MeshDev m) {
  using C = Oi<D, NP, NQ>;
  constexpr int NV = C::NV, NL = C::NL, NVQ = C::NVQ, NPF = C::NPF, NFQ = C::NFQ, NF = C::NF,
                MS = C::MS, NT = C::NT;
  constexpr OiLayout OL{NP, NQ};
  constexpr TabLayout TL{NP};
  __shared__ double smem[C::LDS / 8];
  double* sU = smem;                 // [NV][NL] nodal state
  double* sW = sU + NV * NL;         // [NV][NL] weak-form accumulator
  double* sQ = sW + NV * NL;         // [NV][NVQ] state at the points, then w (rho, m, rho k)
  double* sG = sQ + NV * NVQ;        // [D][NVQ] contravariant velocities at the points
  double* sR = sG + D * NVQ;         // pass scratch
  double* sT = sR + cmax(C::S1, C::S2);  // over-integration tables
  const double* xq = sT + OL.xq();
  const double* wq = sT + OL.wq();
  const double* Bq = sT + OL.bq();
  const double* Dq = sT + OL.dq();
  const double* Bs = sT + OL.bs();
  const double* tab = m.tab;         // nodal tables (uniform reads)

  const int cell = blockIdx.x;
  const int tid = threadIdx.x;
  const unsigned N = (unsigned)m.N;
  const int4 ci = m.cell[cell];
  const int lev = ci.x;
  const int cid[3] = {ci.y, ci.z, ci.w};

  for (int t = tid; t < OL.size(); t += NT) sT[t] = m.oitab[t];
  for (int t = tid; t < NV * NL; t += NT) {
    const int f = t / NL, i = t % NL;
    sU[t] = U[(size_t)f * N + (size_t)cell * NL + i];
    sW[t] = 0.0;
  }
  __syncthreads();

  // ------------------------------------------------------------------ volume: nodes -> points
  {
    double* sA = sR;
    double* sB = sA + NV * C::IA;
    if constexpr (D == 3) {
      pass1d<NT>(Bq, false, NP, NQ, 1, NP * NP, NV, sU, NL, sA, C::IA, false);
      __syncthreads();
      pass1d<NT>(Bq, false, NP, NQ, NQ, NP, NV, sA, C::IA, sB, C::IB, false);
      __syncthreads();
      pass1d<NT>(Bq, false, NP, NQ, NQ * NQ, 1, NV, sB, C::IB, sQ, NVQ, false);
    } else {
      pass1d<NT>(Bq, false, NP, NQ, 1, NP, NV, sU, NL, sA, C::IA, false);
      __syncthreads();
      pass1d<NT>(Bq, false, NP, NQ, NQ, 1, NV, sA, C::IA, sQ, NVQ, false);
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------ flux factors at the points
  // the flux of direction k at point q is (w rho, w m, w rho k) times the contravariant velocity
  // G_k . u, w the point's weight
  for (int q = tid; q < NVQ; q += NT) {
    double X[D], wgt = 1.0;
    int t = q;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int qa = t % NQ;
      t /= NQ;
      X[a] = m.dxl[lev][a] * ((double)cid[a] + 0.5 * (1.0 + xq[qa]));
      wgt *= wq[qa];
    }
    double Gam[D][D], J;
    metric<D, double>(m, lev, X, Gam, J);
    double Uq[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) Uq[f] = sQ[f * NVQ + q];
    const double rho = Uq[0];
    double u[D], m2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) { u[a] = Uq[1 + a] / rho; m2 += Uq[1 + a] * Uq[1 + a]; }
    const double rk = 0.5 * m2 / rho;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double Gu = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) Gu += Gam[k][a] * u[a];
      sG[k * NVQ + q] = Gu;
    }
    sQ[0 * NVQ + q] = wgt * rho;
#pragma unroll
    for (int a = 0; a < D; ++a) sQ[(1 + a) * NVQ + q] = wgt * Uq[1 + a];
    sQ[(1 + D) * NVQ + q] = wgt * rk;
  }
  __syncthreads();

  // ------------------------------------------------------------------ volume: points -> nodes
  // W_i += sum_k sum_q d_k phi_i(x_q) F_k(x_q): along axis k the derivative matrix, else Bq
  {
    double* tA = sR;
    double* tB = tA + NV * C::CA;
    for (int k = 0; k < D; ++k) {
      const double* Gk = sG + k * NVQ;
      if constexpr (D == 3) {
        pass1d<NT>(k == 0 ? Dq : Bq, true, NQ, NP, 1, NQ * NQ, NV, sQ, NVQ, tA, C::CA, false, Gk);
        __syncthreads();
        pass1d<NT>(k == 1 ? Dq : Bq, true, NQ, NP, NP, NQ, NV, tA, C::CA, tB, C::CB, false);
        __syncthreads();
        pass1d<NT>(k == 2 ? Dq : Bq, true, NQ, NP, NP * NP, 1, NV, tB, C::CB, sW, NL, true);
      } else {
        pass1d<NT>(k == 0 ? Dq : Bq, true, NQ, NP, 1, NQ, NV, sQ, NVQ, tA, C::CA, false, Gk);
        __syncthreads();
        pass1d<NT>(k == 1 ? Dq : Bq, true, NQ, NP, NP, 1, NV, tA, C::CA, sW, NL, true);
      }
      __syncthreads();
    }
  }

  // ------------------------------------------------------------------ faces, one axis at a time
  double* sTO = sQ;                  // [2][NV][NPF]
  double* sTN = sTO + C::FO;         // [2][MS][NV][NPF]
  double* sL = sTN + C::FN;          // [2][MS][NV][NFQ]
  double* sGf = sL + C::FL;          // [2][NV][NPF]
  for (int k = 0; k < D; ++k) {
    // node traces: own (LDS) and neighbours (HBM / L2, along their normal lines)
    for (int t = tid; t < 2 * NV * NPF; t += NT) {
      const int s = t / (NV * NPF), v = (t / NPF) % NV, a = t % NPF;
      double o = 0.0;
      for (int n = 0; n < NP; ++n) o += tab[TL.lb() + s * NP + n] * sU[v * NL + compose<D, NP>(k, n, a)];
      sTO[t] = o;
    }
    for (int t = tid; t < 2 * MS * NV * NPF; t += NT) {
      const int s = t / (MS * NV * NPF), sub = (t / (NV * NPF)) % MS, v = (t / NPF) % NV, a = t % NPF;
      const int f = 2 * k + s;
      const int kd = m.fkind[cell * NF + f];
      if (kd == kWall || (kd != kCoarse && sub > 0)) continue;
      const int4 nb4 = m.fnbr[cell * NF + f];
      const int nb = sub == 0 ? nb4.x : sub == 1 ? nb4.y : sub == 2 ? nb4.z : nb4.w;
      double o = 0.0;
      for (int n = 0; n < NP; ++n)
        o += tab[TL.lb() + (1 - s) * NP + n] * U[(size_t)v * N + (size_t)nb * NL + compose<D, NP>(k, n, a)];
      sTN[t] = o;
    }
    __syncthreads();

    // flux at every point of both (sub-)faces, times the face weight
    for (int t = tid; t < 2 * MS * NFQ; t += NT) {
      const int s = t / (MS * NFQ), sub = (t / NFQ) % MS, j = t % NFQ;
      const int f = 2 * k + s;
      const int kd = m.fkind[cell * NF + f];
      if (kd != kCoarse && sub > 0) continue;
      const int j0 = j % NQ, j1 = D == 3 ? j / NQ : 0;
      // this cell's position on its coarse neighbour's face (fine side)
      int cs[2] = {0, 0};
      {
        int tt = 0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax)
          if (ax != k) cs[tt++] = cid[ax] & 1;
      }
      // own-side and neighbour-side interpolation matrices per tangential direction
      const int c0 = sub & 1, c1 = sub >> 1;
      const double* Mo0 = kd == kCoarse ? Bs + c0 * NQ * NP : Bq;
      const double* Mo1 = kd == kCoarse ? Bs + c1 * NQ * NP : Bq;
      const double* Mn0 = kd == kFine ? Bs + cs[0] * NQ * NP : Bq;
      const double* Mn1 = kd == kFine ? Bs + cs[1] * NQ * NP : Bq;
      double tm[NV], tn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double* To = sTO + (s * NV + v) * NPF;
        const double* Tn = sTN + ((s * MS + sub) * NV + v) * NPF;
        double a = 0.0, b = 0.0;
        if constexpr (D == 3) {
#pragma unroll 1
          for (int a1 = 0; a1 < NP; ++a1) {
            double ra = 0.0, rb = 0.0;
#pragma unroll 1
            for (int a0 = 0; a0 < NP; ++a0) {
              ra += Mo0[j0 * NP + a0] * To[a0 + NP * a1];
              rb += Mn0[j0 * NP + a0] * Tn[a0 + NP * a1];
            }
            a += Mo1[j1 * NP + a1] * ra;
            b += Mn1[j1 * NP + a1] * rb;
          }
        } else {
#pragma unroll 1
          for (int a0 = 0; a0 < NP; ++a0) {
            a += Mo0[j0 * NP + a0] * To[a0];
            b += Mn0[j0 * NP + a0] * Tn[a0];
          }
        }
        tm[v] = a;
        tn[v] = b;
      }
      // area-weighted normal at the point, from the integer description of the (sub)face
      const int lf = kd == kCoarse ? lev + 1 : lev;
      int P = kd == kCoarse ? (s ? 2 * (cid[k] + 1) : 2 * cid[k]) : (s ? cid[k] + 1 : cid[k]);
      if (m.per[k] && P >= m.nlev[lf][k]) P -= m.nlev[lf][k];
      double X[D];
      {
        int tt = 0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
          const double dx = m.dxl[lf][ax];
          if (ax == k) {
            X[ax] = dx * (double)P;
          } else {
            const int Tt = kd == kCoarse ? 2 * cid[ax] + ((sub >> tt) & 1) : cid[ax];
            X[ax] = dx * ((double)Tt + 0.5 * (1.0 + xq[tt == 0 ? j0 : j1]));
            ++tt;
          }
        }
      }
      double Gam[D][D], Jf, Nv[D];
      metric<D, double>(m, lf, X, Gam, Jf);
#pragma unroll
      for (int a = 0; a < D; ++a) Nv[a] = Gam[k][a];
      const double wj = D == 3 ? wq[j0] * wq[j1] : wq[j0];
      double F[NV];
      double sgn = s ? 1.0 : -1.0;
      if (kd == kWall) {
        double No[D];
#pragma unroll
        for (int a = 0; a < D; ++a) No[a] = sgn * Nv[a];
        wall_flux<D>(tm, No, F);
        sgn = 1.0;
      } else if (s) {
        rusanov<D>(tm, tn, Nv, F);
      } else {
        rusanov<D>(tn, tm, Nv, F);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) sL[((s * MS + sub) * NV + v) * NFQ + j] = -sgn * wj * F[v];
    }
    __syncthreads();
    // back onto the face nodes (transposed own-side interpolation)
    for (int t = tid; t < 2 * NV * NPF; t += NT) {
      const int s = t / (NV * NPF), v = (t / NPF) % NV, a = t % NPF;
      const int kd = m.fkind[cell * NF + 2 * k + s];
      const int nsub = kd == kCoarse ? MS : 1;
      const int a0 = a % NP, a1 = D == 3 ? a / NP : 0;
      double g = 0.0;
#pragma unroll 1
      for (int sub = 0; sub < nsub; ++sub) {
        const int c0 = sub & 1, c1 = sub >> 1;
        const double* Mo0 = kd == kCoarse ? Bs + c0 * NQ * NP : Bq;
        const double* Mo1 = kd == kCoarse ? Bs + c1 * NQ * NP : Bq;
        const double* Lp = sL + ((s * MS + sub) * NV + v) * NFQ;
#pragma unroll 1
        for (int j = 0; j < NFQ; ++j) {
          const int j0 = j % NQ, j1 = D == 3 ? j / NQ : 0;
          const double b = D == 3 ? Mo0[j0 * NP + a0] * Mo1[j1 * NP + a1] : Mo0[j0 * NP + a0];
          g += b * Lp[j];
        }
      }
      sGf[t] = g;
    }
    __syncthreads();
    // lift both faces along the normal lines into the accumulator (face 2k, then 2k + 1)
    for (int t = tid; t < NV * NL; t += NT) {
      const int v = t / NL, i = t % NL;
      double acc = sW[t];
      acc += tab[TL.lb() + along<D, NP>(i, k)] * sGf[(0 * NV + v) * NPF + tang<D, NP>(i, k)];
      acc += tab[TL.lb() + NP + along<D, NP>(i, k)] * sGf[(1 * NV + v) * NPF + tang<D, NP>(i, k)];
      sW[t] = acc;
    }
    __syncthreads();
  }

  // ------------------------------------------------------------------ finalize
  for (int t = tid; t < NL; t += NT) {
    const int i = t;
    double X[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
      X[a] = m.dxl[lev][a] * ((double)cid[a] + 0.5 * (1.0 + tab[TL.xi() + along<D, NP>(i, a)]));
    double Gam[D][D], J;
    metric<D, double>(m, lev, X, Gam, J);
    double wi = 1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) wi *= tab[TL.w() + along<D, NP>(i, a)];
    const double imass = 1.0 / (wi * J);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double r = sW[v * NL + i] * imass;
      if (v == NV - 1) r -= kG * sU[D * NL + i];
      R[(size_t)v * N + (size_t)cell * NL + i] = r;
    }
  }
}

// (degree, NQ) pairs whose workgroup fits the CU's 160 KiB of LDS
template <int D, int NP, int NQ>
constexpr bool oi_fits() {
  return NQ <= kMaxNq && Oi<D, NP, NQ>::LDS <= 160 * 1024;
}

template <int D, int NP, int NQ>
int run_oi(const MeshDev& m, const double* U, double* R, hipStream_t s) {
  if constexpr (oi_fits<D, NP, NQ>()) {
    if (m.ncell <= 0) return 0;
    hipLaunchKernelGGL((k_exp_oi<D, NP, NQ>), dim3(m.ncell), dim3(Oi<D, NP, NQ>::NT), 0, s, U, R, m);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  } else {
    return -6;
  }
}

template <int D, int NP>
int run_oi_nq(const MeshDev& m, const double* U, double* R, hipStream_t s) {
  switch (m.nq - NP) {
    case 1: return run_oi<D, NP, NP + 1>(m, U, R, s);
    case 2: return run_oi<D, NP, NP + 2>(m, U, R, s);
    case 3: return run_oi<D, NP, NP + 3>(m, U, R, s);
    default: return -6;
  }
}

}  // namespace

int launch_explicit_oi(const MeshDev& m, int degree, const double* U, double* R, hipStream_t s) {
#define DG_OI_DISPATCH(D_)                                  \
  switch (degree) {                                         \
    case 1: return run_oi_nq<D_, 2>(m, U, R, s);            \
    case 2: return run_oi_nq<D_, 3>(m, U, R, s);            \
    case 3: return run_oi_nq<D_, 4>(m, U, R, s);            \
    case 4: return run_oi_nq<D_, 5>(m, U, R, s);            \
    case 5: return run_oi_nq<D_, 6>(m, U, R, s);            \
    default: return -6;                                     \
  }
  if (m.dim == 2) {
    DG_OI_DISPATCH(2)
  } else {
    DG_OI_DISPATCH(3)
  }
#undef DG_OI_DISPATCH
}

}  // namespace dg
