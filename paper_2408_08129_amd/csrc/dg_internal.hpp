// Internal types shared by the host solver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "dg_mesh.hpp"

namespace dg {

constexpr double kG = 9.81;
constexpr double kR = 287.0;
constexpr double kGamma = 1.4;
constexpr double kPi = 3.14159265358979323846;

// Orography and atmosphere parameters (Section 3.1).
struct Terrain {
  int kind;   // DG_ORO_*
  double h0, a, xc, yc;
  double ia2; // 1 / a^2
};

constexpr int kMaxLev = 9;  // levels 0..8

// Device view of the mesh.  Per cell: (level, i0, i1, i2) at its own level (axis order: 3D x,y,z,
// 2D x,z); per face (2 d per cell, face f = 2 k + s): kind and up to 2^(d-1) neighbour ids.
struct MeshDev {
  int dim;
  int ncell;
  long N;                 // nodes per field
  const int4* cell;
  const int* fkind;
  const int4* fnbr;
  const double* tab;      // 1D basis tables (layout: see TabLayout)
  const float* tabf;
  double L[3];
  int nb[3];
  int per[3];
  Terrain ter;
  double invH;                 // 1 / lid height
  double sponge[5];            // absorbing layers: top depth, top rate, lateral width, lateral rate, u_ref
  double dxl[kMaxLev][3];      // cell size per level and axis
  int nlev[kMaxLev][3];        // cells per axis at each level
  // cells whose faces are all conforming or walls (reg) and cells with a 2:1 face (irr), each
  // in mesh order
  const int* reg;
  int nreg;
  const int* irr;
  int nirr;
  // workgroup cell lists of the gradient column kernel: vertical runs of cells joined by
  // conforming bottom / top faces, packed CPB cells per workgroup (-1 pads the last one); flag
  // bit 0 (1): the bottom (top) neighbour is the previous (next) cell of the same workgroup
  const int* runs;
  const int* rflag;
  int nrwg;
  // over-integration of the explicit flux: NQ Gauss points per direction and their tables
  // (OiLayout), or nq = 0
  const double* oitab;
  int nq;
};

// --------------------------------------------------------------- shared launches (segments)
// A kernel launched for one mesh takes its arguments and mesh view by value (Direct).  A shared
// launch over several ensemble members (Shared) takes a table: member k owns the workgroups
// [b0[k], b0[k+1]) of the grid, its arguments a[k] and its mesh view, of which the table holds the
// device copy (the view is too large to repeat per member in the kernel arguments).  Every member
// keeps the grid shape of its own launch, so each member's results are the same bits whatever
// else shares the launch.
constexpr int kMaxSeg = 8;

template <class A>
struct SegTab {
  int n;                       // members in this launch, 1..kMaxSeg
  int b0[kMaxSeg + 1];         // first workgroup of each member; b0[n] = grid size
  const MeshDev* m[kMaxSeg];   // device copies of the members' mesh views (may be null)
  A a[kMaxSeg];
};

template <class A>
struct Direct {
  A a;
  MeshDev m;
  __device__ __forceinline__ int seg() const { return 0; }
  __device__ __forceinline__ const A& args(int) const { return a; }
  __device__ __forceinline__ const MeshDev& mesh(int) const { return m; }
  __device__ __forceinline__ int blk(int) const { return blockIdx.x; }
  __device__ __forceinline__ int nblk(int) const { return gridDim.x; }
};

template <class A>
struct Shared {
  SegTab<A> t;
  // the member that owns this workgroup (uniform across the workgroup)
  __device__ __forceinline__ int seg() const {
    int k = 0;
#pragma unroll
    for (int i = 1; i < kMaxSeg; ++i) k += (i < t.n && (int)blockIdx.x >= t.b0[i]) ? 1 : 0;
    return k;
  }
  __device__ __forceinline__ const A& args(int k) const { return t.a[k]; }
  __device__ __forceinline__ const MeshDev& mesh(int k) const { return *t.m[k]; }
  __device__ __forceinline__ int blk(int k) const { return (int)blockIdx.x - t.b0[k]; }
  __device__ __forceinline__ int nblk(int k) const { return t.b0[k + 1] - t.b0[k]; }
};

// Host side of a shared launch: the members with work (blocks(k) > 0) in order, kMaxSeg per
// launch; launch(table, grid) returns 0 or an error code.
template <class A, class Blocks, class Args, class Launch>
int seg_launch(int n, const MeshDev* const* md, Blocks blocks, Args args, Launch launch) {
  SegTab<A> t{};
  int g = 0;
  auto flush = [&]() {
    if (t.n == 0) return 0;
    for (int i = t.n; i <= kMaxSeg; ++i) t.b0[i] = g;
    const int r = launch(t, g);
    t.n = 0;
    g = 0;
    return r;
  };
  for (int k = 0; k < n; ++k) {
    const int nb = blocks(k);
    if (nb <= 0) continue;
    if (t.n == kMaxSeg) {
      const int r = flush();
      if (r) return r;
    }
    t.b0[t.n] = g;
    t.m[t.n] = md ? md[k] : nullptr;
    t.a[t.n] = args(k);
    t.n++;
    g += nb;
  }
  return flush();
}

// Offsets into the 1D table for NP = r + 1 points.
struct TabLayout {
  int np;
  __host__ __device__ constexpr int xi() const { return 0; }
  __host__ __device__ constexpr int w() const { return np; }
  __host__ __device__ constexpr int dt() const { return 2 * np; }                  // Dt[i][q]
  __host__ __device__ constexpr int lb() const { return 2 * np + np * np; }        // lb[s][a]
  __host__ __device__ constexpr int lbw() const { return 4 * np + np * np; }       // lb/w
  __host__ __device__ constexpr int pi() const { return 6 * np + np * np; }        // Pi[c][j][a]
  __host__ __device__ constexpr int rw() const { return 6 * np + 3 * np * np; }    // Rw[c][a][j]
  __host__ __device__ constexpr int fds() const { return 6 * np + 5 * np * np; }   // S[i][a]
  __host__ __device__ constexpr int fdmu() const { return 6 * np + 6 * np * np; }  // mu[a]
  __host__ __device__ constexpr int size() const { return 7 * np + 6 * np * np; }
};

// Offsets into the over-integration table for NP nodes and NQ quadrature points per direction.
struct OiLayout {
  int np, nq;
  __host__ __device__ constexpr int xq() const { return 0; }                         // points
  __host__ __device__ constexpr int wq() const { return nq; }                        // weights
  __host__ __device__ constexpr int bq() const { return 2 * nq; }                    // Bq[q][j] = l_j(xq_q)
  __host__ __device__ constexpr int dq() const { return 2 * nq + nq * np; }          // Dq[q][j] = l_j'(xq_q)
  __host__ __device__ constexpr int bs() const { return 2 * nq + 2 * nq * np; }      // Bs[h][q][j] = l_j((xq_q + 2h - 1) / 2)
  __host__ __device__ constexpr int size() const { return 2 * nq + 4 * nq * np; }
};
constexpr int kMaxNq = 8;  // over-integration points per direction

// ----------------------------------------------------------------------- operator parameters
// Inputs of the weak gradient M^{-1} B p (output q, d fields).
template <class T>
struct GradArgs {
  const T* p;         // p directly, or v with the Jacobi scaling below
  const T* dinv;      // if non-null: p = scale * dinv * v
  T scale;
  T* q;               // out [d][N]: M^{-1} B p, times h if h is non-null
  const T* h;         // optional pointwise multiplier of the output
  T* z;               // optional: the (scaled) p at the nodes
};

// Inputs of the weak divergence / Helmholtz pass:
//   out = mode_weak ? w_i (acc + amass J p) : acc / J, with
//   acc = (adiv C(h qv) + apen P p) / w_i.
template <class T>
struct DivArgs {
  const T* qv;        // vector field [d][N]
  const T* h;         // multiplier (may be null: 1)
  const T* p;         // scalar for the penalty / mass terms (may be null)
  const T* dinv;      // if non-null: p = scale * dinv * p
  T scale;
  const T* lam;       // per-cell sound speed for the penalty
  T adiv, apen, amass;
  int weak;
  T* out;
  // enthalpy split in one pass (column kernel, h = h - hbar): out also receives
  // hbar C(qv) + adiv M (d hbar/dz) qv_z, with hbar and its height derivative at the nodes
  const T* hb;
  const T* dhb;
};

// Explicit residual R = F_E(U) ([F][N] each).
struct ExpArgs {
  const double* U;
  double* R;
};

// Cell-wise fast-diagonalisation preconditioner: z = P^{-1} (scale v) with, per cell,
// P = Jbar (S^-T (x) ...) [1/(gamma-1) + sum_k alpha_k mu] (S^-1 (x) ...); coef[cell] holds
// (1/Jbar, alpha_0, alpha_1, alpha_2).
template <class T>
struct FdmArgs {
  const T* v;
  T scale;
  const T* coef;
  T* z;
  const double* dscale;  // if non-null: the scale is read from device memory (*dscale) instead
};

// --------------------------------------------------------------------------------- launchers
// Weak gradient / divergence on a list of cells with the general cell kernel.
int launch_grad_cells64(const MeshDev& m, int degree, const GradArgs<double>& a, const int* list, int n, hipStream_t s);
int launch_div_cells64(const MeshDev& m, int degree, const DivArgs<double>& a, const int* list, int n, hipStream_t s);
int launch_grad_cells32(const MeshDev& m, int degree, const GradArgs<float>& a, const int* list, int n, hipStream_t s);
int launch_div_cells32(const MeshDev& m, int degree, const DivArgs<float>& a, const int* list, int n, hipStream_t s);
// the 2:1 face terms of the cells with such faces, added to outputs the column kernels wrote
int launch_grad_hang64(const MeshDev& m, int degree, const GradArgs<double>& a, hipStream_t s);
int launch_div_hang64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s);
int launch_grad_hang32(const MeshDev& m, int degree, const GradArgs<float>& a, hipStream_t s);
int launch_div_hang32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s);
int launch_explicit_hang(const MeshDev& m, int degree, const double* U, double* R, hipStream_t s);
int launch_explicit(const MeshDev& m, int degree, const double* U, double* R, hipStream_t s);
int launch_grad64(const MeshDev& m, int degree, const GradArgs<double>& a, hipStream_t s);
int launch_div64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s);
int launch_grad32(const MeshDev& m, int degree, const GradArgs<float>& a, hipStream_t s);
int launch_div32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s);
int launch_fdm64(const MeshDev& m, int degree, const FdmArgs<double>& a, hipStream_t s);
// the enthalpy-split energy flux in one column pass plus the 2:1 face terms (a.h = h - hbar,
// a.hb = hbar, a.dhb = d hbar / dz)
int launch_div_split64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s);
int launch_div_split32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s);
// explicit residual with its flux integrals over-integrated at m.nq points per direction (all
// cells, general faces); returns -6 for an unsupported (degree, nq)
int launch_explicit_oi(const MeshDev& m, int degree, const double* U, double* R, hipStream_t s);
int launch_fdm32(const MeshDev& m, int degree, const FdmArgs<float>& a, hipStream_t s);

// Shared launches of the column operators over n members of one class (same dimension and degree):
// mh[k] the host copy of member k's mesh view (grid sizes), md[k] its device copy (kernels), a[k]
// its arguments.  Each is the launch of the single-mesh form for every member (column kernel,
// then the 2:1 faces), with the column-form conditions on the arguments (no Jacobi scaling, no
// copy of p; the divergence with h or p, the same for all members); returns -6 otherwise.
int launch_grad_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<double>* a, int degree, hipStream_t s);
int launch_grad_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<float>* a, int degree, hipStream_t s);
int launch_div_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<double>* a, int degree, hipStream_t s);
int launch_div_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<float>* a, int degree, hipStream_t s);
int launch_div_split_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<double>* a, int degree, hipStream_t s);
int launch_div_split_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<float>* a, int degree, hipStream_t s);
int launch_fdm_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const FdmArgs<double>* a, int degree, hipStream_t s);
int launch_fdm_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const FdmArgs<float>* a, int degree, hipStream_t s);
int launch_explicit_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const ExpArgs* a, int degree, hipStream_t s);
// the 2:1-face passes alone (after the column kernels)
int launch_grad_hang_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<double>* a, int degree, hipStream_t s);
int launch_grad_hang_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<float>* a, int degree, hipStream_t s);
int launch_div_hang_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<double>* a, int degree, hipStream_t s);
int launch_div_hang_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<float>* a, int degree, hipStream_t s);
int launch_explicit_hang_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const ExpArgs* a, int degree, hipStream_t s);
// both 2:1-face terms of the enthalpy-split divergence in one pass (a.h = h - hbar, a.hb = hbar)
int launch_div_split_hang64(const MeshDev& m, int degree, const DivArgs<double>& a, hipStream_t s);
int launch_div_split_hang32(const MeshDev& m, int degree, const DivArgs<float>& a, hipStream_t s);
int launch_div_split_hang_seg64(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<double>* a, int degree, hipStream_t s);
int launch_div_split_hang_seg32(int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<float>* a, int degree, hipStream_t s);
// per-cell sound speed (lam) and preconditioner coefficients from h and w J (coef may be null:
// lam only)
int launch_cellcoef(const MeshDev& m, int degree, const double* h, const double* wJ, double dta,
                    double* lam, float* lam32, double* coef, float* coef32, hipStream_t s);
struct CoefArgs {
  const double* h;
  const double* wJ;
  double dta;
  double* lam;
  float* lam32;
  double* coef;
  float* coef32;
};
int launch_cellcoef_seg(int n, const MeshDev* const* mh, const MeshDev* const* md, const CoefArgs* a, int degree,
                        hipStream_t s);

// node geometry: physical coordinates, w J, background p and rho, absorbing-layer rate per node
// (each output optional)
int launch_geometry(const MeshDev& m, int degree, double* x, double* y, double* z, double* wJ,
                    double* pbar, double* rbar, double* tau, int atm_kind, const double* atm,
                    hipStream_t s);

}  // namespace dg
