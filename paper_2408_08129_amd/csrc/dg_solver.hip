// IMEX-RK2 step, pressure fixed-point loop and GMRES on the device, plus the C ABI.
//
// Time integration (arXiv 2408.08129, Section 2): continuity explicit, energy coupled implicitly
// to momentum, second-order IMEX Runge-Kutta (ARK2 of Giraldo, Kelly and Constantinescu, 2013:
// explicit first stage, two implicit stages with diagonal 1 - 1/sqrt(2)).  Each implicit stage
// runs the pressure fixed-point loop of Section 3.2; its linear system, non-symmetric, is solved
// matrix-free with right-preconditioned GMRES.
//
// The implicit stage, with predictor rho_i, m~, e~ and m' = m~ - dt a (rho_i - rhobar) g k:
//   A(h) delta = b - A(h) p',  A = M/(gamma-1) + dt a beta/(2(gamma-1)) P - (dt a)^2 C h M^-1 B,
//   b = M (e~ - |m|^2/(2 rho_i) - pbar/(gamma-1)) - dt a C (h m'),
//   p' += delta;  m = m' - dt a M^-1 B p';  h = gamma (pbar + p') / ((gamma-1) rho_i).
// All vectors live in HBM; the host only drives the loop and solves the small Hessenberg least
// squares problem.  Reductions are two-stage with a fixed shape, so results are bitwise
// reproducible and independent of what else runs on the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "dg_internal.hpp"

namespace dg {
namespace {

constexpr int kMaxV = 32;  // max Krylov vectors per pass (restart <= 31)
// meshes of at most this many nodes per field run the GMRES iteration with one host round trip
constexpr long kOneSyncMaxNodes = 1L << 23;
constexpr int kRedThreads = 256;

thread_local std::string g_last_error;

// Device scratch of the allocation-free diagnostics entry point (dg_diagnostics_noalloc): the
// per-block partial sums of its two reductions (3 values x kMaxGrid blocks for the mass pass,
// kMaxGrid for the maximum) and their results.  One copy per GPU for the life of the process; in
// host code its address is only ever taken through hipGetSymbolAddress (scratch_ptr).
constexpr int kScratchGrid = 2048;
constexpr int kScratchDoubles = 4 * kScratchGrid + 8;
__device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

struct Coef { double c[kMaxV]; };

inline int red_grid(long n) {
  long g = (n + kRedThreads - 1) / kRedThreads;
  return (int)std::max(1L, std::min(2048L, g));
}
constexpr int kMaxGrid = 2048;

// --------------------------------------------------------------------------- reduction helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-reduce NV per-thread sums (fixed order) and write part[i * nb + bid] (block bid of nb).
template <int NV>
__device__ __forceinline__ void block_store(const double (&acc)[NV], double* part, int bid, int nb) {
  __shared__ double s[NV][kRedThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double v = wave_sum(acc[i]);
    if (lane == 0) s[i][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kRedThreads / 64; ++k) t += s[threadIdx.x][k];
    part[(long)threadIdx.x * nb + bid] = t;
  }
}

// Second stage: value i is the sum of part[i * G + 0 .. G), in a fixed order, by one workgroup.
__device__ __forceinline__ double reduce_value(const double* part, int G, int i) {
  __shared__ double s[kRedThreads / 64];
  double t = 0.0;
  for (int b = threadIdx.x; b < G; b += kRedThreads) t += part[(long)i * G + b];
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = t;
  __syncthreads();
  double u = 0.0;
#pragma unroll
  for (int k = 0; k < kRedThreads / 64; ++k) u += s[k];
  return u;  // valid in thread 0
}

// Second stage, one workgroup per value (grid = nv).
__global__ void __launch_bounds__(kRedThreads) k_reduce(const double* part, int G, double* out) {
  const double u = reduce_value(part, G, blockIdx.x);
  if (threadIdx.x == 0) out[blockIdx.x] = u;
}

// The basis kernels stream 16 bytes per lane per access (two doubles or four floats; gfx950
// global accesses need only the element alignment), with a scalar tail for n % W.
template <class T>
struct Vec16 {
  static constexpr int W = 16 / (int)sizeof(T);
  typedef T type __attribute__((ext_vector_type(W), aligned(sizeof(T))));
};

// Reduction pass of the Gram-Schmidt step: for i < NV the products V_i.x and (HASY) V_i.y,
// then x.x and (HASY) x.y, y.y, accumulated in FP64.  Value order in part:
// [V_i.x]_i, [V_i.y]_i, x.x, x.y, y.y (without y: [V_i.x]_i, x.x).
template <int NV, bool HASY, int NA>
__device__ __forceinline__ void dots_point(double (&acc)[NA], double xv, double yv, const double (&v)[NV > 0 ? NV : 1]) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    acc[i] += v[i] * xv;
    if constexpr (HASY) acc[NV + i] += v[i] * yv;
  }
  if constexpr (HASY) {
    acc[2 * NV] += xv * xv;
    acc[2 * NV + 1] += xv * yv;
    acc[2 * NV + 2] += yv * yv;
  } else {
    acc[NV] += xv * xv;
  }
}

template <class T>
struct DotsArgs {
  const T* V;
  long ld;
  const T* x;
  const T* y;
  double* part;
  long n;
};

template <class T, int NV, bool HASY>
__device__ __forceinline__ void gs_dots_body(const DotsArgs<T>& a, int bid, int nb) {
  constexpr int NA = HASY ? 2 * NV + 3 : NV + 1;
  constexpr int W = Vec16<T>::W;
  using VT = typename Vec16<T>::type;
  const T* __restrict__ V = a.V;
  const T* __restrict__ x = a.x;
  const T* __restrict__ y = a.y;
  const long ld = a.ld, n = a.n;
  double acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = 0.0;
  const long gt = (long)bid * kRedThreads + threadIdx.x, gs = (long)nb * kRedThreads;
  const long nvec = n / W;
  for (long e = gt; e < nvec; e += gs) {
    const VT xw = *(const VT*)(x + e * W);
    VT yw = xw;
    if constexpr (HASY) yw = *(const VT*)(y + e * W);
    VT vw[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) vw[i] = *(const VT*)(V + i * ld + e * W);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      double v[NV > 0 ? NV : 1];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = (double)vw[i][k];
      dots_point<NV, HASY>(acc, (double)xw[k], HASY ? (double)yw[k] : 0.0, v);
    }
  }
  for (long e = nvec * W + gt; e < n; e += gs) {
    double v[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = (double)V[i * ld + e];
    dots_point<NV, HASY>(acc, (double)x[e], HASY ? (double)y[e] : 0.0, v);
  }
  block_store<NA>(acc, a.part, bid, nb);
}

template <class T, int NV, bool HASY>
__global__ void __launch_bounds__(kRedThreads) k_gs_dots(const DotsArgs<T> a) {
  gs_dots_body<T, NV, HASY>(a, blockIdx.x, gridDim.x);
}
template <class T, int NV, bool HASY>
__global__ void __launch_bounds__(kRedThreads) k_gs_dots_seg(const Shared<DotsArgs<T>> src) {
  const int k = src.seg();
  gs_dots_body<T, NV, HASY>(src.args(k), src.blk(k), src.nblk(k));
}

// Update pass of the Gram-Schmidt step, FP64 arithmetic:
//   z = y - sum_i b_i V_i - g x      (x as read on entry)
//   x = x - sum_i a_i V_i            (only when NV > 0; in place)
// and part = |z|^2.  The coefficients come as kernel arguments (one mesh) or, for a shared launch,
// from device memory through LDS.
template <class T>
struct UpdArgs {
  const T* V;
  long ld;
  const double* coef;  // shared launches: a at coef[0 .. kMaxV), b at coef[kMaxV .. 2 kMaxV)
  double g;
  T* x;
  const T* y;
  T* z;
  double* part;
  long n;
};
struct CoefRef { const double* c; };

template <class T, int NV, class CA>
__device__ __forceinline__ void update_point(const CA& a, const CA& b, double g, const double (&v)[NV > 0 ? NV : 1],
                                             double xo, double yv, T& zt, T& xt) {
  double zv = yv - g * xo;
  double xn = xo;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    zv -= b.c[i] * v[i];
    xn -= a.c[i] * v[i];
  }
  zt = (T)zv;
  xt = (T)xn;
}

template <class T, int NV, class CA>
__device__ __forceinline__ void gs_update_body(const UpdArgs<T>& u, const CA& a, const CA& b, int bid, int nb) {
  constexpr int W = Vec16<T>::W;
  using VT = typename Vec16<T>::type;
  const T* __restrict__ V = u.V;
  T* __restrict__ x = u.x;
  const T* __restrict__ y = u.y;
  T* __restrict__ z = u.z;
  const long ld = u.ld, n = u.n;
  const double g = u.g;
  double acc[1] = {0.0};
  const long gt = (long)bid * kRedThreads + threadIdx.x, gs = (long)nb * kRedThreads;
  const long nvec = n / W;
  for (long e = gt; e < nvec; e += gs) {
    VT vw[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) vw[i] = *(const VT*)(V + i * ld + e * W);
    const VT xw = *(const VT*)(x + e * W);
    const VT yw = *(const VT*)(y + e * W);
    VT zw, xn;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      double v[NV > 0 ? NV : 1];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = (double)vw[i][k];
      T zt, xt;
      update_point<T, NV>(a, b, g, v, (double)xw[k], (double)yw[k], zt, xt);
      zw[k] = zt;
      xn[k] = xt;
      acc[0] += (double)zt * (double)zt;
    }
    *(VT*)(z + e * W) = zw;
    if (NV > 0) *(VT*)(x + e * W) = xn;
  }
  for (long e = nvec * W + gt; e < n; e += gs) {
    double v[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = (double)V[i * ld + e];
    T zt, xt;
    update_point<T, NV>(a, b, g, v, (double)x[e], (double)y[e], zt, xt);
    z[e] = zt;
    if (NV > 0) x[e] = xt;
    acc[0] += (double)zt * (double)zt;
  }
  block_store<1>(acc, u.part, bid, nb);
}

template <class T, int NV>
__global__ void __launch_bounds__(kRedThreads) k_gs_update(const UpdArgs<T> u, const Coef a, const Coef b) {
  gs_update_body<T, NV>(u, a, b, blockIdx.x, gridDim.x);
}
template <class T, int NV>
__global__ void __launch_bounds__(kRedThreads) k_gs_update_seg(const Shared<UpdArgs<T>> src) {
  __shared__ double sc[2][kMaxV];
  const int k = src.seg();
  const UpdArgs<T>& u = src.args(k);
  if (threadIdx.x < NV) {
    sc[0][threadIdx.x] = u.coef[threadIdx.x];
    sc[1][threadIdx.x] = u.coef[kMaxV + threadIdx.x];
  }
  __syncthreads();
  gs_update_body<T, NV>(u, CoefRef{sc[0]}, CoefRef{sc[1]}, src.blk(k), src.nblk(k));
}

// x += dinv * sum_i c_i V_i  (FP64 accumulation)
template <class T, int NV>
__global__ void k_update(const T* __restrict__ V, long ld, const Coef c, const T* __restrict__ dinv,
                         double* __restrict__ x, long n) {
  constexpr int W = Vec16<T>::W;
  using VT = typename Vec16<T>::type;
  const long gt = (long)blockIdx.x * blockDim.x + threadIdx.x, gs = (long)gridDim.x * blockDim.x;
  const long nvec = n / W;
  for (long e = gt; e < nvec; e += gs) {
    VT vw[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vw[i] = *(const VT*)(V + i * ld + e * W);
    VT dw = vw[0];
    if (dinv) dw = *(const VT*)(dinv + e * W);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < NV; ++i) s += c.c[i] * (double)vw[i][k];
      x[e * W + k] += dinv ? (double)dw[k] * s : s;
    }
  }
  for (long e = nvec * W + gt; e < n; e += gs) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) s += c.c[i] * (double)V[i * ld + e];
    x[e] += dinv ? (double)dinv[e] * s : s;
  }
}

// Second stages of a shared launch: value blk of member k's partials (nv blocks per member), and
// the candidate norm (one block per member).
struct RedArgs {
  const double* part;
  int G;
  double* out;
};
__global__ void __launch_bounds__(kRedThreads) k_reduce_seg(const Shared<RedArgs> src) {
  const int k = src.seg();
  const RedArgs& a = src.args(k);
  const int i = src.blk(k);
  const double u = reduce_value(a.part, a.G, i);
  if (threadIdx.x == 0) a.out[i] = u;
}

#define DG_NV_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) \
  X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31)

#define DG_NV_CASES0(X) X(0) DG_NV_CASES(X)

template <class T>
void launch_gs_dots(int nv, int G, hipStream_t s, const T* V, long ld, const T* x, const T* y, double* part,
                    long n) {
  const DotsArgs<T> a{V, ld, x, y, part, n};
  if (y) {
    switch (nv) {
#define X(K) case K: hipLaunchKernelGGL((k_gs_dots<T, K, true>), dim3(G), dim3(kRedThreads), 0, s, a); break;
      DG_NV_CASES0(X)
#undef X
      default: break;
    }
  } else {
    switch (nv) {
#define X(K) case K: hipLaunchKernelGGL((k_gs_dots<T, K, false>), dim3(G), dim3(kRedThreads), 0, s, a); break;
      DG_NV_CASES0(X)
#undef X
      default: break;
    }
  }
}
template <class T>
void launch_gs_dots_seg(int nv, bool hasy, int g, hipStream_t s, const Shared<DotsArgs<T>>& t) {
  if (hasy) {
    switch (nv) {
#define X(K) case K: hipLaunchKernelGGL((k_gs_dots_seg<T, K, true>), dim3(g), dim3(kRedThreads), 0, s, t); break;
      DG_NV_CASES0(X)
#undef X
      default: break;
    }
  } else {
    switch (nv) {
#define X(K) case K: hipLaunchKernelGGL((k_gs_dots_seg<T, K, false>), dim3(g), dim3(kRedThreads), 0, s, t); break;
      DG_NV_CASES0(X)
#undef X
      default: break;
    }
  }
}
template <class T>
void launch_gs_update(int nv, int G, hipStream_t s, const T* V, long ld, const Coef& a, const Coef& b, double g,
                      T* x, const T* y, T* z, double* part, long n) {
  const UpdArgs<T> u{V, ld, nullptr, g, x, y, z, part, n};
  switch (nv) {
#define X(K) case K: hipLaunchKernelGGL((k_gs_update<T, K>), dim3(G), dim3(kRedThreads), 0, s, u, a, b); break;
    DG_NV_CASES0(X)
#undef X
    default: break;
  }
}
template <class T>
void launch_gs_update_seg(int nv, int g, hipStream_t s, const Shared<UpdArgs<T>>& t) {
  switch (nv) {
#define X(K) case K: hipLaunchKernelGGL((k_gs_update_seg<T, K>), dim3(g), dim3(kRedThreads), 0, s, t); break;
    DG_NV_CASES0(X)
#undef X
    default: break;
  }
}
template <class T>
void launch_update(int nv, dim3 g, hipStream_t s, const T* V, long ld, const Coef& c, const T* dinv, double* x,
                   long n) {
  switch (nv) {
#define X(K) case K: hipLaunchKernelGGL((k_update<T, K>), g, dim3(256), 0, s, V, ld, c, dinv, x, n); break;
    DG_NV_CASES(X)
#undef X
    default: break;
  }
}

__global__ void k_maxabs_ratio(const double* __restrict__ num, const double* __restrict__ den,
                               double* part, long n) {
  __shared__ double s[kRedThreads];
  double m = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(num[e] / den[e]));
  s[threadIdx.x] = m;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Second stage of the candidate-norm reduction of the one-round-trip GMRES iteration: out[0] =
// |v|^2, out[1] = 1/|v| (0 for a zero vector), the scale the next operator application reads.
__device__ __forceinline__ void reduce_norm_body(const double* part, int G, double* out) {
  const double u = reduce_value(part, G, 0);
  if (threadIdx.x == 0) {
    out[0] = u;
    out[1] = u > 0.0 ? 1.0 / sqrt(u) : 0.0;
  }
}
__global__ void __launch_bounds__(kRedThreads) k_reduce_norm(const double* part, int G, double* out) {
  reduce_norm_body(part, G, out);
}
__global__ void __launch_bounds__(kRedThreads) k_reduce_norm_seg(const Shared<RedArgs> src) {
  const int k = src.seg();
  reduce_norm_body(src.args(k).part, src.args(k).G, src.args(k).out);
}

// Second stage of the max reduction: one workgroup, fixed order.
__global__ void __launch_bounds__(kRedThreads) k_reduce_max(const double* part, int G, double* out) {
  __shared__ double s[kRedThreads];
  double m = 0.0;
  for (int b = threadIdx.x; b < G; b += kRedThreads) m = fmax(m, part[b]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}


// ----------------------------------------------------------------------------- pointwise kernels
#define GRID_LOOP(e, n) \
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (n); e += (long)gridDim.x * blockDim.x)

// The pointwise work of the step as functors over n elements: k_pw runs one over a grid, k_pw_seg
// runs one per member in a shared launch.  Each element's arithmetic is the functor's alone.
template <class F>
__global__ void __launch_bounds__(256) k_pw(const F f) {
  GRID_LOOP(e, f.n) f(e);
}
template <class F>
__global__ void __launch_bounds__(256) k_pw_seg(const Shared<F> src) {
  const int k = src.seg();
  const F& f = src.args(k);
  for (long e = (long)src.blk(k) * 256 + threadIdx.x; e < f.n; e += (long)src.nblk(k) * 256) f(e);
}

// p' = p - pbar and h = gamma p / ((gamma - 1) rho) from the state
template <int D>
struct PwPressureH {
  long n, ld;
  const double* U;
  const double* pbar;
  double* pp;
  double* h;
  __device__ void operator()(long e) const {
    const double rho = U[e];
    double m2 = 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) m2 += U[(1 + l) * ld + e] * U[(1 + l) * ld + e];
    const double p = (kGamma - 1.0) * (U[(1 + D) * ld + e] - 0.5 * m2 / rho);
    pp[e] = p - pbar[e];
    h[e] = kGamma * p / ((kGamma - 1.0) * rho);
  }
};

// absorbing layers: R_m -= tau (m - rho u_ref e_x) (Rayleigh friction in the explicit part)
template <int D>
struct PwFriction {
  long n, ld;
  const double* U;
  const double* tau;
  double uref;
  double* R;
  __device__ void operator()(long e) const {
    const double t = tau[e];
    if (t == 0.0) return;
    R[ld + e] -= t * (U[ld + e] - U[e] * uref);
#pragma unroll
    for (int l = 1; l < D; ++l) R[(1 + l) * ld + e] -= t * U[(1 + l) * ld + e];
  }
};

template <int D>
struct PwFiMomentum {
  long n, ld;
  const double* q;
  const double* U;
  const double* rbar;
  double* F;
  __device__ void operator()(long e) const {
    F[e] = 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) F[(1 + l) * ld + e] = -q[l * ld + e];
    F[D * ld + e] -= (U[e] - rbar[e]) * kG;
  }
};

// stage predictor from nj previous stages; Us[0] <- rho_i, mt, et, mp
template <int D>
struct PwPredictor {
  long n, ld;
  const double* U;
  const double* FE0;
  const double* FE1;
  const double* FI0;
  const double* FI1;
  int nj;
  double a0, a1, t0, t1, dt, dta;
  const double* rbar;
  double* Us;
  double* mt;
  double* et;
  double* mp;
  __device__ void operator()(long e) const {
    double rho = FE0[e] * a0;
    if (nj > 1) rho += FE1[e] * a1;
    rho = U[e] + dt * rho;
    Us[e] = rho;
#pragma unroll
    for (int f = 1; f < D + 2; ++f) {
      double s = a0 * FE0[f * ld + e] + t0 * FI0[f * ld + e];
      if (nj > 1) s += a1 * FE1[f * ld + e] + t1 * FI1[f * ld + e];
      const double v = U[f * ld + e] + dt * s;
      if (f <= D) {
        mt[(f - 1) * ld + e] = v;
        mp[(f - 1) * ld + e] = v;
      } else {
        et[e] = v;
      }
    }
    mp[(D - 1) * ld + e] -= dta * (rho - rbar[e]) * kG;
  }
};

// stage start: copy the momentum of U^n
template <int D>
struct PwCopyM {
  long n, ld;
  const double* src;
  double* dst;
  __device__ void operator()(long e) const {
#pragma unroll
    for (int l = 0; l < D; ++l) dst[(1 + l) * ld + e] = src[(1 + l) * ld + e];
  }
};

// coefficients of the fixed-point iterate: h, Jacobi diagonal (inverse), FP32 copies
struct PwCoef {
  long n;
  const double* rho;
  const double* pbar;
  const double* pp;
  const double* wJ;
  const int4* cell;
  int nloc, dim;
  double L0, L1, L2;
  int n0, n1, n2, r1;
  double dta;
  double* h;
  double* dinv;
  float* h32;
  float* dinv32;
  __device__ void operator()(long e) const {
    const double hv = kGamma * (pbar[e] + pp[e]) / ((kGamma - 1.0) * rho[e]);
    const int lev = cell[e / nloc].x;
    const double d0 = L0 / (double)(n0 << lev), d1 = L1 / (double)(n1 << lev);
    double S = (r1 / d0) * (r1 / d0) + (r1 / d1) * (r1 / d1);
    if (dim == 3) {
      const double d2 = L2 / (double)(n2 << lev);
      S += (r1 / d2) * (r1 / d2);
    }
    const double dv = 1.0 / (wJ[e] * (1.0 / (kGamma - 1.0) + dta * dta * hv * S));
    h[e] = hv;
    dinv[e] = dv;
    if (h32) {
      h32[e] = (float)hv;
      dinv32[e] = (float)dv;
    }
  }
};

template <int D>
struct PwRhsAdd {
  long n, ld;
  double* b;
  const double* wJ;
  const double* et;
  const double* Us;
  const double* pbar;
  __device__ void operator()(long e) const {
    const double rho = Us[e];
    double m2 = 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) m2 += Us[(1 + l) * ld + e] * Us[(1 + l) * ld + e];
    b[e] += wJ[e] * (et[e] - 0.5 * m2 / rho - pbar[e] / (kGamma - 1.0));
  }
};

struct PwSub {  // out = a - b
  long n;
  const double* a;
  const double* b;
  double* out;
  __device__ void operator()(long e) const { out[e] = a[e] - b[e]; }
};
struct PwAdd {  // a += b
  long n;
  double* a;
  const double* b;
  __device__ void operator()(long e) const { a[e] += b[e]; }
};
struct PwZero {
  long n;
  double* a;
  __device__ void operator()(long e) const { a[e] = 0.0; }
};
struct PwCopy {
  long n;
  const double* a;
  double* out;
  __device__ void operator()(long e) const { out[e] = a[e]; }
};
struct PwWiden {
  long n;
  const float* a;
  double* out;
  __device__ void operator()(long e) const { out[e] = (double)a[e]; }
};
struct PwScaleCast {  // out = (float)(s a)
  long n;
  const double* a;
  double s;
  float* out;
  __device__ void operator()(long e) const { out[e] = (float)(s * a[e]); }
};
// flag = 1 if any of x[0..n) is not finite (every writer stores the same value)
struct PwNonfinite {
  long n;
  const double* x;
  double* flag;
  __device__ void operator()(long e) const {
    if (!isfinite(x[e])) *flag = 1.0;
  }
};

// Background enthalpy hbar = gamma pbar / ((gamma - 1) rhobar) and its height derivative from the
// closed form of the hydrostatic background: -g + c_p T N^2 / g (stratified), 0 (isothermal).
__global__ void k_hbar(const double* __restrict__ pbar, const double* __restrict__ rbar, int strat, double Nbv,
                       long N, double* __restrict__ hb, double* __restrict__ dhb, float* __restrict__ hb32,
                       float* __restrict__ dhb32) {
  GRID_LOOP(e, N) {
    const double h = kGamma * pbar[e] / ((kGamma - 1.0) * rbar[e]);
    const double T = pbar[e] / (kR * rbar[e]);
    const double d = strat ? -kG + kGamma * kR / (kGamma - 1.0) * T * Nbv * Nbv / kG : 0.0;
    hb[e] = h;
    dhb[e] = d;
    if (hb32) {
      hb32[e] = (float)h;
      dhb32[e] = (float)d;
    }
  }
}

// momentum back-substitution m = m' - dt a q (q = M^-1 B p')
template <int D>
struct PwBacksub {
  long n, ld;
  const double* mp;
  const double* q;
  double dta;
  double* Us;
  __device__ void operator()(long e) const {
#pragma unroll
    for (int l = 0; l < D; ++l) Us[(1 + l) * ld + e] = mp[l * ld + e] - dta * q[l * ld + e];
  }
};

template <int D>
struct PwStageFinish {
  long n, ld;
  double* Us;
  const double* pp;
  const double* pbar;
  const double* mt;
  const double* et;
  double dta;
  double* FI;
  __device__ void operator()(long e) const {
    const double rho = Us[e];
    double m2 = 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) {
      const double m = Us[(1 + l) * ld + e];
      m2 += m * m;
      FI[(1 + l) * ld + e] = (m - mt[l * ld + e]) / dta;
    }
    const double E = (pbar[e] + pp[e]) / (kGamma - 1.0) + 0.5 * m2 / rho;
    Us[(1 + D) * ld + e] = E;
    FI[(1 + D) * ld + e] = (E - et[e]) / dta;
    FI[e] = 0.0;
  }
};

template <int D>
struct PwFinal {
  long n, ld;
  const double* U;
  const double* FE0;
  const double* FE1;
  const double* FE2;
  const double* FI0;
  const double* FI1;
  const double* FI2;
  double b0, b1, b2, dt;
  double* Un;
  __device__ void operator()(long e) const {
    Un[e] = U[e] + dt * (b0 * FE0[e] + b1 * FE1[e] + b2 * FE2[e]);
#pragma unroll
    for (int f = 1; f < D + 2; ++f) {
      const long i = f * ld + e;
      Un[i] = U[i] + dt * ((b0 * FE0[i] + b1 * FE1[i] + b2 * FE2[i]) + (b0 * FI0[i] + b1 * FI1[i] + b2 * FI2[i]));
    }
  }
};

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator: the output mix of the state
// seed + G k.  A node's deviates are keyed by the seed, its cell's (level, i_x, i_y, i_z) and its
// index in the cell, so the noise field does not depend on the cell order or on the launch.
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
constexpr uint64_t kSmGolden = 0x9e3779b97f4a7c15ull;

// Standard normal deviate of node q of a cell with table entry (level, i_x, i_y, i_z) (Box-Muller).
__device__ __forceinline__ double node_normal(uint64_t seed, int4 cl, int D, int q) {
  const int iy = D == 3 ? cl.z : 0, iz = D == 3 ? cl.w : cl.z;
  uint64_t k = sm64_mix(seed + kSmGolden * (uint64_t)(cl.x + 1));
  k = sm64_mix(k + kSmGolden * (uint64_t)(cl.y + 1));
  k = sm64_mix(k + kSmGolden * (uint64_t)(iy + 1));
  k = sm64_mix(k + kSmGolden * (uint64_t)(iz + 1));
  k = sm64_mix(k + kSmGolden * (uint64_t)(q + 1));
  const double u1 = (double)(sm64_mix(k + kSmGolden) >> 11) * 0x1.0p-53;
  const double u2 = (double)(sm64_mix(k + 2 * kSmGolden) >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * kPi * u2);
}

// Hydrostatic background with uniform wind; with sigma > 0 the temperature of every node is
// perturbed by sigma n at constant pressure.
template <int D>
__global__ void k_init_state(const double* __restrict__ pbar, const double* __restrict__ rbar,
                             const int4* __restrict__ cell, int nloc, uint64_t seed, double sigma,
                             double ubar, long N, long ld, double* __restrict__ U) {
  GRID_LOOP(e, N) {
    double rho = rbar[e];
    if (sigma > 0.0) {
      const double T = pbar[e] / (kR * rbar[e]) + sigma * node_normal(seed, cell[e / nloc], D, (int)(e % nloc));
      rho = pbar[e] / (kR * T);
    }
    U[e] = rho;
    U[ld + e] = rho * ubar;
#pragma unroll
    for (int l = 1; l < D; ++l) U[(1 + l) * ld + e] = 0.0;
    U[(1 + D) * ld + e] = pbar[e] / (kGamma - 1.0) + 0.5 * rho * ubar * ubar;
  }
}

inline dim3 pw_grid(long n) {
  long g = (n + 255) / 256;
  return dim3((unsigned)std::max(1L, std::min(g, 65536L)));
}

// ------------------------------------------------------------------------------ basis tables
// Gauss-Legendre points by Newton's method on P_n (long double), Lagrange basis on them.
void gauss_legendre(int n, std::vector<long double>& x, std::vector<long double>& w) {
  x.assign(n, 0);
  w.assign(n, 0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double z = std::cos(pi * (4 * i + 3) / (4 * n + 2));
    long double dp = 1;
    for (int it = 0; it < 200; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      const long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2 / ((1 - z * z) * dp * dp);
  }
}

long double lagrange(const std::vector<long double>& xs, int j, long double t) {
  long double v = 1;
  for (size_t m = 0; m < xs.size(); ++m)
    if ((int)m != j) v *= (t - xs[m]) / (xs[j] - xs[m]);
  return v;
}
long double lagrange_d(const std::vector<long double>& xs, int j, long double t) {
  // derivative via the product rule
  long double s = 0;
  for (size_t m = 0; m < xs.size(); ++m) {
    if ((int)m == j) continue;
    long double term = 1 / (xs[j] - xs[m]);
    for (size_t q = 0; q < xs.size(); ++q)
      if ((int)q != j && q != m) term *= (t - xs[q]) / (xs[j] - xs[q]);
    s += term;
  }
  return s;
}

// Local block of the 1D second-order operator B^T W^-1 B of the weak gradient with central
// fluxes (the 1D analogue of -C M^-1 B at h = 1) on the reference cell [-1, 1], taken from a
// periodic row of three cells, and the generalised eigenpairs L s = mu W s (S^T W S = I) by
// Jacobi rotations on W^-1/2 L W^-1/2.
void fdm_eigen(int np, const std::vector<long double>& x, const std::vector<long double>& w,
               std::vector<double>& S, std::vector<double>& mu) {
  const int nc = 3, n = nc * np;
  std::vector<long double> B((size_t)n * n, 0.0L), lm(np), lp(np);
  for (int a = 0; a < np; ++a) {
    lm[a] = lagrange(x, a, -1.0L);
    lp[a] = lagrange(x, a, 1.0L);
  }
  for (int K = 0; K < nc; ++K) {
    const int Kp = (K + 1) % nc, Km = (K + nc - 1) % nc;
    for (int i = 0; i < np; ++i)
      for (int j = 0; j < np; ++j) {
        B[(size_t)(K * np + i) * n + K * np + j] += -w[j] * lagrange_d(x, i, x[j]) + 0.5L * (lp[i] * lp[j] - lm[i] * lm[j]);
        B[(size_t)(K * np + i) * n + Kp * np + j] += 0.5L * lp[i] * lm[j];
        B[(size_t)(K * np + i) * n + Km * np + j] -= 0.5L * lm[i] * lp[j];
      }
  }
  // L = (B^T W^-1 B) restricted to the middle cell
  std::vector<long double> A((size_t)np * np, 0.0L);
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      long double t = 0.0L;
      for (int r = 0; r < n; ++r)
        t += B[(size_t)r * n + np + i] * B[(size_t)r * n + np + j] / w[r % np];
      A[(size_t)i * np + j] = t / std::sqrt(w[i] * w[j]);  // W^-1/2 L W^-1/2
    }
  std::vector<long double> V((size_t)np * np, 0.0L);
  for (int i = 0; i < np; ++i) V[(size_t)i * np + i] = 1.0L;
  for (int sweep = 0; sweep < 100; ++sweep) {
    long double off = 0.0L;
    for (int p = 0; p < np; ++p)
      for (int q = p + 1; q < np; ++q) off += A[(size_t)p * np + q] * A[(size_t)p * np + q];
    if (off < 1e-36L) break;
    for (int p = 0; p < np; ++p)
      for (int q = p + 1; q < np; ++q) {
        const long double apq = A[(size_t)p * np + q];
        if (std::fabs((double)apq) < 1e-300) continue;
        const long double th = (A[(size_t)q * np + q] - A[(size_t)p * np + p]) / (2.0L * apq);
        const long double t = (th >= 0 ? 1.0L : -1.0L) / (std::fabs((double)th) + std::sqrt(th * th + 1.0L));
        const long double c = 1.0L / std::sqrt(t * t + 1.0L), sn = t * c;
        for (int k = 0; k < np; ++k) {  // rotate columns p, q
          const long double akp = A[(size_t)k * np + p], akq = A[(size_t)k * np + q];
          A[(size_t)k * np + p] = c * akp - sn * akq;
          A[(size_t)k * np + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < np; ++k) {  // rotate rows p, q
          const long double apk = A[(size_t)p * np + k], aqk = A[(size_t)q * np + k];
          A[(size_t)p * np + k] = c * apk - sn * aqk;
          A[(size_t)q * np + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < np; ++k) {
          const long double vkp = V[(size_t)k * np + p], vkq = V[(size_t)k * np + q];
          V[(size_t)k * np + p] = c * vkp - sn * vkq;
          V[(size_t)k * np + q] = sn * vkp + c * vkq;
        }
      }
  }
  S.assign((size_t)np * np, 0.0);
  mu.assign(np, 0.0);
  for (int a = 0; a < np; ++a) {
    mu[a] = (double)A[(size_t)a * np + a];
    for (int i = 0; i < np; ++i) S[(size_t)i * np + a] = (double)(V[(size_t)i * np + a] / std::sqrt(w[i]));
  }
}

// Over-integration table (OiLayout): NQ Gauss points and weights, the nodal basis and its
// derivative at the points, and the basis at the points mapped into either half of [-1, 1].
std::vector<double> make_oi_tables(int np, int nq) {
  OiLayout L{np, nq};
  std::vector<double> t(L.size(), 0.0);
  std::vector<long double> x, w, xq, wq;
  gauss_legendre(np, x, w);
  gauss_legendre(nq, xq, wq);
  for (int q = 0; q < nq; ++q) {
    t[L.xq() + q] = (double)xq[q];
    t[L.wq() + q] = (double)wq[q];
    for (int j = 0; j < np; ++j) {
      t[L.bq() + q * np + j] = (double)lagrange(x, j, xq[q]);
      t[L.dq() + q * np + j] = (double)lagrange_d(x, j, xq[q]);
      for (int h = 0; h < 2; ++h)
        t[L.bs() + (h * nq + q) * np + j] = (double)lagrange(x, j, (xq[q] + 2 * h - 1) / 2);
    }
  }
  return t;
}

std::vector<double> make_tables(int np) {
  TabLayout TL{np};
  std::vector<double> t(TL.size(), 0.0);
  std::vector<long double> x, w;
  gauss_legendre(np, x, w);
  for (int i = 0; i < np; ++i) {
    t[TL.xi() + i] = (double)x[i];
    t[TL.w() + i] = (double)w[i];
  }
  for (int i = 0; i < np; ++i)
    for (int q = 0; q < np; ++q) t[TL.dt() + i * np + q] = (double)(w[q] * lagrange_d(x, i, x[q]) / w[i]);
  for (int s = 0; s < 2; ++s)
    for (int a = 0; a < np; ++a) {
      const long double v = lagrange(x, a, s ? 1.0L : -1.0L);
      t[TL.lb() + s * np + a] = (double)v;
      t[TL.lbw() + s * np + a] = (double)(v / w[a]);
    }
  for (int c = 0; c < 2; ++c)
    for (int j = 0; j < np; ++j)
      for (int a = 0; a < np; ++a) {
        const long double pt = (x[j] + 2 * c - 1) / 2;
        const long double v = lagrange(x, a, pt);
        t[TL.pi() + (c * np + j) * np + a] = (double)v;
        t[TL.rw() + (c * np + a) * np + j] = (double)(w[j] / w[a] * v);
      }
  std::vector<double> S, mu;
  fdm_eigen(np, x, w, S, mu);
  for (int i = 0; i < np * np; ++i) t[TL.fds() + i] = S[i];
  for (int a = 0; a < np; ++a) t[TL.fdmu() + a] = mu[a];
  return t;
}

}  // namespace
}  // namespace dg

// ====================================================================================== context
using namespace dg;

struct dg_ctx {
  HostMesh hm;
  dg_case_desc desc{};
  dg_options opt{};
  int degree = 0, D = 0, F = 0, NL = 0;
  long N = 0, ld = 0;
  hipStream_t stream = nullptr;
  bool timing = false;
  MeshDev md{};
  MeshDev* d_md = nullptr;  // device copy of md (shared launches read the members' views there)
  char* arena = nullptr;
  size_t arena_bytes = 0;
  // mesh
  int4* d_cell = nullptr;
  int* d_fkind = nullptr;
  int4* d_fnbr = nullptr;
  int* d_lists = nullptr;  // cells with conforming faces only, then cells with a 2:1 face
  int* d_runs = nullptr;   // vertical runs for the gradient column kernel (cells, then flags)
  int nrun_slots = 0;
  double* d_tab = nullptr;
  float* d_tabf = nullptr;
  double* d_oitab = nullptr;  // over-integration table (quad_extra > 0)
  // geometry / background
  double *pbar = nullptr, *rbar = nullptr, *wJ = nullptr;
  double* tau = nullptr;  // absorbing-layer rate per node (only with an absorbing layer)
  // enthalpy split: background enthalpy, its height derivative, h - hbar (FP64 / FP32 copies)
  double *hb = nullptr, *dhb = nullptr, *hp = nullptr;
  float *hb32 = nullptr, *dhb32 = nullptr, *hp32 = nullptr;
  // step workspace
  double* FE[3] = {nullptr, nullptr, nullptr};
  double* FI[3] = {nullptr, nullptr, nullptr};
  double *Us = nullptr, *Un = nullptr, *mt = nullptr, *et = nullptr, *mp = nullptr;
  double *pp = nullptr, *h = nullptr, *dinv = nullptr, *q = nullptr, *b = nullptr, *r0 = nullptr;
  double *delta = nullptr, *w = nullptr, *V = nullptr, *lam = nullptr, *z = nullptr;
  // mixed precision
  float *h32 = nullptr, *dinv32 = nullptr, *lam32 = nullptr, *q32 = nullptr, *w32 = nullptr, *V32 = nullptr;
  float* z32 = nullptr;
  double *coef = nullptr, *u = nullptr;
  float *coef32 = nullptr, *u32 = nullptr;
  double* rr = nullptr;
  // reductions: per-block partials; result slots of the members of a team this context leads
  // (device, and pinned host followed by the host staging of the update coefficients); the
  // coefficients of a shared update pass on the device
  double* part = nullptr;
  double* red = nullptr;
  double* hred = nullptr;
  double* tcoef = nullptr;
  int m = 30, m32 = 30;
  // per-launch HIP events (timing on): pairs around launches, tagged with a kernel class
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_cls;
  int ev_n = 0;
  double kbytes[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // per-phase HIP events (timing on): pairs around the phases of a step, tagged with the phase
  std::vector<hipEvent_t> pev;
  std::vector<int> pev_cls;
  int pev_n = 0;
  mutable std::string err;  // last error of a call on this context
};

namespace {

void set_error(const dg_ctx* c, const std::string& msg) {
  g_last_error = msg;
  if (c) c->err = msg;
}

dg_status fail(const dg_ctx* c, dg_status st, const std::string& msg) {
  set_error(c, msg);
  return st;
}

// Device address of the scratch array on the current device, looked up once per device.
dg_status scratch_ptr(const dg_ctx* c, double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(c, DG_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, DG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

constexpr int kEvPool = 8192;

// Teams (lockstep members, see step_team) of at most kTeamMax members.
constexpr int kTeamMax = 32;
// per-member result slot in the lead context's reduction buffer: [0] |v|^2 and [1] 1/|v| of the
// Krylov candidate, [2, 2 + nv) the reduced values of the last reduction, [kFlagAt] the non-finite
// flag of the new state, [kMaxAt] max |w|
constexpr int kResStride = 72;
constexpr int kFlagAt = 68, kMaxAt = 69;
constexpr int kCoefStride = 2 * kMaxV;
static_assert(2 + 2 * (kMaxV - 2) + 3 <= kFlagAt, "result slot too small");  // restart <= kMaxV - 1

// Records a HIP event pair around the launches of its scope when timing is on.
struct Timed {
  dg_ctx* c;
  int slot = -1;
  Timed(dg_ctx* c_, int cls, double bytes = 0.0) : c(c_) {
    if (!c) return;
    if (c->timing) c->kbytes[cls] += bytes;
    if (c->timing && c->ev_n < kEvPool) {
      slot = c->ev_n++;
      c->ev_cls[slot] = cls;
      (void)hipEventRecord(c->ev[2 * slot], c->stream);
    }
  }
  ~Timed() {
    if (slot >= 0) (void)hipEventRecord(c->ev[2 * slot + 1], c->stream);
  }
};
// Records a HIP event pair around a phase of the step when timing is on.
constexpr int kPhasePool = 512;
struct Phase {
  dg_ctx* c;
  int slot = -1;
  Phase(dg_ctx* c_, int ph) : c(c_) {
    if (c && c->timing && c->pev_n < kPhasePool) {
      slot = c->pev_n++;
      c->pev_cls[slot] = ph;
      (void)hipEventRecord(c->pev[2 * slot], c->stream);
    }
  }
  void end() {
    if (slot >= 0) (void)hipEventRecord(c->pev[2 * slot + 1], c->stream);
    slot = -1;
  }
  ~Phase() { end(); }
};

#define TIMED(cls, stmt) \
  do {                   \
    Timed t_(c, cls);    \
    stmt;                \
  } while (0)
// with the algorithmic bytes of the launch
#define TIMEDB(cls, bytes, stmt) \
  do {                           \
    Timed t_(c, cls, bytes);     \
    stmt;                        \
  } while (0)

#define HIPCHK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      set_error(c, std::string(#call) + ": " + hipGetErrorString(e_));          \
      return DG_EDEVICE;                                                          \
    }                                                                             \
  } while (0)
#define LCHK(call)                                                                \
  do {                                                                            \
    int e_ = (call);                                                              \
    if (e_ != 0) {                                                                \
      set_error(c, std::string("launch failed: ") + #call);                     \
      return e_ == -6 ? DG_EUNSUPPORTED : DG_EDEVICE;                             \
    }                                                                             \
  } while (0)

struct Plan {
  std::vector<std::pair<void**, size_t>> items;
  size_t total = 0;
  void add(void** p, size_t bytes) {
    items.push_back({p, bytes});
    total += (bytes + 255) & ~size_t(255);
  }
};

// Cells per workgroup of the Helmholtz column kernels, and the padded length of their run lists.
int col_cpb(const dg_ctx* c) {
  int nc = 1;
  for (int a = 0; a < c->D - 1; ++a) nc *= c->degree + 1;
  return 256 / nc;
}
long run_slots(const dg_ctx* c) {
  const long cpb = col_cpb(c);
  return (c->hm.ncell + cpb - 1) / cpb * cpb;
}

// Vertical runs for the gradient column kernel (Helmholtz pass 1): chains of cells joined by conforming bottom /
// top faces, taken from bottom to top in the order of their lowest cell (Morton), concatenated and
// cut into workgroups of cpb cells.  A cell's flag says whether its bottom (bit 0) or top (bit 1)
// neighbour sits in the previous or next slot of the same workgroup, where the kernel reads that
// neighbour's face trace from LDS instead of gathering its vertical line.
void build_runs(const HostMesh& M, int D, int cpb, std::vector<int>& runs, std::vector<int>& flags) {
  const int NF = 2 * D, fb = 2 * (D - 1), ft = fb + 1;
  const long n = M.ncell;
  std::vector<int> up(n, -1), down(n, -1);
  for (long i = 0; i < n; ++i) {
    if (M.fkind[i * NF + ft] == kConf) up[i] = M.fnbr[(i * NF + ft) * 4];
    if (M.fkind[i * NF + fb] == kConf) down[i] = M.fnbr[(i * NF + fb) * 4];
  }
  runs.clear();
  runs.reserve(n);
  for (long i = 0; i < n; ++i) {
    if (down[i] >= 0) continue;  // not the lowest cell of its chain
    long steps = 0;
    for (long j = i; j >= 0 && steps <= n; j = up[j], ++steps) runs.push_back((int)j);
  }
  const long slots = (n + cpb - 1) / cpb * cpb;
  runs.resize(slots, -1);
  flags.assign(slots, 0);
  for (long k = 0; k < slots; ++k) {
    const int cc = runs[k];
    if (cc < 0) continue;
    if (k % cpb != 0 && runs[k - 1] >= 0 && down[cc] == runs[k - 1]) flags[k] |= 1;
    if ((k + 1) % cpb != 0 && k + 1 < slots && runs[k + 1] >= 0 && up[cc] == runs[k + 1]) flags[k] |= 2;
  }
}

// Every device allocation of a context, in bytes; used by dg_setup and dg_footprint.
void make_plan(dg_ctx* c, Plan& P) {
  const int D = c->D, F = c->F;
  const long ld = c->ld;
  const size_t nc = (size_t)c->hm.ncell;
  const size_t d8 = sizeof(double), f4 = sizeof(float);
  TabLayout TL{c->degree + 1};
  P.add((void**)&c->d_cell, nc * sizeof(int4));
  P.add((void**)&c->d_fkind, nc * 2 * D * sizeof(int));
  P.add((void**)&c->d_lists, nc * sizeof(int));
  P.add((void**)&c->d_runs, (size_t)2 * run_slots(c) * sizeof(int));
  P.add((void**)&c->d_fnbr, nc * 2 * D * sizeof(int4));
  P.add((void**)&c->d_tab, TL.size() * d8);
  P.add((void**)&c->d_tabf, TL.size() * f4);
  if (c->opt.quad_extra > 0) P.add((void**)&c->d_oitab, OiLayout{c->degree + 1, c->degree + 1 + c->opt.quad_extra}.size() * d8);
  P.add((void**)&c->pbar, ld * d8);
  P.add((void**)&c->rbar, ld * d8);
  P.add((void**)&c->wJ, ld * d8);
  if (c->desc.sponge[1] > 0.0 || c->desc.sponge[3] > 0.0) P.add((void**)&c->tau, ld * d8);
  if (c->opt.enthalpy_split) {
    P.add((void**)&c->hb, ld * d8);
    P.add((void**)&c->dhb, ld * d8);
    P.add((void**)&c->hp, ld * d8);
    if (c->opt.precision == DG_FP32_INNER) {
      P.add((void**)&c->hb32, ld * f4);
      P.add((void**)&c->dhb32, ld * f4);
      P.add((void**)&c->hp32, ld * f4);
    }
  }
  for (int j = 0; j < 3; ++j) {
    P.add((void**)&c->FE[j], F * ld * d8);
    P.add((void**)&c->FI[j], F * ld * d8);
  }
  P.add((void**)&c->Us, F * ld * d8);
  P.add((void**)&c->Un, F * ld * d8);
  P.add((void**)&c->mt, D * ld * d8);
  P.add((void**)&c->et, ld * d8);
  P.add((void**)&c->mp, D * ld * d8);
  P.add((void**)&c->pp, ld * d8);
  P.add((void**)&c->h, ld * d8);
  P.add((void**)&c->dinv, ld * d8);
  P.add((void**)&c->q, D * ld * d8);
  P.add((void**)&c->b, ld * d8);
  P.add((void**)&c->r0, ld * d8);
  P.add((void**)&c->delta, ld * d8);
  P.add((void**)&c->w, ld * d8);
  P.add((void**)&c->lam, nc * d8);
  P.add((void**)&c->z, ld * d8);
  P.add((void**)&c->coef, nc * 4 * d8);
  P.add((void**)&c->u, ld * d8);
  if (c->opt.precision == DG_FP32_INNER) {
    P.add((void**)&c->V, 1 * ld * d8);  // outer residual work
    P.add((void**)&c->rr, ld * d8);
    P.add((void**)&c->h32, ld * f4);
    P.add((void**)&c->dinv32, ld * f4);
    P.add((void**)&c->lam32, nc * f4);
    P.add((void**)&c->q32, D * ld * f4);
    P.add((void**)&c->w32, ld * f4);
    P.add((void**)&c->z32, ld * f4);
    P.add((void**)&c->coef32, nc * 4 * f4);
    P.add((void**)&c->u32, ld * f4);
    P.add((void**)&c->V32, (size_t)(c->m32 + 1) * ld * f4);
  } else {
    P.add((void**)&c->V, (size_t)(c->m + 1) * ld * d8);
  }
  P.add((void**)&c->part, (size_t)(2 * kMaxV + 3) * kMaxGrid * d8);
  P.add((void**)&c->red, (size_t)kTeamMax * kResStride * d8);
  P.add((void**)&c->tcoef, (size_t)kTeamMax * kCoefStride * d8);
  P.add((void**)&c->d_md, sizeof(MeshDev));
}

dg_status prepare(dg_ctx* c, const dg_case_desc* desc, int degree, const dg_options* opt) {
  if (!desc) return fail(c, DG_EINVAL, "null description");
  c->desc = *desc;
  if (opt) c->opt = *opt;
  else dg_default_options(&c->opt);
  const dg_options& o = c->opt;
  if (o.fp_iters < 1 || o.fp_iters > 8) return fail(c, DG_EINVAL, "fp_iters must be in [1, 8]");
  if (desc->n_rules > kMaxLev - 1) return fail(c, DG_EINVAL, "at most 8 refinement levels");
  if (!(desc->oro[1] > 0.0) && desc->orography != DG_ORO_FLAT) return fail(c, DG_EINVAL, "orography width must be positive");
  if (o.gmres_restart < 1 || o.gmres_restart > kMaxV - 1) return fail(c, DG_EINVAL, "gmres_restart must be in [1, 31]");
  if (o.inner_restart < 1 || o.inner_restart > kMaxV - 1) return fail(c, DG_EINVAL, "inner_restart must be in [1, 31]");
  if (o.precision != DG_FP64 && o.precision != DG_FP32_INNER) return fail(c, DG_EINVAL, "bad precision");
  if (o.quad_extra < 0) return fail(c, DG_EINVAL, "quad_extra must be >= 0");
  if (o.enthalpy_split != 0 && o.enthalpy_split != 1) return fail(c, DG_EINVAL, "enthalpy_split must be 0 or 1");
  if (o.quad_extra > 3 || degree + 1 + o.quad_extra > kMaxNq)
    return fail(c, DG_EUNSUPPORTED, "over-integration needs quad_extra <= 3 and degree + 1 + quad_extra <= 8");
  if (o.preconditioner != DG_PREC_DIAGONAL && o.preconditioner != DG_PREC_CELL_FDM)
    return fail(c, DG_EINVAL, "bad preconditioner");
  if (desc->orography < 0 || desc->orography > 4) return fail(c, DG_EINVAL, "bad orography kind");
  for (int i = 0; i < 4; ++i)
    if (!(desc->sponge[i] >= 0.0)) return fail(c, DG_EINVAL, "absorbing-layer sizes and rates must be >= 0");
  if (desc->sponge[1] > 0.0 && !(desc->sponge[0] > 0.0 && desc->sponge[0] <= desc->length[2]))
    return fail(c, DG_EINVAL, "top absorbing layer needs 0 < depth <= H");
  if (!std::isfinite(desc->sponge[4])) return fail(c, DG_EINVAL, "absorbing-layer reference wind must be finite");
  if (desc->atmosphere < 0 || desc->atmosphere > 1) return fail(c, DG_EINVAL, "bad atmosphere kind");
  if (desc->oro[0] >= desc->length[2]) return fail(c, DG_EINVAL, "orography higher than the lid");
  std::string err;
  const int rc = build_mesh(c->desc, degree, c->hm, err);
  if (rc != DG_OK) return fail(c, (dg_status)rc, err);
  c->degree = degree;
  c->D = c->hm.dim;
  c->F = c->D + 2;
  c->NL = c->hm.nloc;
  c->N = (long)c->hm.ncell * c->NL;
  c->ld = c->N;  // fields are contiguous: U[f][cell][node]
  c->m = o.gmres_restart;
  c->m32 = o.inner_restart;
  return DG_OK;
}

// ------------------------------------------------------------------------------ lockstep teams
// A team is a set of members (contexts of one class: dimension, degree, precision, preconditioner
// and energy-flux form) advanced through the step in lockstep on one stream.  A team of one with
// direct launches is the single-context step.  Otherwise every operator, Krylov and pointwise
// launch of the step is shared by the members through segment tables, and each host round trip of
// the Krylov iteration serves all of them.  Members keep their own control flow (iteration
// counts, convergence, restarts, failures) by taking part only in the launches they need, and
// their own grid shapes, so a member's results are the same bits alone and in any mix.

struct Team {
  std::vector<dg_ctx*> m;
  hipStream_t s = nullptr;
  bool shared = false;
  dg_ctx* lead = nullptr;
  dg_ctx* tc = nullptr;  // context whose events time the launches (direct launches, timing on)
  std::vector<dg_status> st;
  double* slot(int k) const { return lead->red + (size_t)k * kResStride; }
  const double* hslot(int k) const { return lead->hred + (size_t)k * kResStride; }
  double* hcoef(int k) const { return lead->hred + (size_t)kTeamMax * kResStride + (size_t)k * kCoefStride; }
  const double* dcoef(int k) const { return lead->tcoef + (size_t)k * kCoefStride; }
  bool alive(int k) const { return st[k] == DG_OK; }
  int n() const { return (int)m.size(); }
};

Team solo(dg_ctx* c) {
  Team T;
  T.m = {c};
  T.s = c->stream;
  T.lead = c;
  T.tc = c->timing ? c : nullptr;
  T.st.assign(1, DG_OK);
  return T;
}

// A member leaves the step with an error of its own; the others go on.
void drop(Team& Tm, int k, dg_status rc, const std::string& why) {
  if (!Tm.alive(k)) return;
  Tm.st[k] = rc;
  set_error(Tm.m[k], why);
}
// A failed launch or copy ends the step for every member.
dg_status team_fail(Team& Tm, dg_status rc, const std::string& why) {
  for (int k = 0; k < Tm.n(); ++k) drop(Tm, k, rc, why);
  return rc;
}
#define TCHK(team, call)                                                                    \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return team_fail(team, DG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

std::vector<int> alive_of(const Team& Tm, const std::vector<int>& act) {
  std::vector<int> r;
  for (int k : act)
    if (Tm.alive(k)) r.push_back(k);
  return r;
}

// The members' result slots to the host (one copy, one synchronisation).
dg_status fetch(Team& Tm, const std::vector<int>& act) {
  int hi = -1;
  for (int k : act) hi = std::max(hi, k);
  if (hi < 0) return DG_OK;
  TCHK(Tm, hipMemcpyAsync(Tm.lead->hred, Tm.lead->red, (size_t)(hi + 1) * kResStride * sizeof(double),
                      hipMemcpyDeviceToHost, Tm.s));
  TCHK(Tm, hipStreamSynchronize(Tm.s));
  return DG_OK;
}

// Pointwise functor per member: a direct launch each, or shared launches.
template <class F, class Make>
dg_status pw(Team& Tm, const std::vector<int>& act, Make mk) {
  if (act.empty()) return DG_OK;
  if (!Tm.shared) {
    for (int k : act) {
      const F f = mk(k);
      Timed t_(Tm.tc, 4);
      hipLaunchKernelGGL((k_pw<F>), pw_grid(f.n), dim3(256), 0, Tm.s, f);
    }
  } else {
    std::vector<F> fs;
    fs.reserve(act.size());
    for (int k : act) fs.push_back(mk(k));
    seg_launch<F>((int)fs.size(), nullptr, [&](int i) { return (int)pw_grid(fs[i].n).x; },
                  [&](int i) { return fs[i]; },
                  [&](const SegTab<F>& t, int g) {
                    hipLaunchKernelGGL((k_pw_seg<F>), dim3(g), dim3(256), 0, Tm.s, Shared<F>{t});
                    return 0;
                  });
  }
  TCHK(Tm, hipGetLastError());
  return DG_OK;
}

// Operator per member: the single-mesh launcher (direct), or the shared launcher, which answers
// -6 when the arguments need the general cell kernel (then one launch per member).
template <class A, class Make, class Bytes, class One, class Many>
dg_status op_launch(Team& Tm, const std::vector<int>& act, int cls, Make mk, Bytes bytes, One one, Many many) {
  if (act.empty()) return DG_OK;
  if (!Tm.shared) {
    for (int k : act) {
      const A a = mk(k);
      int r;
      {
        Timed t_(Tm.tc, cls, bytes(k));
        r = one(Tm.m[k], a);
      }
      if (r) return team_fail(Tm, r == -6 ? DG_EUNSUPPORTED : DG_EDEVICE, "operator launch failed");
    }
    return DG_OK;
  }
  std::vector<A> as;
  std::vector<const MeshDev*> mh, md;
  for (int k : act) {
    as.push_back(mk(k));
    mh.push_back(&Tm.m[k]->md);
    md.push_back(Tm.m[k]->d_md);
  }
  int r = many((int)as.size(), mh.data(), md.data(), as.data());
  if (r == -6) {
    r = 0;
    for (size_t i = 0; i < as.size() && !r; ++i) r = one(Tm.m[act[i]], as[i]);
  }
  if (r) return team_fail(Tm, r == -6 ? DG_EUNSUPPORTED : DG_EDEVICE, "operator launch failed");
  return DG_OK;
}

// Precision-dependent buffers and launchers.
template <class T> struct PrecBuf;
template <> struct PrecBuf<double> {
  static double* q(dg_ctx* c) { return c->q; }
  static double* h(dg_ctx* c) { return c->h; }
  static double* z(dg_ctx* c) { return c->z; }
  static double* lam(dg_ctx* c) { return c->lam; }
  static double* coef(dg_ctx* c) { return c->coef; }
  static double* hp(dg_ctx* c) { return c->hp; }
  static double* hb(dg_ctx* c) { return c->hb; }
  static double* dhb(dg_ctx* c) { return c->dhb; }
  static int grad(const MeshDev& m, int deg, const GradArgs<double>& a, hipStream_t s) { return launch_grad64(m, deg, a, s); }
  static int div(const MeshDev& m, int deg, const DivArgs<double>& a, hipStream_t s) { return launch_div64(m, deg, a, s); }
  static int div_split(const MeshDev& m, int deg, const DivArgs<double>& a, hipStream_t s) { return launch_div_split64(m, deg, a, s); }
  static int fdm(const MeshDev& m, int deg, const FdmArgs<double>& a, hipStream_t s) { return launch_fdm64(m, deg, a, s); }
  static constexpr auto grad_seg = launch_grad_seg64;
  static constexpr auto div_seg = launch_div_seg64;
  static constexpr auto div_split_seg = launch_div_split_seg64;
  static constexpr auto fdm_seg = launch_fdm_seg64;
};
template <> struct PrecBuf<float> {
  static float* q(dg_ctx* c) { return c->q32; }
  static float* h(dg_ctx* c) { return c->h32; }
  static float* z(dg_ctx* c) { return c->z32; }
  static float* lam(dg_ctx* c) { return c->lam32; }
  static float* coef(dg_ctx* c) { return c->coef32; }
  static float* hp(dg_ctx* c) { return c->hp32; }
  static float* hb(dg_ctx* c) { return c->hb32; }
  static float* dhb(dg_ctx* c) { return c->dhb32; }
  static int grad(const MeshDev& m, int deg, const GradArgs<float>& a, hipStream_t s) { return launch_grad32(m, deg, a, s); }
  static int div(const MeshDev& m, int deg, const DivArgs<float>& a, hipStream_t s) { return launch_div32(m, deg, a, s); }
  static int div_split(const MeshDev& m, int deg, const DivArgs<float>& a, hipStream_t s) { return launch_div_split32(m, deg, a, s); }
  static int fdm(const MeshDev& m, int deg, const FdmArgs<float>& a, hipStream_t s) { return launch_fdm32(m, deg, a, s); }
  static constexpr auto grad_seg = launch_grad_seg32;
  static constexpr auto div_seg = launch_div_seg32;
  static constexpr auto div_split_seg = launch_div_split_seg32;
  static constexpr auto fdm_seg = launch_fdm_seg32;
};

// Weak gradient per member (args from mk), timing class cls.
template <class T, class Make, class Bytes>
dg_status grad_team(Team& Tm, const std::vector<int>& act, int cls, Make mk, Bytes bytes) {
  using PB = PrecBuf<T>;
  const hipStream_t s = Tm.s;
  const int deg = act.empty() ? 0 : Tm.m[act[0]]->degree;
  return op_launch<GradArgs<T>>(
      Tm, act, cls, mk, bytes, [&](dg_ctx* c, const GradArgs<T>& a) { return PB::grad(c->md, c->degree, a, s); },
      [&](int n, const MeshDev* const* mh, const MeshDev* const* md, const GradArgs<T>* a) {
        return PB::grad_seg(n, mh, md, a, deg, s);
      });
}

// Weak divergence of the implicit energy flux h qv with the penalty / mass terms (a.h = h):
// plain C(h qv), or with the enthalpy split C((h - hbar) qv) + hbar C(qv) + M (d hbar/dz) qv_z,
// the latter in one column pass.
template <class T, class Make, class Bytes>
dg_status energy_div_team(Team& Tm, const std::vector<int>& act, int cls, Make mk, Bytes bytes) {
  using PB = PrecBuf<T>;
  const hipStream_t s = Tm.s;
  if (act.empty()) return DG_OK;
  const int deg = Tm.m[act[0]]->degree;
  if (!Tm.m[act[0]]->opt.enthalpy_split)
    return op_launch<DivArgs<T>>(
        Tm, act, cls, mk, bytes, [&](dg_ctx* c, const DivArgs<T>& a) { return PB::div(c->md, c->degree, a, s); },
        [&](int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<T>* a) {
          return PB::div_seg(n, mh, md, a, deg, s);
        });
  auto mk2 = [&](int k) {
    dg_ctx* c = Tm.m[k];
    DivArgs<T> a = mk(k);
    a.h = PB::hp(c);
    a.hb = PB::hb(c);
    a.dhb = PB::dhb(c);
    return a;
  };
  return op_launch<DivArgs<T>>(
      Tm, act, cls, mk2, bytes, [&](dg_ctx* c, const DivArgs<T>& a) { return PB::div_split(c->md, c->degree, a, s); },
      [&](int n, const MeshDev* const* mh, const MeshDev* const* md, const DivArgs<T>* a) {
        return PB::div_split_seg(n, mh, md, a, deg, s);
      });
}

// h - hbar for the enthalpy split, after h (and h32) changed
dg_status split_update_team(Team& Tm, const std::vector<int>& act) {
  if (act.empty() || !Tm.m[act[0]]->opt.enthalpy_split) return DG_OK;
  dg_status st = pw<PwSub>(Tm, act, [&](int k) { dg_ctx* c = Tm.m[k]; return PwSub{c->N, c->h, c->hb, c->hp}; });
  if (st || Tm.m[act[0]]->opt.precision != DG_FP32_INNER) return st;
  return pw<PwScaleCast>(Tm, act, [&](int k) { dg_ctx* c = Tm.m[k]; return PwScaleCast{c->N, c->hp, 1.0, c->hp32}; });
}

// One term of a Helmholtz application: w = A(h) p in precision T for member k.  With dinv == null
// and scale == 1, p = v is taken as given; else p = scale * dinv * v is formed on the fly and
// written to the z buffer by pass 1.
template <class T>
struct ApItem {
  int k;
  double dta;
  const T* v;
  const T* dinv;
  T scale;
  T* w;
  const double* dscale;  // preconditioned form: scale read from device memory (or null)
};

// Pass 1 writes h M^{-1} B p (and p); pass 2 takes C of it and the penalty and mass terms of p.
template <class T>
dg_status apply_A_team(Team& Tm, const std::vector<ApItem<T>>& it) {
  using PB = PrecBuf<T>;
  std::vector<int> act;
  std::vector<int> idx(Tm.n(), -1);
  for (size_t i = 0; i < it.size(); ++i) {
    act.push_back(it[i].k);
    idx[it[i].k] = (int)i;
  }
  auto given = [&](const ApItem<T>& e) { return e.dinv == nullptr && e.scale == T(1); };
  // pass 1: v (and dinv), h in; h M^-1 B p (d fields) and, if formed here, p out
  dg_status st = grad_team<T>(
      Tm, act, 1,
      [&](int k) {
        const ApItem<T>& e = it[idx[k]];
        dg_ctx* c = Tm.m[k];
        const bool split = c->opt.enthalpy_split != 0;
        return GradArgs<T>{e.v, e.dinv, e.scale, PB::q(c), split ? nullptr : PB::h(c), given(e) ? nullptr : PB::z(c)};
      },
      [&](int k) {
        const ApItem<T>& e = it[idx[k]];
        dg_ctx* c = Tm.m[k];
        return (double)sizeof(T) * c->N * ((e.dinv ? 2 : 1) + 1 + c->D + (given(e) ? 0 : 1));
      });
  if (st) return st;
  // pass 2: d fields and p in; A p out
  return energy_div_team<T>(
      Tm, act, 2,
      [&](int k) {
        const ApItem<T>& e = it[idx[k]];
        dg_ctx* c = Tm.m[k];
        const bool split = c->opt.enthalpy_split != 0;
        const double beta = c->opt.penalty_beta;
        return DivArgs<T>{PB::q(c), split ? PB::h(c) : nullptr, given(e) ? e.v : PB::z(c), nullptr, T(1), PB::lam(c),
                          (T)(-e.dta * e.dta), (T)(e.dta * beta / (2.0 * (kGamma - 1.0))), (T)(1.0 / (kGamma - 1.0)),
                          1, e.w, nullptr, nullptr};
      },
      [&](int k) { dg_ctx* c = Tm.m[k]; return (double)sizeof(T) * c->N * (c->D + 2); });
}

// w = A P^{-1} (scale v): the right-preconditioned operator of the Krylov solve.
template <class T>
dg_status apply_AP_team(Team& Tm, const std::vector<ApItem<T>>& it) {
  using PB = PrecBuf<T>;
  if (it.empty()) return DG_OK;
  if (Tm.m[it[0].k]->opt.preconditioner != DG_PREC_CELL_FDM) return apply_A_team<T>(Tm, it);
  std::vector<int> act;
  std::vector<int> idx(Tm.n(), -1);
  for (size_t i = 0; i < it.size(); ++i) {
    act.push_back(it[i].k);
    idx[it[i].k] = (int)i;
  }
  const hipStream_t s = Tm.s;
  const int deg = Tm.m[act[0]]->degree;
  dg_status st = op_launch<FdmArgs<T>>(
      Tm, act, 4,
      [&](int k) {
        const ApItem<T>& e = it[idx[k]];
        dg_ctx* c = Tm.m[k];
        return FdmArgs<T>{e.v, e.scale, PB::coef(c), PB::z(c), e.dscale};
      },
      [&](int k) { return 2.0 * sizeof(T) * Tm.m[k]->N; },
      [&](dg_ctx* c, const FdmArgs<T>& a) { return PB::fdm(c->md, c->degree, a, s); },
      [&](int n, const MeshDev* const* mh, const MeshDev* const* md, const FdmArgs<T>* a) {
        return PB::fdm_seg(n, mh, md, a, deg, s);
      });
  if (st) return st;
  std::vector<ApItem<T>> it2 = it;
  for (auto& e : it2) {
    e.v = PB::z(Tm.m[e.k]);
    e.dinv = nullptr;
    e.scale = T(1);
    e.dscale = nullptr;
  }
  return apply_A_team<T>(Tm, it2);
}

// One reduction pass per member (Gram-Schmidt form: nv basis vectors, x, optional y), its second
// stage into the member's slot [2, 2 + nvals), nvals = 2 nv + 3 with y, else nv + 1.
template <class T>
struct DotItem {
  int k;
  const T* V;
  const T* x;
  const T* y;
};
template <class T>
dg_status dots_team(Team& Tm, int nv, const std::vector<DotItem<T>>& it) {
  if (it.empty()) return DG_OK;
  const bool hasy = it[0].y != nullptr;
  const int nvals = hasy ? 2 * nv + 3 : nv + 1;
  if (!Tm.shared) {
    for (const auto& e : it) {
      dg_ctx* c = Tm.m[e.k];
      const int G = red_grid(c->N);
      {
        Timed t_(Tm.tc, 3, (nv + (hasy ? 2.0 : 1.0)) * sizeof(T) * c->N);
        launch_gs_dots<T>(nv, G, Tm.s, e.V, c->ld, e.x, e.y, c->part, c->N);
      }
      Timed t_(Tm.tc, 6);
      hipLaunchKernelGGL(k_reduce, dim3(nvals), dim3(kRedThreads), 0, Tm.s, c->part, G, Tm.slot(e.k) + 2);
    }
    TCHK(Tm, hipGetLastError());
    return DG_OK;
  }
  std::vector<DotsArgs<T>> as;
  std::vector<RedArgs> rs;
  for (const auto& e : it) {
    dg_ctx* c = Tm.m[e.k];
    as.push_back(DotsArgs<T>{e.V, c->ld, e.x, e.y, c->part, c->N});
    rs.push_back(RedArgs{c->part, red_grid(c->N), Tm.slot(e.k) + 2});
  }
  const int n = (int)as.size();
  seg_launch<DotsArgs<T>>(n, nullptr, [&](int i) { return red_grid(as[i].n); }, [&](int i) { return as[i]; },
                          [&](const SegTab<DotsArgs<T>>& t, int g) {
                            launch_gs_dots_seg<T>(nv, hasy, g, Tm.s, Shared<DotsArgs<T>>{t});
                            return 0;
                          });
  seg_launch<RedArgs>(n, nullptr, [&](int) { return nvals; }, [&](int i) { return rs[i]; },
                      [&](const SegTab<RedArgs>& t, int g) {
                        hipLaunchKernelGGL(k_reduce_seg, dim3(g), dim3(kRedThreads), 0, Tm.s, Shared<RedArgs>{t});
                        return 0;
                      });
  TCHK(Tm, hipGetLastError());
  return DG_OK;
}

// x.y per member (one reduction pass, one round trip for all); out[k] for the members in act.
template <class T, class X, class Y>
dg_status dot_team(Team& Tm, const std::vector<int>& act, X xof, Y yof, std::vector<double>& out) {
  std::vector<DotItem<T>> it;
  for (int k : act) it.push_back(DotItem<T>{k, nullptr, xof(k), yof(k)});
  dg_status st = dots_team<T>(Tm, 0, it);
  if (st) return st;
  if ((st = fetch(Tm, act))) return st;
  out.assign(Tm.n(), 0.0);
  for (int k : act) out[k] = Tm.hslot(k)[3];
  return DG_OK;
}

struct CycleResult {
  int its = 0;
  double res = 0.0;
  bool converged = false;
};

// Hessenberg bookkeeping of one GMRES cycle: the raw Arnoldi coefficients (needed to correct the
// next column for the delayed re-orthogonalisation) and their Givens-rotated copy.
struct Arnoldi {
  int m;
  std::vector<double> Hr, R, cs, sn, g;
  Arnoldi(int m_, double beta) : m(m_), Hr((size_t)(m_ + 1) * m_, 0.0), R((size_t)(m_ + 1) * m_, 0.0),
                                 cs(m_, 0.0), sn(m_, 0.0), g(m_ + 1, 0.0) { g[0] = beta; }
  double& hr(int i, int j) { return Hr[(size_t)i * m + j]; }
  double& r(int i, int j) { return R[(size_t)i * m + j]; }
  // Rotate column j (entries 0..j+1 given in col) with the rotations 0..j-1, then form rotation j.
  // Returns |residual| after column j; with commit the rotation and the right-hand side are kept.
  double rotate(int j, std::vector<double>& col, bool commit) {
    for (int i = 0; i < j; ++i) {
      const double a = col[i], b = col[i + 1];
      col[i] = cs[i] * a + sn[i] * b;
      col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double den = std::hypot(a, b);
    const double c = den > 0.0 ? a / den : 1.0, s = den > 0.0 ? b / den : 0.0;
    if (commit) {
      for (int i = 0; i <= j; ++i) r(i, j) = col[i];
      r(j, j) = den;
      cs[j] = c;
      sn[j] = s;
      g[j + 1] = -s * g[j];
      g[j] = c * g[j];
      return std::fabs(g[j + 1]);
    }
    return std::fabs(s * g[j]);
  }
};

// One member's GMRES(m) cycle on V[0] (unnormalised, norm beta), stopping at residual <= tol or
// maxits; accumulates x += xscale * P^{-1} V y into the FP64 vector x.
template <class T>
struct Cyc {
  int k;
  T* V;
  T* w;
  const T* dinv;
  int m;
  double beta, tol;
  int maxits;
  double* x;
  double xscale;
  double dta;
  Arnoldi H;
  std::vector<double> s, col, a, t, h;
  double sigma, kappa, res, rho = 0.0;
  int done = -1, jd = 0, fin = 0;
  bool one_rt, run = true;
  Coef ca{}, cb{};
  double gsc = 0.0;
  CycleResult cr;
  Cyc(int k_, T* V_, T* w_, const T* dinv_, int m_, double beta_, double tol_, int maxits_, double* x_,
      double xscale_, double dta_, bool one_rt_)
      : k(k_), V(V_), w(w_), dinv(dinv_), m(m_), beta(beta_), tol(tol_), maxits(maxits_), x(x_), xscale(xscale_),
        dta(dta_), H(m_, beta_), s(m_ + 1, 0.0), col(m_ + 1, 0.0), a(m_ + 1, 0.0), t(m_ + 1, 0.0), h(m_ + 1, 0.0),
        sigma(1.0 / beta_), kappa(1.0), res(beta_), one_rt(one_rt_) {}
  // Column j of the Hessenberg matrix receives the re-orthogonalisation of the candidate that
  // followed it (coefficients av, norm rho2 of the re-orthogonalised candidate).
  void finalize(int j, const double* av, double r2) {
    const double f = 1.0 / (sigma * kappa);
    for (int i = 0; i <= j; ++i) H.hr(i, j) += av ? av[i] * f : 0.0;
    H.hr(j + 1, j) = r2 * f;
    for (int i = 0; i <= j + 1; ++i) col[i] = H.hr(i, j);
    res = H.rotate(j, col, true);
    done = j;
  }
};

// The GMRES cycles of the members in cy, iteration by iteration in lockstep.
//
// Arnoldi with classical Gram-Schmidt and one re-orthogonalisation, the latter delayed by one
// step so that every step costs one reduction pass and one update pass over the basis:
// step j applies the operator to the candidate u_j (projected once), and a single pass returns
// Q^T u_j, Q^T w, u_j.u_j, u_j.w.  From these the candidate is re-orthogonalised and normalised
// (Pythagoras), the previous Hessenberg column receives its correction, the coefficients of
// A q_j follow without touching the vectors again, and one update pass writes both q_j and the
// next candidate.  Basis vectors are stored unnormalised with scale s_i (q_i = s_i V_i).  The
// residual after column j is estimated from the candidate's norm; once it meets the tolerance
// (or the cycle ends) one more reduction pass finalises column j exactly.
//
// Latency-bound sizes run one host round trip per iteration: the update pass leaves the
// candidate's norm and scale on the device (k_reduce_norm), the next operator application reads
// the scale there, and the host receives the norm with the next reduction.  The residual of
// column j is then known only after the operator has been applied to the next candidate, so a
// converging solve pays one extra application; large meshes keep the second round trip.
template <class T>
dg_status gmres_team(Team& Tm, std::vector<Cyc<T>>& cy) {
  const std::string nanmsg = "non-finite value in the Krylov solve";
  double dots[2 * kMaxV + 3];
  for (int j = 0;; ++j) {
    std::vector<int> A;
    for (int i = 0; i < (int)cy.size(); ++i)
      if (cy[i].run && Tm.alive(cy[i].k)) A.push_back(i);
    if (A.empty()) break;
    // operator on the current candidates
    {
      std::vector<ApItem<T>> it;
      for (int i : A) {
        Cyc<T>& c = cy[i];
        const bool dev_sigma = c.one_rt && j > 0;
        it.push_back(ApItem<T>{c.k, c.dta, c.V + (size_t)j * Tm.m[c.k]->ld, c.dinv, (T)c.sigma, c.w,
                               dev_sigma ? Tm.slot(c.k) + 1 : nullptr});
        c.cr.its++;
      }
      dg_status st = apply_AP_team<T>(Tm, it);
      if (st) return st;
    }
    // one reduction: Q_j^T V_j, Q_j^T w, V_j.V_j, V_j.w, w.w
    {
      std::vector<DotItem<T>> it;
      std::vector<int> ks;
      for (int i : A) {
        Cyc<T>& c = cy[i];
        it.push_back(DotItem<T>{c.k, c.V, c.V + (size_t)j * Tm.m[c.k]->ld, c.w});
        ks.push_back(c.k);
      }
      dg_status st = dots_team<T>(Tm, j, it);
      if (!st) st = fetch(Tm, ks);
      if (st) return st;
    }
    std::vector<int> Up;
    for (int i : A) {
      Cyc<T>& c = cy[i];
      const double* hb = Tm.hslot(c.k);
      if (c.one_rt && j > 0) {
        if (!std::isfinite(hb[0])) { drop(Tm, c.k, DG_ENAN, nanmsg); continue; }
        if (hb[0] == 0.0) {
          // A q_{j-1} lies in span(Q_j) exactly: column j-1 is exact with a zero
          c.finalize(j - 1, nullptr, 0.0);
          c.run = false;
          continue;
        }
        c.sigma = hb[1];
      }
      std::copy(hb + 2, hb + 2 + 2 * j + 3, dots);
      bool bad = false;
      for (int q = 0; q < 2 * j + 3; ++q) bad |= !std::isfinite(dots[q]);
      if (bad) { drop(Tm, c.k, DG_ENAN, nanmsg); continue; }
      double aa = 0.0, ab = 0.0;
      for (int q = 0; q < j; ++q) {
        c.a[q] = c.s[q] * c.sigma * dots[q];  // q_q . (sigma V_j)
        c.t[q] = c.s[q] * dots[j + q];        // q_q . w   (kept in t until the correction below)
        aa += c.a[q] * c.a[q];
        ab += c.a[q] * c.t[q];
      }
      const double cc = c.sigma * c.sigma * dots[2 * j];
      const double dd = c.sigma * dots[2 * j + 1];
      const double rho2 = cc - aa;
      if (j > 0 && !(rho2 > 1e-26 * cc)) {
        // the candidate lies in span(Q_j): lucky breakdown, column j-1 is exact with a zero
        if (c.done < j - 1) c.finalize(j - 1, c.a.data(), 0.0);
        c.jd = j;
        c.run = false;
        continue;
      }
      const double rho = std::sqrt(rho2);
      if (j > 0 && c.done < j - 1) {
        c.finalize(j - 1, c.a.data(), rho);
        if (c.res <= c.tol) {
          c.jd = j;
          c.run = false;
          continue;
        }
      }
      // coefficients of A q_j on Q_{j+1}: (w - A Q_j a) / rho with A Q_j = Q_{j+1} Hr
      for (int q = 0; q <= j; ++q) {
        double ti = 0.0;
        for (int r = 0; r < j; ++r) ti += c.H.hr(q, r) * c.a[r];
        c.h[q] = ti;  // (Hr a)_q
      }
      for (int q = 0; q < j; ++q) c.t[q] = (c.t[q] - c.h[q]) / rho;  // h_j[q]
      c.t[j] = ((dd - ab) / rho - c.h[j]) / rho;                      // h_j[j]
      // next candidate V_{j+1} = rho (A q_j - Q_{j+1} h_j) = w - rho Q_{j+1} gv,
      // gv = (Hr a)/rho + h_j
      const double gj = c.h[j] / rho + c.t[j];
      for (int q = 0; q < j; ++q) {
        const double gi = c.h[q] / rho + c.t[q];
        c.cb.c[q] = (rho * gi - gj * c.a[q]) * c.s[q];
        c.ca.c[q] = c.a[q] * c.s[q] / c.sigma;
      }
      c.gsc = gj * c.sigma;
      c.rho = rho;
      Up.push_back(i);
    }
    if (Up.empty()) continue;
    // update pass: q_j and the next candidate; its norm (on the device for one round trip)
    if (!Tm.shared) {
      for (int i : Up) {
        Cyc<T>& c = cy[i];
        dg_ctx* x = Tm.m[c.k];
        const int G = red_grid(x->N);
        T* Vj = c.V + (size_t)j * x->ld;
        T* Vn = c.V + (size_t)(j + 1) * x->ld;
        {
          Timed t_(Tm.tc, 5, (j + 3.0 + (j > 0 ? 1.0 : 0.0)) * sizeof(T) * x->N);
          launch_gs_update<T>(j, G, Tm.s, c.V, x->ld, c.ca, c.cb, c.gsc, Vj, (const T*)c.w, Vn, x->part, x->N);
        }
        Timed t_(Tm.tc, 6);
        if (c.one_rt) hipLaunchKernelGGL(k_reduce_norm, dim3(1), dim3(kRedThreads), 0, Tm.s, x->part, G, Tm.slot(c.k));
        else hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, Tm.s, x->part, G, Tm.slot(c.k) + 2);
      }
    } else {
      std::vector<UpdArgs<T>> us;
      std::vector<RedArgs> one, two;
      int hi = 0;
      for (int i : Up) {
        Cyc<T>& c = cy[i];
        double* hc = Tm.hcoef(c.k);
        for (int q = 0; q < kMaxV; ++q) {
          hc[q] = c.ca.c[q];
          hc[kMaxV + q] = c.cb.c[q];
        }
        hi = std::max(hi, c.k);
      }
      TCHK(Tm, hipMemcpyAsync(Tm.lead->tcoef, Tm.hcoef(0), (size_t)(hi + 1) * kCoefStride * sizeof(double),
                          hipMemcpyHostToDevice, Tm.s));
      for (int i : Up) {
        Cyc<T>& c = cy[i];
        dg_ctx* x = Tm.m[c.k];
        us.push_back(UpdArgs<T>{c.V, x->ld, Tm.dcoef(c.k), c.gsc, c.V + (size_t)j * x->ld, (const T*)c.w,
                                c.V + (size_t)(j + 1) * x->ld, x->part, x->N});
        (c.one_rt ? one : two).push_back(RedArgs{x->part, red_grid(x->N), c.one_rt ? Tm.slot(c.k) : Tm.slot(c.k) + 2});
      }
      seg_launch<UpdArgs<T>>((int)us.size(), nullptr, [&](int q) { return red_grid(us[q].n); },
                             [&](int q) { return us[q]; },
                             [&](const SegTab<UpdArgs<T>>& t, int g) {
                               launch_gs_update_seg<T>(j, g, Tm.s, Shared<UpdArgs<T>>{t});
                               return 0;
                             });
      seg_launch<RedArgs>((int)one.size(), nullptr, [&](int) { return 1; }, [&](int q) { return one[q]; },
                          [&](const SegTab<RedArgs>& t, int g) {
                            hipLaunchKernelGGL(k_reduce_norm_seg, dim3(g), dim3(kRedThreads), 0, Tm.s, Shared<RedArgs>{t});
                            return 0;
                          });
      seg_launch<RedArgs>((int)two.size(), nullptr, [&](int) { return 1; }, [&](int q) { return two[q]; },
                          [&](const SegTab<RedArgs>& t, int g) {
                            hipLaunchKernelGGL(k_reduce_seg, dim3(g), dim3(kRedThreads), 0, Tm.s, Shared<RedArgs>{t});
                            return 0;
                          });
    }
    TCHK(Tm, hipGetLastError());
    std::vector<int> two_k;
    for (int i : Up) {
      Cyc<T>& c = cy[i];
      c.s[j] = c.sigma / c.rho;
      c.kappa = c.rho;
      for (int q = 0; q <= j; ++q) c.H.hr(q, j) = c.t[q];
      c.jd = j + 1;
      if (c.one_rt) {
        if (j + 1 == c.m || c.cr.its >= c.maxits) c.fin = 1;
      } else {
        two_k.push_back(c.k);
      }
    }
    if (!two_k.empty()) {
      dg_status st = fetch(Tm, two_k);
      if (st) return st;
      for (int i : Up) {
        Cyc<T>& c = cy[i];
        if (c.one_rt) continue;
        const double nn = Tm.hslot(c.k)[2];
        if (!std::isfinite(nn)) { drop(Tm, c.k, DG_ENAN, nanmsg); continue; }
        if (nn == 0.0) {
          // A q_j lies in span(Q_{j+1}) exactly
          c.sigma = 1.0;
          c.finalize(j, nullptr, 0.0);
          c.run = false;
          continue;
        }
        c.sigma = 1.0 / std::sqrt(nn);
        // estimate with the candidate's norm, finalise when it meets the tolerance or the cycle ends
        for (int q = 0; q <= j; ++q) c.col[q] = c.t[q];
        c.col[j + 1] = std::sqrt(nn) / c.rho;
        const double est = c.H.rotate(j, c.col, false);
        if (est <= c.tol || j + 1 == c.m || c.cr.its >= c.maxits) c.fin = 2;
      }
    }
    // finalise the last column exactly: Q^T V_{j+1} and |V_{j+1}|^2 (with V_{j+1}'s scale)
    std::vector<DotItem<T>> fit;
    std::vector<int> fks;
    for (int i : Up) {
      Cyc<T>& c = cy[i];
      if (!c.fin || !Tm.alive(c.k)) continue;
      fit.push_back(DotItem<T>{c.k, c.V, c.V + (size_t)(j + 1) * Tm.m[c.k]->ld, nullptr});
      fks.push_back(c.k);
    }
    if (fit.empty()) continue;
    {
      dg_status st = dots_team<T>(Tm, j + 1, fit);
      if (!st) st = fetch(Tm, fks);
      if (st) return st;
    }
    for (int i : Up) {
      Cyc<T>& c = cy[i];
      if (!c.fin || !Tm.alive(c.k)) continue;
      const int fin = c.fin;
      c.fin = 0;
      const double* hb = Tm.hslot(c.k);
      if (fin == 1) {
        if (!std::isfinite(hb[0])) { drop(Tm, c.k, DG_ENAN, nanmsg); continue; }
        if (hb[0] == 0.0) {
          c.finalize(j, nullptr, 0.0);
          c.run = false;
          continue;
        }
        c.sigma = hb[1];
      }
      bool bad = false;
      for (int q = 0; q < j + 2; ++q) bad |= !std::isfinite(hb[2 + q]);
      if (bad) { drop(Tm, c.k, DG_ENAN, nanmsg); continue; }
      double a2 = 0.0;
      for (int q = 0; q <= j; ++q) {
        c.a[q] = c.s[q] * c.sigma * hb[2 + q];
        a2 += c.a[q] * c.a[q];
      }
      const double c2 = c.sigma * c.sigma * hb[2 + j + 1];
      c.finalize(j, c.a.data(), std::sqrt(std::max(c2 - a2, 0.0)));
      if (fin == 1 || c.res <= c.tol || j + 1 == c.m || c.cr.its >= c.maxits) c.run = false;
    }
  }
  // x += P^{-1} (V y) per member
  std::vector<int> fz;
  for (auto& c : cy) {
    if (!Tm.alive(c.k)) continue;
    c.cr.res = c.res;
    c.cr.converged = c.res <= c.tol;
    if (c.jd > 0) fz.push_back(c.k);
  }
  if (fz.empty()) return DG_OK;
  std::vector<int> pos(Tm.n(), -1);
  for (int i = 0; i < (int)cy.size(); ++i) pos[cy[i].k] = i;
  const bool fdm = Tm.m[fz[0]]->opt.preconditioner == DG_PREC_CELL_FDM;
  if (fdm) {
    dg_status st = pw<PwZero>(Tm, fz, [&](int k) { return PwZero{Tm.m[k]->N, Tm.m[k]->u}; });
    if (st) return st;
  }
  for (int k : fz) {
    Cyc<T>& c = cy[pos[k]];
    dg_ctx* x = Tm.m[k];
    const double tsz = (double)sizeof(T) * x->N;
    std::vector<double> y(c.jd, 0.0);
    for (int i = c.jd - 1; i >= 0; --i) {
      double v = c.H.g[i];
      for (int q = i + 1; q < c.jd; ++q) v -= c.H.r(i, q) * y[q];
      y[i] = v / c.H.r(i, i);
    }
    Coef cf{};
    for (int i = 0; i < c.jd; ++i) cf.c[i] = c.xscale * y[i] * c.s[i];
    Timed t_(Tm.tc, 6, c.jd * tsz + 16.0 * x->N + (fdm ? 0.0 : tsz));
    // FDM: combine in FP64 into u, precondition in FP64 below, add; else x += dinv (V y)
    launch_update<T>(c.jd, pw_grid(x->N), Tm.s, (const T*)c.V, x->ld, cf, fdm ? (const T*)nullptr : c.dinv,
                     fdm ? x->u : c.x, x->N);
  }
  TCHK(Tm, hipGetLastError());
  if (!fdm) return DG_OK;
  const int deg = Tm.m[fz[0]]->degree;
  const hipStream_t s = Tm.s;
  dg_status st = op_launch<FdmArgs<double>>(
      Tm, fz, 4, [&](int k) { dg_ctx* x = Tm.m[k]; return FdmArgs<double>{x->u, 1.0, x->coef, x->z, nullptr}; },
      [&](int k) { return 16.0 * Tm.m[k]->N; },
      [&](dg_ctx* x, const FdmArgs<double>& a) { return launch_fdm64(x->md, x->degree, a, s); },
      [&](int n, const MeshDev* const* mh, const MeshDev* const* md, const FdmArgs<double>* a) {
        return launch_fdm_seg64(n, mh, md, a, deg, s);
      });
  if (st) return st;
  return pw<PwAdd>(Tm, fz, [&](int k) { return PwAdd{Tm.m[k]->N, cy[pos[k]].x, Tm.m[k]->z}; });
}

bool one_round_trip(const dg_ctx* c) {
  return c->opt.preconditioner == DG_PREC_CELL_FDM && c->N <= kOneSyncMaxNodes;
}

struct SolveOut {
  int its = 0, outer = 0;
  double relres = 0.0;
};

// Solve A delta = r0 (FP64) for each member in act, delta zeroed here.
dg_status solve64_team(Team& Tm, const std::vector<int>& act, const std::vector<double>& dta,
                       std::vector<SolveOut>& out) {
  dg_status st = pw<PwZero>(Tm, act, [&](int k) { return PwZero{Tm.m[k]->N, Tm.m[k]->delta}; });
  if (st) return st;
  std::vector<double> b2;
  st = dot_team<double>(Tm, act, [&](int k) { return Tm.m[k]->r0; }, [&](int k) { return Tm.m[k]->r0; }, b2);
  if (st) return st;
  std::vector<double> bn(Tm.n(), 0.0), tol(Tm.n(), 0.0), beta(Tm.n(), 0.0);
  std::vector<int> go;
  for (int k : act) {
    dg_ctx* c = Tm.m[k];
    bn[k] = std::sqrt(b2[k]);
    if (!std::isfinite(bn[k])) { drop(Tm, k, DG_ENAN, "non-finite right-hand side"); continue; }
    tol[k] = std::max(c->opt.gmres_rtol * bn[k], c->opt.gmres_atol);
    out[k] = SolveOut{};
    if (bn[k] == 0.0 || bn[k] <= tol[k]) continue;
    beta[k] = bn[k];
    go.push_back(k);
  }
  if (!Tm.shared) {
    for (int k : go) TCHK(Tm, hipMemcpyAsync(Tm.m[k]->V, Tm.m[k]->r0, Tm.m[k]->N * sizeof(double), hipMemcpyDeviceToDevice, Tm.s));
  } else if ((st = pw<PwCopy>(Tm, go, [&](int k) { return PwCopy{Tm.m[k]->N, Tm.m[k]->r0, Tm.m[k]->V}; }))) {
    return st;
  }
  while (!go.empty()) {
    std::vector<Cyc<double>> cy;
    for (int k : go) {
      dg_ctx* c = Tm.m[k];
      cy.emplace_back(k, c->V, c->w, c->dinv, c->m, beta[k], tol[k], c->opt.gmres_maxit - out[k].its, c->delta, 1.0,
                      dta[k], one_round_trip(c));
    }
    if ((st = gmres_team<double>(Tm, cy))) return st;
    std::vector<int> rs;
    for (auto& c : cy) {
      const int k = c.k;
      if (!Tm.alive(k)) continue;
      out[k].its += c.cr.its;
      out[k].relres = c.cr.res / bn[k];
      if (c.cr.converged) continue;
      if (out[k].its >= Tm.m[k]->opt.gmres_maxit) {
        drop(Tm, k, DG_ENOCONV, "GMRES did not reach its tolerance within gmres_maxit iterations");
        continue;
      }
      rs.push_back(k);
    }
    go.clear();
    if (rs.empty()) break;
    // restart from the true residual
    std::vector<ApItem<double>> it;
    for (int k : rs) it.push_back(ApItem<double>{k, dta[k], Tm.m[k]->delta, nullptr, 1.0, Tm.m[k]->w, nullptr});
    if ((st = apply_A_team<double>(Tm, it))) return st;
    if ((st = pw<PwSub>(Tm, rs, [&](int k) { dg_ctx* c = Tm.m[k]; return PwSub{c->N, c->r0, c->w, c->V}; }))) return st;
    if ((st = dot_team<double>(Tm, rs, [&](int k) { return Tm.m[k]->V; }, [&](int k) { return Tm.m[k]->V; }, b2)))
      return st;
    for (int k : rs) {
      beta[k] = std::sqrt(b2[k]);
      out[k].relres = beta[k] / bn[k];
      if (beta[k] > tol[k]) go.push_back(k);
    }
  }
  return DG_OK;
}

// Mixed precision: FP64 defect correction around FP32 GMRES cycles.
dg_status solve_mixed_team(Team& Tm, const std::vector<int>& act, const std::vector<double>& dta,
                           std::vector<SolveOut>& out) {
  dg_status st = pw<PwZero>(Tm, act, [&](int k) { return PwZero{Tm.m[k]->N, Tm.m[k]->delta}; });
  if (st) return st;
  std::vector<double> b2;
  st = dot_team<double>(Tm, act, [&](int k) { return Tm.m[k]->r0; }, [&](int k) { return Tm.m[k]->r0; }, b2);
  if (st) return st;
  std::vector<double> bn(Tm.n(), 0.0), tol(Tm.n(), 0.0), rn(Tm.n(), 0.0);
  std::vector<int> go;
  for (int k : act) {
    dg_ctx* c = Tm.m[k];
    bn[k] = std::sqrt(b2[k]);
    if (!std::isfinite(bn[k])) { drop(Tm, k, DG_ENAN, "non-finite right-hand side"); continue; }
    tol[k] = std::max(c->opt.gmres_rtol * bn[k], c->opt.gmres_atol);
    out[k] = SolveOut{};
    if (bn[k] == 0.0 || bn[k] <= tol[k]) continue;
    rn[k] = bn[k];
    go.push_back(k);
  }
  if (!Tm.shared) {
    for (int k : go) TCHK(Tm, hipMemcpyAsync(Tm.m[k]->rr, Tm.m[k]->r0, Tm.m[k]->N * sizeof(double), hipMemcpyDeviceToDevice, Tm.s));
  } else if ((st = pw<PwCopy>(Tm, go, [&](int k) { return PwCopy{Tm.m[k]->N, Tm.m[k]->r0, Tm.m[k]->rr}; }))) {
    return st;
  }
  const int max_outer = 100;
  while (!go.empty()) {
    std::vector<int> g2;
    for (int k : go) {
      if (out[k].outer >= max_outer || out[k].its >= Tm.m[k]->opt.gmres_maxit)
        drop(Tm, k, DG_ENOCONV, "mixed-precision defect correction did not converge");
      else g2.push_back(k);
    }
    go = g2;
    if (go.empty()) break;
    if ((st = pw<PwScaleCast>(Tm, go, [&](int k) { dg_ctx* c = Tm.m[k]; return PwScaleCast{c->N, c->rr, 1.0 / rn[k], c->V32}; })))
      return st;
    std::vector<double> v2;
    if ((st = dot_team<float>(Tm, go, [&](int k) { return Tm.m[k]->V32; }, [&](int k) { return Tm.m[k]->V32; }, v2)))
      return st;
    std::vector<Cyc<float>> cy;
    for (int k : go) {
      dg_ctx* c = Tm.m[k];
      const double vb = std::sqrt(v2[k]);
      cy.emplace_back(k, c->V32, c->w32, c->dinv32, c->m32, vb, c->opt.inner_rtol * vb, c->opt.inner_maxit, c->delta,
                      rn[k], dta[k], one_round_trip(c));
    }
    if ((st = gmres_team<float>(Tm, cy))) return st;
    std::vector<int> al;
    for (auto& c : cy) {
      if (!Tm.alive(c.k)) continue;
      out[c.k].its += c.cr.its;
      out[c.k].outer++;
      al.push_back(c.k);
    }
    // FP64 residual of the accumulated correction
    std::vector<ApItem<double>> it;
    for (int k : al) it.push_back(ApItem<double>{k, dta[k], Tm.m[k]->delta, nullptr, 1.0, Tm.m[k]->w, nullptr});
    if ((st = apply_A_team<double>(Tm, it))) return st;
    if ((st = pw<PwSub>(Tm, al, [&](int k) { dg_ctx* c = Tm.m[k]; return PwSub{c->N, c->r0, c->w, c->rr}; }))) return st;
    if ((st = dot_team<double>(Tm, al, [&](int k) { return Tm.m[k]->rr; }, [&](int k) { return Tm.m[k]->rr; }, b2)))
      return st;
    go.clear();
    for (int k : al) {
      rn[k] = std::sqrt(b2[k]);
      out[k].relres = rn[k] / bn[k];
      if (rn[k] > tol[k]) go.push_back(k);
    }
  }
  return DG_OK;
}

// ----------------------------------------------------------------------------------- operators
dg_status explicit_team(Team& Tm, const std::vector<int>& act, const std::vector<const double*>& U,
                        const std::vector<double*>& R) {
  if (act.empty()) return DG_OK;
  const hipStream_t s = Tm.s;
  const int deg = Tm.m[act[0]]->degree;
  dg_status st = op_launch<ExpArgs>(
      Tm, act, 0, [&](int k) { return ExpArgs{U[k], R[k]}; },
      [&](int k) { return 16.0 * Tm.m[k]->F * Tm.m[k]->N; },
      [&](dg_ctx* c, const ExpArgs& a) {
        return c->md.nq > 0 ? launch_explicit_oi(c->md, c->degree, a.U, a.R, s) : launch_explicit(c->md, c->degree, a.U, a.R, s);
      },
      [&](int n, const MeshDev* const* mh, const MeshDev* const* md, const ExpArgs* a) {
        return launch_explicit_seg(n, mh, md, a, deg, s);
      });
  if (st) return st;
  std::vector<int> sp;
  for (int k : act)
    if (Tm.m[k]->tau) sp.push_back(k);
  if (sp.empty()) return DG_OK;
  if (Tm.m[sp[0]]->D == 2)
    return pw<PwFriction<2>>(Tm, sp, [&](int k) { dg_ctx* c = Tm.m[k]; return PwFriction<2>{c->N, c->ld, U[k], c->tau, c->desc.sponge[4], R[k]}; });
  return pw<PwFriction<3>>(Tm, sp, [&](int k) { dg_ctx* c = Tm.m[k]; return PwFriction<3>{c->N, c->ld, U[k], c->tau, c->desc.sponge[4], R[k]}; });
}

// Per-cell sound speed and (with coef) preconditioner coefficients of every member from its h.
dg_status cellcoef_team(Team& Tm, const std::vector<int>& act, const std::vector<double>& dta, bool f32, bool coef) {
  if (act.empty()) return DG_OK;
  const hipStream_t s = Tm.s;
  const int deg = Tm.m[act[0]]->degree;
  return op_launch<CoefArgs>(
      Tm, act, 4,
      [&](int k) {
        dg_ctx* c = Tm.m[k];
        return CoefArgs{c->h, c->wJ, dta[k], c->lam, f32 ? c->lam32 : nullptr, coef ? c->coef : nullptr,
                        (coef && f32) ? c->coef32 : nullptr};
      },
      [&](int) { return 0.0; },
      [&](dg_ctx* c, const CoefArgs& a) {
        return launch_cellcoef(c->md, c->degree, a.h, a.wJ, a.dta, a.lam, a.lam32, a.coef, a.coef32, s);
      },
      [&](int n, const MeshDev* const* mh, const MeshDev* const* md, const CoefArgs* a) {
        return launch_cellcoef_seg(n, mh, md, a, deg, s);
      });
}
dg_status lam_team(Team& Tm, const std::vector<int>& act, bool f32) {
  return cellcoef_team(Tm, act, std::vector<double>(Tm.n(), 0.0), f32, false);
}

// F_I(U) into F; uses pp, h, lam, q as scratch
template <int D>
dg_status implicit_team(Team& Tm, const std::vector<int>& act, const std::vector<const double*>& U,
                        const std::vector<double*>& F) {
  dg_status st = pw<PwPressureH<D>>(Tm, act, [&](int k) {
    dg_ctx* c = Tm.m[k];
    return PwPressureH<D>{c->N, c->ld, U[k], c->pbar, c->pp, c->h};
  });
  if (st || (st = lam_team(Tm, act, false)) || (st = split_update_team(Tm, act))) return st;
  st = grad_team<double>(
      Tm, act, 7, [&](int k) { dg_ctx* c = Tm.m[k]; return GradArgs<double>{c->pp, nullptr, 1.0, c->q, nullptr, nullptr}; },
      [&](int) { return 0.0; });
  if (st) return st;
  st = pw<PwFiMomentum<D>>(Tm, act, [&](int k) {
    dg_ctx* c = Tm.m[k];
    return PwFiMomentum<D>{c->N, c->ld, c->q, U[k], c->rbar, F[k]};
  });
  if (st) return st;
  return energy_div_team<double>(
      Tm, act, 7,
      [&](int k) {
        dg_ctx* c = Tm.m[k];
        const double beta = c->opt.penalty_beta;
        return DivArgs<double>{U[k] + c->ld, c->h, c->pp, nullptr, 1.0, c->lam, -1.0, -beta / (2.0 * (kGamma - 1.0)),
                               0.0, 0, F[k] + (size_t)(1 + D) * c->ld, nullptr, nullptr};
      },
      [&](int) { return 0.0; });
}

// mass sum(w J rho) and max |w| of each member's state into its slot ([3] and [kMaxAt])
dg_status diagnostics_team(Team& Tm, const std::vector<int>& act, const std::vector<const double*>& U) {
  std::vector<DotItem<double>> it;
  for (int k : act) it.push_back(DotItem<double>{k, nullptr, Tm.m[k]->wJ, U[k]});
  dg_status st = dots_team<double>(Tm, 0, it);
  if (st) return st;
  for (int k : act) {
    dg_ctx* c = Tm.m[k];
    const int G = red_grid(c->N);
    hipLaunchKernelGGL(k_maxabs_ratio, dim3(G), dim3(kRedThreads), 0, Tm.s, U[k] + (size_t)c->D * c->ld, U[k],
                       c->part + (size_t)3 * kMaxGrid, c->N);
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(kRedThreads), 0, Tm.s, c->part + (size_t)3 * kMaxGrid, G,
                       Tm.slot(k) + kMaxAt);
  }
  TCHK(Tm, hipGetLastError());
  return fetch(Tm, act);
}

// One IMEX-RK2 step of every member (U[k], dt[k]); per-member status in Tm.st.
template <int D>
dg_status step_team(Team& Tm, double* const* U, const double* dt, dg_step_stats* stats) {
  const int n = Tm.n();
  const double g_ = 1.0 - 1.0 / std::sqrt(2.0), d_ = 1.0 / (2.0 * std::sqrt(2.0));
  const double al = (3.0 + 2.0 * std::sqrt(2.0)) / 6.0;
  const double A[3][3] = {{0, 0, 0}, {2 * g_, 0, 0}, {1 - al, al, 0}};
  const double At[3][3] = {{0, 0, 0}, {g_, g_, 0}, {d_, d_, g_}};
  const double bw[3] = {d_, d_, g_};
  std::vector<dg_step_stats> S(n);
  for (auto& x : S) x = dg_step_stats{};
  if (Tm.tc) {
    Tm.tc->ev_n = 0;
    Tm.tc->pev_n = 0;
    for (double& b : Tm.tc->kbytes) b = 0.0;
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<int> act;
  for (int k = 0; k < n; ++k)
    if (Tm.alive(k)) act.push_back(k);
  std::vector<const double*> Uc(n), Usc(n);
  std::vector<double*> R(n);
  for (int k = 0; k < n; ++k) {
    Uc[k] = U[k];
    Usc[k] = Tm.m[k]->Us;
  }
  dg_status st = DG_OK;
#define STEP_CHK(expr) \
  do {                 \
    if ((st = (expr))) return st; \
    act = alive_of(Tm, act); \
  } while (0)
  auto FEof = [&](int j) { for (int k = 0; k < n; ++k) R[k] = Tm.m[k]->FE[j]; return R; };
  auto FIof = [&](int j) { for (int k = 0; k < n; ++k) R[k] = Tm.m[k]->FI[j]; return R; };
  {
    Phase ph(Tm.tc, 0);
    STEP_CHK(explicit_team(Tm, act, Uc, FEof(0)));
  }
  {
    Phase ph(Tm.tc, 1);
    STEP_CHK(implicit_team<D>(Tm, act, Uc, FIof(0)));
  }
  // stage state starts from U^n: momentum, and p' (left in pp by the implicit term)
  {
    Phase ph(Tm.tc, 2);
    STEP_CHK(pw<PwCopyM<D>>(Tm, act, [&](int k) { dg_ctx* c = Tm.m[k]; return PwCopyM<D>{c->N, c->ld, U[k], c->Us}; }));
  }
  std::vector<double> dta(n, 0.0);
  std::vector<SolveOut> so(n);
  for (int i = 1; i <= 2; ++i) {
    const double aii = At[i][i];
    for (int k = 0; k < n; ++k) dta[k] = dt[k] * aii;
    // predictor; Us[0] <- rho_i, mt, et, mp
    {
      Phase ph(Tm.tc, 2);
      STEP_CHK(pw<PwPredictor<D>>(Tm, act, [&](int k) {
        dg_ctx* c = Tm.m[k];
        return PwPredictor<D>{c->N, c->ld, U[k], c->FE[0], c->FE[1], c->FI[0], c->FI[1], i, A[i][0], A[i][1],
                              At[i][0], At[i][1], dt[k], dta[k], c->rbar, c->Us, c->mt, c->et, c->mp};
      }));
    }
    for (int l = 0; l < 8; ++l) {
      std::vector<int> fa;
      for (int k : act)
        if (l < Tm.m[k]->opt.fp_iters) fa.push_back(k);
      if (fa.empty()) break;
      const bool mixed = Tm.m[fa[0]]->opt.precision == DG_FP32_INNER;
      {
        Phase ph3(Tm.tc, 3);
        STEP_CHK(pw<PwCoef>(Tm, fa, [&](int k) {
          dg_ctx* c = Tm.m[k];
          return PwCoef{c->N, c->Us, c->pbar, c->pp, c->wJ, c->d_cell, c->NL, D, c->hm.L[0], c->hm.L[1], c->hm.L[2],
                        c->hm.nb[0], c->hm.nb[1], c->hm.nb[2], c->degree + 1, dta[k], c->h, c->dinv,
                        mixed ? c->h32 : (float*)nullptr, mixed ? c->dinv32 : (float*)nullptr};
        }));
        STEP_CHK(cellcoef_team(Tm, fa, dta, mixed, true));
        STEP_CHK(split_update_team(Tm, fa));
      }
      fa = alive_of(Tm, fa);
      {
        Phase ph(Tm.tc, 4);
        // b = -dta C(h m') + M (e~ - rho k - pbar/(gamma-1))
        STEP_CHK(energy_div_team<double>(
            Tm, fa, 7,
            [&](int k) {
              dg_ctx* c = Tm.m[k];
              return DivArgs<double>{c->mp, c->h, nullptr, nullptr, 1.0, c->lam, -dta[k], 0.0, 0.0, 1, c->b,
                                     nullptr, nullptr};
            },
            [&](int) { return 0.0; }));
        STEP_CHK(pw<PwRhsAdd<D>>(Tm, fa, [&](int k) {
          dg_ctx* c = Tm.m[k];
          return PwRhsAdd<D>{c->N, c->ld, c->b, c->wJ, c->et, c->Us, c->pbar};
        }));
        // r0 = b - A p'
        std::vector<ApItem<double>> it;
        for (int k : fa) it.push_back(ApItem<double>{k, dta[k], Tm.m[k]->pp, nullptr, 1.0, Tm.m[k]->w, nullptr});
        STEP_CHK(apply_A_team<double>(Tm, it));
        STEP_CHK(pw<PwSub>(Tm, fa, [&](int k) { dg_ctx* c = Tm.m[k]; return PwSub{c->N, c->b, c->w, c->r0}; }));
      }
      fa = alive_of(Tm, fa);
      {
        Phase ph(Tm.tc, 5);
        st = mixed ? solve_mixed_team(Tm, fa, dta, so) : solve64_team(Tm, fa, dta, so);
        if (st) return st;
      }
      for (int k : fa) {
        S[k].gmres_iters[i - 1][l] = so[k].its;
        S[k].outer_iters[i - 1][l] = so[k].outer;
        S[k].gmres_relres[i - 1][l] = so[k].relres;
      }
      act = alive_of(Tm, act);
      fa = alive_of(Tm, fa);
      {
        Phase ph(Tm.tc, 6);
        STEP_CHK(pw<PwAdd>(Tm, fa, [&](int k) { return PwAdd{Tm.m[k]->N, Tm.m[k]->pp, Tm.m[k]->delta}; }));
        STEP_CHK(grad_team<double>(
            Tm, fa, 7,
            [&](int k) { dg_ctx* c = Tm.m[k]; return GradArgs<double>{c->pp, nullptr, 1.0, c->q, nullptr, nullptr}; },
            [&](int) { return 0.0; }));
        STEP_CHK(pw<PwBacksub<D>>(Tm, fa, [&](int k) {
          dg_ctx* c = Tm.m[k];
          return PwBacksub<D>{c->N, c->ld, c->mp, c->q, dta[k], c->Us};
        }));
      }
      if (stats) {
        // fixed-point increment |delta| / |p'| (one reduction pass: delta.delta, delta.p', p'.p')
        std::vector<DotItem<double>> it;
        for (int k : fa) it.push_back(DotItem<double>{k, nullptr, Tm.m[k]->delta, Tm.m[k]->pp});
        STEP_CHK(dots_team<double>(Tm, 0, it));
        STEP_CHK(fetch(Tm, fa));
        for (int k : fa) {
          const double* r3 = Tm.hslot(k) + 2;
          S[k].fp_incr[i - 1][l] = r3[2] > 0.0 ? std::sqrt(r3[0] / r3[2]) : std::sqrt(r3[0]);
        }
      }
    }
    {
      Phase ph(Tm.tc, 2);
      STEP_CHK(pw<PwStageFinish<D>>(Tm, act, [&](int k) {
        dg_ctx* c = Tm.m[k];
        return PwStageFinish<D>{c->N, c->ld, c->Us, c->pp, c->pbar, c->mt, c->et, dta[k], c->FI[i]};
      }));
    }
    {
      Phase ph(Tm.tc, 0);
      STEP_CHK(explicit_team(Tm, act, Usc, FEof(i)));
    }
  }
  {
    Phase ph(Tm.tc, 2);
    STEP_CHK(pw<PwFinal<D>>(Tm, act, [&](int k) {
      dg_ctx* c = Tm.m[k];
      return PwFinal<D>{c->N, c->ld, U[k], c->FE[0], c->FE[1], c->FE[2], c->FI[0], c->FI[1], c->FI[2],
                        bw[0], bw[1], bw[2], dt[k], c->Un};
    }));
  }
  Phase ph7(Tm.tc, 7);
  STEP_CHK(pw<PwZero>(Tm, act, [&](int k) { return PwZero{1, Tm.slot(k) + kFlagAt}; }));
  STEP_CHK(pw<PwNonfinite>(Tm, act, [&](int k) {
    dg_ctx* c = Tm.m[k];
    return PwNonfinite{(long)c->F * c->ld, c->Un, Tm.slot(k) + kFlagAt};
  }));
  STEP_CHK(fetch(Tm, act));
  for (int k : act)
    if (Tm.hslot(k)[kFlagAt] != 0.0) drop(Tm, k, DG_ENAN, "non-finite value in the new state");
  act = alive_of(Tm, act);
  if (!Tm.shared) {
      for (int k : act)
      TCHK(Tm, hipMemcpyAsync(U[k], Tm.m[k]->Un, (size_t)Tm.m[k]->F * Tm.m[k]->ld * sizeof(double),
                          hipMemcpyDeviceToDevice, Tm.s));
  } else {
    STEP_CHK(pw<PwCopy>(Tm, act, [&](int k) {
      dg_ctx* c = Tm.m[k];
      return PwCopy{(long)c->F * c->ld, c->Un, U[k]};
    }));
  }
  if (stats) {
    STEP_CHK(diagnostics_team(Tm, act, Uc));
    for (int k : act) {
      S[k].mass = Tm.hslot(k)[3];
      S[k].max_w = Tm.hslot(k)[kMaxAt];
    }
    ph7.end();
    if (Tm.tc) {
      dg_ctx* c = Tm.tc;
      HIPCHK(hipStreamSynchronize(Tm.s));
      S[0].t_step_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      for (int e = 0; e < c->ev_n; ++e) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * e], c->ev[2 * e + 1]));
        S[0].t_kernel_ms[c->ev_cls[e]] += ms;
        S[0].n_kernel[c->ev_cls[e]] += 1;
      }
      for (int k = 0; k < 8; ++k) S[0].bytes_kernel[k] = c->kbytes[k];
      for (int e = 0; e < c->pev_n; ++e) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->pev[2 * e], c->pev[2 * e + 1]));
        S[0].t_phase_ms[c->pev_cls[e]] += ms;
      }
    }
  }
#undef STEP_CHK
  if (stats)
    for (int k = 0; k < n; ++k) stats[k] = S[k];
  return DG_OK;
}

}  // namespace

// ====================================================================================== C ABI
extern "C" {

void dg_default_options(dg_options* o) {
  if (!o) return;
  o->fp_iters = 2;
  o->gmres_restart = 15;
  o->gmres_maxit = 2000;
  o->gmres_rtol = 1e-12;
  o->gmres_atol = 0.0;
  o->precision = DG_FP64;
  o->inner_rtol = 1e-4;
  o->inner_restart = 30;
  o->inner_maxit = 500;
  o->penalty_beta = 1.0;
  o->preconditioner = DG_PREC_CELL_FDM;
  o->quad_extra = 0;
  o->enthalpy_split = 0;
}

const char* dg_last_error(const dg_ctx* c) {
  if (c && !c->err.empty()) return c->err.c_str();
  return g_last_error.c_str();
}

dg_status dg_footprint(const dg_case_desc* desc, int32_t degree, const dg_options* opt, size_t* bytes) {
  if (!bytes) return fail(nullptr, DG_EINVAL, "null output");
  dg_ctx tmp;
  dg_status st = prepare(&tmp, desc, degree, opt);
  if (st) return st;
  Plan P;
  make_plan(&tmp, P);
  *bytes = P.total;
  return DG_OK;
}

dg_status dg_mesh_info(const dg_case_desc* desc, int32_t degree, int64_t* n_cells, int64_t* n_hanging,
                       int32_t* cells_out) {
  if (!desc) return fail(nullptr, DG_EINVAL, "null description");
  HostMesh M;
  std::string err;
  const int rc = build_mesh(*desc, degree, M, err);
  if (rc != DG_OK) return fail(nullptr, (dg_status)rc, err);
  if (n_cells) *n_cells = M.ncell;
  if (n_hanging) *n_hanging = M.nhang;
  if (cells_out) {
    for (int i = 0; i < M.ncell; ++i) {
      const int* ci = &M.cell[4 * i];
      cells_out[4 * i] = ci[0];
      cells_out[4 * i + 1] = ci[1];
      cells_out[4 * i + 2] = M.dim == 3 ? ci[2] : 0;
      cells_out[4 * i + 3] = M.dim == 3 ? ci[3] : ci[2];
    }
  }
  return DG_OK;
}

dg_status dg_setup(const dg_case_desc* desc, int32_t degree, const dg_options* opt, void* stream, dg_ctx** out) {
  if (!out) return fail(nullptr, DG_EINVAL, "null output");
  *out = nullptr;
  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) return fail(nullptr, DG_ENOMEM, "host allocation failed");
  dg_status st = prepare(c, desc, degree, opt);
  if (st) { delete c; return st; }
  c->stream = (hipStream_t)stream;
  {
    double* sp = nullptr;
    st = scratch_ptr(c, &sp);
    if (st) { delete c; return st; }
  }
  Plan P;
  make_plan(c, P);
  hipError_t e = hipMalloc((void**)&c->arena, P.total);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, DG_ENOMEM, std::string("hipMalloc of the workspace failed: ") + hipGetErrorString(e));
  }
  c->arena_bytes = P.total;
  size_t off = 0;
  for (auto& it : P.items) {
    *it.first = c->arena + off;
    off += (it.second + 255) & ~size_t(255);
  }
  e = hipHostMalloc((void**)&c->hred, (size_t)kTeamMax * (kResStride + kCoefStride) * sizeof(double),
                    hipHostMallocDefault);
  if (e != hipSuccess) { dg_destroy(c); return fail(nullptr, DG_ENOMEM, "pinned host allocation failed"); }
  // upload mesh and tables
  const HostMesh& M = c->hm;
  std::vector<int4> cells(M.ncell), nbr((size_t)M.ncell * 2 * c->D);
  for (int i = 0; i < M.ncell; ++i) cells[i] = make_int4(M.cell[4 * i], M.cell[4 * i + 1], M.cell[4 * i + 2], M.cell[4 * i + 3]);
  for (size_t i = 0; i < nbr.size(); ++i) nbr[i] = make_int4(M.fnbr[4 * i], M.fnbr[4 * i + 1], M.fnbr[4 * i + 2], M.fnbr[4 * i + 3]);
  std::vector<double> tab = make_tables(c->degree + 1);
  std::vector<double> oitab;
  if (c->opt.quad_extra > 0) oitab = make_oi_tables(c->degree + 1, c->degree + 1 + c->opt.quad_extra);
  std::vector<float> tabf(tab.begin(), tab.end());
  hipStream_t s = c->stream;
#define SETUP_CHK(call)                                                             \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      std::string msg = std::string(#call) + ": " + hipGetErrorString(e_);         \
      dg_destroy(c);                                                                \
      return fail(nullptr, DG_EDEVICE, msg);                                        \
    }                                                                               \
  } while (0)
  SETUP_CHK(hipMemcpyAsync(c->d_cell, cells.data(), cells.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  SETUP_CHK(hipMemcpyAsync(c->d_fkind, M.fkind.data(), M.fkind.size() * sizeof(int), hipMemcpyHostToDevice, s));
  std::vector<int> lists;
  lists.reserve(M.ncell);
  int nreg = 0;
  {
    const int NF = 2 * c->D;
    std::vector<int> irr;
    for (int i = 0; i < M.ncell; ++i) {
      bool reg = true;
      for (int f = 0; f < NF; ++f) {
        const int k = M.fkind[(size_t)i * NF + f];
        if (k == kFine || k == kCoarse) reg = false;
      }
      if (reg) lists.push_back(i);
      else irr.push_back(i);
    }
    nreg = (int)lists.size();
    lists.insert(lists.end(), irr.begin(), irr.end());
  }
  if (M.ncell > 0)
    SETUP_CHK(hipMemcpyAsync(c->d_lists, lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice, s));
  std::vector<int> runs, rflags;
  build_runs(M, c->D, col_cpb(c), runs, rflags);
  if (runs.size() != (size_t)run_slots(c)) {
    dg_destroy(c);
    return fail(nullptr, DG_EINVAL, "vertical runs do not cover the mesh");
  }
  {
    long seen = 0;
    for (int v : runs) seen += v >= 0;
    if (seen != M.ncell) {
      dg_destroy(c);
      return fail(nullptr, DG_EINVAL, "vertical runs do not cover every cell once");
    }
  }
  c->nrun_slots = (int)runs.size();
  if (!runs.empty()) {
    SETUP_CHK(hipMemcpyAsync(c->d_runs, runs.data(), runs.size() * sizeof(int), hipMemcpyHostToDevice, s));
    SETUP_CHK(hipMemcpyAsync(c->d_runs + runs.size(), rflags.data(), rflags.size() * sizeof(int),
                             hipMemcpyHostToDevice, s));
  }
  SETUP_CHK(hipMemcpyAsync(c->d_fnbr, nbr.data(), nbr.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  SETUP_CHK(hipMemcpyAsync(c->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
  SETUP_CHK(hipMemcpyAsync(c->d_tabf, tabf.data(), tabf.size() * sizeof(float), hipMemcpyHostToDevice, s));
  if (!oitab.empty())
    SETUP_CHK(hipMemcpyAsync(c->d_oitab, oitab.data(), oitab.size() * sizeof(double), hipMemcpyHostToDevice, s));
  MeshDev& md = c->md;
  md.dim = c->D;
  md.ncell = M.ncell;
  md.N = c->ld;  // field stride
  md.cell = c->d_cell;
  md.fkind = c->d_fkind;
  md.fnbr = c->d_fnbr;
  md.reg = c->d_lists;
  md.nreg = nreg;
  md.irr = c->d_lists + nreg;
  md.runs = c->d_runs;
  md.rflag = c->d_runs + c->nrun_slots;
  md.nrwg = c->nrun_slots / col_cpb(c);
  md.nirr = M.ncell - nreg;
  md.tab = c->d_tab;
  md.tabf = c->d_tabf;
  md.oitab = c->d_oitab;
  md.nq = c->opt.quad_extra > 0 ? c->degree + 1 + c->opt.quad_extra : 0;
  for (int a = 0; a < 3; ++a) {
    md.L[a] = M.L[a];
    md.nb[a] = M.nb[a];
    md.per[a] = M.per[a];
  }
  md.ter = Terrain{c->desc.orography, c->desc.oro[0], c->desc.oro[1], c->desc.oro[2], c->desc.oro[3],
                   1.0 / (c->desc.oro[1] * c->desc.oro[1])};
  md.invH = 1.0 / M.L[c->D - 1];
  for (int i = 0; i < 5; ++i) md.sponge[i] = c->desc.sponge[i];
  for (int l = 0; l < kMaxLev; ++l)
    for (int a = 0; a < 3; ++a) {
      md.nlev[l][a] = M.nb[a] << l;
      md.dxl[l][a] = M.L[a] / (double)(M.nb[a] << l);
    }
  {
    MeshDev g = md;
    g.N = c->N;  // geometry kernel iterates over N nodes
    if (launch_geometry(g, c->degree, nullptr, nullptr, nullptr, c->wJ, c->pbar, c->rbar, c->tau,
                        c->desc.atmosphere, c->desc.atm, s)) {
      dg_destroy(c);
      return fail(nullptr, DG_EDEVICE, "geometry kernel launch failed");
    }
    if (c->opt.enthalpy_split)
      hipLaunchKernelGGL(k_hbar, pw_grid(c->N), dim3(256), 0, s, (const double*)c->pbar, (const double*)c->rbar,
                         c->desc.atmosphere == DG_ATM_STRATIFIED ? 1 : 0, c->desc.atm[2], c->N, c->hb, c->dhb,
                         c->hb32, c->dhb32);
  }
  SETUP_CHK(hipMemcpyAsync(c->d_md, &c->md, sizeof(MeshDev), hipMemcpyHostToDevice, s));
  SETUP_CHK(hipStreamSynchronize(s));
#undef SETUP_CHK
  *out = c;
  return DG_OK;
}

void dg_destroy(dg_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  for (auto& e : c->pev) (void)hipEventDestroy(e);
  if (c->arena) (void)hipFree(c->arena);
  if (c->hred) (void)hipHostFree(c->hred);
  delete c;
}

dg_status dg_set_stream(dg_ctx* c, void* stream) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  c->stream = (hipStream_t)stream;
  return DG_OK;
}

dg_status dg_set_timing(dg_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  c->timing = enable != 0;
  if (c->timing && c->ev.empty()) {
    c->ev.resize(2 * kEvPool);
    c->ev_cls.assign(kEvPool, 0);
    for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
    c->pev.resize(2 * kPhasePool);
    c->pev_cls.assign(kPhasePool, 0);
    for (auto& e : c->pev) HIPCHK(hipEventCreate(&e));
  }
  return DG_OK;
}

dg_status dg_sizes(const dg_ctx* c, int64_t* n_cells, int64_t* nodes, int32_t* nf) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  if (n_cells) *n_cells = c->hm.ncell;
  if (nodes) *nodes = c->N;
  if (nf) *nf = c->F;
  return DG_OK;
}

dg_status dg_cell_table(const dg_ctx* c, int32_t* out) {
  if (!c || !out) return fail(nullptr, DG_EINVAL, "null argument");
  for (int i = 0; i < c->hm.ncell; ++i) {
    const int* ci = &c->hm.cell[4 * i];
    out[4 * i] = ci[0];
    if (c->D == 3) {
      out[4 * i + 1] = ci[1];
      out[4 * i + 2] = ci[2];
      out[4 * i + 3] = ci[3];
    } else {
      out[4 * i + 1] = ci[1];
      out[4 * i + 2] = 0;
      out[4 * i + 3] = ci[2];
    }
  }
  return DG_OK;
}

dg_status dg_node_geometry(dg_ctx* c, double* x, double* y, double* z, double* wJ) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  MeshDev g = c->md;
  g.N = c->N;
  if (launch_geometry(g, c->degree, x, y, z, wJ, nullptr, nullptr, nullptr, c->desc.atmosphere, c->desc.atm,
                      c->stream))
    return fail(c, DG_EDEVICE, "geometry kernel launch failed");
  return DG_OK;
}

dg_status dg_init_state(dg_ctx* c, int32_t ic_kind, const double* ic_params, uint64_t noise_seed,
                        double noise_sigma_K, double* U) {
  if (!c || !U || !ic_params) return fail(c, DG_EINVAL, "null argument");
  if (ic_kind != DG_IC_HYDROSTATIC_WIND) return fail(c, DG_EINVAL, "unknown initial-condition kind");
  if (!(noise_sigma_K >= 0.0) || !std::isfinite(noise_sigma_K))
    return fail(c, DG_EINVAL, "noise sigma must be finite and >= 0");
  const double ubar = ic_params[0];
  if (!std::isfinite(ubar)) return fail(c, DG_EINVAL, "wind must be finite");
  if (c->D == 2)
    hipLaunchKernelGGL((k_init_state<2>), pw_grid(c->N), dim3(256), 0, c->stream, c->pbar, c->rbar, c->d_cell,
                       c->NL, noise_seed, noise_sigma_K, ubar, c->N, c->ld, U);
  else
    hipLaunchKernelGGL((k_init_state<3>), pw_grid(c->N), dim3(256), 0, c->stream, c->pbar, c->rbar, c->d_cell,
                       c->NL, noise_seed, noise_sigma_K, ubar, c->N, c->ld, U);
  HIPCHK(hipGetLastError());
  return DG_OK;
}

dg_status dg_explicit_residual(dg_ctx* c, const double* U, double* R) {
  if (!c || !U || !R) return fail(nullptr, DG_EINVAL, "null argument");
  Team T = solo(c);
  const dg_status st = explicit_team(T, {0}, {U}, {R});
  return st ? st : T.st[0];
}

dg_status dg_implicit_term(dg_ctx* c, const double* U, double* F) {
  if (!c || !U || !F) return fail(nullptr, DG_EINVAL, "null argument");
  Team T = solo(c);
  const dg_status st = c->D == 2 ? implicit_team<2>(T, {0}, {U}, {F}) : implicit_team<3>(T, {0}, {U}, {F});
  return st ? st : T.st[0];
}

dg_status dg_apply_helmholtz(dg_ctx* c, double dta, const void* h, const void* p, void* Ap, int32_t prec) {
  if (!c || !h || !p || !Ap) return fail(nullptr, DG_EINVAL, "null argument");
  const long N = c->N;
  Team T = solo(c);
  dg_status st;
  if (prec == DG_FP64) {
    HIPCHK(hipMemcpyAsync(c->h, h, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if ((st = lam_team(T, {0}, false)) || (st = split_update_team(T, {0}))) return st;
    return apply_A_team<double>(T, {ApItem<double>{0, dta, (const double*)p, nullptr, 1.0, (double*)Ap, nullptr}});
  }
  if (prec == DG_FP32_INNER) {
    if (c->opt.precision != DG_FP32_INNER)
      return fail(c, DG_EINVAL, "context was set up without the FP32 workspace (precision option)");
    // h in FP32: copy, and widen to FP64 for the per-cell sound speed
    HIPCHK(hipMemcpyAsync(c->h32, h, N * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    if ((st = pw<PwWiden>(T, {0}, [&](int) { return PwWiden{N, c->h32, c->h}; }))) return st;
    if ((st = lam_team(T, {0}, true)) || (st = split_update_team(T, {0}))) return st;
    return apply_A_team<float>(T, {ApItem<float>{0, dta, (const float*)p, nullptr, 1.0f, (float*)Ap, nullptr}});
  }
  return fail(c, DG_EINVAL, "bad precision");
}

dg_status dg_apply_preconditioner(dg_ctx* c, double dta, const double* h, const void* v, void* z, int32_t prec) {
  if (!c || !h || !v || !z) return fail(nullptr, DG_EINVAL, "null argument");
  const bool mixed = prec == DG_FP32_INNER;
  if (prec != DG_FP64 && !mixed) return fail(c, DG_EINVAL, "bad precision");
  if (mixed && c->opt.precision != DG_FP32_INNER)
    return fail(c, DG_EINVAL, "context was set up without the FP32 workspace (precision option)");
  // per-cell coefficients from h, as in the step (FP64, with an FP32 copy for the mixed form)
  if (launch_cellcoef(c->md, c->degree, h, c->wJ, dta, c->lam, mixed ? c->lam32 : nullptr, c->coef,
                      mixed ? c->coef32 : nullptr, c->stream))
    return fail(c, DG_EDEVICE, "launch failed");
  int rf;
  if (mixed) {
    FdmArgs<float> f{(const float*)v, 1.0f, c->coef32, (float*)z, nullptr};
    rf = launch_fdm32(c->md, c->degree, f, c->stream);
  } else {
    FdmArgs<double> f{(const double*)v, 1.0, c->coef, (double*)z, nullptr};
    rf = launch_fdm64(c->md, c->degree, f, c->stream);
  }
  if (rf) return fail(c, DG_EDEVICE, "launch failed");
  return DG_OK;
}

dg_status imex_rk2_step(dg_ctx* c, double* U, double dt, dg_step_stats* stats) {
  if (!c || !U) return fail(nullptr, DG_EINVAL, "null argument");
  if (!(dt > 0.0)) return fail(c, DG_EINVAL, "dt must be positive");
  Team T = solo(c);
  double* Us[1] = {U};
  const dg_status st = c->D == 2 ? step_team<2>(T, Us, &dt, stats) : step_team<3>(T, Us, &dt, stats);
  return st ? st : T.st[0];
}

dg_status imex_rk2_step_batched(dg_ctx* const* ctxs, double* const* Us, const double* dts, int32_t n,
                                dg_step_stats* stats, int32_t* status) {
  if (n < 0 || (n > 0 && (!ctxs || !Us || !dts))) return fail(nullptr, DG_EINVAL, "bad batch");
  std::vector<dg_status> rc(n, DG_OK);
  std::vector<std::string> msg(n);
  // members of one class share launches: same dimension, degree, precision, preconditioner and
  // energy-flux form (the kernels and the control flow of the step); a class is cut into teams of
  // at most kTeamMax, and the teams run on their own host threads and lead streams
  std::vector<std::vector<int>> teams;
  {
    std::vector<int> cls(n, -1);
    std::vector<int> rep;
    for (int i = 0; i < n; ++i) {
      dg_ctx* c = ctxs[i];
      if (!c || !Us[i]) { rc[i] = DG_EINVAL; msg[i] = "null member"; continue; }
      if (!(dts[i] > 0.0)) { rc[i] = DG_EINVAL; msg[i] = "dt must be positive"; continue; }
      bool dup = false;
      for (int q = 0; q < i && !dup; ++q) dup = ctxs[q] == c && cls[q] >= 0;
      if (dup) { rc[i] = DG_EINVAL; msg[i] = "context appears twice in the batch"; continue; }
      for (int r = 0; r < (int)rep.size() && cls[i] < 0; ++r) {
        const dg_ctx* q = ctxs[rep[r]];
        if (q->D == c->D && q->degree == c->degree && q->opt.precision == c->opt.precision &&
            q->opt.preconditioner == c->opt.preconditioner && q->opt.enthalpy_split == c->opt.enthalpy_split)
          cls[i] = r;
      }
      if (cls[i] < 0) {
        cls[i] = (int)rep.size();
        rep.push_back(i);
      }
    }
    for (int r = 0; r < (int)rep.size(); ++r) {
      std::vector<int> t;
      for (int i = 0; i < n; ++i) {
        if (cls[i] != r) continue;
        t.push_back(i);
        if ((int)t.size() == kTeamMax) {
          teams.push_back(t);
          t.clear();
        }
      }
      if (!t.empty()) teams.push_back(t);
    }
  }
  const auto t0 = std::chrono::steady_clock::now();
  auto run = [&](const std::vector<int>& mem) {
    Team T;
    T.lead = ctxs[mem[0]];
    T.s = T.lead->stream;
    T.shared = true;
    std::vector<double*> U;
    std::vector<double> dt;
    for (int i : mem) {
      T.m.push_back(ctxs[i]);
      U.push_back(Us[i]);
      dt.push_back(dts[i]);
      // work queued on a member's own stream comes first
      if (ctxs[i]->stream != T.s) (void)hipStreamSynchronize(ctxs[i]->stream);
    }
    T.st.assign(mem.size(), DG_OK);
    std::vector<dg_step_stats> S(mem.size());
    const dg_status st = T.m[0]->D == 2 ? step_team<2>(T, U.data(), dt.data(), stats ? S.data() : nullptr)
                                        : step_team<3>(T, U.data(), dt.data(), stats ? S.data() : nullptr);
    (void)hipStreamSynchronize(T.s);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (size_t q = 0; q < mem.size(); ++q) {
      const int i = mem[q];
      rc[i] = st && T.st[q] == DG_OK ? st : T.st[q];
      if (rc[i]) msg[i] = ctxs[i]->err;
      if (stats) {
        stats[i] = S[q];
        stats[i].t_step_ms = ms;
      }
    }
  };
  if (teams.size() == 1) {
    run(teams[0]);
  } else {
    std::vector<std::thread> th;
    for (const auto& t : teams) th.emplace_back(run, std::cref(t));
    for (auto& t : th) t.join();
  }
  dg_status first = DG_OK;
  for (int i = 0; i < n; ++i) {
    if (status) status[i] = rc[i];
    if (rc[i] && first == DG_OK) {
      first = rc[i];
      g_last_error = "member " + std::to_string(i) + ": " + msg[i];
    }
  }
  return first;
}

dg_status dg_diagnostics(dg_ctx* c, const double* U, double* mass, double* max_w) {
  if (!c || !U) return fail(nullptr, DG_EINVAL, "null argument");
  Team T = solo(c);
  const dg_status st = diagnostics_team(T, {0}, {U});
  if (st) return st;
  if (mass) *mass = T.hslot(0)[3];
  if (max_w) *max_w = T.hslot(0)[kMaxAt];
  return DG_OK;
}

dg_status dg_diagnostics_noalloc(dg_ctx* c, const double* U, double* mass, double* max_w) {
  if (!c || !U || !mass || !max_w) return fail(c, DG_EINVAL, "null argument");
  const long N = c->N;
  const int G = red_grid(N);
  if (G > kScratchGrid) return fail(c, DG_EINVAL, "reduction grid exceeds the scratch array");
  double* sp = nullptr;
  dg_status st = scratch_ptr(c, &sp);
  if (st) return st;
  double* part = sp;                      // 3 x G partials of the mass pass
  double* pmax = sp + 3 * kScratchGrid;   // G partials of the maximum
  double* res = sp + 4 * kScratchGrid;    // [0..2] the mass pass's sums, [3] the maximum
  // every partial the second stages read is written by the first stages of this call
  launch_gs_dots<double>(0, G, c->stream, (const double*)nullptr, c->ld, c->wJ, U, part, N);
  hipLaunchKernelGGL(k_reduce, dim3(3), dim3(kRedThreads), 0, c->stream, part, G, res);
  hipLaunchKernelGGL(k_maxabs_ratio, dim3(G), dim3(kRedThreads), 0, c->stream, U + (size_t)c->D * c->ld, U, pmax, N);
  hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(kRedThreads), 0, c->stream, pmax, G, res + 3);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(mass, res + 1, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(max_w, res + 3, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DG_OK;
}

}  // extern "C"
