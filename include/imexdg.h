/*
 * imexdg.h — C ABI of the MI355X (gfx950) IMEX-DG library for the compressible Euler equations.
 *
 * The method is the one of Orlando, Benacchio, Bonaventura, "Efficient and scalable atmospheric
 * dynamics simulations using non-conforming meshes" (arXiv 2408.08129):
 *   - Section 2, Eq. (1): Euler equations for rho, rho u, rho E in SI units (g = 9.81, R = 287,
 *     gamma = 1.4) on a domain of dimension d = 2 (x-z slice) or 3;
 *   - Section 2: DG in space on quadrilaterals / hexahedra with 2:1 non-conforming faces, second
 *     order IMEX Runge-Kutta in time, continuity explicit and energy coupled implicitly to momentum;
 *   - Section 3.2: matrix-free operator action; the pressure fixed-point loop of each implicit
 *     stage solves a non-symmetric linear system with GMRES;
 *   - Section 3.1: terrain-following geometry over orography (Eq. (3) and variants) and the
 *     stratified hydrostatic atmosphere of Eq. (4)-(5).
 *
 * Conventions shared by every call.
 *   - Status: every function returns dg_status (DG_OK = 0, errors negative); no exception crosses
 *     the ABI.  dg_last_error(ctx) returns a message for the last error.
 *   - Memory: pointers named *_dev are device pointers (HIP device memory, e.g. torch tensors on a
 *     ROCm device), borrowed for the duration of the call.  All device work is ordered on the HIP
 *     stream given to dg_setup (or dg_set_stream); a call returns when its work is queued, except
 *     calls that return host values (they synchronise that stream).
 *   - Layout of a state U: FP64, structure of arrays U[f][cell][node] with fields
 *     f = (rho, rho u, rho w, rho E) in 2D and (rho, rho u, rho v, rho w, rho E) in 3D; cells in
 *     the order reported by dg_cell_table; nodes at the tensor Gauss-Legendre points of degree r,
 *     lexicographic with x fastest (2D: x then z).  Scalars (pressure, enthalpy) are [cell][node].
 *   - Ownership: the context owns the mesh tables and all workspace, allocated in dg_setup and
 *     released by dg_destroy.  One context must not be used by two threads at once; different
 *     contexts are independent.
 */
#ifndef IMEXDG_H
#define IMEXDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DG_OK = 0,
  DG_EINVAL = -1,       /* invalid argument or mesh description (e.g. 2:1 violation) */
  DG_ENOMEM = -2,       /* device or host allocation failed */
  DG_EDEVICE = -3,      /* a HIP runtime call failed */
  DG_ENOCONV = -4,      /* a GMRES solve missed its tolerance within its iteration limit */
  DG_ENAN = -5,         /* a non-finite value appeared in the new state */
  DG_EUNSUPPORTED = -6  /* degree / dimension not compiled in */
} dg_status;

typedef enum { DG_FP64 = 0, DG_FP32_INNER = 1 } dg_precision;
typedef enum { DG_PREC_DIAGONAL = 0, DG_PREC_CELL_FDM = 1 } dg_preconditioner;

enum { DG_ORO_FLAT = 0, DG_ORO_AGNESI = 1, DG_ORO_BELL = 2, DG_ORO_GAUSS_HILL = 3, DG_ORO_GAUSS_RIDGE = 4 };
enum { DG_ATM_ISOTHERMAL = 0, DG_ATM_STRATIFIED = 1 };

#define DG_MAX_RULES 8

/* Refinement rule of level l (applied to cells of level l-1): refine when the logical cell centre
 * has zeta < zeta_max and |x - x_c| < half_width_x (if > 0) and |y - y_c| < half_width_y (if > 0,
 * 3D only).  Section 3.1 / Fig. 1: finer cells near the orography, coarser aloft. */
typedef struct {
  double zeta_max, x_c, half_width_x, y_c, half_width_y;
} dg_refine_rule;

/* Problem description, plain data copied at setup.
 *   sponge = (top depth, top rate, lateral width, lateral rate, u_ref): absorbing layers for the
 *     non-reflecting boundaries of Section 3.1 (whose form the paper leaves to cited work):
 *     Rayleigh friction d m/dt = -tau (m - rho u_ref e_x) in the explicit part, tau = top rate
 *     sin^2(pi/2 (z - z_s)/depth) above z_s = H - depth (physical height z) plus lateral rate
 *     sin^2(pi/2 (1 - dist/width)) within width of each lateral side (x = 0, x = Lx, and in 3D
 *     y = 0, y = Ly), walled or periodic (at a periodic seam the layer absorbs what leaves one side
 *     before it re-enters on the other); rates <= 0 switch a layer off.
 *   dim: 2 (x-z slice) or 3; nbase: base cells along x, y, z (y ignored in 2D);
 *   length: Lx, Ly, H in metres (H = rigid-lid height); periodic_x / periodic_y: 1 periodic,
 *   0 slip walls; bottom and top are slip walls;
 *   orography: DG_ORO_*, oro = (height, width a or sigma, x_c, y_c):
 *     AGNESI h a^2/(a^2+(x-x_c)^2); BELL h/(1+((x-x_c)/a)^2+((y-y_c)/a)^2)^(3/2) (Section 3.1,
 *     Eq. (3)); GAUSS_HILL h exp(-r^2/(2 sigma^2)); GAUSS_RIDGE h exp(-((x-x_c)/a)^2);
 *   atmosphere: DG_ATM_ISOTHERMAL atm = (p0, T0) or DG_ATM_STRATIFIED atm = (p_ref, T_ref, N)
 *     (Section 3.1, Eq. (4)-(5), with the factor g^2/N^2 that makes the state hydrostatic). */
typedef struct {
  int32_t dim;
  int32_t nbase[3];
  double length[3];
  int32_t periodic_x, periodic_y;
  int32_t n_rules;
  dg_refine_rule rules[DG_MAX_RULES];
  int32_t orography;
  double oro[4];
  int32_t atmosphere;
  double atm[3];
  double sponge[5];
} dg_case_desc;

/* Solver options (Section 3.2: fixed-point loop + GMRES).
 *   fp_iters: fixed-point iterations per implicit stage (>= 1);
 *   gmres_restart, gmres_maxit, gmres_rtol, gmres_atol: right-preconditioned GMRES(m), stop when
 *     ||r||_2 <= max(rtol ||r0||_2, atol);
 *   precision: DG_FP64, or DG_FP32_INNER (FP64 defect correction around an FP32 GMRES whose
 *     operator, preconditioner and basis are FP32; inner_rtol / inner_restart / inner_maxit);
 *   penalty_beta: weight of the pressure-jump penalty in the implicit energy flux;
 *   preconditioner: DG_PREC_DIAGONAL (a diagonal scaling) or DG_PREC_CELL_FDM (cell-wise fast
 *     diagonalisation of a separable approximation of the cell block); changes iteration counts
 *     only, not the converged solution;
 *   quad_extra: over-integration of the explicit advective flux (de-aliasing of the nonlinear
 *     terms): its volume and face integrals use degree + 1 + quad_extra Gauss points per direction
 *     (on a 2:1 face the fine sub-face's points), the mass matrix stays the nodal one and the
 *     gravity work pointwise; 0 (default) keeps the nodal rule.  quad_extra <= 3 and
 *     degree + 1 + quad_extra <= 8, else DG_EUNSUPPORTED; negative: DG_EINVAL;
 *   enthalpy_split: 1 splits the implicit energy flux div(h m) into the perturbation part
 *     div((h - hbar) m) and the background part hbar div(m) + m . grad(hbar), the latter with the
 *     continuity equation's discrete divergence and the exact height derivative of the background
 *     enthalpy hbar = gamma pbar / ((gamma - 1) rhobar); this keeps the discrete buoyancy balance
 *     of grid-scale modes stable in a stratified atmosphere (with the plain flux they grow, with
 *     e-folding times of 20-60 s; long runs also need penalty_beta = 0).  0 (default): plain. */
typedef struct {
  int32_t fp_iters;
  int32_t gmres_restart;
  int32_t gmres_maxit;
  double gmres_rtol;
  double gmres_atol;
  int32_t precision;
  double inner_rtol;
  int32_t inner_restart;
  int32_t inner_maxit;
  double penalty_beta;
  int32_t preconditioner;
  int32_t quad_extra;
  int32_t enthalpy_split;
} dg_options;

/* Per-step statistics ([implicit stage][fixed-point iteration]) of the pressure fixed-point loop
 * and its GMRES solves (Section 3.2). */
typedef struct {
  int32_t gmres_iters[2][8];    /* Krylov iterations (FP32 inner iterations in mixed mode) */
  int32_t outer_iters[2][8];    /* defect-correction sweeps (mixed mode), 0 for FP64 */
  double gmres_relres[2][8];    /* final ||r|| / ||r0|| */
  double fp_incr[2][8];         /* fixed-point increment ||delta||_2 / ||p'||_2 after the iteration */
  double t_phase_ms[8];         /* with dg_set_timing on: device time per phase of the step, from HIP
                                   events at the phase boundaries on the context's stream:
                                   0 explicit residuals, 1 implicit term at U^n, 2 stage predictors,
                                   stage ends and final combination, 3 fixed-point coefficients,
                                   4 Helmholtz right-hand side and initial residual, 5 Krylov
                                   solves, 6 back-substitution, 7 non-finite check, copy-out and
                                   diagnostics */
  double t_kernel_ms[8];        /* with dg_set_timing on: device time summed per kernel class,
                                   from HIP events around every launch on the context's stream:
                                   0 explicit residual, 1 Helmholtz apply pass 1 (h M^-1 B p),
                                   2 Helmholtz apply pass 2 (divergence, penalty, mass),
                                   3 Gram-Schmidt reduction pass (k_gs_dots), 4 pointwise vector
                                   work and preconditioner, 5 Gram-Schmidt update pass
                                   (k_gs_update), 6 Krylov solution update and final reductions,
                                   7 the other operator passes (right-hand side divergence,
                                   implicit term, back-substitution gradient) */
  int32_t n_kernel[8];          /* launches per class (timing on) */
  double bytes_kernel[8];       /* algorithmic HBM bytes per class (timing on): the arrays each
                                   launch must read and write once, as the kernels are designed */
  double t_step_ms;             /* host wall time of the step (timing on) */
  double mass, max_w;           /* diagnostics of the new state */
} dg_step_stats;

typedef struct dg_ctx dg_ctx;

/* Fills *opt with the defaults: fp_iters 2, GMRES(15), rtol 1e-12, atol 0, maxit 2000, FP64,
 * inner_rtol 1e-4, inner_restart 30, inner_maxit 500, penalty_beta 1, DG_PREC_CELL_FDM.
 * (GMRES restart 15 keeps the iteration counts of restart 30 on the 3D hill case at about half
 * the orthogonalisation traffic.) */
void dg_default_options(dg_options* opt);

/* Sets up the discretisation of Section 2 on the mesh of Section 3.1 / Fig. 1: builds the mesh
 * (base grid refined by the rules, 2:1 balance check, Morton order of the leaves), uploads its
 * tables and allocates the whole workspace (dg_footprint bytes) on the current device.
 * degree r in [1, 5]: the paper runs r = 4 (and r = 2 in its scaling study, Section 3.2); r = 6
 * would need 343-node cells, beyond the 256-thread workgroups and the static LDS budget of the
 * cell kernels, so it is rejected with DG_EUNSUPPORTED.  desc and opt (NULL: defaults) are copied;
 * stream: a hipStream_t (NULL = default stream); *out receives the new context, owned by the
 * caller until dg_destroy.  Errors: DG_EINVAL (null pointers, bad description, 2:1 violation),
 * DG_EUNSUPPORTED, DG_ENOMEM (device memory), DG_EDEVICE; *out is left NULL on error. */
dg_status dg_setup(const dg_case_desc* desc, int32_t degree, const dg_options* opt, void* stream,
                   dg_ctx** out);

/* Exact device bytes dg_setup would allocate for this description (mesh tables, geometry and the
 * step and Krylov workspace of Section 3.2's solver), without allocating or touching the device;
 * used to admit ensemble members by HBM footprint.  Errors as dg_setup. */
dg_status dg_footprint(const dg_case_desc* desc, int32_t degree, const dg_options* opt,
                       size_t* bytes);

/* Host-only mesh query (no device work): number of cells, number of hanging sub-faces (each
 * counted once) and, if cells_out != NULL, the cell table in the order dg_setup uses
 * (4 int32 per cell, as dg_cell_table).  Errors as dg_setup. */
dg_status dg_mesh_info(const dg_case_desc* desc, int32_t degree, int64_t* n_cells,
                       int64_t* n_hanging, int32_t* cells_out);

/* Replaces the HIP stream on which the context orders its work (the caller keeps ownership of the
 * stream and synchronises any switch).  DG_EINVAL for a null ctx. */
dg_status dg_set_stream(dg_ctx* ctx, void* stream);

/* enable != 0: every later step records HIP events around its launches and phases (the per-class
 * and per-phase device times of dg_step_stats); allocates the event pool on first use.
 * DG_EINVAL for a null ctx, DG_EDEVICE if an event cannot be created. */
dg_status dg_set_timing(dg_ctx* ctx, int32_t enable);

/* Cells, nodes per scalar field N = cells (r + 1)^d (the per-scalar unknown count of Section 3.2)
 * and fields d + 2 (Eq. (1): rho, the d momentum components, rho E); any output may be NULL. */
dg_status dg_sizes(const dg_ctx* ctx, int64_t* n_cells, int64_t* nodes_per_field,
                   int32_t* n_fields);

/* The cells of the non-conforming mesh (Section 3.1, Fig. 1) in the order of the state arrays.
 * host_out: caller-owned, 4 int32 per cell: (level, i_x, i_y, i_z) at the cell's own level
 * (i_y = 0 in 2D); the cell's logical box is [i L / (n 2^level), (i + 1) L / (n 2^level)) per
 * axis.  DG_EINVAL for null pointers. */
dg_status dg_cell_table(const dg_ctx* ctx, int32_t* host_out);

/* Geometry of the terrain-following map over the orography of Section 3.1 at every node.
 * Device outputs (caller-owned, N doubles each, any may be NULL), [cell][node]: physical x, y, z
 * and the quadrature weight times the Jacobian determinant (the diagonal mass matrix).
 * Errors: DG_EINVAL for a null ctx, DG_EDEVICE. */
dg_status dg_node_geometry(dg_ctx* ctx, double* x_dev, double* y_dev, double* z_dev,
                           double* wJ_dev);

/* Initial-condition kinds of dg_init_state. */
enum { DG_IC_HYDROSTATIC_WIND = 0 };

/* Initial state (Section 3.1, Eq. (4)-(5)) written to U_dev (caller-owned, F x N doubles, layout
 * of U).  DG_IC_HYDROSTATIC_WIND: the hydrostatic background of the context's atmosphere with the
 * uniform wind (ic_params[0], 0, 0) m/s.  With noise_sigma_K > 0 every node's temperature is
 * perturbed by sigma * n at constant pressure (rho = pbar / (R (Tbar + sigma n))), where n is a
 * standard normal deviate drawn in the library from SplitMix64 (Steele, Lea, Flood 2014) used as a
 * counter-based generator keyed by the node's identity, so the field does not depend on the
 * cell order or on the launch:
 *   mix(z) = z ^ (z >> 30), * 0xbf58476d1ce4e5b9; ^ (>> 27), * 0x94d049bb133111eb; ^ (>> 31)
 *   (64-bit wrap-around arithmetic), G = 0x9e3779b97f4a7c15,
 *   k = mix(seed + G (level + 1)); k = mix(k + G (i_x + 1)); k = mix(k + G (i_y + 1));
 *   k = mix(k + G (i_z + 1)); k = mix(k + G (node + 1))   (cell table entries, node in the cell),
 *   u1 = (mix(k + G) >> 11) 2^-53, u2 = (mix(k + 2 G) >> 11) 2^-53,
 *   n = sqrt(-2 ln(1 - u1)) cos(2 pi u2)   (Box-Muller).
 * Errors: DG_EINVAL for a null ctx / U_dev / ic_params, an unknown ic_kind or a negative or
 * non-finite sigma; U_dev is not written then. */
dg_status dg_init_state(dg_ctx* ctx, int32_t ic_kind, const double* ic_params, uint64_t noise_seed,
                        double noise_sigma_K, double* U_dev);

/* R = M^{-1} (explicit weak form): the explicit part of the IMEX split of Section 2 (continuity,
 * the advective momentum flux and the kinetic-energy flux of Eq. (1), with a Rusanov flux on the
 * advective speed, slip walls, 2:1 faces on the fine side, and the gravity work -rho g w on the
 * energy), plus the absorbing-layer friction if the case has layers.  U_dev and R_dev:
 * caller-owned device arrays of F x N doubles (layout of U), not aliased.  Errors: DG_EINVAL for
 * null pointers, DG_EDEVICE for a failed launch. */
dg_status dg_explicit_residual(dg_ctx* ctx, const double* U_dev, double* R_dev);

/* F = M^{-1} (implicit weak form) at U, the implicit part of the IMEX split of Section 2
 * (pressure gradient and buoyancy in the momentum, the enthalpy flux in the energy):
 * (0, -B p' - M (rho - rhobar) g k, -C(h m) - beta/(2(gamma-1)) P p'), with p' = p - pbar.
 * U_dev, F_dev: caller-owned device arrays of F x N doubles (the density row of F is not written).
 * Uses the context's workspace; errors as dg_explicit_residual. */
dg_status dg_implicit_term(dg_ctx* ctx, const double* U_dev, double* F_dev);

/* The operator of the pressure system of Section 3.2 (non-symmetric, applied matrix-free):
 * Ap = A(h) p = M p/(gamma-1) + dt_a beta/(2(gamma-1)) P p - dt_a^2 C (h M^{-1} B p), in weak
 * (test-space) form; P uses per-cell sound speeds from h.  h_dev, p_dev, Ap_dev: caller-owned
 * device arrays of N values, float with prec = DG_FP32_INNER (context set up with that precision,
 * else DG_EINVAL), double with DG_FP64.  Uses the context's workspace; not reentrant per context.
 * Errors: DG_EINVAL (null pointers, bad prec), DG_EDEVICE. */
dg_status dg_apply_helmholtz(dg_ctx* ctx, double dt_a, const void* h_dev, const void* p_dev,
                             void* Ap_dev, int32_t prec);

/* z = P^{-1} v: the cell-wise fast-diagonalisation preconditioner of the Helmholtz operator that
 * right-preconditions the GMRES solves (DG_PREC_CELL_FDM; an extension: the paper names stronger
 * preconditioning as future work, Section 3.2), with its per-cell coefficients formed from h as in
 * the step:
 *   P^{-1} = (1/Jbar) (S x S [x S]) diag(1 / (1/(gamma-1) + sum_k alpha_k mu_{i_k})) (S x S [x S])^T,
 *   alpha_k = dt_a^2 hbar (2/D_k)^2,
 * per cell, with hbar and Jbar the means of h and of the map's Jacobian over the cell's nodes,
 * D_k the cell size (the vertical one times the mean terrain stretching Jbar / prod(D_k / 2)),
 * and (mu, S) the generalised eigenpairs L s = mu W s, S^T W S = I, of the middle-cell block L of
 * the 1D central-flux operator B^T W^{-1} B on a periodic row of three reference cells (W the
 * Gauss weights).  The node order is that of U (x fastest).  h_dev, v_dev, z_dev: caller-owned
 * device arrays of N values; h is double for both precisions, v and z are float with
 * prec = DG_FP32_INNER (context set up with that precision, else DG_EINVAL), double otherwise.
 * Null pointers or an unknown prec give DG_EINVAL.  Overwrites the context's per-cell
 * coefficients and sound speeds (the step and dg_apply_helmholtz recompute them); not reentrant
 * per context. */
dg_status dg_apply_preconditioner(dg_ctx* ctx, double dt_a, const double* h_dev, const void* v_dev,
                                  void* z_dev, int32_t prec);

/* One step of the second-order IMEX Runge-Kutta method of Section 2 (ARK2 of Giraldo, Kelly and
 * Constantinescu 2013: explicit first stage, two implicit stages), each implicit stage running the
 * pressure fixed-point loop with GMRES of Section 3.2, in place on U_dev (caller-owned F x N
 * doubles).  stats (host, may be NULL) receives iteration counts, residuals, fixed-point
 * increments, the diagnostics of the new state and, with timing on, device times.  Errors:
 * DG_EINVAL (null pointers, dt <= 0), DG_ENOCONV (a solve missed its tolerance within maxit),
 * DG_ENAN (a non-finite value in a solve or in the new state), DG_EDEVICE; on any error U is left
 * unchanged. */
dg_status imex_rk2_step(dg_ctx* ctx, double* U_dev, double dt, dg_step_stats* stats);

/* One step for each of n contexts (ensemble members of any mesh size; the serving form of the
 * step that Section 3.2 sizes per node): members of one class (same dimension, degree, precision,
 * preconditioner and energy-flux form) advance in lockstep and share every launch of the step.
 * Each operator, Krylov and pointwise kernel takes a segment table: member k owns a contiguous
 * range of the grid's workgroups, with its own arguments and mesh view, and keeps the grid shape
 * of its own launch.  Each host round trip of the Krylov iteration fetches the reductions of all
 * members at once.  Members keep their own iteration counts, restarts and failures.  A member's
 * new state is the same bits alone (n = 1) and in any mix.  A class is cut into teams of at most
 * 32 members, with up to 8 members per launch.  Each team runs on the stream of its first member,
 * from a host thread of its own; work already queued on the other members' streams is waited
 * for first, and the call returns when every team is done.  stats: array of n or NULL
 * (t_step_ms = time from the call to the member's team completion); status: array of n or NULL
 * (per-member result).  Returns DG_OK or the first member error; a member that fails keeps its
 * state, the others advance.  A context may appear once per call: a repeat gets DG_EINVAL and is
 * not stepped. */
dg_status imex_rk2_step_batched(dg_ctx* const* ctxs, double* const* U_devs, const double* dts,
                                int32_t n, dg_step_stats* stats, int32_t* status);

/* Invariants of the step (mass is conserved to rounding by the explicit continuity equation,
 * Section 2): total mass sum(w J rho) and max |w| = max |rho w| / rho over the nodes, as host
 * outputs (either may be NULL); synchronises the context's stream.  Errors: DG_EINVAL for a null
 * ctx or U_dev, DG_EDEVICE. */
dg_status dg_diagnostics(dg_ctx* ctx, const double* U_dev, double* mass, double* max_w);

/* dg_diagnostics for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same two reductions, the same
 * results bit for bit, with their partial sums in a fixed 64 KiB device array of the library (one
 * per GPU, held until the process ends) instead of the context's workspace, and the maximum's
 * second stage on the device.  Calls no hipMalloc, hipFree or allocating routine; mass and max_w
 * are host pointers (written before the call returns: the call synchronises the context's
 * stream).  The array is shared by every call on a GPU and keeps the last call's contents: calls
 * that overlap on one GPU (other threads, other streams) race and must be serialised by the
 * caller.  Any mesh size fits (the reductions use at most 2048 workgroups).  Errors: DG_EINVAL
 * for null pointers, DG_EDEVICE for a failed HIP call. */
dg_status dg_diagnostics_noalloc(dg_ctx* ctx, const double* U_dev, double* mass, double* max_w);

/* Message of the last error: the context's own (set by any call on it, including the member steps
 * of imex_rk2_step_batched, which run on other threads) if ctx is non-NULL and has one, else the
 * calling thread's (setup and argument errors).  The string stays valid until the next call on
 * that context or thread. */
const char* dg_last_error(const dg_ctx* ctx);

/* Releases the context's device memory, events and pinned host buffer (waits for its stream). */
void dg_destroy(dg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* IMEXDG_H */
