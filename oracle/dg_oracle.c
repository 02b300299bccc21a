/*
 * Plain FP64 CPU oracle for the DG operators of the IMEX-DG compressible Euler solver
 * (Orlando, Benacchio, Bonaventura, "Efficient and scalable atmospheric dynamics simulations
 * using non-conforming meshes", arXiv 2408.08129).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the HIP
 * library is compared against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code with the GPU library.
 *
 * What it computes (all in FP64, dense, no sum factorisation):
 *   - Section 2, Eq. (1): the compressible Euler equations in SI units with g = 9.81, R = 287,
 *     gamma = 1.4; the explicit part of the IMEX split (Section 2: continuity explicit, energy
 *     coupled implicitly to momentum) is the advective flux div(rho u), div(rho u (x) u),
 *     div(rho k u) plus the gravity work -rho g w;
 *   - the DG space of Section 2: tensor-product polynomials of degree r on quadrilaterals /
 *     hexahedra, nodal Lagrange basis at the Gauss-Legendre points, quadrature on the same points;
 *   - meshes with 2:1 non-conforming faces (Section 1 and Section 3.1, Fig. 1): face integrals of
 *     a hanging face are evaluated on the fine sub-faces, where the coarse polynomial is evaluated
 *     directly at the fine quadrature points;
 *   - the matrix-free operators of the implicit pressure system (Section 3.2: only the action of
 *     the linear operators is computed): the weak gradient B, the weak divergence C and the
 *     pressure-jump penalty P.
 * Every basis value is evaluated by multiplying 1D Lagrange polynomials at the point in question;
 * traces are full sums over all cell nodes; volume integrals are full double loops over
 * quadrature points and test functions.
 *
 * Geometry: one global terrain-following map x = X, y = Y, z = zeta + h(x, y) (1 - zeta / H)
 * (orography of Section 3.1, Eq. (3), and its 2D / Gaussian variants), composed with the affine
 * map of each cell of the logical box.  Face geometry is always evaluated from the integer
 * description of the (sub)face, so both sides of every face see identical numbers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OC_G 9.81
#define OC_R 287.0
#define OC_GAMMA 1.4

#define OC_MAXNP 8 /* degree <= 7 */
#define OC_MAXNQ 12 /* explicit-flux quadrature points per direction */
#define OC_MAXRULES 8

enum { OC_FLAT = 0, OC_AGNESI = 1, OC_BELL = 2, OC_GAUSS_HILL = 3, OC_GAUSS_RIDGE = 4 };
enum { OC_ISOTHERMAL = 0, OC_STRATIFIED = 1 };
enum { OC_WALL = 0, OC_CONF = 1, OC_FINE = 2, OC_COARSE = 3 };

typedef struct {
  int32_t dim, degree;
  int32_t nbase[3];    /* base cells along x, y, z (y unused in 2D) */
  int32_t periodic[2]; /* x, y lateral periodicity (1) or walls (0); z: bottom wall, top lid */
  int32_t n_rules;
  int32_t oro_kind;
  int32_t atm_kind;
  int32_t pad_;
  double length[3];              /* Lx, Ly, H [m] */
  double rules[OC_MAXRULES][5];  /* zeta_max, x_c, half-width x (<=0: any), y_c, half-width y */
  double oro[4];                 /* height, width (a or sigma), x_c, y_c */
  double atm[3];                 /* isothermal: p0, T0; stratified: p_ref, T_ref, N */
  double grav;                   /* gravitational acceleration g of Eq. (1) (9.81; 0 switches the
                                    gravity terms off, isothermal atmosphere only) */
} oc_case;

typedef struct {
  oc_case cs;
  int d, r, np1, nloc, nfp;
  int n[3];      /* base cells per axis (axis order: 3D x,y,z; 2D x,z) */
  double L[3];   /* extents per axis */
  int per[3];    /* periodic per axis */
  int lmax;
  int ncell;
  int *lev, *idx; /* idx[cell*3 + axis] at the cell's own level */
  int *fkind;     /* [cell][2d] */
  int *fnbr;      /* [cell][2d][4] */
  int nhang;      /* number of hanging sub-faces (counted once) */
  double xi[OC_MAXNP], w[OC_MAXNP];
  double *gradL;  /* [q][i][k] = d/dxi_k L_i (xi_q) */
  double *faceL;  /* [face][fp][i] = L_i at the face point of face (k,s) */
  double *subL;   /* [face][sub][fp][i] = L_i at the fine sub-face point, in coarse coordinates */
  double *wq;     /* volume weights [q] */
  double *wf;     /* face weights [fp] */
  /* over-integration of the explicit flux: nq Gauss points per direction (0: not set) */
  int nq, nvq, nfq;
  double xq[OC_MAXNQ], wq1[OC_MAXNQ];
  double *phiQ;   /* [qv][i] = L_i at volume quadrature point qv */
  double *gradQ;  /* [qv][i][k] = d/dxi_k L_i at qv */
  double *wvq;    /* [qv] volume weights */
  double *faceQ;  /* [face][j][i] = L_i at face quadrature point j of face (k,s) */
  double *subQ;   /* [face][sub][j][i] = L_i at the fine sub-face quadrature point, coarse coords */
  double *wfq;    /* [j] face weights */
} oc_mesh;

/* ------------------------------------------------------------------------------------------ */
/* 1D Gauss-Legendre rule: Newton iteration on the Legendre polynomial P_n, three-term recurrence */

static void legendre(int n, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *p = p1;
  *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

void oc_gauss(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double t = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, t, &p, &dp);
      double dt = p / dp;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    double p, dp;
    legendre(n, t, &p, &dp);
    x[n - 1 - i] = t; /* ascending order */
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

/* Lagrange polynomial j on the nodes xs[0..n) and its derivative, evaluated at x. */
static double lag(int n, const double* xs, int j, double x) {
  double v = 1.0;
  for (int m = 0; m < n; ++m)
    if (m != j) v *= (x - xs[m]) / (xs[j] - xs[m]);
  return v;
}
static double dlag(int n, const double* xs, int j, double x) {
  double s = 0.0;
  for (int m = 0; m < n; ++m) {
    if (m == j) continue;
    double t = 1.0 / (xs[j] - xs[m]);
    for (int q = 0; q < n; ++q)
      if (q != j && q != m) t *= (x - xs[q]) / (xs[j] - xs[q]);
    s += t;
  }
  return s;
}

void oc_lagrange_eval(int n, const double* xs, double x, double* val, double* der) {
  for (int j = 0; j < n; ++j) {
    val[j] = lag(n, xs, j, x);
    der[j] = dlag(n, xs, j, x);
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Orography (Section 3.1, Eq. (3) and variants) and its horizontal derivatives */

static void terrain(const oc_case* c, double x, double y, double* h, double* hx, double* hy) {
  double h0 = c->oro[0], a = c->oro[1], xc = c->oro[2], yc = c->oro[3];
  double dx = x - xc, dy = y - yc;
  *h = 0.0; *hx = 0.0; *hy = 0.0;
  switch (c->oro_kind) {
    case OC_AGNESI: { /* h0 a^2 / (a^2 + (x-xc)^2), independent of y */
      double q = a * a + dx * dx;
      *h = h0 * a * a / q;
      *hx = -2.0 * dx * h0 * a * a / (q * q);
      break;
    }
    case OC_BELL: { /* h0 / (1 + (dx/a)^2 + (dy/a)^2)^(3/2); in 2D dy = 0 */
      if (c->dim == 2) dy = 0.0;
      double t = 1.0 + (dx * dx + dy * dy) / (a * a);
      *h = h0 / pow(t, 1.5);
      double dhdt = -1.5 * h0 / pow(t, 2.5);
      *hx = dhdt * 2.0 * dx / (a * a);
      *hy = (c->dim == 2) ? 0.0 : dhdt * 2.0 * dy / (a * a);
      break;
    }
    case OC_GAUSS_HILL: { /* h0 exp(-(dx^2 + dy^2) / (2 sigma^2)); in 2D dy = 0 */
      if (c->dim == 2) dy = 0.0;
      *h = h0 * exp(-(dx * dx + dy * dy) / (2.0 * a * a));
      *hx = -dx / (a * a) * (*h);
      *hy = (c->dim == 2) ? 0.0 : -dy / (a * a) * (*h);
      break;
    }
    case OC_GAUSS_RIDGE: { /* h0 exp(-((x - xc)/a)^2), ridge along y */
      *h = h0 * exp(-(dx * dx) / (a * a));
      *hx = -2.0 * dx / (a * a) * (*h);
      break;
    }
    default:
      break;
  }
}

/* Hydrostatic background (Section 3.1, Eq. (4)-(5) with the g^2 / N^2 factor that makes
 * dp/dz = -rho g hold; or an isothermal atmosphere). */
static void background_g(int kind, const double* atm, double g, double z, double* p, double* rho) {
  if (kind == OC_ISOTHERMAL) {
    double p0 = atm[0], T0 = atm[1];
    *p = p0 * exp(-g * z / (OC_R * T0));
    *rho = *p / (OC_R * T0);
  } else {
    double pref = atm[0], Tref = atm[1], N = atm[2];
    double G = (OC_GAMMA - 1.0) / OC_GAMMA;
    double rhoref = pref / (OC_R * Tref);
    double s = exp(-N * N * z / g);
    double base = 1.0 - (g * g / (N * N)) * G * (rhoref / pref) * (1.0 - s);
    *p = pref * pow(base, 1.0 / G);
    *rho = rhoref * pow(*p / pref, 1.0 / OC_GAMMA) * s;
  }
}

void oc_background(int kind, const double* atm, double z, double* p, double* rho) {
  background_g(kind, atm, OC_G, z, p, rho);
}

/* Metric of the map (cell affine map at level lev composed with the terrain-following map) at
 * logical point X (axis order).  Gam[k][l] = det(J) * (J^{-1})_{kl}: row k is the area-weighted
 * normal of a reference face of constant xi_k; detJ its Jacobian determinant; zph the height. */
static void metric(const oc_mesh* m, int lev, const double* X, double Gam[3][3], double* detJ,
                   double* zph) {
  const oc_case* c = &m->cs;
  int d = m->d;
  double H = m->L[d - 1];
  double half[3];
  for (int a = 0; a < d; ++a) half[a] = 0.5 * m->L[a] / (m->n[a] * (double)(1 << lev));
  double x = X[0], y = (d == 3) ? X[1] : 0.0, zeta = X[d - 1];
  double h, hx, hy;
  terrain(c, x, y, &h, &hx, &hy);
  double Jt = 1.0 - h / H;
  double sx = hx * (1.0 - zeta / H), sy = hy * (1.0 - zeta / H);
  memset(Gam, 0, sizeof(double) * 9);
  if (d == 3) {
    double a = half[0], b = half[1], e = half[2], f = e * Jt;
    Gam[0][0] = b * f;
    Gam[1][1] = a * f;
    Gam[2][0] = -a * b * sx;
    Gam[2][1] = -a * b * sy;
    Gam[2][2] = a * b;
    *detJ = a * b * f;
  } else {
    double a = half[0], e = half[1], f = e * Jt;
    Gam[0][0] = f;
    Gam[1][0] = -a * sx;
    Gam[1][1] = a;
    *detJ = a * f;
  }
  *zph = zeta + h * (1.0 - zeta / H);
}

/* ------------------------------------------------------------------------------------------ */
/* Mesh: base grid refined by rules on cell centres; 2:1 balance required */

static int tang(int d, int k, int t) { /* t-th tangential axis of a face normal to k */
  if (d == 2) return k == 0 ? 1 : 0;
  int ax[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  return ax[k][t];
}

typedef struct { int lev, idx[3]; } oc_cellrec;

static int cmp_cells(const void* A, const void* B) {
  const oc_cellrec* a = (const oc_cellrec*)A;
  const oc_cellrec* b = (const oc_cellrec*)B;
  if (a->lev != b->lev) return a->lev - b->lev;
  for (int k = 2; k >= 0; --k)
    if (a->idx[k] != b->idx[k]) return a->idx[k] - b->idx[k];
  return 0;
}

void oc_mesh_free(oc_mesh* m);

/* Returns 0 on success, -1 on an invalid description, -2 on a 2:1 violation. */
int oc_mesh_build(const oc_case* cs, oc_mesh** out) {
  *out = NULL;
  if (cs->dim != 2 && cs->dim != 3) return -1;
  if (cs->degree < 1 || cs->degree > OC_MAXNP - 1) return -1;
  if (cs->n_rules < 0 || cs->n_rules > OC_MAXRULES) return -1;
  if (!(cs->grav > 0.0) && !(cs->grav == 0.0 && cs->atm_kind == OC_ISOTHERMAL)) return -1;
  oc_mesh* m = (oc_mesh*)calloc(1, sizeof(oc_mesh));
  m->cs = *cs;
  int d = m->d = cs->dim;
  m->r = cs->degree;
  m->np1 = cs->degree + 1;
  m->nloc = 1;
  for (int a = 0; a < d; ++a) m->nloc *= m->np1;
  m->nfp = m->nloc / m->np1;
  for (int a = 0; a < d; ++a) {
    int da = (d == 3) ? a : (a == 0 ? 0 : 2);
    m->n[a] = cs->nbase[da];
    m->L[a] = cs->length[da];
    m->per[a] = (a < d - 1) ? cs->periodic[a] : 0;
    if (m->n[a] < 1) { free(m); return -1; }
  }
  m->lmax = cs->n_rules;

  /* refine level by level */
  int cap = 1;
  for (int a = 0; a < d; ++a) cap *= m->n[a];
  oc_cellrec* cur = (oc_cellrec*)malloc(sizeof(oc_cellrec) * cap);
  int ncur = 0;
  for (int k2 = 0; k2 < (d == 3 ? m->n[2] : 1); ++k2)
    for (int k1 = 0; k1 < m->n[1]; ++k1)
      for (int k0 = 0; k0 < m->n[0]; ++k0) {
        oc_cellrec c = {0, {k0, k1, (d == 3) ? k2 : 0}};
        cur[ncur++] = c;
      }
  oc_cellrec* leaves = NULL;
  int nleaves = 0, capl = 0;
  for (int lev = 0; lev <= m->lmax; ++lev) {
    oc_cellrec* next = NULL;
    int nnext = 0, capn = 0;
    for (int i = 0; i < ncur; ++i) {
      oc_cellrec c = cur[i];
      int refine = 0;
      if (lev < m->lmax) {
        const double* ru = cs->rules[lev];
        double ctr[3];
        for (int a = 0; a < d; ++a)
          ctr[a] = (c.idx[a] + 0.5) * m->L[a] / (m->n[a] * (double)(1 << lev));
        double zc = ctr[d - 1];
        refine = zc < ru[0];
        if (refine && ru[2] > 0) refine = fabs(ctr[0] - ru[1]) < ru[2];
        if (refine && d == 3 && ru[4] > 0) refine = fabs(ctr[1] - ru[3]) < ru[4];
      }
      if (refine) {
        int nch = 1 << d;
        if (nnext + nch > capn) {
          capn = 2 * (nnext + nch);
          next = (oc_cellrec*)realloc(next, sizeof(oc_cellrec) * capn);
        }
        for (int ch = 0; ch < nch; ++ch) {
          oc_cellrec cc;
          cc.lev = lev + 1;
          for (int a = 0; a < 3; ++a) cc.idx[a] = 0;
          for (int a = 0; a < d; ++a) cc.idx[a] = 2 * c.idx[a] + ((ch >> a) & 1);
          next[nnext++] = cc;
        }
      } else {
        if (nleaves + 1 > capl) {
          capl = 2 * (nleaves + 1);
          leaves = (oc_cellrec*)realloc(leaves, sizeof(oc_cellrec) * capl);
        }
        leaves[nleaves++] = c;
      }
    }
    free(cur);
    cur = next;
    ncur = nnext;
    if (ncur == 0) break;
  }
  free(cur);
  qsort(leaves, nleaves, sizeof(oc_cellrec), cmp_cells);
  int used_lmax = 0;
  for (int i = 0; i < nleaves; ++i)
    if (leaves[i].lev > used_lmax) used_lmax = leaves[i].lev;
  m->lmax = used_lmax;
  m->ncell = nleaves;
  m->lev = (int*)malloc(sizeof(int) * nleaves);
  m->idx = (int*)malloc(sizeof(int) * 3 * nleaves);
  for (int i = 0; i < nleaves; ++i) {
    m->lev[i] = leaves[i].lev;
    for (int a = 0; a < 3; ++a) m->idx[3 * i + a] = leaves[i].idx[a];
  }
  free(leaves);

  /* finest-grid owner map */
  long fn[3] = {1, 1, 1};
  for (int a = 0; a < d; ++a) fn[a] = (long)m->n[a] << m->lmax;
  long ftot = fn[0] * fn[1] * fn[2];
  int* owner = (int*)malloc(sizeof(int) * ftot);
  for (int c = 0; c < m->ncell; ++c) {
    int S = 1 << (m->lmax - m->lev[c]);
    long lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) {
      lo[a] = (long)m->idx[3 * c + a] * S;
      hi[a] = lo[a] + S;
    }
    for (long z = lo[2]; z < hi[2]; ++z)
      for (long y = lo[1]; y < hi[1]; ++y)
        for (long x = lo[0]; x < hi[0]; ++x) owner[(z * fn[1] + y) * fn[0] + x] = c;
  }

  int nf = 2 * d;
  m->fkind = (int*)malloc(sizeof(int) * nf * m->ncell);
  m->fnbr = (int*)malloc(sizeof(int) * 4 * nf * m->ncell);
  int bad = 0;
  long nhang = 0;
  for (int c = 0; c < m->ncell; ++c) {
    int l = m->lev[c];
    int S = 1 << (m->lmax - l);
    for (int k = 0; k < d; ++k)
      for (int s = 0; s < 2; ++s) {
        int f = 2 * k + s;
        int* kind = &m->fkind[c * nf + f];
        int* nb = &m->fnbr[(c * nf + f) * 4];
        nb[0] = nb[1] = nb[2] = nb[3] = -1;
        long pos[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) pos[a] = (long)m->idx[3 * c + a] * S;
        pos[k] = s ? pos[k] + S : pos[k] - 1;
        if (pos[k] < 0 || pos[k] >= fn[k]) {
          if (!m->per[k]) { *kind = OC_WALL; continue; }
          pos[k] = (pos[k] + fn[k]) % fn[k];
        }
        int o = owner[(pos[2] * fn[1] + pos[1]) * fn[0] + pos[0]];
        int lo = m->lev[o];
        if (lo == l) {
          *kind = OC_CONF;
          nb[0] = o;
        } else if (lo == l - 1) {
          *kind = OC_FINE;
          nb[0] = o;
        } else if (lo == l + 1) {
          *kind = OC_COARSE;
          int half = S / 2;
          for (int sub = 0; sub < (1 << (d - 1)); ++sub) {
            long q[3] = {pos[0], pos[1], pos[2]};
            for (int t = 0; t < d - 1; ++t) {
              int ta = tang(d, k, t);
              q[ta] += ((sub >> t) & 1) * half;
            }
            int o2 = owner[(q[2] * fn[1] + q[1]) * fn[0] + q[0]];
            if (m->lev[o2] != l + 1) bad = 1;
            nb[sub] = o2;
          }
          nhang += 1 << (d - 1);
        } else {
          bad = 1;
        }
      }
  }
  free(owner);
  m->nhang = (int)nhang;
  if (bad) { oc_mesh_free(m); return -2; }

  /* 1D rule and dense tables */
  oc_gauss(m->np1, m->xi, m->w);
  int np1 = m->np1, nloc = m->nloc, nfp = m->nfp;
  m->wq = (double*)malloc(sizeof(double) * nloc);
  m->wf = (double*)malloc(sizeof(double) * nfp);
  m->gradL = (double*)malloc(sizeof(double) * nloc * nloc * d);
  m->faceL = (double*)malloc(sizeof(double) * nf * nfp * nloc);
  m->subL = (double*)malloc(sizeof(double) * nf * (1 << (d - 1)) * nfp * nloc);
  int ii[3];
  for (int q = 0; q < nloc; ++q) {
    int t = q;
    double wv = 1.0;
    for (int a = 0; a < d; ++a) { ii[a] = t % np1; t /= np1; wv *= m->w[ii[a]]; }
    m->wq[q] = wv;
  }
  for (int fp = 0; fp < nfp; ++fp) {
    int t = fp;
    double wv = 1.0;
    for (int a = 0; a < d - 1; ++a) { wv *= m->w[t % np1]; t /= np1; }
    m->wf[fp] = wv;
  }
  /* volume: gradient of every basis function at every quadrature point */
  for (int q = 0; q < nloc; ++q) {
    double xq[3];
    int t = q;
    for (int a = 0; a < d; ++a) { xq[a] = m->xi[t % np1]; t /= np1; }
    for (int i = 0; i < nloc; ++i) {
      int ia[3];
      int u = i;
      for (int a = 0; a < d; ++a) { ia[a] = u % np1; u /= np1; }
      for (int k = 0; k < d; ++k) {
        double v = 1.0;
        for (int a = 0; a < d; ++a)
          v *= (a == k) ? dlag(np1, m->xi, ia[a], xq[a]) : lag(np1, m->xi, ia[a], xq[a]);
        m->gradL[(q * nloc + i) * d + k] = v;
      }
    }
  }
  /* faces: every basis function at every face point, own and sub-face (coarse coordinates) */
  for (int k = 0; k < d; ++k)
    for (int s = 0; s < 2; ++s) {
      int f = 2 * k + s;
      for (int sub = 0; sub <= (1 << (d - 1)); ++sub) {
        for (int fp = 0; fp < nfp; ++fp) {
          double pt[3];
          pt[k] = s ? 1.0 : -1.0;
          int t = fp;
          for (int tt = 0; tt < d - 1; ++tt) {
            int ta = tang(d, k, tt);
            double xj = m->xi[t % np1];
            t /= np1;
            if (sub == 0) pt[ta] = xj;
            else pt[ta] = 0.5 * (xj + 2.0 * (((sub - 1) >> tt) & 1) - 1.0);
          }
          for (int i = 0; i < nloc; ++i) {
            int u = i;
            double v = 1.0;
            for (int a = 0; a < d; ++a) { v *= lag(np1, m->xi, u % np1, pt[a]); u /= np1; }
            if (sub == 0) m->faceL[(f * nfp + fp) * nloc + i] = v;
            else m->subL[((f * (1 << (d - 1)) + (sub - 1)) * nfp + fp) * nloc + i] = v;
          }
        }
      }
    }
  *out = m;
  return 0;
}

void oc_mesh_free(oc_mesh* m) {
  if (!m) return;
  free(m->lev); free(m->idx); free(m->fkind); free(m->fnbr);
  free(m->gradL); free(m->faceL); free(m->subL); free(m->wq); free(m->wf);
  free(m->phiQ); free(m->gradQ); free(m->wvq); free(m->faceQ); free(m->subQ); free(m->wfq);
  free(m);
}

/* Over-integration (quadrature of the explicit flux integrals with nq >= r + 1 Gauss points per
 * direction): the basis and its gradient at the volume points, the basis at the points of every
 * face and of every fine sub-face (in the coarse cell's coordinates), and the weights.  Returns 0,
 * or -1 for an nq out of range. */
int oc_set_quadrature(oc_mesh* m, int nq) {
  int d = m->d, np1 = m->np1, nloc = m->nloc, nf = 2 * d, nsub = 1 << (d - 1);
  if (nq < np1 || nq > OC_MAXNQ) return -1;
  free(m->phiQ); free(m->gradQ); free(m->wvq); free(m->faceQ); free(m->subQ); free(m->wfq);
  m->nq = nq;
  oc_gauss(nq, m->xq, m->wq1);
  int nvq = 1, nfq = 1;
  for (int a = 0; a < d; ++a) nvq *= nq;
  for (int a = 0; a < d - 1; ++a) nfq *= nq;
  m->nvq = nvq;
  m->nfq = nfq;
  m->phiQ = (double*)malloc(sizeof(double) * nvq * nloc);
  m->gradQ = (double*)malloc(sizeof(double) * nvq * nloc * d);
  m->wvq = (double*)malloc(sizeof(double) * nvq);
  m->faceQ = (double*)malloc(sizeof(double) * nf * nfq * nloc);
  m->subQ = (double*)malloc(sizeof(double) * nf * nsub * nfq * nloc);
  m->wfq = (double*)malloc(sizeof(double) * nfq);
  for (int q = 0; q < nvq; ++q) {
    double xqv[3], wv = 1.0;
    int t = q;
    for (int a = 0; a < d; ++a) { xqv[a] = m->xq[t % nq]; wv *= m->wq1[t % nq]; t /= nq; }
    m->wvq[q] = wv;
    for (int i = 0; i < nloc; ++i) {
      int ia[3], u = i;
      for (int a = 0; a < d; ++a) { ia[a] = u % np1; u /= np1; }
      double v = 1.0;
      for (int a = 0; a < d; ++a) v *= lag(np1, m->xi, ia[a], xqv[a]);
      m->phiQ[q * nloc + i] = v;
      for (int k = 0; k < d; ++k) {
        double g = 1.0;
        for (int a = 0; a < d; ++a)
          g *= (a == k) ? dlag(np1, m->xi, ia[a], xqv[a]) : lag(np1, m->xi, ia[a], xqv[a]);
        m->gradQ[(q * nloc + i) * d + k] = g;
      }
    }
  }
  for (int j = 0; j < nfq; ++j) {
    int t = j;
    double wv = 1.0;
    for (int a = 0; a < d - 1; ++a) { wv *= m->wq1[t % nq]; t /= nq; }
    m->wfq[j] = wv;
  }
  for (int k = 0; k < d; ++k)
    for (int s = 0; s < 2; ++s) {
      int f = 2 * k + s;
      for (int sub = 0; sub <= nsub; ++sub)
        for (int j = 0; j < nfq; ++j) {
          double pt[3];
          pt[k] = s ? 1.0 : -1.0;
          int t = j;
          for (int tt = 0; tt < d - 1; ++tt) {
            int ta = tang(d, k, tt);
            double xj = m->xq[t % nq];
            t /= nq;
            pt[ta] = sub == 0 ? xj : 0.5 * (xj + 2.0 * (((sub - 1) >> tt) & 1) - 1.0);
          }
          for (int i = 0; i < nloc; ++i) {
            int u = i;
            double v = 1.0;
            for (int a = 0; a < d; ++a) { v *= lag(np1, m->xi, u % np1, pt[a]); u /= np1; }
            if (sub == 0) m->faceQ[(f * nfq + j) * nloc + i] = v;
            else m->subQ[((f * nsub + (sub - 1)) * nfq + j) * nloc + i] = v;
          }
        }
    }
  return 0;
}

int oc_ncell(const oc_mesh* m) { return m->ncell; }
int oc_nloc(const oc_mesh* m) { return m->nloc; }
int oc_nhang(const oc_mesh* m) { return m->nhang; }
int oc_lmax(const oc_mesh* m) { return m->lmax; }

/* (level, i_x, i_y, i_z) of every cell, at its own level; i_y = 0 in 2D. */
void oc_cell_table(const oc_mesh* m, int32_t* out) {
  for (int c = 0; c < m->ncell; ++c) {
    out[4 * c] = m->lev[c];
    if (m->d == 3) {
      for (int a = 0; a < 3; ++a) out[4 * c + 1 + a] = m->idx[3 * c + a];
    } else {
      out[4 * c + 1] = m->idx[3 * c];
      out[4 * c + 2] = 0;
      out[4 * c + 3] = m->idx[3 * c + 1];
    }
  }
}

/* logical coordinates of node q of cell c */
static void node_X(const oc_mesh* m, int c, int q, double* X) {
  int l = m->lev[c];
  int t = q;
  for (int a = 0; a < m->d; ++a) {
    double dx = m->L[a] / (m->n[a] * (double)(1 << l));
    X[a] = dx * (m->idx[3 * c + a] + 0.5 * (1.0 + m->xi[t % m->np1]));
    t /= m->np1;
  }
}

/* Physical coordinates, quadrature weight times Jacobian, per node; layout [cell][node]. */
void oc_node_geometry(const oc_mesh* m, double* x, double* y, double* z, double* wJ) {
  for (int c = 0; c < m->ncell; ++c)
    for (int q = 0; q < m->nloc; ++q) {
      double X[3], Gam[3][3], J, zp;
      node_X(m, c, q, X);
      metric(m, m->lev[c], X, Gam, &J, &zp);
      long n = (long)c * m->nloc + q;
      x[n] = X[0];
      y[n] = (m->d == 3) ? X[1] : 0.0;
      z[n] = zp;
      wJ[n] = m->wq[q] * J;
    }
}

/* Background pressure and density at every node. */
void oc_background_nodes(const oc_mesh* m, double* pbar, double* rbar) {
  for (int c = 0; c < m->ncell; ++c)
    for (int q = 0; q < m->nloc; ++q) {
      double X[3], Gam[3][3], J, zp;
      node_X(m, c, q, X);
      metric(m, m->lev[c], X, Gam, &J, &zp);
      long n = (long)c * m->nloc + q;
      background_g(m->cs.atm_kind, m->cs.atm, m->cs.grav, zp, &pbar[n], &rbar[n]);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Face bookkeeping: for face f = 2k + s of cell c, and (for coarse faces) sub-face sub, give the
 * fine level, the integer face position along k, the tangential integer indices at the fine
 * level, whether c is the left (lower-k) side, and the basis tables of c and of the neighbour. */

typedef struct {
  int lev;       /* level at which the (sub)face is described */
  long P;        /* face position along k, in cells of that level, reduced if periodic */
  long T[3];     /* tangential indices at that level (entries for axis k unused) */
  int left;      /* 1 if c lies on the lower side of the face */
  int nb;        /* neighbour cell (or -1 on a wall) */
  const double* myL;  /* [fp][nloc] basis of c at the face points */
  const double* nbL;  /* [fp][nloc] basis of the neighbour at the face points */
} oc_facepts;

static void face_points(const oc_mesh* m, int c, int f, int sub, oc_facepts* fp) {
  int d = m->d, k = f / 2, s = f % 2, nf = 2 * d, nfp = m->nfp, nloc = m->nloc;
  int l = m->lev[c];
  int kind = m->fkind[c * nf + f];
  const int* nb = &m->fnbr[(c * nf + f) * 4];
  int fo = 2 * k + (1 - s); /* the neighbour's face index */
  fp->left = s;
  if (kind == OC_COARSE) {
    fp->lev = l + 1;
    fp->P = s ? 2L * (m->idx[3 * c + k] + 1) : 2L * m->idx[3 * c + k];
    for (int t = 0; t < d - 1; ++t) {
      int ta = tang(d, k, t);
      fp->T[ta] = 2L * m->idx[3 * c + ta] + ((sub >> t) & 1);
    }
    fp->nb = nb[sub];
    fp->myL = &m->subL[((f * (1 << (d - 1)) + sub) * nfp) * nloc];
    fp->nbL = &m->faceL[(fo * nfp) * nloc];
  } else {
    fp->lev = l;
    fp->P = s ? (long)m->idx[3 * c + k] + 1 : (long)m->idx[3 * c + k];
    for (int t = 0; t < d - 1; ++t) {
      int ta = tang(d, k, t);
      fp->T[ta] = m->idx[3 * c + ta];
    }
    fp->nb = (kind == OC_WALL) ? -1 : nb[0];
    fp->myL = &m->faceL[(f * nfp) * nloc];
    if (kind == OC_FINE) {
      int csub = 0;
      for (int t = 0; t < d - 1; ++t) csub |= (m->idx[3 * c + tang(d, k, t)] & 1) << t;
      fp->nbL = &m->subL[((fo * (1 << (d - 1)) + csub) * nfp) * nloc];
    } else {
      fp->nbL = &m->faceL[(fo * nfp) * nloc];
    }
  }
  long nk = (long)m->n[k] << fp->lev;
  if (m->per[k]) fp->P = ((fp->P % nk) + nk) % nk;
}

/* Area-weighted normal (pointing from the lower to the upper side along k) at face point j. */
static void face_normal(const oc_mesh* m, int k, const oc_facepts* fp, int j, double* N) {
  int d = m->d;
  double X[3];
  X[k] = m->L[k] / (m->n[k] * (double)(1 << fp->lev)) * (double)fp->P;
  int t = j;
  for (int tt = 0; tt < d - 1; ++tt) {
    int ta = tang(d, k, tt);
    double dx = m->L[ta] / (m->n[ta] * (double)(1 << fp->lev));
    X[ta] = dx * (fp->T[ta] + 0.5 * (1.0 + m->xi[t % m->np1]));
    t /= m->np1;
  }
  double Gam[3][3], J, zp;
  metric(m, fp->lev, X, Gam, &J, &zp);
  for (int a = 0; a < d; ++a) N[a] = Gam[k][a];
}

static double dense_trace(const double* Lrow, const double* u, int nloc) {
  double s = 0.0;
  for (int i = 0; i < nloc; ++i) s += Lrow[i] * u[i];
  return s;
}

/* ------------------------------------------------------------------------------------------ */
/* Explicit advective flux (IMEX split of Section 2: continuity explicit, energy implicitly
 * coupled to momentum), Rusanov numerical flux with the advective speed |u.n|. */

static void adv_flux_n(int d, const double* U, const double* N, double* out) {
  double rho = U[0], mn = 0.0, m2 = 0.0;
  for (int l = 0; l < d; ++l) { mn += U[1 + l] * N[l]; m2 += U[1 + l] * U[1 + l]; }
  double un = mn / rho;
  out[0] = mn;
  for (int l = 0; l < d; ++l) out[1 + l] = U[1 + l] * un;
  out[1 + d] = 0.5 * m2 / rho * un;
}

static void rusanov(int d, const double* UL, const double* UR, const double* N, double* out) {
  double FL[5], FR[5];
  adv_flux_n(d, UL, N, FL);
  adv_flux_n(d, UR, N, FR);
  double vl = 0.0, vr = 0.0;
  for (int l = 0; l < d; ++l) { vl += UL[1 + l] * N[l]; vr += UR[1 + l] * N[l]; }
  vl = fabs(vl / UL[0]);
  vr = fabs(vr / UR[0]);
  double lam = vl > vr ? vl : vr;
  for (int f = 0; f < d + 2; ++f) out[f] = 0.5 * (FL[f] + FR[f]) - 0.5 * lam * (UR[f] - UL[f]);
}

/* Rusanov flux against the mirror state (rho, m - 2 (m.n) n, rhoE) at a wall with outward
 * area-weighted normal N: mass and energy fluxes vanish, momentum gets (m.N)(v + |v|) N / |N|^2
 * with v = (m.N) / rho. */
static void wall_flux(int d, const double* U, const double* N, double* out) {
  double mn = 0.0, nn = 0.0;
  for (int l = 0; l < d; ++l) { mn += U[1 + l] * N[l]; nn += N[l] * N[l]; }
  double v = mn / U[0];
  out[0] = 0.0;
  for (int l = 0; l < d; ++l) out[1 + l] = mn * (v + fabs(v)) * N[l] / nn;
  out[1 + d] = 0.0;
}

/* The slip-wall flux at one point, exported for the oracle's own tests (closed-form check against
 * the Rusanov flux with the mirror state). */
void oc_wall_flux(int d, const double* U, const double* N, double* out) { wall_flux(d, U, N, out); }

/* R = M^{-1} (explicit weak form): the explicit time derivative of U, layout [field][cell][node].
 * Volume: + int F . grad(phi_i); faces: - int (F^.n) phi_i; gravity work -g (rho w) on energy. */
void oc_explicit_residual(const oc_mesh* m, const double* U, double* R) {
  int d = m->d, nloc = m->nloc, nfp = m->nfp, nf = 2 * d, NF = d + 2;
  long N = (long)m->ncell * nloc;
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < m->ncell; ++c) {
    double W[5][OC_MAXNP * OC_MAXNP * OC_MAXNP];
    double Uq[5], Gam[3][3], J, zp, X[3];
    for (int f = 0; f < NF; ++f)
      for (int i = 0; i < nloc; ++i) W[f][i] = 0.0;
    /* volume */
    for (int q = 0; q < nloc; ++q) {
      for (int f = 0; f < NF; ++f) Uq[f] = U[f * N + (long)c * nloc + q];
      node_X(m, c, q, X);
      metric(m, m->lev[c], X, Gam, &J, &zp);
      double rho = Uq[0], m2 = 0.0, u[3];
      for (int l = 0; l < d; ++l) { u[l] = Uq[1 + l] / rho; m2 += Uq[1 + l] * Uq[1 + l]; }
      double rk = 0.5 * m2 / rho;
      for (int k = 0; k < d; ++k) {
        /* contravariant component k of each field's flux */
        double Gu = 0.0; /* Gam[k] . u */
        for (int l = 0; l < d; ++l) Gu += Gam[k][l] * u[l];
        double Gk[5];
        Gk[0] = rho * Gu;
        for (int l = 0; l < d; ++l) Gk[1 + l] = Uq[1 + l] * Gu;
        Gk[1 + d] = rk * Gu;
        for (int i = 0; i < nloc; ++i) {
          double gl = m->gradL[(q * nloc + i) * d + k] * m->wq[q];
          for (int f = 0; f < NF; ++f) W[f][i] += gl * Gk[f];
        }
      }
    }
    /* faces */
    for (int f = 0; f < nf; ++f) {
      int kind = m->fkind[c * nf + f];
      int k = f / 2;
      int nsub = (kind == OC_COARSE) ? (1 << (d - 1)) : 1;
      for (int sub = 0; sub < nsub; ++sub) {
        oc_facepts fp;
        face_points(m, c, f, sub, &fp);
        for (int j = 0; j < nfp; ++j) {
          double Nv[3], Um[5], Un[5], Fh[5];
          face_normal(m, k, &fp, j, Nv);
          for (int g = 0; g < NF; ++g) Um[g] = dense_trace(&fp.myL[j * nloc], &U[g * N + (long)c * nloc], nloc);
          double sign = fp.left ? 1.0 : -1.0;
          if (kind == OC_WALL) {
            double No[3];
            for (int a = 0; a < d; ++a) No[a] = sign * Nv[a];
            wall_flux(d, Um, No, Fh);
            sign = 1.0;
          } else {
            for (int g = 0; g < NF; ++g)
              Un[g] = dense_trace(&fp.nbL[j * nloc], &U[g * N + (long)fp.nb * nloc], nloc);
            if (fp.left) rusanov(d, Um, Un, Nv, Fh);
            else rusanov(d, Un, Um, Nv, Fh);
          }
          double wj = m->wf[j];
          for (int i = 0; i < nloc; ++i) {
            double li = fp.myL[j * nloc + i] * wj * sign;
            for (int g = 0; g < NF; ++g) W[g][i] -= li * Fh[g];
          }
        }
      }
    }
    for (int q = 0; q < nloc; ++q) {
      node_X(m, c, q, X);
      metric(m, m->lev[c], X, Gam, &J, &zp);
      double mJ = m->wq[q] * J;
      for (int f = 0; f < NF; ++f) R[f * N + (long)c * nloc + q] = W[f][q] / mJ;
      R[(1 + d) * N + (long)c * nloc + q] -= m->cs.grav * U[d * N + (long)c * nloc + q];
    }
  }
}

/* The over-integrated explicit residual: the same weak form as oc_explicit_residual, with the
 * volume and face integrals of the flux taken with nq Gauss points per direction (the state
 * interpolated there from the nodes); on a 2:1 face the points are those of the fine sub-face, as
 * for the nodal rule.  The mass matrix stays the nodal one and the gravity work stays pointwise. */
static void face_points_q(const oc_mesh* m, int c, int f, int sub, oc_facepts* fp) {
  face_points(m, c, f, sub, fp);
  int d = m->d, k = f / 2, s = f % 2, nf = 2 * d, nfq = m->nfq, nloc = m->nloc, nsub = 1 << (d - 1);
  int kind = m->fkind[c * nf + f];
  int fo = 2 * k + (1 - s);
  if (kind == OC_COARSE) {
    fp->myL = &m->subQ[((f * nsub + sub) * nfq) * nloc];
    fp->nbL = &m->faceQ[(fo * nfq) * nloc];
  } else {
    fp->myL = &m->faceQ[(f * nfq) * nloc];
    if (kind == OC_FINE) {
      int csub = 0;
      for (int t = 0; t < d - 1; ++t) csub |= (m->idx[3 * c + tang(d, k, t)] & 1) << t;
      fp->nbL = &m->subQ[((fo * nsub + csub) * nfq) * nloc];
    } else {
      fp->nbL = &m->faceQ[(fo * nfq) * nloc];
    }
  }
}

static void face_normal_q(const oc_mesh* m, int k, const oc_facepts* fp, int j, double* N) {
  int d = m->d;
  double X[3];
  X[k] = m->L[k] / (m->n[k] * (double)(1 << fp->lev)) * (double)fp->P;
  int t = j;
  for (int tt = 0; tt < d - 1; ++tt) {
    int ta = tang(d, k, tt);
    double dx = m->L[ta] / (m->n[ta] * (double)(1 << fp->lev));
    X[ta] = dx * (fp->T[ta] + 0.5 * (1.0 + m->xq[t % m->nq]));
    t /= m->nq;
  }
  double Gam[3][3], J, zp;
  metric(m, fp->lev, X, Gam, &J, &zp);
  for (int a = 0; a < d; ++a) N[a] = Gam[k][a];
}

int oc_explicit_residual_oi(const oc_mesh* m, const double* U, double* R) {
  if (m->nq == 0) return -1;
  int d = m->d, nloc = m->nloc, nf = 2 * d, NF = d + 2, nq = m->nq, nvq = m->nvq, nfq = m->nfq;
  long N = (long)m->ncell * nloc;
#pragma omp parallel for schedule(dynamic, 4)
  for (int c = 0; c < m->ncell; ++c) {
    double W[5][OC_MAXNP * OC_MAXNP * OC_MAXNP];
    int l = m->lev[c];
    for (int f = 0; f < NF; ++f)
      for (int i = 0; i < nloc; ++i) W[f][i] = 0.0;
    /* volume, at the nq^d quadrature points */
    for (int q = 0; q < nvq; ++q) {
      double Uq[5], X[3], Gam[3][3], J, zp;
      for (int f = 0; f < NF; ++f) Uq[f] = dense_trace(&m->phiQ[q * nloc], &U[f * N + (long)c * nloc], nloc);
      int t = q;
      for (int a = 0; a < d; ++a) {
        double dx = m->L[a] / (m->n[a] * (double)(1 << l));
        X[a] = dx * (m->idx[3 * c + a] + 0.5 * (1.0 + m->xq[t % nq]));
        t /= nq;
      }
      metric(m, l, X, Gam, &J, &zp);
      double rho = Uq[0], m2 = 0.0, u[3];
      for (int a = 0; a < d; ++a) { u[a] = Uq[1 + a] / rho; m2 += Uq[1 + a] * Uq[1 + a]; }
      double rk = 0.5 * m2 / rho;
      for (int k = 0; k < d; ++k) {
        double Gu = 0.0;
        for (int a = 0; a < d; ++a) Gu += Gam[k][a] * u[a];
        double Gk[5];
        Gk[0] = rho * Gu;
        for (int a = 0; a < d; ++a) Gk[1 + a] = Uq[1 + a] * Gu;
        Gk[1 + d] = rk * Gu;
        for (int i = 0; i < nloc; ++i) {
          double gl = m->gradQ[(q * nloc + i) * d + k] * m->wvq[q];
          for (int f = 0; f < NF; ++f) W[f][i] += gl * Gk[f];
        }
      }
    }
    /* faces, at the nq^(d-1) points of every (sub-)face */
    for (int f = 0; f < nf; ++f) {
      int kind = m->fkind[c * nf + f];
      int k = f / 2;
      int nsub = (kind == OC_COARSE) ? (1 << (d - 1)) : 1;
      for (int sub = 0; sub < nsub; ++sub) {
        oc_facepts fp;
        face_points_q(m, c, f, sub, &fp);
        for (int j = 0; j < nfq; ++j) {
          double Nv[3], Um[5], Un[5], Fh[5];
          face_normal_q(m, k, &fp, j, Nv);
          for (int g = 0; g < NF; ++g) Um[g] = dense_trace(&fp.myL[j * nloc], &U[g * N + (long)c * nloc], nloc);
          double sign = fp.left ? 1.0 : -1.0;
          if (kind == OC_WALL) {
            double No[3];
            for (int a = 0; a < d; ++a) No[a] = sign * Nv[a];
            wall_flux(d, Um, No, Fh);
            sign = 1.0;
          } else {
            for (int g = 0; g < NF; ++g)
              Un[g] = dense_trace(&fp.nbL[j * nloc], &U[g * N + (long)fp.nb * nloc], nloc);
            if (fp.left) rusanov(d, Um, Un, Nv, Fh);
            else rusanov(d, Un, Um, Nv, Fh);
          }
          double wj = m->wfq[j];
          for (int i = 0; i < nloc; ++i) {
            double li = fp.myL[j * nloc + i] * wj * sign;
            for (int g = 0; g < NF; ++g) W[g][i] -= li * Fh[g];
          }
        }
      }
    }
    for (int q = 0; q < nloc; ++q) {
      double X[3], Gam[3][3], J, zp;
      node_X(m, c, q, X);
      metric(m, l, X, Gam, &J, &zp);
      double mJ = m->wq[q] * J;
      for (int f = 0; f < NF; ++f) R[f * N + (long)c * nloc + q] = W[f][q] / mJ;
      R[(1 + d) * N + (long)c * nloc + q] -= m->cs.grav * U[d * N + (long)c * nloc + q];
    }
  }
  return 0;
}

/* q = M^{-1} B p: weak gradient, B p . phi = -int p div(phi) + int p^ phi.n, with the central
 * value p^ = (p- + p+)/2 on interior and hanging faces and p^ = p- on walls.  q layout [d][N]. */
void oc_grad(const oc_mesh* m, const double* p, double* qout) {
  int d = m->d, nloc = m->nloc, nfp = m->nfp, nf = 2 * d;
  long N = (long)m->ncell * nloc;
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < m->ncell; ++c) {
    double W[3][OC_MAXNP * OC_MAXNP * OC_MAXNP];
    double Gam[3][3], J, zp, X[3];
    for (int l = 0; l < d; ++l)
      for (int i = 0; i < nloc; ++i) W[l][i] = 0.0;
    for (int q = 0; q < nloc; ++q) {
      double pq = p[(long)c * nloc + q];
      node_X(m, c, q, X);
      metric(m, m->lev[c], X, Gam, &J, &zp);
      for (int i = 0; i < nloc; ++i)
        for (int k = 0; k < d; ++k) {
          double gl = m->gradL[(q * nloc + i) * d + k] * m->wq[q] * pq;
          for (int l = 0; l < d; ++l) W[l][i] -= gl * Gam[k][l];
        }
    }
    for (int f = 0; f < nf; ++f) {
      int kind = m->fkind[c * nf + f];
      int k = f / 2;
      int nsub = (kind == OC_COARSE) ? (1 << (d - 1)) : 1;
      for (int sub = 0; sub < nsub; ++sub) {
        oc_facepts fp;
        face_points(m, c, f, sub, &fp);
        for (int j = 0; j < nfp; ++j) {
          double Nv[3];
          face_normal(m, k, &fp, j, Nv);
          double pm = dense_trace(&fp.myL[j * nloc], &p[(long)c * nloc], nloc);
          double ph = pm;
          if (kind != OC_WALL) {
            double pn = dense_trace(&fp.nbL[j * nloc], &p[(long)fp.nb * nloc], nloc);
            ph = fp.left ? 0.5 * (pm + pn) : 0.5 * (pn + pm);
          }
          double sign = fp.left ? 1.0 : -1.0;
          for (int i = 0; i < nloc; ++i) {
            double li = fp.myL[j * nloc + i] * m->wf[j] * sign * ph;
            for (int l = 0; l < d; ++l) W[l][i] += li * Nv[l];
          }
        }
      }
    }
    for (int q = 0; q < nloc; ++q) {
      node_X(m, c, q, X);
      metric(m, m->lev[c], X, Gam, &J, &zp);
      double mJ = m->wq[q] * J;
      for (int l = 0; l < d; ++l) qout[l * N + (long)c * nloc + q] = W[l][q] / mJ;
    }
  }
}

/* C w (weak, not divided by the mass): C w . psi = -int w . grad(psi) + int psi {{w}}.n, with
 * the average of the two traces on interior and hanging faces and zero normal flux on walls.
 * w layout [d][N]; out layout [N]. */
void oc_div(const oc_mesh* m, const double* wv, double* out) {
  int d = m->d, nloc = m->nloc, nfp = m->nfp, nf = 2 * d;
  long N = (long)m->ncell * nloc;
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < m->ncell; ++c) {
    double W[OC_MAXNP * OC_MAXNP * OC_MAXNP];
    double Gam[3][3], J, zp, X[3];
    for (int i = 0; i < nloc; ++i) W[i] = 0.0;
    for (int q = 0; q < nloc; ++q) {
      node_X(m, c, q, X);
      metric(m, m->lev[c], X, Gam, &J, &zp);
      for (int k = 0; k < d; ++k) {
        double Gk = 0.0;
        for (int l = 0; l < d; ++l) Gk += Gam[k][l] * wv[l * N + (long)c * nloc + q];
        for (int i = 0; i < nloc; ++i) W[i] -= m->gradL[(q * nloc + i) * d + k] * m->wq[q] * Gk;
      }
    }
    for (int f = 0; f < nf; ++f) {
      int kind = m->fkind[c * nf + f];
      if (kind == OC_WALL) continue;
      int k = f / 2;
      int nsub = (kind == OC_COARSE) ? (1 << (d - 1)) : 1;
      for (int sub = 0; sub < nsub; ++sub) {
        oc_facepts fp;
        face_points(m, c, f, sub, &fp);
        for (int j = 0; j < nfp; ++j) {
          double Nv[3];
          face_normal(m, k, &fp, j, Nv);
          double wm = 0.0, wn = 0.0;
          for (int l = 0; l < d; ++l) {
            wm += Nv[l] * dense_trace(&fp.myL[j * nloc], &wv[l * N + (long)c * nloc], nloc);
            wn += Nv[l] * dense_trace(&fp.nbL[j * nloc], &wv[l * N + (long)fp.nb * nloc], nloc);
          }
          double wh = fp.left ? 0.5 * (wm + wn) : 0.5 * (wn + wm);
          double sign = fp.left ? 1.0 : -1.0;
          for (int i = 0; i < nloc; ++i) W[i] += fp.myL[j * nloc + i] * m->wf[j] * sign * wh;
        }
      }
    }
    for (int q = 0; q < nloc; ++q) out[(long)c * nloc + q] = W[q];
  }
}

/* Pressure-jump penalty (weak): P p . psi = sum over interior and hanging faces of
 * int psi lam_f (p_own - p_other) dS with lam_f = max(lam[c], lam[nb]); zero on walls.
 * The factor beta / (2 (gamma - 1)) is applied by the caller. */
void oc_penalty(const oc_mesh* m, const double* lam, const double* p, double* out) {
  int d = m->d, nloc = m->nloc, nfp = m->nfp, nf = 2 * d;
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < m->ncell; ++c) {
    double W[OC_MAXNP * OC_MAXNP * OC_MAXNP];
    for (int i = 0; i < nloc; ++i) W[i] = 0.0;
    for (int f = 0; f < nf; ++f) {
      int kind = m->fkind[c * nf + f];
      if (kind == OC_WALL) continue;
      int k = f / 2;
      int nsub = (kind == OC_COARSE) ? (1 << (d - 1)) : 1;
      for (int sub = 0; sub < nsub; ++sub) {
        oc_facepts fp;
        face_points(m, c, f, sub, &fp);
        double lf = lam[c] > lam[fp.nb] ? lam[c] : lam[fp.nb];
        for (int j = 0; j < nfp; ++j) {
          double Nv[3], nn = 0.0;
          face_normal(m, k, &fp, j, Nv);
          for (int a = 0; a < d; ++a) nn += Nv[a] * Nv[a];
          double pm = dense_trace(&fp.myL[j * nloc], &p[(long)c * nloc], nloc);
          double pn = dense_trace(&fp.nbL[j * nloc], &p[(long)fp.nb * nloc], nloc);
          double v = lf * sqrt(nn) * (pm - pn) * m->wf[j];
          for (int i = 0; i < nloc; ++i) W[i] += fp.myL[j * nloc + i] * v;
        }
      }
    }
    for (int q = 0; q < nloc; ++q) out[(long)c * nloc + q] = W[q];
  }
}

/* Logical cell sizes per axis for every cell (used by the diagonal preconditioner). */
void oc_cell_sizes(const oc_mesh* m, double* out) {
  for (int c = 0; c < m->ncell; ++c)
    for (int a = 0; a < 3; ++a)
      out[3 * c + a] = (a < m->d) ? m->L[a] / (m->n[a] * (double)(1 << m->lev[c])) : 0.0;
}

/* Outward area-weighted normals at the bottom-wall face points of every bottom cell, with the
 * physical coordinates of those points: out rows (x, y, z, N_x, N_y, N_z). Returns the count. */
int oc_bottom_normals(const oc_mesh* m, double* out) {
  int d = m->d, nf = 2 * d, nfp = m->nfp, cnt = 0;
  int f = 2 * (d - 1);
  for (int c = 0; c < m->ncell; ++c) {
    if (m->fkind[c * nf + f] != OC_WALL) continue;
    oc_facepts fp;
    face_points(m, c, f, 0, &fp);
    for (int j = 0; j < nfp; ++j) {
      double Nv[3];
      face_normal(m, d - 1, &fp, j, Nv);
      double X[3];
      X[d - 1] = 0.0;
      int t = j;
      for (int tt = 0; tt < d - 1; ++tt) {
        int ta = tang(d, d - 1, tt);
        double dx = m->L[ta] / (m->n[ta] * (double)(1 << fp.lev));
        X[ta] = dx * (fp.T[ta] + 0.5 * (1.0 + m->xi[t % m->np1]));
        t /= m->np1;
      }
      double h, hx, hy;
      terrain(&m->cs, X[0], d == 3 ? X[1] : 0.0, &h, &hx, &hy);
      double* o = &out[6 * cnt];
      o[0] = X[0];
      o[1] = d == 3 ? X[1] : 0.0;
      o[2] = h;
      o[3] = -Nv[0];
      o[4] = d == 3 ? -Nv[1] : 0.0;
      o[5] = -Nv[d - 1];
      ++cnt;
    }
  }
  return cnt;
}
