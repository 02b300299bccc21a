"""Brute-force assembly of the implicit pressure operator (no GPU).

The weak operators of the implicit stage (the gradient B, the divergence C, the pressure-jump
penalty P and the mass matrix M; Section 3.2 applies them matrix-free) are assembled here as dense
global matrices, cell by cell and face by face, from their definitions alone: Gauss-Legendre
quadrature from numpy, Lagrange polynomials written out as products, the terrain-following map
x = X, y = Y, z = zeta + h(x, y)(1 - zeta/H) differentiated in closed form (terrain slopes by the
complex step), face neighbours found by comparing the cells' logical boxes, and face normals from
the cross product of the face's tangent vectors.  Nothing here calls the oracle's operators; the
oracle only supplies its cell list and node order.  The assembled

    A = M/(gamma-1) + dt_a beta/(2(gamma-1)) P - dt_a^2 C diag(h) M^-1 B

must equal the oracle's matrix-free operator, column by column, on the 7-cell 2D and 15-cell 3D
meshes with 2:1 faces, over terrain, with periodic sides and walls.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from tests import _exact as E

GAMMA = 1.4


def tiny2d(r, h0, periodic):
    """2x2 base quads, the lower-left cell refined once: 7 cells, hanging faces along x and z."""
    return O.Case(dim=2, degree=r, nbase=(2, 1, 2), length=(1000.0, 1.0, 1000.0), periodic=periodic,
                  rules=[(500.0, 250.0, 250.0, 0, 0)], oro_kind=O.GAUSS_HILL,
                  oro=(h0, 300.0, 500.0, 0.0), atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0))


def tiny3d(r, h0, periodic):
    """2x2x2 base hexes, one corner cell refined once: 15 cells."""
    return O.Case(dim=3, degree=r, nbase=(2, 2, 2), length=(1000.0, 1000.0, 1000.0), periodic=periodic,
                  rules=[(500.0, 250.0, 250.0, 250.0, 250.0)], oro_kind=O.GAUSS_HILL,
                  oro=(h0, 300.0, 500.0, 500.0), atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0))


def lagrange(nodes, t):
    """Values and derivatives of the Lagrange polynomials on `nodes` at the points t."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(nodes)
    val = np.ones((len(t), n))
    der = np.zeros((len(t), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                val[:, j] *= (t - nodes[m]) / (nodes[j] - nodes[m])
        for m in range(n):
            if m == j:
                continue
            term = np.full(len(t), 1.0 / (nodes[j] - nodes[m]))
            for q in range(n):
                if q != j and q != m:
                    term *= (t - nodes[q]) / (nodes[j] - nodes[q])
            der[:, j] += term
    return val, der


class Assembly:
    """Dense M, B, C, P of one mesh, built from the definitions."""

    def __init__(self, case: O.Case, cells: np.ndarray):
        self.c = case
        self.d = d = case.dim
        self.r = case.degree
        self.np1 = self.r + 1
        self.nloc = self.np1 ** d
        self.cells = cells
        self.ncell = len(cells)
        self.N = self.ncell * self.nloc
        self.xi, self.wg = np.polynomial.legendre.leggauss(self.np1)
        # axes in the oracle's node order: 2D (x, z), 3D (x, y, z); the vertical axis is last
        self.L = [case.length[0], case.length[2]] if d == 2 else list(case.length)
        self.nb = [case.nbase[0], case.nbase[2]] if d == 2 else list(case.nbase)
        self.per = [case.periodic[0], 0] if d == 2 else [case.periodic[0], case.periodic[1], 0]
        self.H = case.length[2]
        # logical box of every cell: lower corner and size per axis
        self.lo = np.zeros((self.ncell, d))
        self.size = np.zeros((self.ncell, d))
        for c, (lev, ix, iy, iz) in enumerate(cells):
            idx = [ix, iz] if d == 2 else [ix, iy, iz]
            for a in range(d):
                self.size[c, a] = self.L[a] / (self.nb[a] * 2 ** lev)
                self.lo[c, a] = idx[a] * self.size[c, a]
        # reference node k of a cell: per-axis index tuple (x fastest)
        self.multi = list(itertools.product(range(self.np1), repeat=d))
        self.multi = [tuple(reversed(m)) for m in self.multi]

    # -------------------------------------------------------------- geometry of the global map
    def _h(self, X):
        y = X[1] if self.d == 3 else 0.0 * X[0]
        h = E.terrain(self.c.oro_kind, self.c.oro, self.d, X[0], y)
        hx, hy = E.terrain_slopes(self.c.oro_kind, self.c.oro, self.d, X[0], y)
        return h, hx, hy

    def jacobian(self, X):
        """d(x_phys)/d(X_logical) at logical points X (shape d x npts) -> (npts, d, d)."""
        d = self.d
        h, hx, hy = self._h(X)
        zeta = X[d - 1]
        J = np.zeros((X.shape[1], d, d))
        for a in range(d - 1):
            J[:, a, a] = 1.0
        J[:, d - 1, 0] = hx * (1.0 - zeta / self.H)
        if d == 3:
            J[:, d - 1, 1] = hy * (1.0 - zeta / self.H)
        J[:, d - 1, d - 1] = 1.0 - h / self.H
        return J

    # ---------------------------------------------------------------------- basis at a point
    def basis(self, c, X):
        """Values (npts, nloc) and physical gradients (npts, nloc, d) of cell c's basis at
        logical points X (d x npts)."""
        d = self.d
        ref = [(X[a] - self.lo[c, a]) / self.size[c, a] * 2.0 - 1.0 for a in range(d)]
        v1 = []
        d1 = []
        for a in range(d):
            v, dv = lagrange(self.xi, ref[a])
            v1.append(v)
            d1.append(dv * 2.0 / self.size[c, a])            # d/dX_a
        npts = X.shape[1]
        val = np.ones((npts, self.nloc))
        gradX = np.ones((npts, self.nloc, d))
        for k, m in enumerate(self.multi):
            for a in range(d):
                val[:, k] *= v1[a][:, m[a]]
                for b in range(d):
                    gradX[:, k, b] *= (d1[a][:, m[a]] if a == b else v1[a][:, m[a]])
        J = self.jacobian(X)
        Jinv = np.linalg.inv(J)
        grad = np.einsum("pkb,pbx->pkx", gradX, Jinv)      # grad_x phi = grad_X phi J^-1
        return val, grad

    def nodes(self, c):
        """Logical coordinates (d x nloc) and weights x det J of cell c's nodes."""
        d = self.d
        X = np.zeros((d, self.nloc))
        w = np.ones(self.nloc)
        for k, m in enumerate(self.multi):
            for a in range(d):
                X[a, k] = self.lo[c, a] + 0.5 * self.size[c, a] * (1.0 + self.xi[m[a]])
                w[k] *= self.wg[m[a]] * 0.5 * self.size[c, a]
        return X, w * np.linalg.det(self.jacobian(X))

    # ----------------------------------------------------------------------------- faces
    def faces(self):
        """Every (sub)face once: (axis k, lower cell or None, upper cell or None, logical points
        (d x nq), weights, area-weighted normal (nq x d) pointing to increasing X_k)."""
        d = self.d
        out = []
        for k in range(d):
            tang = [a for a in range(d) if a != k]
            for cl in range(self.ncell):
                xk = self.lo[cl, k] + self.size[cl, k]
                for cu in range(self.ncell):
                    xu = self.lo[cu, k]
                    same = abs(xk - xu) < 1e-9
                    seam = self.per[k] and abs(xk - self.L[k]) < 1e-9 and abs(xu) < 1e-9
                    if not (same or seam):
                        continue
                    lo_t, hi_t = [], []
                    ok = True
                    for a in tang:
                        l0 = max(self.lo[cl, a], self.lo[cu, a])
                        h0 = min(self.lo[cl, a] + self.size[cl, a], self.lo[cu, a] + self.size[cu, a])
                        if h0 - l0 < 1e-9:
                            ok = False
                        lo_t.append(l0)
                        hi_t.append(h0)
                    if ok:
                        # the seam's geometry is taken at its reduced position X_k = 0
                        out.append((k, cl, cu, self._face_quad(k, 0.0 if seam else xk, tang, lo_t, hi_t)))
            # walls: lower faces at X_k = 0 and upper faces at X_k = L_k without a periodic partner
            if not self.per[k]:
                for c in range(self.ncell):
                    t_lo = [self.lo[c, a] for a in tang]
                    t_hi = [self.lo[c, a] + self.size[c, a] for a in tang]
                    if abs(self.lo[c, k]) < 1e-9:
                        out.append((k, None, c, self._face_quad(k, 0.0, tang, t_lo, t_hi)))
                    if abs(self.lo[c, k] + self.size[c, k] - self.L[k]) < 1e-9:
                        out.append((k, c, None, self._face_quad(k, self.L[k], tang, t_lo, t_hi)))
        return out

    def _face_quad(self, k, xk, tang, lo_t, hi_t):
        d = self.d
        pts = list(itertools.product(range(self.np1), repeat=d - 1))
        X = np.zeros((d, len(pts)))
        w = np.ones(len(pts))
        X[k] = xk
        for j, m in enumerate(pts):
            for t, a in enumerate(tang):
                X[a, j] = lo_t[t] + 0.5 * (hi_t[t] - lo_t[t]) * (1.0 + self.xi[m[t]])
                w[j] *= self.wg[m[t]] * 0.5 * (hi_t[t] - lo_t[t])
        # tangent vectors d(x_phys)/dX_a for the tangential axes, normal by the cross product
        J = self.jacobian(X)
        if d == 2:
            t = J[:, :, tang[0]]
            n = np.stack([t[:, 1], -t[:, 0]], axis=1)        # rotate: X_k increases to the right
            if k == 1:
                n = -n
        else:
            t0, t1 = J[:, :, tang[0]], J[:, :, tang[1]]
            n = np.cross(t0, t1)
            if k == 1:
                n = -n                                        # (x, z) tangents for a y-face
        return X, w, n

    # ---------------------------------------------------------------------------- operators
    def assemble(self, h, lam_cell):
        d, N, nl = self.d, self.N, self.nloc
        M = np.zeros(N)
        B = np.zeros((d * N, N))          # weak gradient: row (k, node i), column node j
        C = np.zeros((N, d * N))          # weak divergence
        P = np.zeros((N, N))              # pressure-jump penalty
        for c in range(self.ncell):
            X, wJ = self.nodes(c)
            sl = slice(c * nl, (c + 1) * nl)
            M[sl] = wJ
            _, grad = self.basis(c, X)                    # at the nodes (collocated quadrature)
            for k in range(d):
                # -int p d_k phi_i = -sum_q wJ_q p_q d_k phi_i(x_q)
                B[k * N + c * nl:k * N + (c + 1) * nl, sl] += -(grad[:, :, k] * wJ[:, None]).T
                # -int w_k d_k psi_i
                C[sl, k * N + c * nl:k * N + (c + 1) * nl] += -(grad[:, :, k] * wJ[:, None]).T
        for k, cl, cu, (X, w, n) in self.faces():
            sides = []
            for cell, sgn in ((cl, 1.0), (cu, -1.0)):
                if cell is None:
                    sides.append(None)
                    continue
                Xc = X.copy()
                if self.per[k] and Xc[k, 0] == 0.0 and sgn > 0:
                    Xc[k] = self.L[k]                       # the seam seen from its lower cell
                val, _ = self.basis(cell, Xc)
                sides.append((cell, sgn, val))
            if sides[0] is None or sides[1] is None:         # wall: p^ = p-, no divergence flux
                cell, sgn, val = sides[0] or sides[1]
                sl = slice(cell * nl, (cell + 1) * nl)
                for kk in range(d):
                    B[kk * N + cell * nl:kk * N + (cell + 1) * nl, sl] += \
                        np.einsum("p,pi,pj->ij", w * sgn * n[:, kk], val, val)
                continue
            lamf = max(lam_cell[cl], lam_cell[cu])
            area = np.linalg.norm(n, axis=1)
            for (ca, sa, va) in sides:
                sla = slice(ca * nl, (ca + 1) * nl)
                for (cb, _, vb) in sides:
                    slb = slice(cb * nl, (cb + 1) * nl)
                    for kk in range(d):
                        # int {p} phi_i n_k (outward for a) and int psi_i {w}.n
                        blk = 0.5 * np.einsum("p,pi,pj->ij", w * sa * n[:, kk], va, vb)
                        B[kk * N + ca * nl:kk * N + (ca + 1) * nl, slb] += blk
                        C[sla, kk * N + cb * nl:kk * N + (cb + 1) * nl] += blk
                    # int lam_f (p_a - p_b) psi_i
                    s = 1.0 if ca == cb else -1.0
                    P[sla, slb] += s * lamf * np.einsum("p,pi,pj->ij", w * area, va, vb)
        return M, B, C, P


def _matrix(apply, n):
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = apply(e)
    return A


@pytest.mark.parametrize("mk,r,periodic", [(tiny2d, 2, (1, 1)), (tiny2d, 3, (0, 0)),
                                           (tiny3d, 2, (1, 1)), (tiny3d, 2, (0, 1))])
def test_assembled_operators_equal_matrix_free(mk, r, periodic):
    case = mk(r, 120.0, periodic)
    o = O.Oracle(case)
    asm = Assembly(case, o.cells)
    rng = np.random.default_rng(17)
    h = 1e5 * (3.0 + rng.uniform(0, 1, o.N))
    lam = np.sqrt((GAMMA - 1.0) * h).reshape(o.ncell, o.nloc).max(axis=1)
    M, B, C, P = asm.assemble(h, lam)
    N, d = o.N, o.d
    assert np.max(np.abs(M - o.wJ)) < 1e-12 * np.max(M)
    # the oracle's weak gradient M^-1 B, divergence C and penalty, one column at a time
    Bo = np.zeros((d * N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        Bo[:, j] = (o.wJ[None, :] * o.grad(e)).ravel()
    assert np.max(np.abs(Bo - B)) < 1e-11 * np.max(np.abs(B))
    Co = np.zeros((N, d * N))
    for j in range(d * N):
        e = np.zeros(d * N)
        e[j] = 1.0
        Co[:, j] = o.div(e.reshape(d, N))
    assert np.max(np.abs(Co - C)) < 1e-11 * np.max(np.abs(C))
    Po = _matrix(lambda e: o.penalty(lam, e), N)
    assert np.max(np.abs(Po - P)) < 1e-11 * np.max(np.abs(P))
    dta = 0.8
    Aref = (np.diag(M) / (GAMMA - 1.0) + dta * o.beta / (2 * (GAMMA - 1.0)) * P
            - dta ** 2 * C @ (np.tile(h / M, d)[:, None] * B))
    Ao = _matrix(lambda e: o.helmholtz(dta, h, lam, e), N)
    assert np.max(np.abs(Ao - Aref)) < 1e-11 * np.max(np.abs(Aref))
