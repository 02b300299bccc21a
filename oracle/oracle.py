"""Plain FP64 CPU oracle of the IMEX-DG compressible Euler step.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline leg of
the benchmark; the GPU library never imports or links it, and it shares no code with it.

The spatial operators (explicit residual, weak gradient B, weak divergence C, pressure penalty P,
geometry, mesh) are in ``dg_oracle.c`` as dense loops.  This module composes them, following the
paper (Orlando, Benacchio, Bonaventura, arXiv 2408.08129):

* Section 2, Eq. (1): Euler equations in SI units, g = 9.81, R = 287, gamma = 1.4, rhoE = rho e +
  rho k with k = |u|^2 / 2;
* Section 2: continuity explicit, energy coupled implicitly to momentum; a second-order IMEX-RK
  method (ARK2 of Giraldo, Kelly, Constantinescu 2013: explicit stage 1, two implicit stages with
  diagonal 1 - 1/sqrt(2));
* Section 3.2: each implicit stage runs a fixed-point loop for the pressure whose linear system is
  non-symmetric and solved with GMRES, applying the operators matrix-free;
* Section 3.1, Eq. (4)-(5): the stratified initial state (with the factor g^2 / N^2 that makes it
  hydrostatic), or an isothermal atmosphere;
* Section 3.1: the test runs with non-reflecting top and lateral boundaries whose form the paper
  defers to cited work.  Reading used here: absorbing layers of Rayleigh friction on the momentum,
  d m / dt = -tau (m - rho u_ref e_x), explicit, with the sin^2 rate profile of Klemp and Lilly
  (1978) below the lid and along the lateral sides, walled or periodic (mass and total energy
  untouched: the layer turns the damped kinetic energy into heat).
* Optional enthalpy split of the implicit energy flux (enthalpy_split=True): the background part
  of div(h m) is taken as hbar div(m) + m . grad(hbar), with the continuity equation's discrete
  divergence and the exact height derivative of the background enthalpy, so that the discrete
  buoyancy balance of grid-scale modes keeps the sign of N^2.

The pressure unknown of the implicit stage is the perturbation p' = p - pbar from the analytic
hydrostatic background evaluated at every node, so that an atmosphere at rest has exactly zero
tendencies.  The implicit stage solves, for the increment delta of p' at fixed-point iterate l,

    A(h^l) delta = b^l - A(h^l) p'^l,
    A(h) = M / (gamma - 1) + dt a P(h) - (dt a)^2 C diag(h) M^{-1} B,
    b^l  = M (e~ - rho k^l - pbar / (gamma - 1)) - dt a C (h^l m'),

where h = gamma p / ((gamma - 1) rho) is the specific enthalpy, m' the momentum predictor including
the implicit buoyancy -dt a (rho - rhobar) g k, and the momentum follows as
m = m' - dt a M^{-1} B p'.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

G = 9.81
RGAS = 287.0
GAMMA = 1.4

FLAT, AGNESI, BELL, GAUSS_HILL, GAUSS_RIDGE = range(5)
ISOTHERMAL, STRATIFIED = range(2)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build_oracle(force: bool = False) -> str:
    """Compile dg_oracle.c with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                               "-fopenmp", "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp,
                               "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Case(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("degree", ctypes.c_int32),
        ("nbase", ctypes.c_int32 * 3), ("periodic", ctypes.c_int32 * 2),
        ("n_rules", ctypes.c_int32), ("oro_kind", ctypes.c_int32), ("atm_kind", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("length", ctypes.c_double * 3), ("rules", (ctypes.c_double * 5) * 8),
        ("oro", ctypes.c_double * 4), ("atm", ctypes.c_double * 3), ("grav", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build_oracle())
        P = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.oc_mesh_build.argtypes = [ctypes.POINTER(_Case), ctypes.POINTER(P)]
        L.oc_mesh_build.restype = ctypes.c_int
        L.oc_mesh_free.argtypes = [P]
        for name in ("oc_ncell", "oc_nloc", "oc_nhang", "oc_lmax"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = ctypes.c_int
        L.oc_cell_table.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.oc_node_geometry.argtypes = [P, dp, dp, dp, dp]
        L.oc_background_nodes.argtypes = [P, dp, dp]
        L.oc_explicit_residual.argtypes = [P, dp, dp]
        L.oc_explicit_residual_oi.argtypes = [P, dp, dp]
        L.oc_explicit_residual_oi.restype = ctypes.c_int
        L.oc_set_quadrature.argtypes = [P, ctypes.c_int]
        L.oc_set_quadrature.restype = ctypes.c_int
        L.oc_grad.argtypes = [P, dp, dp]
        L.oc_div.argtypes = [P, dp, dp]
        L.oc_penalty.argtypes = [P, dp, dp, dp]
        L.oc_cell_sizes.argtypes = [P, dp]
        L.oc_bottom_normals.argtypes = [P, dp]
        L.oc_bottom_normals.restype = ctypes.c_int
        L.oc_wall_flux.argtypes = [ctypes.c_int, dp, dp, dp]
        L.oc_gauss.argtypes = [ctypes.c_int, dp, dp]
        L.oc_lagrange_eval.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp, dp]
        L.oc_background.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp, dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gauss(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().oc_gauss(n, _p(x), _p(w))
    return x, w


def wall_flux(d: int, U: np.ndarray, N: np.ndarray) -> np.ndarray:
    """The oracle's slip-wall flux at one point: conserved state U (d + 2 values) and outward
    area-weighted normal N (d values)."""
    out = np.zeros(d + 2)
    lib().oc_wall_flux(d, _p(np.ascontiguousarray(U, dtype=np.float64)),
                       _p(np.ascontiguousarray(N, dtype=np.float64)), _p(out))
    return out


def lagrange_eval(nodes: np.ndarray, x: float):
    n = len(nodes)
    v = np.zeros(n)
    d = np.zeros(n)
    lib().oc_lagrange_eval(n, _p(np.ascontiguousarray(nodes, dtype=np.float64)), float(x), _p(v), _p(d))
    return v, d


def background(kind: int, atm, z: float):
    a = np.array(list(atm) + [0.0] * (3 - len(atm)), dtype=np.float64)
    p = ctypes.c_double()
    r = ctypes.c_double()
    lib().oc_background(kind, _p(a), float(z), ctypes.byref(p), ctypes.byref(r))
    return p.value, r.value


@dataclass
class Case:
    """Problem description: logical box, base grid, refinement rules, orography, atmosphere."""
    dim: int
    degree: int
    nbase: tuple
    length: tuple
    periodic: tuple = (1, 1)
    rules: list = field(default_factory=list)  # (zeta_max, x_c, hw_x, y_c, hw_y)
    oro_kind: int = FLAT
    oro: tuple = (0.0, 1.0, 0.0, 0.0)
    atm_kind: int = ISOTHERMAL
    atm: tuple = (1.0e5, 250.0, 0.0)
    # absorbing layers: (top depth, top rate, lateral width, lateral rate, reference wind u_ref)
    sponge: tuple = (0.0, 0.0, 0.0, 0.0, 0.0)
    # gravitational acceleration of Eq. (1); 0 (isothermal atmosphere only) switches the gravity
    # terms off, for the exact isentropic-vortex solution of the Euler equations
    gravity: float = G

    def to_struct(self) -> _Case:
        c = _Case()
        c.dim = self.dim
        c.degree = self.degree
        for i in range(3):
            c.nbase[i] = int(self.nbase[i])
            c.length[i] = float(self.length[i])
        c.periodic[0] = int(self.periodic[0])
        c.periodic[1] = int(self.periodic[1])
        c.n_rules = len(self.rules)
        for i, r in enumerate(self.rules):
            for j in range(5):
                c.rules[i][j] = float(r[j])
        c.oro_kind = self.oro_kind
        for i in range(4):
            c.oro[i] = float(self.oro[i])
        c.atm_kind = self.atm_kind
        atm = list(self.atm) + [0.0] * (3 - len(self.atm))
        for i in range(3):
            c.atm[i] = float(atm[i])
        c.grav = float(self.gravity)
        return c


class MeshError(RuntimeError):
    pass


class Oracle:
    """Mesh + operators + IMEX-RK2 step of the oracle for one case."""

    # ARK2 (Giraldo, Kelly, Constantinescu 2013) in Butcher form.
    ARK_G = 1.0 - 1.0 / math.sqrt(2.0)
    ARK_D = 1.0 / (2.0 * math.sqrt(2.0))
    ARK_A = (3.0 + 2.0 * math.sqrt(2.0)) / 6.0

    def __init__(self, case: Case, beta: float = 1.0, quad_extra: int = 0, enthalpy_split: bool = False):
        self.case = case
        self.beta = beta
        self.quad_extra = quad_extra
        self.enthalpy_split = enthalpy_split
        self._cs = case.to_struct()
        h = ctypes.c_void_p()
        rc = lib().oc_mesh_build(ctypes.byref(self._cs), ctypes.byref(h))
        if rc != 0:
            raise MeshError("oracle mesh build failed (%d)" % rc)
        self._m = h
        L = lib()
        self.d = case.dim
        self.r = case.degree
        self.nf = self.d + 2
        self.ncell = L.oc_ncell(h)
        self.nloc = L.oc_nloc(h)
        self.nhang = L.oc_nhang(h)
        self.lmax = L.oc_lmax(h)
        self.g = float(case.gravity)
        self.N = self.ncell * self.nloc
        cells = np.zeros((self.ncell, 4), dtype=np.int32)
        L.oc_cell_table(h, cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self.cells = cells
        self.x = np.zeros(self.N)
        self.y = np.zeros(self.N)
        self.z = np.zeros(self.N)
        self.wJ = np.zeros(self.N)
        L.oc_node_geometry(h, _p(self.x), _p(self.y), _p(self.z), _p(self.wJ))
        self.pbar = np.zeros(self.N)
        self.rbar = np.zeros(self.N)
        L.oc_background_nodes(h, _p(self.pbar), _p(self.rbar))
        sz = np.zeros((self.ncell, 3))
        L.oc_cell_sizes(h, _p(sz))
        self.cell_sizes = sz
        self.tau = self.sponge_rate()
        self.hbar, self.dhbar = self.background_enthalpy()
        if quad_extra > 0:
            # over-integration of the explicit flux: r + 1 + quad_extra Gauss points per direction
            if L.oc_set_quadrature(h, self.r + 1 + quad_extra) != 0:
                raise ValueError("quad_extra out of range")
        g, a, dd = self.ARK_G, self.ARK_A, self.ARK_D
        self.A = np.array([[0, 0, 0], [2 * g, 0, 0], [1 - a, a, 0]], dtype=np.float64)
        self.At = np.array([[0, 0, 0], [g, g, 0], [dd, dd, g]], dtype=np.float64)
        self.b = np.array([dd, dd, g])
        self.bt = np.array([dd, dd, g])

    def __del__(self):
        try:
            lib().oc_mesh_free(self._m)
        except Exception:
            pass

    # ---------------------------------------------------------------------------- absorbing layers
    def sponge_rate(self) -> np.ndarray:
        """Rayleigh friction rate tau at every node (physical coordinates): below the lid,
        tau_t sin^2(pi/2 (z - z_s) / (H - z_s)) for z > z_s = H - depth; along each lateral side
        (x = 0, x = Lx and, in 3D, y = 0, y = Ly; walled or periodic: at a periodic seam the
        layer absorbs what leaves on one side before it comes back on the other),
        tau_l sin^2(pi/2 (1 - dist / width)) for dist < width; the rates add."""
        depth, rate_t, width, rate_l, _ = (float(v) for v in self.case.sponge)
        c = self.case
        H = float(c.length[2])
        tau = np.zeros(self.N)
        if depth > 0.0 and rate_t > 0.0:
            zs = H - depth
            t = np.clip((self.z - zs) / depth, 0.0, None)
            tau += np.where(self.z > zs, rate_t * np.sin(0.5 * math.pi * t) ** 2, 0.0)
        if width > 0.0 and rate_l > 0.0:
            walls = [(0, self.x, float(c.length[0]))]
            if self.d == 3:
                walls.append((1, self.y, float(c.length[1])))
            for ax, coord, L in walls:
                dist = np.minimum(coord, L - coord)
                t = np.clip(1.0 - dist / width, 0.0, None)
                tau += np.where(dist < width, rate_l * np.sin(0.5 * math.pi * t) ** 2, 0.0)
        return tau

    # -------------------------------------------------------------------------------- operators
    def explicit_residual(self, U: np.ndarray) -> np.ndarray:
        """M^{-1} times the explicit weak form, plus the absorbing-layer friction on the momentum."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        R = np.zeros_like(U)
        if self.quad_extra > 0:
            lib().oc_explicit_residual_oi(self._m, _p(U), _p(R))
        else:
            lib().oc_explicit_residual(self._m, _p(U), _p(R))
        if np.any(self.tau > 0.0):
            uref = float(self.case.sponge[4])
            R[1:1 + self.d] -= self.tau[None, :] * U[1:1 + self.d]
            R[1] += self.tau * U[0] * uref
        return R

    def background_enthalpy(self):
        """Enthalpy of the hydrostatic background at the nodes, hbar = gamma pbar / ((gamma-1) rhobar),
        and its vertical derivative from the closed form of the background (dp/dz = -rho g):
        d hbar / dz = -g + c_p T N^2 / g in the stratified atmosphere, 0 in the isothermal one."""
        hbar = GAMMA * self.pbar / ((GAMMA - 1.0) * self.rbar)
        if self.case.atm_kind == STRATIFIED:
            Nb = float(self.case.atm[2])
            T = self.pbar / (RGAS * self.rbar)
            dhbar = -self.g + GAMMA * RGAS / (GAMMA - 1.0) * T * Nb * Nb / self.g
        else:
            dhbar = np.zeros(self.N)
        return hbar, dhbar

    def enthalpy_flux_div(self, h: np.ndarray, m: np.ndarray) -> np.ndarray:
        """Weak divergence of the implicit energy flux h m.  Plain: C(h m).  With the enthalpy
        split the background part is written as hbar div(m) + m . grad(hbar) with the same discrete
        divergence C as the continuity equation and the exact gradient of hbar (which depends on
        the height only): C((h - hbar) m) + hbar C(m) + M (d hbar/dz) m_z."""
        if not self.enthalpy_split:
            return self.div(h[None, :] * m)
        return (self.div((h - self.hbar)[None, :] * m) + self.hbar * self.div(m)
                + self.wJ * self.dhbar * m[self.d - 1])

    def grad(self, p: np.ndarray) -> np.ndarray:
        """M^{-1} B p, shape (d, N)."""
        p = np.ascontiguousarray(p, dtype=np.float64)
        q = np.zeros((self.d, self.N))
        lib().oc_grad(self._m, _p(p), _p(q))
        return q

    def div(self, w: np.ndarray) -> np.ndarray:
        """C w in weak form, w of shape (d, N)."""
        w = np.ascontiguousarray(w, dtype=np.float64)
        out = np.zeros(self.N)
        lib().oc_div(self._m, _p(w), _p(out))
        return out

    def penalty(self, lam_cell: np.ndarray, p: np.ndarray) -> np.ndarray:
        """Jump penalty sum over faces of lam_f |N| (p_own - p_other) psi, weak form."""
        lam_cell = np.ascontiguousarray(lam_cell, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        out = np.zeros(self.N)
        lib().oc_penalty(self._m, _p(lam_cell), _p(p), _p(out))
        return out

    def bottom_normals(self) -> np.ndarray:
        out = np.zeros((self.ncell * self.nloc, 6))
        n = lib().oc_bottom_normals(self._m, _p(out))
        return out[:n]

    # ------------------------------------------------------------------- pointwise thermodynamics
    def pressure(self, U: np.ndarray) -> np.ndarray:
        rho = U[0]
        m2 = np.sum(U[1:1 + self.d] ** 2, axis=0)
        return (GAMMA - 1.0) * (U[1 + self.d] - 0.5 * m2 / rho)

    def enthalpy(self, p: np.ndarray, rho: np.ndarray) -> np.ndarray:
        return GAMMA * p / ((GAMMA - 1.0) * rho)

    def cell_sound_speed(self, h: np.ndarray) -> np.ndarray:
        """Per-cell maximum of c = sqrt((gamma - 1) h)."""
        c = np.sqrt((GAMMA - 1.0) * h)
        return c.reshape(self.ncell, self.nloc).max(axis=1)

    # ------------------------------------------------------------------------- implicit operator
    def helmholtz(self, dta: float, h: np.ndarray, lam: np.ndarray, p: np.ndarray) -> np.ndarray:
        """A(h) p = M p / (gamma-1) + dt a beta/(2(gamma-1)) P p - (dt a)^2 C (h M^{-1} B p)."""
        q = self.grad(p)
        out = self.wJ * p / (GAMMA - 1.0)
        if self.beta != 0.0:
            out = out + dta * self.beta / (2.0 * (GAMMA - 1.0)) * self.penalty(lam, p)
        out = out - dta * dta * self.enthalpy_flux_div(h, q)
        return out

    def jacobi_diag(self, dta: float, h: np.ndarray) -> np.ndarray:
        """Diagonal scaling used as preconditioner: w J [1/(gamma-1) + (dt a)^2 h sum_k ((r+1)/D_k)^2]
        with D_k the logical cell size along axis k."""
        r1 = self.r + 1
        s = np.sum((r1 / self.cell_sizes[:, :self.d]) ** 2, axis=1)
        s = np.repeat(s, self.nloc)
        return self.wJ * (1.0 / (GAMMA - 1.0) + dta * dta * h * s)

    # -------------------------------------------- cell-wise fast-diagonalisation preconditioner
    # Not from the paper (which names stronger preconditioning as future work, Section 3.2): the
    # right preconditioner of the GPU path's Krylov solves, written here from its definition.
    @staticmethod
    def fdm_line_operator(r: int, nc: int = 3):
        """The 1D second-order operator G = B^T W^{-1} B on a periodic row of nc reference cells
        [-1, 1] (cell K covers [2K - 1, 2K + 1]), with B the weak gradient of a nodal degree-r field
        on the Gauss points with the central flux {p} at the two cell ends:
            (B p)_i = -sum_j w_j p_j l_i'(x_j) + l_i(1) {p}(1) - l_i(-1) {p}(-1),
        and W the Gauss weights.  Returns (L, G, W), L the block of G on cell 1 (the preconditioner
        uses nc = 3: the middle cell)."""
        n1 = r + 1
        x, w = gauss(n1)
        lm = lagrange_eval(x, -1.0)[0]
        lp = lagrange_eval(x, 1.0)[0]
        dl = np.array([lagrange_eval(x, xj)[1] for xj in x])  # dl[j, i] = l_i'(x_j)
        B = np.zeros((nc * n1, nc * n1))
        for K in range(nc):
            own = slice(K * n1, (K + 1) * n1)
            right = slice(((K + 1) % nc) * n1, ((K + 1) % nc + 1) * n1)
            left = slice(((K - 1) % nc) * n1, ((K - 1) % nc + 1) * n1)
            B[own, own] += -(dl * w[:, None]).T  # -sum_j w_j l_i'(x_j) p_j
            B[own, own] += 0.5 * np.outer(lp, lp) - 0.5 * np.outer(lm, lm)
            B[own, right] += 0.5 * np.outer(lp, lm)
            B[own, left] -= 0.5 * np.outer(lm, lp)
        W = np.tile(w, nc)
        G = B.T @ (B / W[:, None])
        return G[n1:2 * n1, n1:2 * n1], G, W

    @classmethod
    def fdm_eigen(cls, r: int):
        """Generalised eigenpairs L s = mu W s of the middle-cell block, S^T W S = I."""
        from scipy.linalg import eigh
        L, _, W = cls.fdm_line_operator(r)
        mu, S = eigh(L, np.diag(W[:r + 1]))
        return mu, S

    def node_weights(self) -> np.ndarray:
        """Tensor Gauss weight of every node of a cell (x fastest, the vertical axis slowest)."""
        _, w = gauss(self.r + 1)
        wn = w
        for _ in range(self.d - 1):
            wn = np.kron(w, wn)
        return wn

    def fdm_coefficients(self, dta: float, h: np.ndarray):
        """Per cell: Jbar = mean over the nodes of the map's Jacobian wJ / w, hbar = mean of h,
        alpha_k = dta^2 hbar (2 / D_k)^2 with D_k the cell size and the vertical one multiplied by
        the mean terrain stretching Jbar / prod(D_k / 2).  Returns (Jbar, alpha[ncell, d])."""
        J = (self.wJ.reshape(self.ncell, self.nloc) / self.node_weights()[None, :])
        Jbar = J.mean(axis=1)
        hbar = np.asarray(h, dtype=np.float64).reshape(self.ncell, self.nloc).mean(axis=1)
        D = self.cell_sizes[:, :self.d].copy()
        stretch = Jbar / np.prod(0.5 * D, axis=1)
        D[:, self.d - 1] *= stretch
        alpha = dta * dta * hbar[:, None] * (2.0 / D) ** 2
        return Jbar, alpha

    def fdm_apply(self, dta: float, h: np.ndarray, v: np.ndarray) -> np.ndarray:
        """z = (1/Jbar) (S x .. x S) diag(1 / (1/(gamma-1) + sum_k alpha_k mu_{i_k})) (S x .. x S)^T v
        in every cell (i_k the index along axis k; the transforms act along each axis of the cell's
        node array)."""
        n1, d = self.r + 1, self.d
        mu, S = self.fdm_eigen(self.r)
        Jbar, alpha = self.fdm_coefficients(dta, h)
        V = np.asarray(v, dtype=np.float64).reshape((self.ncell,) + (n1,) * d)  # [cell][(z,) y/z .. x]
        if d == 3:
            Vh = np.einsum("za,yb,xc,nzyx->nabc", S, S, S, V)
            den = (1.0 / (GAMMA - 1.0) + alpha[:, 2, None, None, None] * mu[None, :, None, None]
                   + alpha[:, 1, None, None, None] * mu[None, None, :, None]
                   + alpha[:, 0, None, None, None] * mu[None, None, None, :])
            Z = np.einsum("za,yb,xc,nabc->nzyx", S, S, S, Vh / den)
        else:
            Vh = np.einsum("za,xc,nzx->nac", S, S, V)
            den = (1.0 / (GAMMA - 1.0) + alpha[:, 1, None, None] * mu[None, :, None]
                   + alpha[:, 0, None, None] * mu[None, None, :])
            Z = np.einsum("za,xc,nac->nzx", S, S, Vh / den)
        return (Z / Jbar.reshape((-1,) + (1,) * d)).reshape(-1)

    # ------------------------------------------------------------------------------------ GMRES
    @staticmethod
    def gmres(apply, b: np.ndarray, dinv: np.ndarray, rtol: float, atol: float, restart: int,
              maxit: int):
        """Right-preconditioned restarted GMRES(m) with modified Gram-Schmidt and Givens rotations,
        zero initial guess; stops when the residual 2-norm is <= max(rtol |b|, atol).
        Returns (x, iterations, final residual norm, converged)."""
        n = b.shape[0]
        x = np.zeros(n)
        bnorm = float(np.linalg.norm(b))
        tol = max(rtol * bnorm, atol)
        if bnorm <= tol or bnorm == 0.0:
            return x, 0, bnorm, True
        its = 0
        r = b.copy()
        beta = bnorm
        while True:
            V = np.zeros((restart + 1, n))
            Hs = np.zeros((restart + 1, restart))
            cs = np.zeros(restart)
            sn = np.zeros(restart)
            g = np.zeros(restart + 1)
            V[0] = r / beta
            g[0] = beta
            j_done = 0
            res = beta
            for j in range(restart):
                w = apply(dinv * V[j])
                for i in range(j + 1):
                    Hs[i, j] = float(np.dot(V[i], w))
                    w = w - Hs[i, j] * V[i]
                Hs[j + 1, j] = float(np.linalg.norm(w))
                if Hs[j + 1, j] != 0.0:
                    V[j + 1] = w / Hs[j + 1, j]
                for i in range(j):
                    t = cs[i] * Hs[i, j] + sn[i] * Hs[i + 1, j]
                    Hs[i + 1, j] = -sn[i] * Hs[i, j] + cs[i] * Hs[i + 1, j]
                    Hs[i, j] = t
                den = math.hypot(Hs[j, j], Hs[j + 1, j])
                cs[j] = Hs[j, j] / den
                sn[j] = Hs[j + 1, j] / den
                Hs[j, j] = den
                Hs[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                its += 1
                j_done = j + 1
                res = abs(g[j + 1])
                if res <= tol or its >= maxit:
                    break
            y = np.zeros(j_done)
            for i in range(j_done - 1, -1, -1):
                y[i] = (g[i] - np.dot(Hs[i, i + 1:j_done], y[i + 1:j_done])) / Hs[i, i]
            x = x + dinv * (V[:j_done].T @ y)
            if res <= tol:
                return x, its, res, True
            if its >= maxit:
                r = b - apply(x)
                return x, its, float(np.linalg.norm(r)), False
            r = b - apply(x)
            beta = float(np.linalg.norm(r))
            if beta <= tol:
                return x, its, beta, True

    # ------------------------------------------------------------------------ initial-state noise
    def temperature_noise(self, seed: int, sigma: float) -> np.ndarray:
        """sigma times a standard normal deviate per node, from SplitMix64 (Steele, Lea, Flood 2014)
        used as a counter-based generator keyed by the seed, the node's cell (level, i_x, i_y, i_z)
        and its index in the cell, then Box-Muller:
            mix(z) = z ^ (z >> 30), times 0xbf58476d1ce4e5b9, ^ (>> 27), times 0x94d049bb133111eb,
                     ^ (>> 31), in 64-bit wrap-around arithmetic;  G = 0x9e3779b97f4a7c15;
            k = mix(seed + G (level + 1)), then k = mix(k + G (i + 1)) for i_x, i_y, i_z and the
            node index;  u1, u2 = the top 53 bits of mix(k + G), mix(k + 2 G) times 2^-53;
            n = sqrt(-2 ln(1 - u1)) cos(2 pi u2)."""
        u64 = np.uint64
        G_ = u64(0x9e3779b97f4a7c15)

        def mix(z):
            z = (z ^ (z >> u64(30))) * u64(0xbf58476d1ce4e5b9)
            z = (z ^ (z >> u64(27))) * u64(0x94d049bb133111eb)
            return z ^ (z >> u64(31))

        with np.errstate(over="ignore"):
            cells = np.repeat(self.cells.astype(np.uint64), self.nloc, axis=0)
            node = np.tile(np.arange(self.nloc, dtype=np.uint64), self.ncell)
            k = mix(u64(seed) + G_ * (cells[:, 0] + u64(1)))
            for col in (cells[:, 1], cells[:, 2], cells[:, 3], node):
                k = mix(k + G_ * (col + u64(1)))
            u1 = (mix(k + G_) >> u64(11)).astype(np.float64) * 2.0 ** -53
            u2 = (mix(k + u64(2) * G_) >> u64(11)).astype(np.float64) * 2.0 ** -53
        return sigma * np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * math.pi * u2)

    # ------------------------------------------------------------------------------ time step
    def initial_state(self, ubar: float = 0.0, dT: np.ndarray | None = None) -> np.ndarray:
        """Hydrostatic background with uniform horizontal wind ubar; with a temperature
        perturbation dT the pressure is kept and the density recomputed from p = rho R T."""
        rho = self.rbar.copy()
        if dT is not None:
            T = self.pbar / (RGAS * self.rbar) + dT
            rho = self.pbar / (RGAS * T)
        U = np.zeros((self.nf, self.N))
        U[0] = rho
        U[1] = rho * ubar
        U[1 + self.d] = self.pbar / (GAMMA - 1.0) + 0.5 * rho * ubar * ubar
        return U

    def implicit_term(self, U: np.ndarray) -> np.ndarray:
        """F_I(U) = (0, -M^{-1} B p' - (rho - rhobar) g k, -M^{-1} (C(h m) + beta/(2(gamma-1)) P p'))."""
        d = self.d
        rho = U[0]
        p = self.pressure(U)
        pp = p - self.pbar
        h = self.enthalpy(p, rho)
        lam = self.cell_sound_speed(h)
        F = np.zeros_like(U)
        q = self.grad(pp)
        F[1:1 + d] = -q
        F[d] -= (rho - self.rbar) * self.g
        e = self.enthalpy_flux_div(h, U[1:1 + d])
        if self.beta != 0.0:
            e = e + self.beta / (2.0 * (GAMMA - 1.0)) * self.penalty(lam, pp)
        F[1 + d] = -e / self.wJ
        return F

    def step(self, U: np.ndarray, dt: float, fp_iters: int = 2, rtol: float = 1e-12,
             atol: float = 0.0, restart: int = 30, maxit: int = 2000, stats: dict | None = None):
        """One IMEX-RK2 step; returns the new state (the input is not modified)."""
        d = self.d
        A, At, b, bt = self.A, self.At, self.b, self.bt
        FE = [self.explicit_residual(U)]
        FI = [self.implicit_term(U)]
        its_log = []
        pp_prev = self.pressure(U) - self.pbar
        m_prev = U[1:1 + d].copy()
        for i in (1, 2):
            aii = At[i, i]
            dta = dt * aii
            rho_i = U[0] + dt * sum(A[i, j] * FE[j][0] for j in range(i))
            mt = U[1:1 + d] + dt * sum(A[i, j] * FE[j][1:1 + d] + At[i, j] * FI[j][1:1 + d]
                                       for j in range(i))
            et = U[1 + d] + dt * sum(A[i, j] * FE[j][1 + d] + At[i, j] * FI[j][1 + d]
                                     for j in range(i))
            mprime = mt.copy()
            mprime[d - 1] -= dta * (rho_i - self.rbar) * self.g
            pp = pp_prev.copy()
            m = m_prev.copy()
            for _ in range(fp_iters):
                h = self.enthalpy(self.pbar + pp, rho_i)
                rk = 0.5 * np.sum(m * m, axis=0) / rho_i
                lam = self.cell_sound_speed(h)
                rhs = self.wJ * (et - rk - self.pbar / (GAMMA - 1.0)) - dta * self.enthalpy_flux_div(h, mprime)
                op = lambda v, h=h, lam=lam: self.helmholtz(dta, h, lam, v)
                r0 = rhs - op(pp)
                dinv = 1.0 / self.jacobi_diag(dta, h)
                delta, its, res, ok = self.gmres(op, r0, dinv, rtol, atol, restart, maxit)
                if not ok:
                    raise RuntimeError("oracle GMRES did not converge (%d its, res %g)" % (its, res))
                its_log.append(its)
                pp = pp + delta
                m = mprime - dta * self.grad(pp)
            Ei = (self.pbar + pp) / (GAMMA - 1.0) + 0.5 * np.sum(m * m, axis=0) / rho_i
            Ui = np.concatenate([rho_i[None], m, Ei[None]], axis=0)
            Fi = np.zeros_like(U)
            Fi[1:1 + d] = (m - mt) / dta
            Fi[1 + d] = (Ei - et) / dta
            FI.append(Fi)
            FE.append(self.explicit_residual(Ui))
            pp_prev = pp
            m_prev = m
        Un = U + dt * sum(b[j] * FE[j] + bt[j] * FI[j] for j in range(3))
        if stats is not None:
            stats["gmres_iters"] = its_log
        return Un

    # ------------------------------------------------------------------------------ diagnostics
    def mass(self, U: np.ndarray) -> float:
        return float(np.sum(self.wJ * U[0]))

    def max_w(self, U: np.ndarray) -> float:
        return float(np.max(np.abs(U[self.d] / U[0])))


def courant(degree: int, speed: float, dt: float, cell_sizes, dim: int) -> float:
    """Courant number of Section 3: r c dt sqrt(d) / H with H the minimum cell diameter (the
    printed formula is garbled; this reading gives r c dt / dx on cubes)."""
    diam = math.sqrt(sum(float(s) ** 2 for s in cell_sizes))
    return degree * speed * dt * math.sqrt(dim) / diam


def dofs_per_scalar(ncells: int, degree: int, dim: int) -> int:
    """Unknowns per scalar field: cells x (r+1)^d (Section 3.2)."""
    return int(ncells) * (degree + 1) ** dim
