"""Closed-form fields for the oracle's accuracy pins, written from the equations alone.

Nothing here calls the oracle: these are the terrain profiles of Section 3.1 (Eq. (3) and its
variants), a smooth state that is tangent to the terrain-following coordinate surfaces (so slip
walls see no normal momentum), the exact explicit tendency of Eq. (1) for that state, and the
isentropic vortex, an exact translating solution of the Euler equations without gravity.
Derivatives are taken by the complex step, f'(x) = Im f(x + i e) / e, which is exact to rounding
for analytic functions.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4
CSTEP = 1e-30

FLAT, AGNESI, BELL, GAUSS_HILL, GAUSS_RIDGE = range(5)


def terrain(kind, oro, dim, x, y):
    """Height h(x, y) of the orographies (complex-safe)."""
    h0, a, xc, yc = (float(v) for v in oro)
    dx = x - xc
    dy = (y - yc) if dim == 3 else 0.0 * dx
    if kind == FLAT:
        return 0.0 * dx
    if kind == AGNESI:                       # h a^2 / ((x - xc)^2 + a^2)
        return h0 * a * a / (dx * dx + a * a)
    if kind == BELL:                         # Eq. (3): h_c / [1 + (dx/a)^2 + (dy/a)^2]^(3/2)
        return h0 / (1.0 + (dx / a) ** 2 + (dy / a) ** 2) ** 1.5
    if kind == GAUSS_HILL:                   # h exp(-(dx^2 + dy^2) / (2 sigma^2))
        return h0 * np.exp(-(dx * dx + dy * dy) / (2.0 * a * a))
    if kind == GAUSS_RIDGE:                  # h exp(-((x - xc)/a)^2), independent of y
        return h0 * np.exp(-(dx / a) ** 2)
    raise ValueError(kind)


def terrain_slopes(kind, oro, dim, x, y):
    """(h_x, h_y) by the complex step."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    hx = np.imag(terrain(kind, oro, dim, x + 1j * CSTEP, y + 0j)) / CSTEP
    hy = np.imag(terrain(kind, oro, dim, x + 0j, y + 1j * CSTEP)) / CSTEP
    return hx, hy


class TangentState:
    """A smooth state on the domain (0, Lx) x (0, Ly) x (terrain, H) with lateral slip walls:
    u vanishes at x = 0, Lx and v at y = 0, Ly, and w = (u h_x + v h_y)(1 - zeta/H), so the
    velocity is tangent to every coordinate surface zeta = const of the terrain-following map
    (in particular to the ground and to the lid).  Density and pressure are generic."""

    def __init__(self, dim, length, oro_kind, oro):
        self.d = dim
        self.Lx, self.Ly, self.H = (float(v) for v in length)
        self.kind = oro_kind
        self.oro = oro

    def fields(self, x, y, z):
        """(rho, u, v, w, p) at physical points (complex-safe)."""
        Lx, Ly, H = self.Lx, self.Ly, self.H
        h = terrain(self.kind, self.oro, self.d, x, y)
        zeta = H * (z - h) / (H - h)
        # slopes of the coordinate surfaces: dz/dx and dz/dy at constant zeta
        # the complex step cannot nest, so the slope inside the state is a fourth-order difference:
        # an analytic function of (x, y) that is tangent to the coordinate surfaces up to 1e-12
        hx = self._slope(x, y, 0, 1e-4 * Lx)
        hy = self._slope(x, y, 1, 1e-4 * Ly) if self.d == 3 else 0.0 * x
        sx, sz = np.pi * x / Lx, np.pi * zeta / H
        rho = 1.1 * (1.0 + 0.1 * np.cos(sx) * np.cos(sz) + 0.05 * np.sin(2 * sz))
        u = 12.0 * np.sin(sx) * (1.0 + 0.25 * np.cos(sz + 0.3))
        if self.d == 3:
            sy = np.pi * y / Ly
            rho = rho * (1.0 + 0.05 * np.cos(sy) * np.sin(sx + sz))
            u = u * (1.0 + 0.1 * np.cos(sy))
            v = 8.0 * np.sin(sy) * (1.0 + 0.2 * np.sin(sz) * np.cos(sx))
        else:
            v = 0.0 * x
        w = (u * hx + v * hy) * (1.0 - zeta / H)
        p = 9.0e4 * (1.0 + 0.03 * np.sin(sx + 0.5) * np.cos(0.5 * sz) - 0.1 * zeta / H)
        return rho, u, v, w, p

    def _slope(self, x, y, axis, e):
        f = lambda a, b: terrain(self.kind, self.oro, self.d, a, b)
        if axis == 0:
            return (-f(x + 2 * e, y) + 8 * f(x + e, y) - 8 * f(x - e, y) + f(x - 2 * e, y)) / (12 * e)
        return (-f(x, y + 2 * e) + 8 * f(x, y + e) - 8 * f(x, y - e) + f(x, y - 2 * e)) / (12 * e)

    def conserved(self, x, y, z):
        """Conserved variables in the oracle's field order."""
        rho, u, v, w, p = self.fields(x, y, z)
        vel = [u, v, w] if self.d == 3 else [u, w]
        k = 0.5 * sum(c * c for c in vel)
        return [rho] + [rho * c for c in vel] + [p / (GAMMA - 1.0) + rho * k]

    def explicit_tendency(self, x, y, z, g):
        """-div(rho u), -div(rho u (x) u), -div(rho k u) - g rho w in physical coordinates."""
        d = self.d

        def fluxes(X, Y, Z):
            rho, u, v, w, p = self.fields(X, Y, Z)
            vel = [u, v, w] if d == 3 else [u, w]
            k = 0.5 * sum(c * c for c in vel)
            # F[field][direction]
            F = [[rho * vel[j] for j in range(d)]]
            for i in range(d):
                F.append([rho * vel[i] * vel[j] for j in range(d)])
            F.append([rho * k * vel[j] for j in range(d)])
            return F

        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        z = np.asarray(z, dtype=np.float64)
        shifts = []
        for j in range(d):
            X, Y, Z = x + 0j, y + 0j, z + 0j
            if j == 0:
                X = X + 1j * CSTEP
            elif j == 1 and d == 3:
                Y = Y + 1j * CSTEP
            else:
                Z = Z + 1j * CSTEP
            shifts.append(fluxes(X, Y, Z))
        R = []
        for f in range(d + 2):
            R.append(-sum(np.imag(shifts[j][f][j]) / CSTEP for j in range(d)))
        rho, u, v, w, p = self.fields(x, y, z)
        R[d + 1] = R[d + 1] - g * rho * w
        return R


def isentropic_vortex(x, z, t, xc, zc, radius, strength, uinf, rho_inf, p_inf):
    """Conserved variables (rho, rho u, rho w, rho E) of the isentropic vortex translating with
    (uinf, 0) in the x-z plane, an exact solution of the Euler equations without gravity.
    With c0 = sqrt(p_inf / rho_inf) and the distance r in units of radius:
        delta (u, w) = strength c0 / (2 pi) exp((1 - r^2) / 2) (-(z - zc), x - xc) / radius,
        T / T_inf = 1 - (gamma - 1) strength^2 / (8 gamma pi^2) exp(1 - r^2),
        rho = rho_inf (T / T_inf)^(1/(gamma - 1)),  p = p_inf (rho / rho_inf)^gamma."""
    c0 = np.sqrt(p_inf / rho_inf)
    X = (x - xc - uinf * t) / radius
    Z = (z - zc) / radius
    r2 = X * X + Z * Z
    f = np.exp(0.5 * (1.0 - r2))
    du = -strength * c0 / (2 * np.pi) * f * Z
    dw = strength * c0 / (2 * np.pi) * f * X
    th = 1.0 - (GAMMA - 1.0) * strength ** 2 / (8.0 * GAMMA * np.pi ** 2) * f * f
    rho = rho_inf * th ** (1.0 / (GAMMA - 1.0))
    p = p_inf * (rho / rho_inf) ** GAMMA
    u = uinf + du
    w = dw
    return np.stack([rho, rho * u, rho * w, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + w * w)])
