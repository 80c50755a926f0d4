"""Manufactured solution of the 2D Euler equations and its source term.

TEST INFRASTRUCTURE (see the package docstring). The residual of Eq.
(residual) carries a cell-averaged source S_h, and the cell-wise
semi-discrete form of Eq. (governing_cv) holds the exact solution steady when
S is the divergence of the inviscid flux of Eq. (QF) evaluated on it. Here the
"exact solution" is a chosen smooth periodic field (the method of manufactured
solutions: Roache 2002; Roy 2005 for the Euler form used as a template), and
its source is that divergence, differentiated by hand with the product rule.
Fed the cell averages of both, the discrete residual is the scheme's
truncation error, which falls as h^2 for a second-order scheme.

With a viscosity the same fields serve the Navier-Stokes form of Eq.
(governing): the source becomes the divergence of the inviscid flux minus the
divergence of the viscous flux F_nu of Eq. (QF) (Stokes stresses, heat flux
k dT/dx_d with T = p / rho and k = mu gamma / ((gamma - 1) Pr)), also
differentiated by hand (``viscous_divergence``, ``ns_source``).

Fields on the periodic unit square (x, y in [0, 1]):
  rho = 1   + 0.15 sin(2 pi x) + 0.10 cos(2 pi y)
  u   = 0.7 + 0.05 sin(2 pi x) + 0.05 cos(4 pi y)
  v   = 0.9 + 0.05 cos(4 pi x) + 0.08 sin(2 pi y)
  p   = 1   + 0.20 cos(2 pi x) + 0.05 sin(2 pi y)
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi

# (mean, (amp, kx, 'sin'|'cos') in x, (amp, ky, 'sin'|'cos') in y) per primitive
FIELDS = {
    "rho": (1.0, (0.15, 1, "sin"), (0.10, 1, "cos")),
    "u": (0.7, (0.05, 1, "sin"), (0.05, 2, "cos")),
    "v": (0.9, (0.05, 2, "cos"), (0.08, 1, "sin")),
    "p": (1.0, (0.20, 1, "cos"), (0.05, 1, "sin")),
}


def _term(t, s):
    """Value and derivative of amp * sin|cos(2 pi k s)."""
    amp, k, kind = t
    w = TWO_PI * k
    if kind == "sin":
        return amp * np.sin(w * s), amp * w * np.cos(w * s)
    return amp * np.cos(w * s), -amp * w * np.sin(w * s)


def primitive(name, x, y):
    """(value, d/dx, d/dy) of a primitive field at points (x, y)."""
    mean, tx, ty = FIELDS[name]
    fx, dfx = _term(tx, x)
    fy, dfy = _term(ty, y)
    return mean + fx + fy, dfx + 0.0 * y, dfy + 0.0 * x


def conserved(x, y, gamma=1.4):
    """(rho, rho u, rho v, E) at points (x, y)."""
    r, _, _ = primitive("rho", x, y)
    u, _, _ = primitive("u", x, y)
    v, _, _ = primitive("v", x, y)
    p, _, _ = primitive("p", x, y)
    E = p / (gamma - 1.0) + 0.5 * r * (u * u + v * v)
    return np.stack([r, r * u, r * v, E])


def source(x, y, gamma=1.4):
    """S = d F/dx + d G/dy of the inviscid fluxes on the manufactured fields."""
    r, rx, ry = primitive("rho", x, y)
    u, ux, uy = primitive("u", x, y)
    v, vx, vy = primitive("v", x, y)
    p, px, py = primitive("p", x, y)
    q2 = u * u + v * v
    E = p / (gamma - 1.0) + 0.5 * r * q2
    Ex = px / (gamma - 1.0) + 0.5 * rx * q2 + r * (u * ux + v * vx)
    Ey = py / (gamma - 1.0) + 0.5 * ry * q2 + r * (u * uy + v * vy)
    # F = (rho u, rho u^2 + p, rho u v, u (E + p)),  G = (rho v, rho u v, rho v^2 + p, v (E + p))
    s0 = (rx * u + r * ux) + (ry * v + r * vy)
    s1 = (rx * u * u + 2.0 * r * u * ux + px) + (ry * u * v + r * uy * v + r * u * vy)
    s2 = (rx * u * v + r * ux * v + r * u * vx) + (ry * v * v + 2.0 * r * v * vy + py)
    s3 = (ux * (E + p) + u * (Ex + px)) + (vy * (E + p) + v * (Ey + py))
    return np.stack([s0, s1, s2, s3])


def cell_averages(fn, n, order=4):
    """Cell averages of fn(x, y) -> (4, ...) over an n x n grid of the unit
    square by order x order Gauss-Legendre quadrature; shape (4, n, n) [v][j][i]."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    h = 1.0 / n
    centres = (np.arange(n) + 0.5) * h
    out = np.zeros((4, n, n))
    for a, wa in zip(xg, wg):
        for b, wb in zip(xg, wg):
            X = centres[None, :] + 0.5 * h * a
            Y = centres[:, None] + 0.5 * h * b
            out += 0.25 * wa * wb * fn(np.broadcast_to(X, (n, n)), np.broadcast_to(Y, (n, n)))
    return out


# ---------------------------------------------------------------------------
# 3D: the same construction on the periodic unit cube, with w and z terms.
#   rho = 1   + 0.15 sin(2 pi x) + 0.10 cos(2 pi y) + 0.08 sin(2 pi z)
#   u   = 0.6 + 0.05 sin(2 pi x) + 0.05 cos(4 pi y) + 0.04 cos(2 pi z)
#   v   = 0.5 + 0.05 cos(4 pi x) + 0.08 sin(2 pi y) + 0.03 sin(2 pi z)
#   w   = 0.4 + 0.04 sin(2 pi x) + 0.03 cos(2 pi y) + 0.06 cos(2 pi z)
#   p   = 1   + 0.20 cos(2 pi x) + 0.05 sin(2 pi y) + 0.07 cos(4 pi z)

FIELDS3 = {
    "rho": (1.0, (0.15, 1, "sin"), (0.10, 1, "cos"), (0.08, 1, "sin")),
    "u": (0.6, (0.05, 1, "sin"), (0.05, 2, "cos"), (0.04, 1, "cos")),
    "v": (0.5, (0.05, 2, "cos"), (0.08, 1, "sin"), (0.03, 1, "sin")),
    "w": (0.4, (0.04, 1, "sin"), (0.03, 1, "cos"), (0.06, 1, "cos")),
    "p": (1.0, (0.20, 1, "cos"), (0.05, 1, "sin"), (0.07, 2, "cos")),
}


def primitive3(name, x, y, z):
    """(value, d/dx, d/dy, d/dz) of a 3D primitive field."""
    mean, tx, ty, tz = FIELDS3[name]
    fx, dfx = _term(tx, x)
    fy, dfy = _term(ty, y)
    fz, dfz = _term(tz, z)
    zero = 0.0 * (x + y + z)
    return mean + fx + fy + fz, dfx + zero, dfy + zero, dfz + zero


def conserved3(x, y, z, gamma=1.4):
    r = primitive3("rho", x, y, z)[0]
    vel = [primitive3(c, x, y, z)[0] for c in ("u", "v", "w")]
    p = primitive3("p", x, y, z)[0]
    E = p / (gamma - 1.0) + 0.5 * r * sum(c * c for c in vel)
    return np.stack([r] + [r * c for c in vel] + [E])


def source3(x, y, z, gamma=1.4):
    """S = sum_d d F_d / d x_d of the 3D inviscid fluxes, by the product rule."""
    r, *dr = primitive3("rho", x, y, z)
    vel = [primitive3(c, x, y, z) for c in ("u", "v", "w")]
    V = [q[0] for q in vel]
    dV = [q[1:] for q in vel]          # dV[i][d] = d V_i / d x_d
    p, *dp = primitive3("p", x, y, z)
    q2 = sum(c * c for c in V)
    E = p / (gamma - 1.0) + 0.5 * r * q2
    dE = [dp[d] / (gamma - 1.0) + 0.5 * dr[d] * q2 + r * sum(V[i] * dV[i][d] for i in range(3)) for d in range(3)]
    S = [0.0 * x for _ in range(5)]
    for d in range(3):
        # F_d = (rho V_d, rho V_1 V_d + p delta_1d, ..., V_d (E + p))
        S[0] = S[0] + dr[d] * V[d] + r * dV[d][d]
        for i in range(3):
            S[1 + i] = S[1 + i] + dr[d] * V[i] * V[d] + r * dV[i][d] * V[d] + r * V[i] * dV[d][d] + (dp[d] if i == d else 0.0)
        S[4] = S[4] + dV[d][d] * (E + p) + V[d] * (dE[d] + dp[d])
    return np.stack(S)


def cell_averages3(fn, n, order=3):
    """Cell averages of fn(x, y, z) -> (5, ...) over an n^3 grid of the unit cube; shape (5, n, n, n) [v][k][j][i]."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    out = np.zeros((5, n, n, n))
    for a, wa in zip(xg, wg):
        for b, wb in zip(xg, wg):
            for e, we in zip(xg, wg):
                Z, Y, X = np.meshgrid(c + 0.5 * h * e, c + 0.5 * h * b, c + 0.5 * h * a, indexing="ij")
                out += 0.125 * wa * wb * we * fn(X, Y, Z)
    return out


# ---------------------------------------------------------------------------
# Navier-Stokes: the divergence of the viscous flux on the manufactured fields
# (2D or 3D), for constant mu. Every field is a sum of one-variable terms, so
# mixed second derivatives of the velocity vanish and, with
# tau_bd = mu (du_b/dx_d + du_d/dx_b) - 2/3 mu delta_bd div(u),
#   sum_d d tau_bd / dx_d = mu (lap u_b + 1/3 d/dx_b div u) = mu (lap u_b + 1/3 d2u_b/dx_b2),
#   sum_d d Theta_d / dx_d = sum_bd du_b/dx_d tau_bd + sum_b u_b sum_d d tau_bd/dx_d + k lap T,
# with Theta_d = sum_b u_b tau_bd + k dT/dx_d. T = p / rho is not a sum of
# one-variable terms; only its pure second derivatives enter:
#   T_d = (p_d - T rho_d) / rho,  T_dd = (p_dd - 2 T_d rho_d - T rho_dd) / rho.

def _term2(t, s):
    """Value, first and second derivative of amp * sin|cos(2 pi k s)."""
    amp, k, kind = t
    w = TWO_PI * k
    if kind == "sin":
        f = amp * np.sin(w * s)
        return f, amp * w * np.cos(w * s), -w * w * f
    f = amp * np.cos(w * s)
    return f, -amp * w * np.sin(w * s), -w * w * f


def _field_derivs(table, name, coords):
    """(value, [d/dx_d], [d2/dx_d2]) of a primitive field of `table` at the points."""
    mean, *terms = table[name]
    zero = 0.0 * sum(coords)
    val, d1, d2 = mean + zero, [], []
    for t, c in zip(terms, coords):
        f, df, ddf = _term2(t, c)
        val = val + f
        d1.append(df + zero)
        d2.append(ddf + zero)
    return val, d1, d2


def viscous_divergence(coords, mu, prandtl, gamma=1.4):
    """sum_d d F_nu,d / d x_d on the manufactured fields: (0, momentum..., energy).
    coords = (x, y) uses the 2D fields, (x, y, z) the 3D ones."""
    nd = len(coords)
    table = FIELDS if nd == 2 else FIELDS3
    names = ("u", "v") if nd == 2 else ("u", "v", "w")
    vel = [_field_derivs(table, c, coords) for c in names]
    r, rd, rdd = _field_derivs(table, "rho", coords)
    p, pd, pdd = _field_derivs(table, "p", coords)
    T = p / r
    Td = [(pd[d] - T * rd[d]) / r for d in range(nd)]
    Tdd = [(pdd[d] - 2.0 * Td[d] * rd[d] - T * rdd[d]) / r for d in range(nd)]
    kc = mu * gamma / ((gamma - 1.0) * prandtl)
    div = sum(vel[d][1][d] for d in range(nd))
    tau = [[mu * (vel[b][1][d] + vel[d][1][b]) - (2.0 / 3.0 * mu * div if b == d else 0.0)
            for d in range(nd)] for b in range(nd)]
    mom = [mu * (sum(vel[b][2][d] for d in range(nd)) + vel[b][2][b] / 3.0) for b in range(nd)]
    en = kc * sum(Tdd)
    for b in range(nd):
        en = en + vel[b][0] * mom[b]
        for d in range(nd):
            en = en + vel[b][1][d] * tau[b][d]
    zero = 0.0 * r
    return np.stack([zero] + [m + zero for m in mom] + [en])


def ns_source(x, y, mu, prandtl=0.72, gamma=1.4):
    """Source of the 2D manufactured solution for the Navier-Stokes equations."""
    return source(x, y, gamma) - viscous_divergence((x, y), mu, prandtl, gamma)


def ns_source3(x, y, z, mu, prandtl=0.72, gamma=1.4):
    """Source of the 3D manufactured solution for the Navier-Stokes equations."""
    return source3(x, y, z, gamma) - viscous_divergence((x, y, z), mu, prandtl, gamma)
