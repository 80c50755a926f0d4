"""Exact solution of the 1D Riemann problem for the Euler equations.

TEST INFRASTRUCTURE (pins the oracle's Sod-tube runs). Follows Toro,
"Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4: Newton
iteration on the pressure function f(p) = f_L(p) + f_R(p) + (u_R - u_L) for
the star pressure, then sampling of the self-similar solution at x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _f_side(p, rho_k, p_k, c_k, gam):
    """Toro's f_K(p) and its derivative (shock branch for p > p_k, else rarefaction)."""
    if p > p_k:
        A = 2.0 / ((gam + 1.0) * rho_k)
        B = (gam - 1.0) / (gam + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        return (p - p_k) * s, s * (1.0 - 0.5 * (p - p_k) / (B + p))
    e = (gam - 1.0) / (2.0 * gam)
    f = 2.0 * c_k / (gam - 1.0) * ((p / p_k) ** e - 1.0)
    df = 1.0 / (rho_k * c_k) * (p / p_k) ** (-(gam + 1.0) / (2.0 * gam))
    return f, df


def star_state(left, right, gam=1.4, tol=1e-14, maxit=100):
    """Star-region pressure and velocity for left/right (rho, u, p)."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL = math.sqrt(gam * pL / rL)
    cR = math.sqrt(gam * pR / rR)
    # two-rarefaction initial guess
    e = (gam - 1.0) / (2.0 * gam)
    p = ((cL + cR - 0.5 * (gam - 1.0) * (uR - uL)) / (cL / pL ** e + cR / pR ** e)) ** (1.0 / e)
    p = max(p, 1e-12)
    for _ in range(maxit):
        fL, dL = _f_side(p, rL, pL, cL, gam)
        fR, dR = _f_side(p, rR, pR, cR, gam)
        pn = p - (fL + fR + uR - uL) / (dL + dR)
        pn = max(pn, 1e-14)
        if abs(pn - p) / (0.5 * (pn + p)) < tol:
            p = pn
            break
        p = pn
    fL, _ = _f_side(p, rL, pL, cL, gam)
    fR, _ = _f_side(p, rR, pR, cR, gam)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def star_densities(left, right, gam=1.4):
    rL, uL, pL = left
    rR, uR, pR = right
    p, u = star_state(left, right, gam)
    g1 = (gam - 1.0) / (gam + 1.0)

    def side(rk, pk):
        if p > pk:  # shock
            return rk * (p / pk + g1) / (g1 * p / pk + 1.0)
        return rk * (p / pk) ** (1.0 / gam)  # rarefaction

    return side(rL, pL), side(rR, pR)


def sample(left, right, s, gam=1.4):
    """(rho, u, p) at similarity coordinate s = (x - x0)/t, vectorised over s."""
    s = np.asarray(s, dtype=np.float64)
    rL, uL, pL = left
    rR, uR, pR = right
    cL = math.sqrt(gam * pL / rL)
    cR = math.sqrt(gam * pR / rR)
    p_s, u_s = star_state(left, right, gam)
    rsL, rsR = star_densities(left, right, gam)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    g1 = (gam - 1.0) / (gam + 1.0)
    for idx, x in np.ndenumerate(s):
        if x <= u_s:  # left of contact
            if p_s > pL:  # left shock
                S = uL - cL * math.sqrt((gam + 1.0) / (2.0 * gam) * p_s / pL + (gam - 1.0) / (2.0 * gam))
                st = (rL, uL, pL) if x <= S else (rsL, u_s, p_s)
            else:  # left rarefaction
                cs = cL * (p_s / pL) ** ((gam - 1.0) / (2.0 * gam))
                head, tail = uL - cL, u_s - cs
                if x <= head:
                    st = (rL, uL, pL)
                elif x >= tail:
                    st = (rsL, u_s, p_s)
                else:
                    fac = 2.0 / (gam + 1.0) + g1 / cL * (uL - x)
                    st = (rL * fac ** (2.0 / (gam - 1.0)),
                          2.0 / (gam + 1.0) * (cL + 0.5 * (gam - 1.0) * uL + x),
                          pL * fac ** (2.0 * gam / (gam - 1.0)))
        else:  # right of contact
            if p_s > pR:  # right shock
                S = uR + cR * math.sqrt((gam + 1.0) / (2.0 * gam) * p_s / pR + (gam - 1.0) / (2.0 * gam))
                st = (rR, uR, pR) if x >= S else (rsR, u_s, p_s)
            else:  # right rarefaction
                cs = cR * (p_s / pR) ** ((gam - 1.0) / (2.0 * gam))
                head, tail = uR + cR, u_s + cs
                if x >= head:
                    st = (rR, uR, pR)
                elif x <= tail:
                    st = (rsR, u_s, p_s)
                else:
                    fac = 2.0 / (gam + 1.0) - g1 / cR * (uR - x)
                    st = (rR * fac ** (2.0 / (gam - 1.0)),
                          2.0 / (gam + 1.0) * (-cR + 0.5 * (gam - 1.0) * uR + x),
                          pR * fac ** (2.0 * gam / (gam - 1.0)))
        rho[idx], u[idx], p[idx] = st
    return rho, u, p


def shock_speed(left, right, gam=1.4):
    """Speed of the right-moving shock (when the right wave is a shock)."""
    rR, uR, pR = right
    cR = math.sqrt(gam * pR / rR)
    p_s, _ = star_state(left, right, gam)
    return uR + cR * math.sqrt((gam + 1.0) / (2.0 * gam) * p_s / pR + (gam - 1.0) / (2.0 * gam))
