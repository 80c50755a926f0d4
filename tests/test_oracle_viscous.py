"""Pins of the oracle's viscous flux (F_nu,n of Eq. (QF), in the residual of
Eq. (residual)): closed-form face fluxes of linear fields, the hand-derived
Navier-Stokes manufactured source against finite differences of a textbook
viscous flux, second-order truncation error of the Navier-Stokes residual in
2D and 3D (and its failure when the viscous source is left out), discrete
conservation, axis symmetry, the Euler residual recovered bit for bit at
zero viscosity, and the explicit diffusion limit of the time step."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from oracle import mms

GAMMA = 1.4
PR = 0.72


def box(n, ndim=2, mu=0.05, bc=None, hi=1.0):
    nn = tuple(n) if isinstance(n, (tuple, list)) else (n,) * ndim
    nn = nn + (1,) * (3 - len(nn))
    return SimpleNamespace(ndim=ndim, n=nn, lo=(0.0, 0.0, 0.0), hi=(hi, hi, hi),
                           bc=bc or ((0, 0), (0, 0), (0, 0)), gamma=GAMMA, cfl=0.5, mu=mu, prandtl=PR)


def conserved(g, rho, vel, p):
    U = np.zeros((g.ndim + 2,) + rho.shape)
    U[0] = rho
    ke = np.zeros_like(rho)
    for d in range(g.ndim):
        U[1 + d] = rho * vel[d]
        ke += vel[d] ** 2
    U[-1] = p / (GAMMA - 1.0) + 0.5 * rho * ke
    return U


def centres(g):
    dx = [(g.hi[d] - g.lo[d]) / g.n[d] for d in range(3)]
    c = [(np.arange(g.n[d]) + 0.5) * dx[d] for d in range(3)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    return X, Y, Z


def test_linear_shear_face_flux():
    # u = a y, v = 0, rho = p = 1: tau_xy = mu a on every face, the y face
    # carries (0, mu a, 0, u_f mu a) with u_f the face's velocity, the x face
    # (0, 0, mu a, v mu a = 0)
    g = box((6, 8), mu=0.07, bc=((0, 0), (1, 1), (0, 0)))
    X, Y, _ = centres(g)
    a = 0.3
    U = conserved(g, np.ones_like(X), (a * Y, 0 * Y), np.ones_like(X))
    i, j = 2, 3
    Fy = oracle.visc_face_flux(g, U, 1, i, j)
    yf = (j + 1) / 8.0
    assert np.allclose(Fy, [0.0, 0.07 * a, 0.0, a * yf * 0.07 * a], rtol=1e-13, atol=1e-16)
    Fx = oracle.visc_face_flux(g, U, 0, i, j)
    assert np.allclose(Fx, [0.0, 0.0, 0.07 * a, 0.0], rtol=1e-13, atol=1e-16)


def test_dilatation_and_stokes_hypothesis():
    # u = a x, v = b y: tau_xx = mu (2a - 2/3 (a + b)), tau_yy = mu (2b - 2/3 (a + b)),
    # tau_xy = 0 (Stokes' hypothesis: the bulk viscosity is -2/3 mu)
    g = box((8, 8), mu=0.1, bc=((1, 1), (1, 1), (0, 0)))
    X, Y, _ = centres(g)
    for a, b in ((0.2, -0.1), (0.15, 0.15)):
        U = conserved(g, np.ones_like(X), (a * X, b * Y), np.ones_like(X))
        Fx = oracle.visc_face_flux(g, U, 0, 3, 4)
        Fy = oracle.visc_face_flux(g, U, 1, 3, 4)
        txx = 0.1 * (2 * a - 2.0 / 3.0 * (a + b))
        tyy = 0.1 * (2 * b - 2.0 / 3.0 * (a + b))
        xf, yf = 4 / 8.0, 5 / 8.0   # the x face between columns 3, 4 and the y face between rows 4, 5
        assert np.allclose(Fx[:3], [0.0, txx, 0.0], rtol=1e-12, atol=1e-15)
        assert np.allclose(Fy[:3], [0.0, 0.0, tyy], rtol=1e-12, atol=1e-15)
        # Theta = u . tau (T uniform) with the velocity at the face
        assert abs(Fx[3] - a * xf * txx) <= 1e-13
        assert abs(Fy[3] - b * yf * tyy) <= 1e-13
        # the 2D trace: tau_xx + tau_yy = 2 mu div u - 4/3 mu div u = 2/3 mu div u
        assert abs(Fx[1] + Fy[2] - 0.1 * (2.0 / 3.0) * (a + b)) <= 1e-15


def test_heat_conduction_face_flux():
    # fluid at rest with T = p / rho linear in x: the energy flux is k dT/dx,
    # k = mu gamma / ((gamma - 1) Pr); nothing else
    g = box((10, 4), mu=0.02, bc=((1, 1), (0, 0), (0, 0)))
    X, Y, _ = centres(g)
    s = 0.5
    p = 1.0 + s * X        # rho = 1, so T = p
    U = conserved(g, np.ones_like(X), (0 * X, 0 * X), p)
    F = oracle.visc_face_flux(g, U, 0, 4, 1)
    k = 0.02 * GAMMA / ((GAMMA - 1.0) * PR)
    assert np.allclose(F, [0.0, 0.0, 0.0, k * s], rtol=1e-12, atol=1e-16)
    assert np.allclose(oracle.visc_face_flux(g, U, 1, 4, 1), 0.0, atol=1e-16)


def textbook_viscous_flux(coords, mu, ax):
    """F_nu along axis ax at points, from the analytic gradients of the manufactured fields."""
    nd = len(coords)
    table = mms.FIELDS if nd == 2 else mms.FIELDS3
    names = ("u", "v") if nd == 2 else ("u", "v", "w")
    V, dV = [], []
    for c in names:
        val, d1, _ = mms._field_derivs(table, c, coords)
        V.append(val)
        dV.append(d1)
    r, rd, _ = mms._field_derivs(table, "rho", coords)
    p, pd, _ = mms._field_derivs(table, "p", coords)
    T = p / r
    Tn = (pd[ax] - T * rd[ax]) / r
    div = sum(dV[d][d] for d in range(nd))
    tau = [mu * (dV[b][ax] + dV[ax][b]) - (2.0 / 3.0 * mu * div if b == ax else 0.0) for b in range(nd)]
    k = mu * GAMMA / ((GAMMA - 1.0) * PR)
    th = k * Tn + sum(V[b] * tau[b] for b in range(nd))
    return np.stack([0.0 * r] + tau + [th])


@pytest.mark.parametrize("nd", [2, 3])
def test_viscous_divergence_matches_finite_differences(nd):
    rng = np.random.default_rng(4)
    pts = [rng.random(300) for _ in range(nd)]
    h = 1e-5
    fd = 0.0
    for d in range(nd):
        up = [c + (h if e == d else 0.0) for e, c in enumerate(pts)]
        dn = [c - (h if e == d else 0.0) for e, c in enumerate(pts)]
        fd = fd + (textbook_viscous_flux(up, 0.3, d) - textbook_viscous_flux(dn, 0.3, d)) / (2 * h)
    S = mms.viscous_divergence(pts, 0.3, PR)
    for v in range(1, nd + 2):
        assert np.abs(S[v] - fd[v]).max() <= 1e-7 * np.abs(S[v]).max(), v
        assert np.abs(S[v]).max() > 0.05, v   # not a trivial field


def ns_truncation(n, mu, with_viscous_source=True, limiter=False):
    g = box(n, 2, mu=mu)
    U = mms.cell_averages(mms.conserved, n)
    src = (lambda X, Y: mms.ns_source(X, Y, mu, PR)) if with_viscous_source else mms.source
    S = mms.cell_averages(src, n)
    te = oracle.residual(g, U, limiter=limiter, source=S) * n ** 2
    return np.sqrt((te ** 2).mean(axis=(1, 2)))


def test_navier_stokes_truncation_error_second_order():
    mu = 0.05
    errs = [ns_truncation(n, mu) for n in (32, 64, 128)]
    for v in range(4):
        orders = [math.log2(errs[i][v] / errs[i + 1][v]) for i in range(2)]
        assert 1.85 <= orders[-1] <= 2.25, (v, orders)
    # the viscous terms are not negligible: leaving their source out leaves an
    # O(1) residual in the momenta and energy that does not fall with h
    bad = [ns_truncation(n, mu, with_viscous_source=False) for n in (32, 64)]
    for v in (1, 2, 3):
        assert bad[1][v] > 0.9 * bad[0][v] and bad[1][v] > 20 * errs[1][v], v


def test_navier_stokes_truncation_error_second_order_3d():
    mu = 0.05
    errs = []
    for n in (16, 32):
        g = box(n, 3, mu=mu)
        U = mms.cell_averages3(mms.conserved3, n)
        S = mms.cell_averages3(lambda X, Y, Z: mms.ns_source3(X, Y, Z, mu, PR), n)
        te = oracle.residual(g, U, limiter=False, source=S) * n ** 3
        errs.append(np.sqrt((te ** 2).mean(axis=(1, 2, 3))))
    for v in range(5):
        order = math.log2(errs[0][v] / errs[1][v])
        assert 1.8 <= order <= 2.3, (v, order)


def smooth_state(g, seed):
    rng = np.random.default_rng(seed)
    X, Y, Z = centres(g)
    ph = rng.random(8) * 2 * math.pi
    w = 2 * math.pi
    rho = 1.0 + 0.2 * np.sin(w * X + ph[0]) * np.cos(w * Y + ph[1]) + 0.1 * np.sin(w * Z + ph[6])
    vel = [0.3 * np.sin(w * Y + ph[2]) + 0.1 * np.cos(w * Z + ph[7]), -0.2 * np.cos(w * X + ph[3]),
           0.25 * np.sin(w * (X + Y) + ph[5])][:g.ndim]
    p = 1.0 + 0.15 * np.cos(w * (X - Y) + ph[4])
    return conserved(g, rho, vel, p)


@pytest.mark.parametrize("ndim", [2, 3])
def test_periodic_conservation(ndim):
    g = box((12, 10, 8)[:ndim], ndim, mu=0.08)
    U = smooth_state(g, 1)
    R = oracle.residual(g, U, limiter=True)
    for v in range(ndim + 2):
        assert abs(R[v].sum()) <= 1e-14 * np.abs(R[v]).sum() + 1e-16, v


def test_axis_symmetry_2d():
    # transposing the grid (x <-> y, u <-> v) transposes the residual
    g = box((9, 9), mu=0.06)
    U = smooth_state(g, 2)
    UT = U[[0, 2, 1, 3]].transpose(0, 1, 3, 2)
    R = oracle.residual(g, U)
    RT = oracle.residual(g, UT)
    assert np.allclose(RT, R[[0, 2, 1, 3]].transpose(0, 1, 3, 2), rtol=0, atol=1e-13 * np.abs(R).max())


def test_axis_symmetry_3d():
    # cycling the axes x -> y -> z -> x (and the momenta with them) cycles the residual
    g = box((7, 7, 7), 3, mu=0.06)
    U = smooth_state(g, 3)
    # new coordinates (x', y', z') = (y, z, x): with array axes (z, y, x) the new
    # array at [x, z, y] is the old one at [z, y, x], and the new momenta
    # (x', y', z') are the old (y, z, x) ones
    perm = [0, 2, 3, 1, 4]
    UC = U[perm].transpose(0, 3, 1, 2)
    R = oracle.residual(g, U)
    RC = oracle.residual(g, UC)
    assert np.allclose(RC, R[perm].transpose(0, 3, 1, 2), rtol=0, atol=1e-13 * np.abs(R).max())


@pytest.mark.parametrize("bc", [((0, 0), (0, 0), (0, 0)), ((1, 1), (2, 2), (0, 0))])
def test_zero_viscosity_is_the_euler_residual(bc):
    g0 = box((10, 8), mu=0.0, bc=bc)
    U = smooth_state(g0, 4)
    ge = SimpleNamespace(**{k: v for k, v in vars(g0).items() if k not in ("mu", "prandtl")})
    assert np.array_equal(oracle.residual(g0, U), oracle.residual(ge, U))
    assert oracle.dt(g0, U)[0] == oracle.dt(ge, U)[0]


def test_time_step_diffusion_limit():
    # fluid at rest, rho = 2, p = 1: lambda = sum_d c / dx_d + 2 nu sum_d 1/dx_d^2,
    # nu = (mu / rho) max(4/3, gamma / Pr)
    g = box((8, 16), mu=0.01, hi=1.0)
    X, _, _ = centres(g)
    U = conserved(g, 2.0 + 0 * X, (0 * X, 0 * X), 1.0 + 0 * X)
    c = math.sqrt(GAMMA * 1.0 / 2.0)
    nu = 0.01 / 2.0 * max(4.0 / 3.0, GAMMA / PR)
    lam = c * 8 + c * 16 + 2.0 * nu * (64 + 256)
    dt, fl = oracle.dt(g, U)
    assert fl == 0 and abs(dt - 0.5 / lam) <= 1e-15 * dt


def test_reverse_gradient_refuses_viscosity():
    g = box((6, 6), mu=0.01)
    U = smooth_state(g, 5)
    with pytest.raises(NotImplementedError):
        oracle.residual_vjp(g, U, U)
