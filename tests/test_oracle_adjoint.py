"""Pins of the oracle's reverse-mode gradient: dot-product tests against the
complex-step tangent, a full brute-force Jacobian on a tiny grid, and finite
differences of the tangent itself."""
import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs


def grids():
    g1, U1 = inputs.vortex_case(12, seed=1)
    U1 = inputs.gaussian_bumps(g1, U1, 1, amp=0.05)
    g2 = inputs.grid2d(9, 7, hi=(1.0, 1.0), bc=((1, 1), (0, 0)))
    U2 = inputs.sod_state(g2, (0.8, 0.6, 0.0), (0.5, 0.5, 0.0))
    g3 = inputs.grid3d(6, 5, 4)
    U3 = inputs.sod_state(g3, inputs.sod_rotated_normal(2), (0.5, 0.5, 0.5))
    rng = np.random.default_rng(0)
    U3[1:4] += 0.05 * rng.standard_normal(U3[1:4].shape) * U3[0]
    g4 = inputs.grid2d(10, 1, hi=(1.0, 1.0), bc=((1, 1), (0, 0)))
    U4 = inputs.sod_axis_state(g4, 0)
    U4[1] += 0.1
    return [("periodic_vortex", g1, U1), ("transmissive_tilted_sod", g2, U2), ("3d_sod", g3, U3),
            ("single_row", g4, U4)]


GRIDS = grids()


@pytest.mark.parametrize("name,g,U", GRIDS, ids=[x[0] for x in GRIDS])
def test_residual_dot_product(name, g, U):
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal(U.shape)
        w = rng.standard_normal(U.shape)
        _, Jv = oracle.residual_cs(g, U, v)
        JTw = oracle.residual_vjp(g, U, w)
        a, b = np.sum(Jv * w), np.sum(v * JTw)
        assert abs(a - b) <= 1e-12 * max(abs(a), np.abs(Jv).sum()), (a, b)


@pytest.mark.parametrize("name,g,U", GRIDS, ids=[x[0] for x in GRIDS])
def test_step_dot_product(name, g, U):
    rng = np.random.default_rng(4)
    dt = 0.5 * oracle.dt(g, U)[0]
    for _ in range(2):
        v = rng.standard_normal(U.shape)
        w = rng.standard_normal(U.shape)
        _, Jv = oracle.rk3_step_cs(g, U, v, dt)
        JTw = oracle.rk3_step_vjp(g, U, dt, w)
        a, b = np.sum(Jv * w), np.sum(v * JTw)
        assert abs(a - b) <= 1e-12 * max(abs(a), np.abs(Jv).sum()), (a, b)


def test_full_jacobian_brute_force():
    # every column of dStep/dU by the complex step equals the corresponding row of the reverse
    g = inputs.grid2d(4, 3, hi=(1.0, 1.0), bc=((0, 0), (1, 1)))
    rng = np.random.default_rng(5)
    U = inputs.sod_state(g, (0.6, 0.8, 0.0), (0.4, 0.5, 0.0))
    U[1:3] += 0.1 * rng.standard_normal(U[1:3].shape)
    dt = 0.4 * oracle.dt(g, U)[0]
    n = U.size
    J = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        J[:, c] = oracle.rk3_step_cs(g, U, e.reshape(U.shape), dt)[1].ravel()
    JT = np.zeros((n, n))
    for r in range(n):
        e = np.zeros(n)
        e[r] = 1.0
        JT[r, :] = oracle.rk3_step_vjp(g, U, dt, e.reshape(U.shape)).ravel()
    assert np.allclose(JT, J, rtol=0, atol=1e-13 * np.abs(J).max())


def smooth_cases():
    g1, U1 = inputs.vortex_case(12, seed=1)
    g2 = inputs.grid2d(11, 9, bc=((1, 1), (1, 1)))
    U2 = inputs.vortex_state(g2, (4.6, 5.3), 3.0)
    g3 = inputs.grid3d(5, 6, 4, bc=((1, 1), (0, 0), (1, 1)))
    rng = np.random.default_rng(2)
    U3 = inputs.primitive_to_conserved(
        g3, 1.0 + 0.1 * rng.random(g3.shape[1:]), tuple(0.2 * rng.standard_normal(g3.shape[1:]) for _ in range(3)),
        1.0 + 0.1 * rng.random(g3.shape[1:]))
    return [("periodic_vortex", g1, U1), ("transmissive_vortex", g2, U2), ("3d_random_smooth", g3, U3)]


SMOOTH = smooth_cases()


@pytest.mark.parametrize("name,g,U", SMOOTH, ids=[x[0] for x in SMOOTH])
def test_tangent_matches_finite_differences(name, g, U):
    # central differences of the real step along random directions with the
    # limiter off (the scheme is then smooth: no minmod kinks)
    rng = np.random.default_rng(6)
    dt = 0.5 * oracle.dt(g, U)[0]
    v = rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True) * 1e-2
    _, Jv = oracle.rk3_step_cs(g, U, v, dt, limiter=False)
    h = 1e-5
    fd = (oracle.rk3_step(g, U + h * v, dt, limiter=False) - oracle.rk3_step(g, U - h * v, dt, limiter=False)) / (2 * h)
    assert np.abs(fd - Jv).max() <= 1e-7 * np.abs(Jv).max()
