"""Pins of the oracle's inflow boundary (the supersonic inlet of Sec. "A Test
Case" takes in a given state): the given state flowing in stays uniform, an
inflow face equals a grid two cells longer that holds the given state there,
and the residual's transposed derivative leaves the fixed ghost cells out
(dot-product test against complex-step derivatives)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

INFLOW = 3


def inflow_grid(nx, ny, state):
    g = inputs.grid2d(nx, ny, hi=(1.0, 1.0), bc=((INFLOW, 1), (0, 0)))
    st = np.zeros((3, 2, 4))
    st[0, 0] = state
    return dataclasses.replace(g, bc_state=st)


def inflow_state(mach=2.0, angle=0.1):
    rho, p, gam = 1.0, 1.0 / 1.4, 1.4
    c = np.sqrt(gam * p / rho)
    u, v = mach * c * np.cos(angle), mach * c * np.sin(angle)
    return np.array([rho, rho * u, rho * v, p / (gam - 1) + 0.5 * rho * (u * u + v * v)])


def wavy(g, seed):
    rng = np.random.default_rng(seed)
    nx, ny = g.n[0], g.n[1]
    X, Y = np.meshgrid((np.arange(nx) + 0.5) / nx, (np.arange(ny) + 0.5) / ny)
    ph = rng.uniform(0, 6.28, 3)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X + ph[0]) * np.cos(2 * np.pi * Y)
    u = 1.2 + 0.2 * np.cos(2 * np.pi * Y + ph[1])
    v = 0.1 * np.sin(2 * np.pi * X + ph[2])
    p = 0.8 + 0.1 * np.cos(2 * np.pi * (X + Y))
    return inputs.primitive_to_conserved(g, rho[None], (u[None], v[None]), p[None])


@pytest.mark.parametrize("limiter", [True, False, "vanleer"])
def test_uniform_inflow_is_steady(limiter):
    q = inflow_state()
    g = inflow_grid(23, 9, q)
    U = np.broadcast_to(q[:, None, None, None], (4, 1, 9, 23)).copy()
    assert np.abs(oracle.residual(g, U, limiter=limiter)).max() <= 1e-14 * np.abs(q).max()


@pytest.mark.parametrize("limiter", [True, False])
def test_inflow_face_equals_a_longer_grid_holding_the_state(limiter):
    q = inflow_state(1.5, 0.3)
    n, ny = 30, 12
    g = inflow_grid(n, ny, q)
    U = wavy(g, 1)
    ge = inputs.grid2d(n + 2, ny, lo=(-2.0 / n, 0.0), hi=(1.0, 1.0), bc=((1, 1), (0, 0)))
    Ue = np.concatenate([np.broadcast_to(q[:, None, None, None], (4, 1, ny, 2)), U], axis=3)
    R = oracle.residual(g, U, limiter=limiter)
    Re = oracle.residual(ge, Ue, limiter=limiter)
    assert np.allclose(R, Re[:, :, :, 2:], rtol=0, atol=1e-13 * np.abs(R).max())


def test_transposed_derivative_leaves_the_fixed_ghosts_out():
    g = inflow_grid(16, 7, inflow_state(1.7, 0.2))
    U = wavy(g, 2)
    rng = np.random.default_rng(3)
    for _ in range(3):
        V = rng.standard_normal(U.shape)
        w = rng.standard_normal(U.shape)
        _, JV = oracle.residual_cs(g, U, V, limiter=False)
        JTw = oracle.residual_vjp(g, U, w, limiter=False)
        assert abs((w * JV).sum() - (JTw * V).sum()) <= 1e-12 * np.abs(w * JV).sum()
