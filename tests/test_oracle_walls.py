"""Pins of the oracle's slip wall (the reading for the solid boundaries of the
supersonic inlet of Sec. "A Test Case"): a closed box conserves mass
and energy exactly, a box at rest stays at rest, mirror-symmetric states stay
symmetric, and a walled grid equals the periodic grid of twice the size that
holds the state and its mirror image."""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

WALL = 2


def box(nx, ny, bc=((WALL, WALL), (WALL, WALL)), hi=(1.0, 1.0)):
    return inputs.grid2d(nx, ny, hi=hi, bc=bc)


def pulse_state(g, seed=0, vel=0.1):
    """Smooth pressure and density pulse with a smooth velocity field."""
    rng = np.random.default_rng(seed)
    nx, ny = g.n[0], g.n[1]
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    cx, cy = rng.uniform(0.3, 0.7, 2)
    b = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / 0.02)
    rho = 1.0 + 0.3 * b
    p = 1.0 + 0.5 * b
    u = vel * np.sin(np.pi * X) * np.cos(2 * np.pi * Y + 0.3)
    v = vel * np.cos(np.pi * X + 0.2) * np.sin(2 * np.pi * Y)
    return inputs.primitive_to_conserved(g, rho[None], (u[None], v[None]), p[None])


@pytest.mark.parametrize("limiter", [True, False])
def test_closed_box_conserves_mass_and_energy(limiter):
    g = box(40, 33)
    U = pulse_state(g, 1)
    R = oracle.residual(g, U, limiter=limiter)
    scale = np.abs(R).max()
    assert scale > 1e-3
    assert abs(R[0].sum()) <= 1e-13 * scale * R[0].size
    assert abs(R[3].sum()) <= 1e-13 * scale * R[3].size
    # the walls push on the momentum: its sum is not zero
    assert abs(R[1].sum()) > 1e-6 * scale


def test_box_at_rest_stays_at_rest():
    g = box(24, 17)
    U = inputs.primitive_to_conserved(g, np.full((1, 17, 24), 1.3), (np.zeros((1, 17, 24)),) * 2,
                                      np.full((1, 17, 24), 0.7))
    assert np.abs(oracle.residual(g, U)).max() == 0.0


def test_wall_equals_periodic_mirror_domain():
    # x walls on n cells == periodic on 2n cells holding [mirror(U) reversed, U]
    n, ny = 20, 13
    g = box(n, ny, bc=((WALL, WALL), (0, 0)))
    U = pulse_state(g, 2, vel=0.3)
    gd = inputs.grid2d(2 * n, ny, hi=(2.0, 1.0), bc=((0, 0), (0, 0)))
    M = U[:, :, :, ::-1].copy()
    M[1] = -M[1]
    Ud = np.concatenate([M, U], axis=3)
    for lim in (True, False, "vanleer"):
        R = oracle.residual(g, U, limiter=lim)
        Rd = oracle.residual(gd, Ud, limiter=lim)
        assert np.allclose(R, Rd[:, :, :, n:], rtol=0, atol=1e-14 * np.abs(R).max()), lim
    # the same along y
    gy = box(ny, n, bc=((0, 0), (WALL, WALL)))
    Uy = pulse_state(gy, 3, vel=0.3)
    gyd = inputs.grid2d(ny, 2 * n, hi=(1.0, 2.0), bc=((0, 0), (0, 0)))
    My = Uy[:, :, ::-1, :].copy()
    My[2] = -My[2]
    Ryd = oracle.residual(gyd, np.concatenate([My, Uy], axis=2))
    assert np.allclose(oracle.residual(gy, Uy), Ryd[:, :, n:, :], rtol=0, atol=1e-14 * np.abs(Ryd).max())


def test_mirror_symmetric_state_stays_symmetric():
    g = box(30, 22)
    U = pulse_state(g, 4)
    M = U[:, :, :, ::-1].copy()
    M[1] = -M[1]
    Us = 0.5 * (U + M)               # symmetric about x = 1/2, u antisymmetric
    U1, _, fl = oracle.run(g, Us, 5)
    assert fl == 0
    M1 = U1[:, :, :, ::-1].copy()
    M1[1] = -M1[1]
    assert np.allclose(U1, M1, rtol=0, atol=1e-13)


def test_wall_needs_two_cells():
    g = inputs.grid2d(8, 1, hi=(1.0, 1.0), bc=((0, 0), (WALL, WALL)))
    with pytest.raises(ValueError):
        oracle.residual(g, np.ones((4, 1, 1, 8)))
