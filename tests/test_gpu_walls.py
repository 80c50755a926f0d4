"""Slip walls (FV_BC_WALL) on the HIP split path against the FP64 oracle:
residual, steps and the adjoint step on closed and partly closed boxes in 2D
and 3D; launch tables give the same bits; the same boxes on the fused path."""
import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

pytestmark = pytest.mark.gpu

WALL = 2
TOL = 1e-12


def assert_pervar_close(got, ref, tol, what):
    for v in range(ref.shape[0]):
        scale = max(np.abs(ref[v]).max(), 1e-300)
        err = np.abs(got[v] - ref[v]).max()
        assert err <= tol * scale, f"{what} var {v}: max err {err:.3e} vs scale {scale:.3e}"


def pulse(g, seed, vel=0.2):
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in g.n)
    ax = [(np.arange(m) + 0.5) / m for m in (nx, ny, nz)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    c = rng.uniform(0.3, 0.7, 3)
    r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + ((Z - c[2]) ** 2 if g.ndim == 3 else 0.0)
    b = np.exp(-r2 / 0.02)
    vels = [vel * np.sin(np.pi * X) * np.cos(2 * np.pi * Y + 0.3),
            vel * np.cos(np.pi * X + 0.2) * np.sin(2 * np.pi * Y),
            vel * np.sin(2 * np.pi * Z + 0.1) * np.cos(np.pi * X)][:g.ndim]
    return inputs.primitive_to_conserved(g, 1.0 + 0.3 * b, vels, 1.0 + 0.5 * b)


def cases():
    g1 = inputs.grid2d(40, 33, hi=(1.0, 1.0), bc=((WALL, WALL), (WALL, WALL)))
    g2 = inputs.grid2d(37, 26, hi=(1.0, 1.0), bc=((WALL, 1), (0, 0)))        # wall inflow side, open outlet
    g3 = inputs.grid3d(18, 11, 9, bc=((WALL, WALL), (0, 0), (WALL, 1)))
    return [("box_2d", g1, pulse(g1, 1)), ("wall_outlet_2d", g2, pulse(g2, 2)), ("walls_3d", g3, pulse(g3, 3))]


CASES = cases()
IDS = [c[0] for c in CASES]


def test_fused_walls_several_strips():
    # a closed box wider than one 60-column strip (x walls in the first and the
    # ragged last strip), van Leer and minmod, against the oracle; two
    # per-stage tables give the same bits
    import torch
    from paper_2306_14011_amd import fv
    g = inputs.grid2d(133, 47, hi=(2.0, 0.8), bc=((WALL, WALL), (WALL, WALL)))
    U = pulse(g, 7)
    for lim in (True, "vanleer"):
        h = g if lim is True else __import__("copy").copy(g)
        h.limiter = lim
        outs = []
        for seg, waves in (([0, 0, 0], [0, 0, 0]), ([8, 20, 12], [3, 0, 21])):
            s = fv.Solver(h)
            s.set_path(fv.FV_PATH_FUSED, 0, 0)
            s.set_fused_launch(seg, waves)
            s.set_state(U)
            dts = torch.zeros(4, dtype=torch.float64, device="cuda")
            s.step(4, dt_out=dts)
            rc, flags = s.status()
            assert flags == 0
            outs.append((s.get_state(), dts.cpu().numpy()))
            s.close()
        ref, rdt, _ = oracle.run(h, U, 4, limiter=lim)
        assert np.allclose(outs[0][1], rdt, rtol=1e-13, atol=0), lim
        assert_pervar_close(outs[0][0], ref, 1e-11, f"box {lim}")
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1]), lim


def test_fused3d_walls_several_tiles():
    # a 3D grid of several 32 x 7 tiles in x and y, walls on both x sides and
    # the low y side, an inflow face on the high z side, transmissive low z:
    # against the oracle, and two per-stage tables give the same bits
    import math
    import torch
    from paper_2306_14011_amd import fv
    g = inputs.grid3d(71, 23, 19, bc=((WALL, WALL), (WALL, 1), (1, 3)))
    q = np.zeros((3, 2, 5))
    q[2, 1] = (1.0, 0.1, 0.0, -0.9 * math.sqrt(g.gamma), 1.0 / (g.gamma - 1.0) + 0.5 * (0.01 + 0.81 * g.gamma))
    g.bc_state = q
    U = pulse(g, 11)
    outs = []
    for seg, waves in (([0, 0, 0], [0, 0, 0]), ([8, 4, 12], [5, 0, 9])):
        s = fv.Solver(g)
        s.set_path(fv.FV_PATH_FUSED, 0, 0)
        s.set_fused_launch(seg, waves)
        s.set_state(U)
        dts = torch.zeros(3, dtype=torch.float64, device="cuda")
        s.step(3, dt_out=dts)
        rc, flags = s.status()
        assert flags == 0
        outs.append((s.get_state(), dts.cpu().numpy()))
        s.close()
    ref, rdt, _ = oracle.run(g, U, 3)
    assert np.allclose(outs[0][1], rdt, rtol=1e-13, atol=0)
    assert_pervar_close(outs[0][0], ref, 1e-11, "walls 3d")
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_batch_with_walled_grids_matches_oracle():
    # a batch of the 2D walled grids and a periodic vortex runs the boundary
    # variant of the stage kernels; each grid against its own oracle run, and
    # two schedules give the same bits
    from paper_2306_14011_amd import fv
    g0, U0 = inputs.vortex_case(40, seed=5)
    grids = [CASES[0][1], CASES[1][1], g0]
    states = [CASES[0][2], CASES[1][2], U0]
    outs = []
    for seg in (8, 20):
        B = fv.Batch(grids, seg=seg)
        B.set_states(states)
        B.step(4)
        rc, flags = B.status()
        assert flags == 0
        outs.append((B.get_states(), B.dt()))
        B.close()
    for gi, (g, U) in enumerate(zip(grids, states)):
        ref, rdts, _ = oracle.run(g, U, 4)
        assert abs(outs[0][1][gi] - rdts[-1]) <= 1e-13 * rdts[-1], gi
        assert_pervar_close(outs[0][0][gi], ref, 1e-11, f"grid {gi}")
        assert np.array_equal(outs[0][0][gi], outs[1][0][gi])


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_residual_with_walls_matches_oracle(name, g, U):
    from paper_2306_14011_amd import fv
    s = fv.Solver(g)
    s.set_state(U)
    R = s.residual().cpu().numpy()
    s.close()
    ref = oracle.residual(g, U)
    assert_pervar_close(R, ref, TOL, name)
    if name == "box_2d":
        # closed box: no mass or energy crosses the walls
        assert abs(R[0].sum()) <= 1e-13 * np.abs(R).max() * R[0].size
        assert abs(R[3].sum()) <= 1e-13 * np.abs(R).max() * R[3].size


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_steps_with_walls_match_oracle(name, g, U):
    import torch
    from paper_2306_14011_amd import fv
    n = 5
    outs = []
    for launch in (None, [32, 128, 16, 512, 64, 64, 4096, 128, 0, 64, 64, 256, 0, 1024]):
        s = fv.Solver(g)
        if launch is not None:
            s.set_launch(launch)
        s.set_state(U)
        dts = torch.zeros(n, dtype=torch.float64, device="cuda")
        s.step(n, dt_out=dts)
        rc, flags = s.status()
        assert flags == 0
        outs.append((s.get_state(), dts.cpu().numpy()))
        s.close()
    ref, rdt, rfl = oracle.run(g, U, n)
    assert rfl == 0
    assert np.allclose(outs[0][1], rdt, rtol=1e-12, atol=0)
    assert_pervar_close(outs[0][0], ref, TOL, name)
    assert np.array_equal(outs[0][0], outs[1][0])      # launch tables give the same bits


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_adjoint_step_with_walls_matches_oracle(name, g, U):
    # unlimited scheme: minmod's derivative jumps where a slope crosses zero
    import dataclasses

    import torch
    from paper_2306_14011_amd import fv
    g = dataclasses.replace(g, limiter=False)
    rng = np.random.default_rng(5)
    dt = 0.8 * oracle.dt(g, U)[0]
    lam = rng.standard_normal(U.shape)
    s = fv.Solver(g)
    s.set_state(U)
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    L = torch.as_tensor(np.ascontiguousarray(lam)).cuda()
    fv.fv_adjoint_step(s.ctx, s.U.data_ptr(), dtt.data_ptr(), L.data_ptr())
    got = L.cpu().numpy()
    s.close()
    ref = oracle.rk3_step_vjp(g, U, dt, lam, limiter=False)
    for v in range(U.shape[0]):
        assert np.abs(got[v] - ref[v]).max() <= 1e-10 * np.abs(ref[v]).max(), (name, v)


@pytest.mark.parametrize("limiter", [True, "vanleer", False], ids=["minmod", "vanleer", "unlimited"])
@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_fused_path_with_walls_matches_oracle(name, g, U, limiter):
    # walls on the fused path (2D and 3D): the kernels' boundary variant maps
    # ghost rows, columns and planes to the mirror cells with the normal
    # momentum reversed; two per-stage tables give the same bits
    import copy

    import torch
    from paper_2306_14011_amd import fv
    h = copy.copy(g)
    h.limiter = limiter
    n = 4
    outs = []
    for seg, waves in (([0, 0, 0], [0, 0, 0]), ([4, 12, 8], [0, 7, 64])):
        s = fv.Solver(h)
        s.set_path(fv.FV_PATH_FUSED, 0, 0)
        s.set_fused_launch(seg, waves)
        s.set_state(U)
        dts = torch.zeros(n, dtype=torch.float64, device="cuda")
        s.step(n, dt_out=dts)
        rc, flags = s.status()
        assert flags == 0
        outs.append((s.get_state(), dts.cpu().numpy()))
        s.close()
    ref, rdt, _ = oracle.run(h, U, n, limiter=limiter)
    assert np.allclose(outs[0][1], rdt, rtol=1e-13, atol=0)
    assert_pervar_close(outs[0][0], ref, 1e-11, name)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
