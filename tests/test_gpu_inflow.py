"""Inflow faces (FV_BC_INFLOW, a given ghost state) on the HIP split path
against the FP64 oracle: an inlet-like 2D channel (supersonic inflow, slip
walls, outflow) and a 3D grid, residual, steps and the adjoint step; launch
tables give the same bits; both on the fused path too."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

pytestmark = pytest.mark.gpu

INFLOW, WALL, OUT = 3, 2, 1
TOL = 1e-12


def assert_pervar_close(got, ref, tol, what):
    for v in range(ref.shape[0]):
        scale = max(np.abs(ref[v]).max(), 1e-300)
        err = np.abs(got[v] - ref[v]).max()
        assert err <= tol * scale, f"{what} var {v}: max err {err:.3e} vs scale {scale:.3e}"


def free_stream(ndim, mach=2.0, angle=0.1):
    rho, p, gam = 1.0, 1.0 / 1.4, 1.4
    c = np.sqrt(gam * p / rho)
    vel = [mach * c * np.cos(angle), mach * c * np.sin(angle), 0.05 * mach * c][:ndim]
    return np.array([rho] + [rho * u for u in vel] + [p / (gam - 1) + 0.5 * rho * sum(u * u for u in vel)])


def bumped(g, q, seed):
    rng = np.random.default_rng(seed)
    U = np.broadcast_to(q.reshape((-1,) + (1,) * 3), g.shape).copy()
    nx, ny, nz = (int(v) for v in g.n)
    ax = [(np.arange(m) + 0.5) / m for m in (nx, ny, nz)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    c = rng.uniform(0.3, 0.7, 3)
    b = 0.3 * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + ((Z - c[2]) ** 2 if g.ndim == 3 else 0)) / 0.02)
    U *= (1.0 + b)[None]                   # denser blob moving with the stream
    return U


def cases():
    q2 = free_stream(2)
    g2 = inputs.grid2d(61, 23, hi=(2.0, 1.0), bc=((INFLOW, OUT), (WALL, WALL)))
    st2 = np.zeros((3, 2, 4))
    st2[0, 0] = q2
    g2 = dataclasses.replace(g2, bc_state=st2)
    q3 = free_stream(3)
    g3 = inputs.grid3d(21, 10, 9, bc=((INFLOW, OUT), (0, 0), (WALL, INFLOW)))
    st3 = np.zeros((3, 2, 5))
    st3[0, 0] = q3
    st3[2, 1] = q3 * np.array([1.0, 1.0, 1.0, -1.0, 1.0])   # flow entering through the top z face
    g3 = dataclasses.replace(g3, bc_state=st3)
    return [("inlet_channel_2d", g2, bumped(g2, q2, 1)), ("inflow_3d", g3, bumped(g3, q3, 2))]


CASES = cases()
IDS = [c[0] for c in CASES]


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_residual_with_inflow_matches_oracle(name, g, U):
    from paper_2306_14011_amd import fv
    s = fv.Solver(g)
    s.set_state(U)
    R = s.residual().cpu().numpy()
    s.close()
    assert_pervar_close(R, oracle.residual(g, U), TOL, name)


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_steps_with_inflow_match_oracle(name, g, U):
    import torch
    from paper_2306_14011_amd import fv
    n = 6
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
    assert np.array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_adjoint_step_with_inflow_matches_oracle(name, g, U):
    import torch
    from paper_2306_14011_amd import fv
    g = dataclasses.replace(g, limiter=False)
    rng = np.random.default_rng(6)
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


@pytest.mark.parametrize("name,g,U", CASES, ids=[c[0] for c in CASES])
def test_fused_path_with_inflow_matches_oracle(name, g, U):
    # the inlet channel (2D) and the 3D grid with inflow, walls and outflow on
    # the fused path
    import torch
    from paper_2306_14011_amd import fv
    n = 5
    s = fv.Solver(g)
    s.set_path(fv.FV_PATH_FUSED, 8, 0)
    s.set_state(U)
    dts = torch.zeros(n, dtype=torch.float64, device="cuda")
    s.step(n, dt_out=dts)
    rc, flags = s.status()
    got = s.get_state()
    s.close()
    assert flags == 0
    ref, rdt, _ = oracle.run(g, U, n)
    assert np.allclose(dts.cpu().numpy(), rdt, rtol=1e-13, atol=0)
    assert_pervar_close(got, ref, 1e-11, name)


def test_large_inlet_channel_matches_oracle():
    # many tiles and a ragged last block of every kernel: 517 x 389 cells,
    # supersonic inflow, slip walls, outflow, 4 steps
    import torch
    from paper_2306_14011_amd import fv
    q = free_stream(2, mach=2.5, angle=0.15)
    g = inputs.grid2d(517, 389, hi=(2.0, 1.5), bc=((INFLOW, OUT), (WALL, WALL)))
    st = np.zeros((3, 2, 4))
    st[0, 0] = q
    g = dataclasses.replace(g, bc_state=st)
    U = bumped(g, q, 7)
    s = fv.Solver(g)
    s.set_state(U)
    assert_pervar_close(s.residual().cpu().numpy(), oracle.residual(g, U), TOL, "residual")
    dts = torch.zeros(4, dtype=torch.float64, device="cuda")
    s.step(4, dt_out=dts)
    got = s.get_state()
    s.close()
    ref, rdt, _ = oracle.run(g, U, 4)
    assert np.allclose(dts.cpu().numpy(), rdt, rtol=1e-12, atol=0)
    assert_pervar_close(got, ref, TOL, "4 steps")
    # the same channel on the fused path (ragged strips and segments)
    s = fv.Solver(g)
    s.set_path(fv.FV_PATH_FUSED, 0, 0)
    s.set_state(U)
    s.step(4)
    got_f = s.get_state()
    s.close()
    assert_pervar_close(got_f, ref, 1e-11, "4 fused steps")
