"""Curvilinear 2D grids on the HIP split and fused paths against the FP64
oracle: residual and steps (dt included) on wavy periodic grids, on a
rotated grid with walls and on a ramp inlet (supersonic inflow, slip walls
along a compression ramp, outflow), for minmod, van Leer and the unlimited
scheme; launch tables (split) and per-stage tables (fused) give the same
bits; a uniform flow stays uniform; the identity map reproduces the
uniform-grid path; the adjoint step and viscous curvilinear grids refuse."""
import copy
import math

import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

pytestmark = pytest.mark.gpu

WALL, INFLOW = 2, 3


def assert_pervar_close(got, ref, tol, what):
    for v in range(ref.shape[0]):
        scale = max(np.abs(ref[v]).max(), 1e-300)
        err = np.abs(got[v] - ref[v]).max()
        assert err <= tol * scale, f"{what} var {v}: max err {err:.3e} vs scale {scale:.3e}"


def box_nodes(g):
    x = g.lo[0] + (g.hi[0] - g.lo[0]) * np.arange(g.n[0] + 1) / g.n[0]
    y = g.lo[1] + (g.hi[1] - g.lo[1]) * np.arange(g.n[1] + 1) / g.n[1]
    Y, X = np.meshgrid(y, x, indexing="ij")
    return np.stack([X, Y])


def curved(g, nodes):
    h = copy.copy(g)
    h.nodes = nodes
    return h


def wavy_state(g, nodes, seed):
    rng = np.random.default_rng(seed)
    x, y = inputs.node_centroids(nodes)
    L = (g.hi[0] - g.lo[0], g.hi[1] - g.lo[1])
    ph = rng.random(5) * 2 * math.pi
    rho = 1.0 + 0.2 * np.sin(2 * math.pi * x / L[0] + ph[0]) * np.cos(2 * math.pi * y / L[1] + ph[1])
    u = 0.5 + 0.3 * np.sin(2 * math.pi * y / L[1] + ph[2])
    v = -0.3 + 0.3 * np.cos(2 * math.pi * x / L[0] + ph[3])
    p = 1.0 + 0.2 * np.cos(2 * math.pi * (x / L[0] - y / L[1]) + ph[4])
    return inputs.primitive_to_conserved(g, rho[None], (u[None], v[None]), p[None])


def ramp_inlet(nx=60, ny=24, angle_deg=10.0, mach=2.5):
    """A 2D inlet-like channel: supersonic inflow on the left, outflow on the
    right, a slip-wall floor that turns up by `angle_deg` at x = 1 (a
    compression ramp: an oblique shock), a flat slip-wall ceiling at y = 1.2."""
    g = inputs.grid2d(nx, ny, hi=(3.0, 1.2), bc=((INFLOW, 1), (WALL, WALL)))
    xi = 3.0 * np.arange(nx + 1) / nx
    floor = np.where(xi > 1.0, (xi - 1.0) * math.tan(math.radians(angle_deg)), 0.0)
    eta = np.arange(ny + 1) / ny
    X = np.broadcast_to(xi[None, :], (ny + 1, nx + 1))
    Y = floor[None, :] + eta[:, None] * (1.2 - floor[None, :])
    nodes = np.stack([X, Y]).copy()
    c = math.sqrt(g.gamma)
    u = mach * c
    q = np.zeros((3, 2, 5))
    q[0, 0, :4] = (1.0, u, 0.0, 1.0 / (g.gamma - 1.0) + 0.5 * u * u)
    g.bc_state = q
    U = np.broadcast_to(q[0, 0, :4, None, None, None], (4, 1, ny, nx)).copy()
    return curved(g, nodes), U


def cases():
    out = []
    g = inputs.grid2d(36, 28, hi=(2.0, 1.5))
    nodes = inputs.wavy_nodes(36, 28, hi=(2.0, 1.5), amp=0.05, rot=0.3)
    out.append(("wavy_periodic", curved(g, nodes), wavy_state(g, nodes, 1)))
    g = inputs.grid2d(33, 25, hi=(2.0, 1.5), bc=((1, 1), (0, 0)))
    nodes = inputs.wavy_nodes(33, 25, hi=(2.0, 1.5), amp=0.04)
    out.append(("wavy_transmissive_x", curved(g, nodes), wavy_state(g, nodes, 2)))
    g = inputs.grid2d(30, 22, hi=(1.5, 1.1), bc=((WALL, WALL), (WALL, 1)))
    X, Y = box_nodes(g)
    th = 0.6
    nodes = np.stack([math.cos(th) * X - math.sin(th) * Y, math.sin(th) * X + math.cos(th) * Y])
    out.append(("rotated_walls", curved(g, nodes), wavy_state(g, nodes, 3)))
    h, U = ramp_inlet()
    out.append(("ramp_inlet", h, U))
    return out


CASES = cases()
IDS = [c[0] for c in CASES]


def spec_with(g, limiter):
    h = copy.copy(g)
    h.limiter = limiter
    return h


@pytest.mark.parametrize("limiter", [True, "vanleer", False], ids=["minmod", "vanleer", "unlimited"])
@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_curvilinear_residual_matches_oracle(name, g, U, limiter):
    from paper_2306_14011_amd import fv
    h = spec_with(g, limiter)
    s = fv.Solver(h)
    s.set_state(U)
    R = s.residual().cpu().numpy()
    s.close()
    ref = oracle.residual(h, U, limiter=limiter)
    if name == "ramp_inlet":
        # the uniform inflow state: only the ramp's cells see a residual
        assert np.abs(ref).max() > 1e-3
    assert_pervar_close(R, ref, 1e-12, name)


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_curvilinear_steps_match_oracle(name, g, U):
    import torch
    from paper_2306_14011_amd import fv
    n = 5
    outs = []
    for launch in (None, [32, 128, 16, 512, 0, 0, 4096, 128, 0, 64, 64, 256, 0, 1024]):
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
    assert np.allclose(outs[0][1], rdt, rtol=1e-13, atol=0), (outs[0][1], rdt)
    assert_pervar_close(outs[0][0], ref, 1e-11, name)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("limiter", [True, "vanleer", False], ids=["minmod", "vanleer", "unlimited"])
@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_curvilinear_fused_steps_match_oracle(name, g, U, limiter):
    # the fused stage kernels' curvilinear variant: metric streams per face and
    # cell, the Roe flux along each face normal, walls reflected about their
    # normals; 5 steps, dt included, two per-stage tables give the same bits
    import torch
    from paper_2306_14011_amd import fv
    h = spec_with(g, limiter)
    n = 5
    outs = []
    for seg, waves in (([0, 0, 0], [0, 0, 0]), ([8, 4, 12], [3, 0, 64])):
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
    ref, rdt, rfl = oracle.run(h, U, n, limiter=limiter)
    assert rfl == 0
    assert np.allclose(outs[0][1], rdt, rtol=1e-13, atol=0), (outs[0][1], rdt)
    assert_pervar_close(outs[0][0], ref, 1e-11, name)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("limiter", [True, False], ids=["minmod", "unlimited"])
def test_curvilinear_fused_several_strips(limiter):
    # wider than one 60-column strip, with ragged last strips and segments:
    # a wavy grid with walls on both y sides, and the ramp inlet at 131 x 45
    import torch
    from paper_2306_14011_amd import fv
    g = inputs.grid2d(143, 61, hi=(3.0, 1.2), bc=((1, 1), (WALL, WALL)))
    nodes = inputs.wavy_nodes(143, 61, hi=(3.0, 1.2), amp=0.03)
    cases_ = [("wavy_walls", curved(g, nodes), wavy_state(g, nodes, 6)), ("ramp", *ramp_inlet(131, 45))]
    for name, h, U in cases_:
        h = spec_with(h, limiter)
        outs = []
        for seg, waves in (([0, 0, 0], [0, 0, 0]), ([8, 16, 12], [5, 0, 40])):
            s = fv.Solver(h)
            s.set_path(fv.FV_PATH_FUSED, 0, 0)
            s.set_fused_launch(seg, waves)
            s.set_state(U)
            dts = torch.zeros(3, dtype=torch.float64, device="cuda")
            s.step(3, dt_out=dts)
            rc, flags = s.status()
            assert flags == 0
            outs.append((s.get_state(), dts.cpu().numpy()))
            s.close()
        ref, rdt, _ = oracle.run(h, U, 3, limiter=limiter)
        assert np.allclose(outs[0][1], rdt, rtol=1e-13, atol=0), name
        assert_pervar_close(outs[0][0], ref, 1e-11, name)
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1]), name


def test_curvilinear_fused_source_matches_oracle():
    # the source term on a curvilinear grid enters as -area S per cell
    import torch
    from paper_2306_14011_amd import fv
    name, g, U = CASES[0]
    rng = np.random.default_rng(7)
    S = 0.05 * rng.standard_normal(U.shape)
    n = 3
    s = fv.Solver(g)
    s.set_path(fv.FV_PATH_FUSED, 0, 0)
    s.set_state(U)
    St = torch.as_tensor(np.ascontiguousarray(S)).cuda()
    s.set_source(St)
    dts = torch.zeros(n, dtype=torch.float64, device="cuda")
    s.step(n, dt_out=dts)
    got = s.get_state()
    s.close()
    ref, rdt, _ = oracle.run(g, U, n, source=S)
    assert np.allclose(dts.cpu().numpy(), rdt, rtol=1e-13, atol=0)
    assert_pervar_close(got, ref, 1e-11, name)


def test_uniform_flow_stays_uniform_on_the_gpu():
    from paper_2306_14011_amd import fv
    g = inputs.grid2d(40, 30, hi=(2.0, 1.5))
    h = curved(g, inputs.wavy_nodes(40, 30, hi=(2.0, 1.5), amp=0.06, rot=0.5))
    U = inputs.primitive_to_conserved(g, np.full((1, 30, 40), 1.2), (np.full((1, 30, 40), 0.6),
                                      np.full((1, 30, 40), -0.3)), np.full((1, 30, 40), 0.8))
    s = fv.Solver(h)
    s.set_state(U)
    R = s.residual().cpu().numpy()
    s.step(5)
    U5 = s.get_state()
    s.close()
    assert np.abs(R).max() <= 1e-13
    assert np.abs(U5 - U).max() <= 1e-13
    f = fv.Solver(h)
    f.set_path(fv.FV_PATH_FUSED, 0, 0)
    f.set_state(U)
    f.step(5)
    F5 = f.get_state()
    f.close()
    assert np.abs(F5 - U).max() <= 1e-13


def test_identity_map_matches_the_uniform_grid_path():
    from paper_2306_14011_amd import fv
    g = inputs.grid2d(31, 23, hi=(1.5, 1.1), bc=((WALL, 1), (0, 0)))
    U = wavy_state(g, box_nodes(g), 4)
    out = []
    for spec in (g, curved(g, box_nodes(g))):
        s = fv.Solver(spec)
        s.set_state(U)
        out.append(s.residual().cpu().numpy())
        s.close()
    assert np.abs(out[1] - out[0]).max() <= 1e-14 * np.abs(out[0]).max()


def test_curvilinear_refusals():
    import torch
    from paper_2306_14011_amd import fv
    g = inputs.grid2d(12, 10)
    h = curved(g, box_nodes(g))
    s = fv.Solver(h)
    s.set_state(wavy_state(g, box_nodes(g), 5))
    lam = torch.ones(g.shape, dtype=torch.float64, device="cuda")
    dt = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    with pytest.raises(fv.FvError) as e:
        fv.fv_adjoint_step(s.ctx, s.U.data_ptr(), dt.data_ptr(), lam.data_ptr())
    assert e.value.code == fv.FV_ENOTSUP
    s.close()
    v = copy.copy(h)
    v.mu = 0.01
    with pytest.raises(fv.FvError) as e:
        fv.Solver(v)
    assert e.value.code == fv.FV_EINVAL
