"""The source term of Eq. (residual) on the HIP path against the FP64 oracle:
residual, split and fused steps in 2D and 3D, and the adjoint step whose
recomputed stage states carry the source. Inputs: the seeded smooth source of
`inputs.smooth_source` on the parity workloads' states."""
import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def assert_pervar_close(got, ref, tol, what):
    for v in range(ref.shape[0]):
        scale = max(np.abs(ref[v]).max(), 1e-300)
        err = np.abs(got[v] - ref[v]).max()
        assert err <= tol * scale, f"{what} var {v}: max err {err:.3e} vs scale {scale:.3e}"


def cases():
    g1, U1 = inputs.vortex_bumps_case(96, seed=3)
    g2 = inputs.grid2d(131, 70, bc=((1, 1), (0, 0)))          # ragged strips, transmissive x
    U2 = inputs.vortex_state(g2, inputs.vortex_centre(5), 3.0)
    g3 = inputs.grid3d(37, 22, 17)
    U3 = inputs.sod_state(g3, inputs.sod_rotated_normal(2), (0.5, 0.5, 0.5))
    return [("vortex_bumps_96", g1, U1), ("vortex_131x70", g2, U2), ("sod3d_37x22x17", g3, U3)]


CASES = cases()
IDS = [c[0] for c in CASES]


def solver(g, U, S, path=None):
    from paper_2306_14011_amd import fv
    s = fv.Solver(g)
    s.set_state(U)
    s.set_source(S)
    if path is not None:
        s.set_path(path, 0, 0)
    return s


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_residual_with_source_matches_oracle(name, g, U):
    S = inputs.smooth_source(g, 1)
    s = solver(g, U, S)
    R = s.residual().cpu().numpy()
    assert_pervar_close(R, oracle.residual(g, U, source=S), TOL, name)
    # removing the source gives back the plain residual, bitwise
    s.set_source(None)
    R0 = s.residual().cpu().numpy()
    s.close()
    from paper_2306_14011_amd import fv
    t = fv.Solver(g)
    t.set_state(U)
    assert np.array_equal(R0, t.residual().cpu().numpy())
    t.close()
    assert_pervar_close(R0, oracle.residual(g, U), TOL, name + " no source")


@pytest.mark.parametrize("path", ["split", "fused"])
@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_steps_with_source_match_oracle(name, g, U, path):
    import torch
    from paper_2306_14011_amd import fv
    S = inputs.smooth_source(g, 2)
    s = solver(g, U, S, fv.FV_PATH_FUSED if path == "fused" else None)
    n = 4
    dts = torch.zeros(n, dtype=torch.float64, device="cuda")
    s.step(n, dt_out=dts)
    rc, flags = s.status()
    got = s.get_state()
    s.close()
    ref, rdt, rfl = oracle.run(g, U, n, source=S)
    assert flags == 0 and rfl == 0
    # dt of every step comes from the wave speed of the state with the source's share
    assert np.allclose(dts.cpu().numpy(), rdt, rtol=1e-12, atol=0)
    assert_pervar_close(got, ref, TOL, f"{name} {path}")
    # and the source moved the result: not the source-free trajectory
    free, _, _ = oracle.run(g, U, n)
    assert np.abs(got - free).max() > 1e-6 * np.abs(free).max()


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_adjoint_step_with_source_matches_oracle(name, g, U):
    # on the unlimited scheme: the test is about the stage states the
    # derivative is taken at, and minmod's derivative jumps where a slope of
    # those states crosses zero, so two states a rounding apart can take
    # different branches (seen on the 131 x 70 case: 1e-16 agreement except a
    # few cells at 5e-3 relative); the minmod adjoint is checked on states
    # without such crossings in the adjoint tests
    import dataclasses

    import torch
    from paper_2306_14011_amd import fv
    g = dataclasses.replace(g, limiter=False)
    if g.ndim == 3:
        # the unlimited scheme over-shoots the Sod jump into negative pressure:
        # a smooth 3D state of the same grid instead
        W = inputs.smooth_source(g, 11, amp=0.05)
        U = inputs.primitive_to_conserved(g, 1.0 + W[0], (0.3 + W[1], 0.2 + W[2], 0.1 + W[3]), 1.0 + W[4])
    S = inputs.smooth_source(g, 3)
    rng = np.random.default_rng(4)
    dt = 0.8 * oracle.dt(g, U)[0]
    lam = rng.standard_normal(U.shape)
    s = solver(g, U, S)
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    L = torch.as_tensor(np.ascontiguousarray(lam)).cuda()
    fv.fv_adjoint_step(s.ctx, s.U.data_ptr(), dtt.data_ptr(), L.data_ptr())
    got = L.cpu().numpy()
    s.close()
    ref = oracle.rk3_step_vjp(g, U, dt, lam, limiter=False, source=S)
    for v in range(U.shape[0]):
        assert np.abs(got[v] - ref[v]).max() <= 1e-10 * np.abs(ref[v]).max(), (name, v)
    # the source changes the linearisation point, so the derivative differs from the source-free one
    free = oracle.rk3_step_vjp(g, U, dt, lam, limiter=False)
    assert np.abs(ref - free).max() > 1e-9 * np.abs(free).max()
