"""HIP path vs the FP64 oracle, through the C ABI.

Tolerance: per cell and variable, |gpu - oracle| <= 1e-12 * max_cells |oracle_v|
(a per-variable scale because the momenta cross zero). The binding check is
one step from an identical input; trajectories are checked too. Launch
configurations must give bitwise-identical states.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _fv():
    from paper_2306_14011_amd import fv
    return fv


def assert_pervar_close(got, ref, tol=TOL, what="", scales=None):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape
    for v in range(ref.shape[0]):
        scale = max(np.abs(ref[v]).max(), 1e-300) if scales is None else scales[v]
        err = np.abs(got[v] - ref[v]).max()
        assert err <= tol * scale, f"{what} var {v}: max err {err:.3e} vs scale {scale:.3e}"


def run_gpu(spec, U0, nsteps, dt_in=None, launch=None):
    import torch
    fv = _fv()
    s = fv.Solver(spec)
    if launch is not None:
        s.set_launch(launch)
    s.set_state(U0)
    dts = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda")
    dti = None
    if dt_in is not None:
        dti = torch.as_tensor(np.asarray(dt_in, dtype=np.float64)).cuda()
    s.step(nsteps, dt_in=dti, dt_out=dts)
    rc, flags = s.status()
    out = s.get_state()
    s.close()
    return out, dts.cpu().numpy()[:nsteps], flags


def gpu_residual(spec, U0, launch=None):
    fv = _fv()
    s = fv.Solver(spec)
    if launch is not None:
        s.set_launch(launch)
    s.set_state(U0)
    R = s.residual().cpu().numpy()
    s.close()
    return R


CASES_2D = [
    ("vortex64", lambda: inputs.vortex_case(64, seed=0)),
    ("ragged_bumps", lambda: (lambda g: (g, inputs.gaussian_bumps(g, inputs.vortex_state(g, (4.2, 5.7)), 1, amp=0.05)))(inputs.grid2d(77, 45))),
    ("transmissive_sod_x", lambda: (lambda g: (g, inputs.sod_axis_state(g, 0)))(inputs.grid2d(131, 3, bc=((1, 1), (0, 0))))),
    ("transmissive_sod_y", lambda: (lambda g: (g, inputs.sod_axis_state(g, 1)))(inputs.grid2d(2, 70, bc=((1, 1), (1, 1))))),
    ("tilted_sod_2d", lambda: (lambda g: (g, inputs.sod_state(g, (0.8, 0.6, 0.0), (0.5, 0.5, 0.0))))(inputs.grid2d(50, 41, hi=(1.0, 1.0), bc=((1, 1), (0, 0))))),
    ("single_cell_axis", lambda: (lambda g: (g, inputs.sod_axis_state(g, 0)))(inputs.grid2d(66, 1, bc=((1, 1), (0, 0))))),
]


def case_3d(n=(20, 17, 13), seed=3):
    g = inputs.grid3d(*n)
    return g, inputs.sod_state(g, inputs.sod_rotated_normal(seed), (0.5, 0.5, 0.5))


@pytest.mark.parametrize("name,make", CASES_2D, ids=[c[0] for c in CASES_2D])
def test_residual_matches_oracle_2d(name, make):
    g, U0 = make()
    assert_pervar_close(gpu_residual(g, U0), oracle.residual(g, U0), what=name)


def test_residual_matches_oracle_3d():
    g, U0 = case_3d()
    rng = np.random.default_rng(0)
    U0[1:4] += 0.1 * rng.standard_normal(U0[1:4].shape) * U0[0]
    assert_pervar_close(gpu_residual(g, U0), oracle.residual(g, U0), what="3d")


@pytest.mark.parametrize("name,make", CASES_2D, ids=[c[0] for c in CASES_2D])
def test_one_step_matches_oracle_2d(name, make):
    g, U0 = make()
    got, dts, flags = run_gpu(g, U0, 1)
    ref, rdts, rflags = oracle.run(g, U0, 1)
    assert flags == 0 and rflags == 0
    assert abs(dts[0] - rdts[0]) <= 1e-14 * rdts[0]
    assert_pervar_close(got, ref, what=name)


def test_one_step_matches_oracle_3d():
    g, U0 = case_3d()
    got, dts, flags = run_gpu(g, U0, 1)
    ref, rdts, _ = oracle.run(g, U0, 1)
    assert flags == 0
    assert abs(dts[0] - rdts[0]) <= 1e-14 * rdts[0]
    assert_pervar_close(got, ref, what="3d")


def test_vortex_100_steps_trajectory():
    # 64^2 periodic vortex, beta 5, CFL 0.5, 100 steps: the measured small case
    g, U0 = inputs.vortex_case(64, seed=0)
    got, dts, flags = run_gpu(g, U0, 100)
    ref, rdts, rflags = oracle.run(g, U0, 100)
    assert flags == 0 and rflags == 0
    assert np.allclose(dts, rdts, rtol=1e-12, atol=0)
    # every step is Lipschitz in its input, so per-step roundoff stays small
    assert_pervar_close(got, ref, tol=1e-11, what="100 steps")


def test_3d_sod_several_steps():
    g, U0 = case_3d((24, 18, 16), seed=7)
    got, dts, _ = run_gpu(g, U0, 5)
    ref, rdts, _ = oracle.run(g, U0, 5)
    assert np.allclose(dts, rdts, rtol=1e-12, atol=0)
    assert_pervar_close(got, ref, tol=1e-11, what="3d 5 steps")


def test_frozen_dt_path():
    g, U0 = inputs.vortex_case(40, seed=5)
    dt_in = np.array([0.011, 0.02, 0.005])
    got, dts, _ = run_gpu(g, U0, 3, dt_in=dt_in)
    ref, _, _ = oracle.run(g, U0, 3, dt_in=dt_in)
    assert np.array_equal(dts, dt_in)
    assert_pervar_close(got, ref, what="frozen dt")


def test_freestream_exact_on_gpu():
    g = inputs.grid3d(9, 11, 6, bc=((1, 1), (0, 0), (1, 1)))
    shp = g.shape[1:]
    U0 = inputs.primitive_to_conserved(g, np.full(shp, 1.3), (np.full(shp, 0.3), np.full(shp, -0.4), np.full(shp, 0.1)), np.full(shp, 0.8))
    R = gpu_residual(g, U0)
    assert np.all(R == 0.0)


def test_periodic_conservation_on_gpu():
    g, U0 = inputs.vortex_bumps_case(96, seed=2)
    got, _, _ = run_gpu(g, U0, 3)
    tot0 = U0.sum(axis=(1, 2, 3))
    tot1 = got.sum(axis=(1, 2, 3))
    assert np.allclose(tot1, tot0, rtol=1e-13, atol=1e-12)


def random_launch(rng, ndim):
    p = []
    for s in range(3):
        bx = int(2 ** rng.integers(4, 9))          # 16..256
        t = int(2 ** rng.integers(max(6, int(math.log2(bx))), 11))
        p += [bx, t]
    for s in range(4):
        gang = int(rng.choice([0, 1, 256, 512, 1024, 2048]))
        t = int(2 ** rng.integers(6, 11))
        p += [gang, t]
    return p


def test_launch_configurations_are_bitwise_invariant():
    fv = _fv()
    rng = np.random.default_rng(123)
    for g, U0 in (inputs.vortex_bumps_case(72, seed=1), case_3d((19, 14, 11), seed=2)):
        base, _, _ = run_gpu(g, U0, 2)
        for _ in range(12):
            p = random_launch(rng, g.ndim)
            got, _, _ = run_gpu(g, U0, 2, launch=p)
            assert np.array_equal(got, base), p


def test_invalid_launch_rejected_and_kept():
    fv = _fv()
    g, U0 = inputs.vortex_case(16)
    s = fv.Solver(g)
    before = s.get_launch()
    bad = list(before)
    bad[0] = 48  # not a power of two
    with pytest.raises(fv.FvError) as e:
        s.set_launch(bad)
    assert e.value.code == fv.FV_EINVAL
    assert s.get_launch() == before
    bad = list(before)
    bad[2], bad[3] = 512, 256   # block width above threads
    with pytest.raises(fv.FvError):
        s.set_launch(bad)
    assert s.get_launch() == before
    s.close()


def test_nonphysical_state_sets_flags():
    fv = _fv()
    g, U0 = inputs.vortex_case(32)
    bad = U0.copy()
    bad[3, 0, 5, 7] = -1.0        # negative pressure
    s = fv.Solver(g)
    s.set_state(bad)
    s.step(1)
    rc, flags = s.status()
    assert rc == fv.FV_ENONPHYS and flags & fv.FV_FLAG_P
    s.clear_status()
    s.set_state(U0)
    s.step(1)
    rc, flags = s.status()
    assert rc == fv.FV_OK and flags == 0
    bad = U0.copy()
    bad[0, 0, 1, 2] = float("nan")
    s.set_state(bad)
    s.step(1)
    rc, flags = s.status()
    assert flags & fv.FV_FLAG_NAN
    s.close()


def test_full_size_2d_one_step():
    # 2048^2 vortex + 32 Gaussian bumps, one step in the bench's default launch
    g, U0 = inputs.vortex_bumps_case(2048, seed=0)
    got, dts, flags = run_gpu(g, U0, 1)
    ref, rdts, _ = oracle.run(g, U0, 1)
    assert flags == 0
    assert abs(dts[0] - rdts[0]) <= 1e-14 * rdts[0]
    assert_pervar_close(got, ref, what="2048^2")


def sod256_front_origins(P, seed):
    """Patch origins on the tilted front of the 256^3 Sod workload: five at
    seeded (y, z), two across the periodic y seam and two across the z seam
    (where the tilted plane, not periodic itself, also jumps)."""
    from tests.patch_util import sod_front_origins
    n = 256
    normal = inputs.sod_rotated_normal(0)
    rng = np.random.default_rng(seed)
    out = sod_front_origins(n, normal, P, rng, 5)
    for i, o in enumerate(sod_front_origins(n, normal, P, rng, 4)):
        o = list(o)
        o[1 + i // 2] = n - P // 2      # the patch centre sits on the seam
        out.append(tuple(o))
    return out


def test_full_size_3d_sampled_patches():
    # 256^3 rotated Sod: one step on the GPU; the oracle recomputes 20^3
    # patches on the front and across the periodic seams with the GPU's dt
    # (a cell depends on cells at most 6 away, so the inner 8^3 are exact)
    from tests.patch_util import check_patches
    g, U0 = inputs.sod3d_case(256, seed=0)
    got, dts, flags = run_gpu(g, U0, 1)
    dt_ref, _ = oracle.dt(g, U0)
    assert flags == 0
    assert abs(dts[0] - dt_ref) <= 1e-14 * dt_ref
    n, worst = check_patches(got, U0, g, dts, sod256_front_origins(20, 9), 20, 6, min_change=1e-3,
                             what="split 256^3")
    print(n, worst)


def test_full_size_3d_three_steps_sampled_patches():
    # three steps at the GPU's dt sequence: 48^3 patches, exact in their inner
    # 12^3 (18 cells of halo for 3 steps x 3 stages x 2 cells)
    from tests.patch_util import check_patches
    g, U0 = inputs.sod3d_case(256, seed=0)
    got, dts, flags = run_gpu(g, U0, 3)
    assert flags == 0
    # the first dt is the oracle's on the full grid; the later ones depend on
    # the full state, so the patches take the GPU's sequence
    dt_ref, _ = oracle.dt(g, U0)
    assert abs(dts[0] - dt_ref) <= 1e-14 * dt_ref
    origins = sod256_front_origins(48, 17)[:4] + sod256_front_origins(48, 17)[5:7]
    n, worst = check_patches(got, U0, g, dts, origins, 48, 18, min_change=1e-3, what="split 256^3, 3 steps")
    print(n, worst)
