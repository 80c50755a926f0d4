"""Residual L2 norm (the convergence monitor of the relative residual history
of Sec. "A Test Case") through the C ABI against the FP64 oracle, and a
convergence history on an inlet-like channel: supersonic inflow at an angle
into slip walls, outflow, from a disturbed free stream."""
import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

pytestmark = pytest.mark.gpu


def cases():
    import tests.test_gpu_inflow as T
    g1, U1 = inputs.vortex_bumps_case(96, seed=3)
    g3 = inputs.grid3d(23, 14, 11)
    U3 = inputs.sod_state(g3, inputs.sod_rotated_normal(2), (0.5, 0.5, 0.5))
    return [("vortex_bumps_96", g1, U1), T.CASES[0], ("sod3d", g3, U3)]


CASES = cases()
IDS = [c[0] for c in CASES]


@pytest.mark.parametrize("name,g,U", CASES, ids=IDS)
def test_norm_matches_oracle(name, g, U):
    from paper_2306_14011_amd import fv
    s = fv.Solver(g)
    s.set_state(U)
    a = s.residual_norm()
    b = s.residual_norm()
    assert np.array_equal(a, b)                      # fixed summation order
    ref = oracle.residual_norm(g, U)
    assert np.allclose(a, ref, rtol=1e-12, atol=0), (a, ref)
    s.step(10)
    U10, _, _ = oracle.run(g, U, 10)
    assert np.allclose(s.residual_norm(), oracle.residual_norm(g, U10), rtol=1e-9, atol=0)
    s.close()


def test_inlet_channel_converges():
    from paper_2306_14011_amd import fv
    name, g, U = CASES[1]
    s = fv.Solver(g)
    s.set_state(U)
    hist = [s.residual_norm()]
    for _ in range(8):
        s.step(100)
        hist.append(s.residual_norm())
    rc, flags = s.status()
    s.close()
    assert flags == 0
    rel = np.array(hist) / hist[0]
    print(rel[:, 0])
    # the disturbance leaves through the outflow: the relative residual of
    # every variable falls by more than three orders over 800 steps (the
    # oracle: 3.1e-1, 1.2e-1, ... 1.8e-4 for the density)
    assert np.all(rel[-1] < 1e-3), rel[-1]
    assert np.all(rel[6] < rel[2])
