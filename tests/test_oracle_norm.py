"""The residual norm of the oracle (the convergence monitor of the relative
residual history of Sec. "A Test Case") pinned on hand-computed arrays."""
import numpy as np

import oracle
from paper_2306_14011_amd import inputs


def test_norm_of_hand_computed():
    # four variables over a 2 x 2 grid of cells; the norms are worked out by
    # hand: sqrt((9 + 16) / 4) = 2.5, sqrt(4 / 4) = 1, sqrt(16 / 4) = 2, sqrt(36 / 4) = 3
    R = np.array([[3.0, 4.0, 0.0, 0.0],
                  [1.0, 1.0, 1.0, 1.0],
                  [2.0, -2.0, 2.0, -2.0],
                  [0.0, 0.0, 0.0, 6.0]]).reshape(4, 1, 2, 2)
    assert np.array_equal(oracle.norm_of(R), [2.5, 1.0, 2.0, 3.0])
    # the cell count, not nvar * ncell, divides: a 3D layout of the same cells
    assert np.array_equal(oracle.norm_of(R.reshape(4, 2, 1, 2)), [2.5, 1.0, 2.0, 3.0])
    # five variables over three cells
    R5 = np.array([[1.0, 2.0, 2.0], [0.0, 0.0, 3.0], [0.0] * 3, [-3.0, 0.0, 0.0], [6.0, 6.0, 6.0]]).reshape(5, 1, 1, 3)
    assert np.allclose(oracle.norm_of(R5), [np.sqrt(3.0), np.sqrt(3.0), 0.0, np.sqrt(3.0), 6.0], rtol=1e-15, atol=0)


def test_residual_norm_is_norm_of_residual():
    g, U = inputs.vortex_bumps_case(48, seed=1)
    a = oracle.residual_norm(g, U)
    b = oracle.norm_of(oracle.residual(g, U))
    assert np.array_equal(a, b)
    assert np.all(a > 0)
    # a uniform state has a zero residual and so a zero norm
    Uf = np.broadcast_to(U[:, :, :1, :1], U.shape).copy()
    assert np.array_equal(oracle.residual_norm(g, Uf), np.zeros(4))
