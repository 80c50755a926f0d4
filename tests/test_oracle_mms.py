"""Pins of the oracle's source term (Eq. (residual)) with a manufactured
solution: the analytic source against finite differences of the flux, the
residual's truncation error at second order, the source entering as
-|Omega| S, and a manufactured steady state held by the time stepper."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from oracle import mms

GAMMA = 1.4


def unit_square(n):
    return SimpleNamespace(ndim=2, n=(n, n, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                           bc=((0, 0), (0, 0), (0, 0)), gamma=GAMMA, cfl=0.5)


def flux(Q, ax):
    """Inviscid flux of Eq. (QF) along x (ax 0) or y (ax 1), textbook form."""
    r, mx, my, E = Q
    u, v = mx / r, my / r
    p = (GAMMA - 1.0) * (E - 0.5 * r * (u * u + v * v))
    vn = u if ax == 0 else v
    return np.stack([r * vn, mx * vn + (p if ax == 0 else 0.0), my * vn + (p if ax == 1 else 0.0), (E + p) * vn])


def test_source_is_the_flux_divergence():
    rng = np.random.default_rng(0)
    x, y = rng.random(200), rng.random(200)
    h = 1e-5
    fd = ((flux(mms.conserved(x + h, y), 0) - flux(mms.conserved(x - h, y), 0)) / (2 * h)
          + (flux(mms.conserved(x, y + h), 1) - flux(mms.conserved(x, y - h), 1)) / (2 * h))
    S = mms.source(x, y)
    for v in range(4):
        assert np.abs(S[v] - fd[v]).max() <= 1e-7 * np.abs(S[v]).max(), v
    # not a trivial field: every component of the source is O(1)
    assert all(np.abs(S[v]).max() > 0.1 for v in range(4))


def test_cell_averages_of_a_constant_and_of_a_mode():
    n = 16
    one = mms.cell_averages(lambda X, Y: np.stack([np.ones_like(X)] * 4), n)
    assert np.allclose(one, 1.0, rtol=0, atol=1e-15)
    avg = mms.cell_averages(lambda X, Y: np.stack([np.sin(2 * math.pi * X)] * 4), n)[0]
    i = np.arange(n)
    exact = (np.cos(2 * math.pi * i / n) - np.cos(2 * math.pi * (i + 1) / n)) * n / (2 * math.pi)
    assert np.allclose(avg, exact[None, :], rtol=0, atol=1e-12)


def test_source_enters_as_minus_volume_times_s():
    n = 24
    spec = unit_square(n)
    U = mms.cell_averages(mms.conserved, n)
    S = np.random.default_rng(1).standard_normal((4, n, n))
    R0 = oracle.residual(spec, U)
    R1 = oracle.residual(spec, U, source=S)
    vol = 1.0 / n ** 2
    assert np.allclose(R1 - R0, -vol * S, rtol=0, atol=4e-16 * np.abs(R0).max())
    with pytest.raises(ValueError):
        oracle.residual(spec, U, source=S[:3])


@pytest.mark.parametrize("limiter,lo,hi", [(False, 1.85, 2.25), (True, 1.3, 2.25)])
def test_truncation_error_order(limiter, lo, hi):
    # residual of the cell-averaged manufactured solution with its cell-averaged
    # source, per unit volume: the truncation error, O(h^2) for the unlimited
    # kappa = -1 scheme; minmod clips the slopes at the field's extrema
    errs = []
    for n in (32, 64, 128):
        spec = unit_square(n)
        U = mms.cell_averages(mms.conserved, n)
        S = mms.cell_averages(mms.source, n)
        te = oracle.residual(spec, U, limiter=limiter, source=S) * n ** 2
        errs.append(np.sqrt((te ** 2).mean(axis=(1, 2))))
        if n == 32:
            # without the source the residual is the O(1) flux divergence
            r0 = oracle.residual(spec, U, limiter=limiter) * n ** 2
            assert np.sqrt((r0 ** 2).mean()) > 10 * np.sqrt((te ** 2).mean())
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    print(limiter, errs, orders)
    assert np.all(orders[-1] >= lo) and np.all(orders[-1] <= hi), orders


def test_manufactured_steady_state_is_held():
    # with its source the manufactured state drifts by the truncation error
    # only; without it, it moves at the rate of the flux divergence
    n = 32
    spec = unit_square(n)
    U0 = mms.cell_averages(mms.conserved, n)
    S = mms.cell_averages(mms.source, n)
    U1, dts, fl = oracle.run(spec, U0, 20, limiter=False, source=S)
    U2, _, _ = oracle.run(spec, U0, 20, limiter=False)
    assert fl == 0 and dts.min() > 0
    d_src = np.abs(U1 - U0).max()
    d_free = np.abs(U2 - U0).max()
    assert d_src * 30 < d_free, (d_src, d_free)


def flux3(Q, ax):
    r, m, E = Q[0], Q[1:4], Q[4]
    V = m / r
    p = (GAMMA - 1.0) * (E - 0.5 * r * (V * V).sum(axis=0))
    out = [r * V[ax]] + [m[i] * V[ax] + (p if i == ax else 0.0) for i in range(3)] + [(E + p) * V[ax]]
    return np.stack(out)


def test_3d_source_is_the_flux_divergence():
    rng = np.random.default_rng(5)
    x, y, z = rng.random(150), rng.random(150), rng.random(150)
    h = 1e-5
    e = [np.array([h, 0, 0]), np.array([0, h, 0]), np.array([0, 0, h])]
    fd = 0.0
    for ax in range(3):
        hp = mms.conserved3(x + e[ax][0], y + e[ax][1], z + e[ax][2])
        hm = mms.conserved3(x - e[ax][0], y - e[ax][1], z - e[ax][2])
        fd = fd + (flux3(hp, ax) - flux3(hm, ax)) / (2 * h)
    S = mms.source3(x, y, z)
    for v in range(5):
        assert np.abs(S[v] - fd[v]).max() <= 1e-7 * np.abs(S[v]).max(), v


def test_3d_truncation_error_is_second_order():
    errs = []
    for n in (24, 48):
        spec = SimpleNamespace(ndim=3, n=(n, n, n), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                               bc=((0, 0), (0, 0), (0, 0)), gamma=GAMMA, cfl=0.5)
        U = mms.cell_averages3(mms.conserved3, n)
        S = mms.cell_averages3(mms.source3, n)
        te = oracle.residual(spec, U, limiter=False, source=S) * n ** 3
        errs.append(np.sqrt((te ** 2).mean(axis=(1, 2, 3))))
    orders = np.log2(errs[0] / errs[1])
    print(orders)
    assert np.all(orders > 1.85) and np.all(orders < 2.3), orders   # 12 -> 24 is not yet asymptotic (w: 1.67)
