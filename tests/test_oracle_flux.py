"""Pins of the oracle's face-level pieces: limiter, MUSCL, physical and Roe flux.

Each check is fixed by the mathematics (hand-computed values, textbook
identities, symmetries), never by re-running the oracle's own formula.
"""
import math

import numpy as np
import pytest

import oracle

GAM = 1.4


def textbook_minmod(a, b):
    """minmod(a, b): zero unless a and b share a strict sign, else the smaller magnitude."""
    if a > 0 and b > 0:
        return min(a, b)
    if a < 0 and b < 0:
        return max(a, b)
    return 0.0


@pytest.mark.parametrize("num,den", [
    (1.0, 2.0), (2.0, 1.0), (-1.0, -4.0), (-4.0, -1.0), (3.0, -1.0), (-3.0, 1.0),
    (0.0, 1.0), (1.0, 0.0), (0.0, 0.0), (2.0, 2.0), (-0.5, -0.5), (0.75, 3.0),
    (5e-310, 1e-300), (1e300, 1e-300), (-8.0, 0.25),
])
def test_limited_slope_is_minmod(num, den):
    # Psi(num/den)*den with the minmod Psi is minmod(den, num); dyadic values make it exact
    assert oracle.limited(num, den) == textbook_minmod(den, num)


def test_psi_minmod_shape():
    assert oracle.psi_minmod(-2.0) == 0.0
    assert oracle.psi_minmod(0.0) == 0.0
    assert oracle.psi_minmod(0.25) == 0.25
    assert oracle.psi_minmod(1.0) == 1.0
    assert oracle.psi_minmod(7.0) == 1.0
    assert oracle.limited(3.0, 1.0, limiter=False) == 1.0  # Psi = 1 when the limiter is off


def test_muscl_hand_values():
    # linear data: both face states are the exact midpoint value, for any kappa
    for kappa in (-1.0, 0.0, 1.0 / 3.0, 1.0):
        assert oracle.muscl(0.0, 1.0, 2.0, 3.0, kappa=kappa) == (1.5, 1.5)
    # one-sided data 0, 0, 1, 3 with kappa = -1, limiter off:
    #   QL = 0 + (0 - 0)/2 = 0,  QR = 1 - (3 - 1)/2 = 0
    assert oracle.muscl(0.0, 0.0, 1.0, 3.0, limiter=False) == (0.0, 0.0)
    # same data, minmod: QL = 0 + minmod(0, 1)/2 = 0, QR = 1 - minmod(2, 1)/2 = 0.5
    assert oracle.muscl(0.0, 0.0, 1.0, 3.0) == (0.0, 0.5)
    # a local maximum at k: the left state falls back to first order
    qL, qR = oracle.muscl(0.0, 2.0, 1.0, 0.0)
    assert qL == 2.0 and qR == 1.0 - 0.5 * textbook_minmod(-1.0, -1.0)
    # kappa = 1, limiter off: central average of Q_k and Q_{k+1} on both sides
    assert oracle.muscl(5.0, 1.0, 3.0, -7.0, limiter=False, kappa=1.0) == (2.0, 2.0)


def test_muscl_kappa_family_pins():
    """Eq. (flux) with epsilon = 1. (a) With the minmod limiter Psi+ and Psi-
    give the same limited difference (minmod is symmetric), so kappa drops
    out: every kappa gives Q_k + minmod / 2. (b) kappa = 1/3 without limiter
    reproduces the face value of a quadratic from its cell averages (third
    order): averages of x^2 over unit cells centred on -1, 0, 1, 2 are
    k^2 + 1/12, and both states at x = 1/2 are 1/4. (c) kappa = 0 (Fromm)
    uses the central difference (Q_{k+1} - Q_{k-1}) / 4."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        q = rng.normal(size=4)
        base = oracle.muscl(*q, kappa=-1.0)
        for kappa in (0.0, 1.0 / 3.0, 1.0):
            got = oracle.muscl(*q, kappa=kappa)
            assert np.allclose(got, base, rtol=1e-15, atol=1e-15), (q, kappa)
    avg = [k * k + 1.0 / 12.0 for k in (-1, 0, 1, 2)]
    qL, qR = oracle.muscl(*avg, limiter=False, kappa=1.0 / 3.0)
    assert abs(qL - 0.25) < 1e-15 and abs(qR - 0.25) < 1e-15
    # the other members are not exact for it: kappa = -1 gives 1/12 + 1/2 (1/12 - 13/12)
    qL_up, _ = oracle.muscl(*avg, limiter=False, kappa=-1.0)
    assert abs(qL_up - (1.0 / 12.0 - 0.5)) < 1e-15
    qL0, qR0 = oracle.muscl(0.0, 1.0, 5.0, 2.0, limiter=False, kappa=0.0)
    assert qL0 == 1.0 + (5.0 - 0.0) / 4.0 and qR0 == 5.0 - (2.0 - 1.0) / 4.0


def test_muscl_quick_member_pin():
    """kappa = 1/2 without limiter is Leonard's QUICK: quadratic upstream
    interpolation, exact for point values of any quadratic. With q(x) =
    a + b x + c x^2 sampled at the cell centres -1, 0, 1, 2, both states at
    the face x = 1/2 equal q(1/2); kappa = 1/3 (exact for cell averages) and
    kappa = -1 miss it by multiples of c."""
    rng = np.random.default_rng(11)
    for _ in range(100):
        a, b, c = rng.normal(size=3)
        pts = [a + b * x + c * x * x for x in (-1.0, 0.0, 1.0, 2.0)]
        exact = a + 0.5 * b + 0.25 * c
        qL, qR = oracle.muscl(*pts, limiter=False, kappa=0.5)
        assert abs(qL - exact) <= 1e-14 * (1 + abs(exact)) and abs(qR - exact) <= 1e-14 * (1 + abs(exact))
        # kappa = 1/3 is off by c / 12 on the left (point values, not averages)
        qL3, _ = oracle.muscl(*pts, limiter=False, kappa=1.0 / 3.0)
        assert abs((qL3 - exact) - (-c / 12.0)) <= 1e-13 * (1 + abs(c))
    # the hand value of x^2 at 1/2 from 1, 0, 1, 4: 0 + (1/8)(0 - 1) + (3/8)(1 - 0)
    assert oracle.muscl(1.0, 0.0, 1.0, 4.0, limiter=False, kappa=0.5) == (0.25, 0.25)


def test_van_leer_limiter_pins():
    """van Leer's Psi(r) = (r + |r|)/(1 + |r|): Psi(1) = 1, zero for r <= 0,
    symmetric (Psi(r)/r = Psi(1/r)), inside Sweby's second-order TVD region
    (between minmod and superbee), and its limited difference is the harmonic
    form 2ab/(a + b) for slopes of one sign. Being symmetric, it makes kappa
    drop out of Eq. (flux) as minmod does."""
    assert oracle.psi_vanleer(1.0) == 1.0
    assert oracle.psi_vanleer(0.0) == 0.0 and oracle.psi_vanleer(-3.0) == 0.0
    assert oracle.psi_vanleer(3.0) == 1.5
    rng = np.random.default_rng(8)
    for r in np.exp(rng.uniform(-6, 6, 200)):
        psi = oracle.psi_vanleer(r)
        assert abs(psi / r - oracle.psi_vanleer(1.0 / r)) <= 1e-15 * max(1.0, psi / r)
        lo = min(r, 1.0)
        hi = max(min(2.0 * r, 1.0), min(r, 2.0))
        assert lo - 1e-15 <= psi <= hi + 1e-15, r
    assert oracle.limited(3.0, 1.0, "vanleer") == 1.5      # 2*3*1/(3+1)
    assert oracle.limited(-2.0, -6.0, "vanleer") == -3.0   # 2*(-2)(-6)/(-8)
    assert oracle.limited(2.0, -1.0, "vanleer") == 0.0
    assert oracle.limited(0.0, 5.0, "vanleer") == 0.0
    # hand face states: cells 0, 1, 4, 5: QL = 1 + vl(1, 3)/2 = 1.75, QR = 4 - vl(3, 1)/2 = 3.25
    for kappa in (-1.0, 0.0, 1.0 / 3.0, 1.0):
        assert oracle.muscl(0.0, 1.0, 4.0, 5.0, limiter="vanleer", kappa=kappa) == (1.75, 3.25)
    for _ in range(100):
        q = rng.normal(size=4)
        base = oracle.muscl(*q, limiter="vanleer")
        assert np.allclose(oracle.muscl(*q, limiter="vanleer", kappa=1.0 / 3.0), base, rtol=1e-15, atol=1e-15)


def test_physical_flux_hand_values():
    # rho = 1, u = (2, 0), p = 1 -> E = 1/0.4 + 0.5*4 = 4.5
    Q = [1.0, 2.0, 0.0, 4.5]
    assert np.allclose(oracle.phys_flux(2, 0, Q), [2.0, 5.0, 0.0, 11.0], rtol=0, atol=1e-14)
    assert np.allclose(oracle.phys_flux(2, 1, Q), [0.0, 0.0, 1.0, 0.0], rtol=0, atol=1e-14)
    # 3D: rho = 2, u = (1, -1, 0.5), p = 3: E = 3/0.4 + 0.5*2*2.25 = 9.75
    Q = [2.0, 2.0, -2.0, 1.0, 9.75]
    Fz = oracle.phys_flux(3, 2, Q)
    assert np.allclose(Fz, [1.0, 1.0, -1.0, 0.5 + 3.0, (9.75 + 3.0) * 0.5], rtol=0, atol=1e-14)


def random_state(rng, ndim, mach_max=0.8):
    rho = rng.uniform(0.2, 3.0)
    p = rng.uniform(0.2, 3.0)
    c = math.sqrt(GAM * p / rho)
    u = rng.uniform(-1, 1, ndim) * mach_max * c / math.sqrt(ndim)
    return np.array([rho, *(rho * u), p / (GAM - 1) + 0.5 * rho * (u @ u)])


@pytest.mark.parametrize("ndim", [2, 3])
def test_roe_consistency_bitwise(ndim):
    rng = np.random.default_rng(1)
    for _ in range(50):
        Q = random_state(rng, ndim)
        for ax in range(ndim):
            assert np.array_equal(oracle.roe_flux(ndim, ax, Q, Q), oracle.phys_flux(ndim, ax, Q))


def supersonic_pair(rng, ndim, ax, sign):
    """Two states whose normal velocity exceeds the sound speed on both sides."""
    out = []
    for _ in range(2):
        rho = rng.uniform(0.5, 2.0)
        p = rng.uniform(0.5, 2.0)
        c = math.sqrt(GAM * p / rho)
        u = rng.uniform(-0.3, 0.3, ndim) * c
        u[ax] = sign * rng.uniform(3.0, 5.0) * c
        out.append(np.array([rho, *(rho * u), p / (GAM - 1) + 0.5 * rho * (u @ u)]))
    return out


@pytest.mark.parametrize("ndim", [2, 3])
def test_roe_supersonic_upwinding(ndim):
    # all Roe wave speeds > 0: sum_k lambda_k alpha_k r_k = F(QR) - F(QL) (Roe's property),
    # hence F = F(QL); all < 0 gives F(QR). This pins every wave strength, speed and
    # eigenvector component of the dissipation term.
    rng = np.random.default_rng(2)
    for _ in range(40):
        for ax in range(ndim):
            QL, QR = supersonic_pair(rng, ndim, ax, +1)
            F = oracle.roe_flux(ndim, ax, QL, QR)
            FL = oracle.phys_flux(ndim, ax, QL)
            assert np.allclose(F, FL, rtol=1e-12, atol=1e-12 * np.abs(FL).max())
            QL, QR = supersonic_pair(rng, ndim, ax, -1)
            F = oracle.roe_flux(ndim, ax, QL, QR)
            FR = oracle.phys_flux(ndim, ax, QR)
            assert np.allclose(F, FR, rtol=1e-12, atol=1e-12 * np.abs(FR).max())


def test_roe_stationary_contact_exact():
    # density jump at rest with equal pressure: Roe's flux keeps the contact exactly
    p = 0.7
    QL = np.array([1.0, 0.0, 0.0, p / (GAM - 1)])
    QR = np.array([0.125, 0.0, 0.0, p / (GAM - 1)])
    F = oracle.roe_flux(2, 0, QL, QR)
    assert np.allclose(F, [0.0, p, 0.0, 0.0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("ndim", [2, 3])
def test_roe_mirror_symmetry(ndim):
    # reflecting the normal axis and swapping sides flips the sign of every flux
    # component except the normal momentum
    rng = np.random.default_rng(3)
    for _ in range(40):
        for ax in range(ndim):
            QL = random_state(rng, ndim, 1.5)
            QR = random_state(rng, ndim, 1.5)
            M = np.ones(ndim + 2)
            M[1 + ax] = -1.0
            F = oracle.roe_flux(ndim, ax, QL, QR)
            Fm = oracle.roe_flux(ndim, ax, QR * M, QL * M)
            assert np.allclose(Fm, -F * M, rtol=1e-13, atol=1e-13 * np.abs(F).max())


@pytest.mark.parametrize("ndim", [2, 3])
def test_roe_axis_permutation(ndim):
    # the flux along axis a of a state equals the x flux of the state with the
    # velocity components of axes a and 0 exchanged, components exchanged back
    rng = np.random.default_rng(4)
    for _ in range(40):
        QL = random_state(rng, ndim, 1.5)
        QR = random_state(rng, ndim, 1.5)
        for ax in range(1, ndim):
            perm = list(range(ndim + 2))
            perm[1], perm[1 + ax] = perm[1 + ax], perm[1]
            Fa = oracle.roe_flux(ndim, ax, QL, QR)
            F0 = oracle.roe_flux(ndim, 0, QL[perm], QR[perm])
            # bitwise in 2D; in 3D |u|^2 is summed in another order, so roundoff
            assert np.allclose(Fa, F0[perm], rtol=1e-14, atol=1e-14 * np.abs(Fa).max())


def test_roe_upwind_limit_small_jump():
    # for a small jump the Roe flux approaches F(Q) - |A| dQ / 2 with A the flux Jacobian;
    # checked against a finite-difference Jacobian of the physical flux, eigen-decomposed
    rng = np.random.default_rng(5)
    Q = random_state(rng, 2)
    dQ = rng.standard_normal(4) * 1e-6
    QL, QR = Q - dQ / 2, Q + dQ / 2
    h = 1e-7
    A = np.zeros((4, 4))
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        A[:, j] = (oracle.phys_flux(2, 0, Q + e) - oracle.phys_flux(2, 0, Q - e)) / (2 * h)
    w, V = np.linalg.eig(A)
    absA = (V @ np.diag(np.abs(w)) @ np.linalg.inv(V)).real
    expect = 0.5 * (oracle.phys_flux(2, 0, QL) + oracle.phys_flux(2, 0, QR)) - 0.5 * absA @ dQ
    F = oracle.roe_flux(2, 0, QL, QR)
    assert np.allclose(F, expect, rtol=0, atol=1e-11)
