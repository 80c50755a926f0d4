"""FP64 CPU oracle: plain, slow, obviously correct reference results.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the bench's
CPU-baseline leg import this package. The HIP product path never imports,
links or calls it, and it shares no code with that path: both sides take the
same seeded inputs from ``paper_2306_14011_amd.inputs`` and nothing else.

Contents:
  * ``liboracle.so`` (from ``fv_oracle.cpp``): MUSCL-minmod, Roe flux, residual,
    CFL wave-speed reduction and SSP-RK3 step (Eq. QF, residual, flux of the
    paper), complex-step derivatives of the residual and the step, and the
    reverse-mode gradient of the residual and of one step at frozen dt.
  * ``exact.py``: Toro's exact Riemann solver for the Sod tube.
  * ``mlp.py``: the runtime-regression network of the autotuner in FP64.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

c_double_p = ctypes.POINTER(ctypes.c_double)
c_u32_p = ctypes.POINTER(ctypes.c_uint32)


class OrGrid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("source", ctypes.c_void_p),
        ("bc_state", ((ctypes.c_double * 5) * 2) * 3),
        ("mu", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("nodes", ctypes.c_void_p),
    ]


FLAG_NAN = 1
FLAG_RHO = 2
FLAG_P = 4


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        L.or_psi_minmod.restype = ctypes.c_double
        L.or_psi_minmod.argtypes = [ctypes.c_double]
        L.or_psi_vanleer.restype = ctypes.c_double
        L.or_psi_vanleer.argtypes = [ctypes.c_double]
        L.or_limited.restype = ctypes.c_double
        L.or_limited.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.or_muscl.restype = None
        L.or_muscl.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, ctypes.c_double, c_double_p, c_double_p]
        L.or_phys_flux.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, c_double_p, c_double_p]
        L.or_roe_flux.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, c_double_p, c_double_p, c_double_p]
        g = ctypes.POINTER(OrGrid)
        L.or_residual.argtypes = [g, c_double_p, c_double_p]
        L.or_residual_cs.argtypes = [g, c_double_p, c_double_p, ctypes.c_double, c_double_p, c_double_p]
        L.or_max_wavespeed.restype = ctypes.c_double
        L.or_max_wavespeed.argtypes = [g, c_double_p, c_u32_p]
        L.or_dt.restype = ctypes.c_double
        L.or_dt.argtypes = [g, c_double_p, c_u32_p]
        L.or_rk3_step.argtypes = [g, c_double_p, ctypes.c_double]
        L.or_rk3_step_cs.argtypes = [g, c_double_p, c_double_p, ctypes.c_double, ctypes.c_double,
                                     c_double_p, c_double_p]
        L.or_run.argtypes = [g, c_double_p, ctypes.c_int32, c_double_p, c_double_p, c_u32_p]
        L.or_residual_vjp.argtypes = [g, c_double_p, c_double_p, c_double_p]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_max_threads.restype = ctypes.c_int
        L.or_visc_face_flux.argtypes = [g, c_double_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, c_double_p]
        L.or_rk3_step_vjp.argtypes = [g, c_double_p, ctypes.c_double, c_double_p]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(c_double_p)


def limiter_code(limiter):
    """OrGrid.limiter of a limiter choice: True or "minmod" -> 1, "vanleer" -> 2,
    False or None -> 0 (Psi = 1)."""
    if limiter == "vanleer":
        return 2
    if limiter is True or limiter == "minmod":
        return 1
    if limiter is False or limiter is None:
        return 0
    raise ValueError(f"unknown limiter {limiter!r}")


def make_grid(spec, limiter=True, kappa=-1.0, source=None):
    """OrGrid from any object with ndim, n, lo, hi, bc, gamma, cfl attributes.
    source: cell-averaged source S, shape (nvar, nz, ny, nx) or (nvar, ny, nx),
    or None for S = 0 (Eq. residual)."""
    g = OrGrid()
    for d in range(spec.ndim):
        if 2 in (int(spec.bc[d][0]), int(spec.bc[d][1])) and int(spec.n[d]) < 2:
            raise ValueError("a slip wall needs at least 2 cells on its axis")
    if source is not None:
        src = np.ascontiguousarray(source, dtype=np.float64)
        if src.size != (spec.ndim + 2) * int(np.prod([int(v) for v in spec.n])):
            raise ValueError("source has the wrong number of cells or variables")
        g._source_ref = src          # kept alive with the struct
        g.source = src.ctypes.data
    g.ndim = spec.ndim
    g.limiter = limiter_code(limiter)
    for d in range(3):
        g.n[d] = int(spec.n[d])
        g.dx[d] = (spec.hi[d] - spec.lo[d]) / spec.n[d]
        g.bc[d][0] = int(spec.bc[d][0])
        g.bc[d][1] = int(spec.bc[d][1])
    g.gamma = float(spec.gamma)
    g.cfl = float(spec.cfl)
    g.kappa = float(kappa)
    g.mu = float(getattr(spec, "mu", 0.0))
    g.prandtl = float(getattr(spec, "prandtl", 0.72))
    if g.mu < 0.0 or not g.prandtl > 0.0:
        raise ValueError("viscosity must be >= 0 and the Prandtl number > 0")
    nodes = getattr(spec, "nodes", None)
    if nodes is not None:
        if spec.ndim != 2:
            raise NotImplementedError("curvilinear grids are 2D here")
        if g.mu > 0.0:
            raise NotImplementedError("the viscous flux is taken on uniform grids only")
        nd = np.ascontiguousarray(nodes, dtype=np.float64)
        if nd.shape != (2, int(spec.n[1]) + 1, int(spec.n[0]) + 1):
            raise ValueError("nodes must have shape (2, ny + 1, nx + 1)")
        g._nodes_ref = nd
        g.nodes = nd.ctypes.data
    st = getattr(spec, "bc_state", None)
    if st is not None:
        st = np.asarray(st, dtype=np.float64)
        for a in range(3):
            for sd in range(2):
                for v in range(min(5, st.shape[2])):
                    g.bc_state[a][sd][v] = float(st[a, sd, v])
    return g


def _arr(U):
    return np.ascontiguousarray(U, dtype=np.float64)


def psi_minmod(r):
    return lib().or_psi_minmod(float(r))


def psi_vanleer(r):
    return lib().or_psi_vanleer(float(r))


def limited(num, den, limiter=True):
    return lib().or_limited(float(num), float(den), limiter_code(limiter))


def muscl(qm1, q0, qp1, qp2, limiter=True, kappa=-1.0):
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().or_muscl(qm1, q0, qp1, qp2, limiter_code(limiter), kappa, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def phys_flux(ndim, ax, Q, gamma=1.4):
    Q = _arr(Q)
    F = np.zeros(ndim + 2)
    lib().or_phys_flux(ndim, ax, gamma, _p(Q), _p(F))
    return F


def roe_flux(ndim, ax, QL, QR, gamma=1.4):
    QL = _arr(QL)
    QR = _arr(QR)
    F = np.zeros(ndim + 2)
    lib().or_roe_flux(ndim, ax, gamma, _p(QL), _p(QR), _p(F))
    return F


def residual(spec, U, limiter=True, kappa=-1.0, source=None):
    g = make_grid(spec, limiter, kappa, source)
    U = _arr(U)
    R = np.zeros_like(U)
    lib().or_residual(ctypes.byref(g), _p(U), _p(R))
    return R


def norm_of(R):
    """Per-variable L2 norm of a residual array R of shape (nvar, cells...):
    norm_v = sqrt(sum over the cells of R_v^2 / ncell), ncell being the number
    of cells (not nvar * ncell). The convergence monitor behind the relative
    residual history of Sec. "A Test Case"; the paper gives no normalisation,
    and the relative history (each norm over the first) does not depend on it."""
    R = np.asarray(R, dtype=np.float64)
    R = R.reshape(R.shape[0], -1)
    return np.sqrt((R * R).sum(axis=1) / R.shape[1])


def residual_norm(spec, U, limiter=True, kappa=-1.0, source=None):
    """Per-variable L2 norm of the residual of U (``norm_of`` of ``residual``)."""
    return norm_of(residual(spec, U, limiter, kappa, source))


def residual_cs(spec, U, V, h=1e-30, limiter=True):
    g = make_grid(spec, limiter)
    U = _arr(U)
    V = _arr(V)
    R = np.zeros_like(U)
    dR = np.zeros_like(U)
    lib().or_residual_cs(ctypes.byref(g), _p(U), _p(V), h, _p(R), _p(dR))
    return R, dR


def visc_face_flux(spec, U, ax, i, j, k=0):
    """Viscous flux F_nu,n (Eq. QF, n = e_ax) through the face between cell
    (i, j, k) and its neighbour along axis ax (indices may lie one cell
    outside the grid: they go through the boundary maps)."""
    g = make_grid(spec)
    U = _arr(U)
    F = np.zeros(spec.ndim + 2)
    lib().or_visc_face_flux(ctypes.byref(g), _p(U), int(ax), int(i), int(j), int(k), _p(F))
    return F


def max_wavespeed(spec, U):
    g = make_grid(spec)
    U = _arr(U)
    fl = ctypes.c_uint32(0)
    lam = lib().or_max_wavespeed(ctypes.byref(g), _p(U), ctypes.byref(fl))
    return lam, fl.value


def dt(spec, U):
    g = make_grid(spec)
    U = _arr(U)
    fl = ctypes.c_uint32(0)
    v = lib().or_dt(ctypes.byref(g), _p(U), ctypes.byref(fl))
    return v, fl.value


def rk3_step(spec, U, dt_, limiter=True, kappa=-1.0, source=None):
    g = make_grid(spec, limiter, kappa, source)
    U = _arr(U).copy()
    lib().or_rk3_step(ctypes.byref(g), _p(U), float(dt_))
    return U


def rk3_step_cs(spec, U, V, dt_, h=1e-30, limiter=True):
    g = make_grid(spec, limiter)
    U = _arr(U)
    V = _arr(V)
    Un = np.zeros_like(U)
    dUn = np.zeros_like(U)
    lib().or_rk3_step_cs(ctypes.byref(g), _p(U), _p(V), h, float(dt_), _p(Un), _p(dUn))
    return Un, dUn


def run(spec, U, nsteps, dt_in=None, limiter=True, kappa=-1.0, source=None):
    """Advance ``nsteps`` SSP-RK3 steps; returns (U, dt per step, flags)."""
    g = make_grid(spec, limiter, kappa, source)
    U = _arr(U).copy()
    dts = np.zeros(max(nsteps, 1))
    fl = ctypes.c_uint32(0)
    dti = None
    if dt_in is not None:
        dti = _arr(dt_in)
    lib().or_run(ctypes.byref(g), _p(U), int(nsteps), _p(dti) if dti is not None else None,
                 _p(dts), ctypes.byref(fl))
    return U, dts[:nsteps], fl.value


def _inviscid_only(spec):
    if getattr(spec, "mu", 0.0) > 0.0:
        raise NotImplementedError("the reverse gradient covers the inviscid residual only")
    if getattr(spec, "nodes", None) is not None:
        raise NotImplementedError("the reverse gradient covers uniform grids only")


def residual_vjp(spec, U, w, limiter=True):
    """(dR/dU)^T w."""
    _inviscid_only(spec)
    g = make_grid(spec, limiter)
    U = _arr(U)
    w = _arr(w)
    mu = np.zeros_like(U)
    lib().or_residual_vjp(ctypes.byref(g), _p(U), _p(w), _p(mu))
    return mu


def rk3_step_vjp(spec, U, dt_, lam, limiter=True, kappa=-1.0, source=None):
    """dJ/dU^n from dJ/dU^{n+1} = lam for one step at frozen dt (a source
    moves the stage states the derivative is taken at, not the derivative's form)."""
    _inviscid_only(spec)
    g = make_grid(spec, limiter, kappa, source)
    U = _arr(U)
    lam = _arr(lam).copy()
    lib().or_rk3_step_vjp(ctypes.byref(g), _p(U), float(dt_), _p(lam))
    return lam


def omp_threads():
    """Threads the oracle's OpenMP loops use now."""
    return int(lib().or_max_threads())


def set_threads(n):
    """Sets the threads of the oracle's OpenMP loops (n >= 1)."""
    lib().or_set_threads(int(n))
