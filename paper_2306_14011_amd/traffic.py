"""Algorithmic (compulsory) HBM bytes of each kernel launch of the split step.

Counts every array element a kernel must read or write once, FP64 = 8 B,
ignoring halo re-reads, ghost layers and cache effects. These are the bytes
the roofline fractions are quoted against.

Per launch, with V = nvar, N = interior cells, F_d = faces on axis d:
  flux_d    read U (V N) + write F_d (V F_d)
  residual  read every F_d + write R (V N)
  update    read R, U^n [, U_s] + write U_{s+1}: 3 V N (stage 1), 4 V N (stages 2, 3)
  bc        read + write the ghost cells: 2 V G, G = sum_d 4 prod_{d' != d} n_d'
  cfl       read U (V N)
Per cell-update of the whole step (3 stages + one dt reduction), 2D: 1056 B,
3D: 1694 B (plus the ghost fill).

Algorithmic FP64 flops of the fused 2D stage (an FMA counts 2), counted
from the source (constants below): per cell and axis one MUSCL difference
and two face states, per face one Roe flux, per cell the residual and the
stage combination, and in the last stage the CFL wave speed.
"""
from __future__ import annotations

SITES = ("flux_x", "flux_y", "flux_z", "residual", "update", "bc", "cfl")


def faces(spec):
    nx, ny, nz = (int(v) for v in spec.n)
    f = [(nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)]
    return f[: spec.ndim] + [0] * (3 - spec.ndim)


def ghost_cells(spec):
    nx, ny, nz = (int(v) for v in spec.n)
    g = 4 * ny * nz + 4 * nx * nz
    if spec.ndim == 3:
        g += 4 * nx * ny
    return g


def site_bytes(spec):
    """Algorithmic bytes per launch of each site (update averaged over its 3 stages)."""
    V = spec.ndim + 2
    N = spec.ncells
    F = faces(spec)
    b = {}
    for d, name in enumerate(("flux_x", "flux_y", "flux_z")):
        b[name] = 8 * V * (N + F[d]) if d < spec.ndim else 0
    b["residual"] = 8 * V * (sum(F) + N)
    b["update"] = 8 * V * N * (3 + 4 + 4) / 3.0
    b["bc"] = 8 * V * 2 * ghost_cells(spec)
    b["cfl"] = 8 * V * N
    return b


def step_bytes(spec):
    """Algorithmic bytes of one full step (3 stages + dt reduction)."""
    b = site_bytes(spec)
    per_stage = sum(b[f"flux_{a}"] for a in "xyz") + b["residual"] + b["bc"] + b["update"]
    return 3 * per_stage + b["cfl"]


def fused_step_bytes(spec):
    """Compulsory bytes of a step whose stages each read U_s (and U^n) once and
    write U_{s+1} once: 2 + 3 + 3 = 8 states per step."""
    return 8 * (spec.ndim + 2) * spec.ncells * 8


# Algorithmic FP64 flops, counted from the device source with an FMA as 2,
# min / max / abs as 0 and each shared subexpression once:
#   MUSCL per cell and axis: 4 variables x (the backward difference D[i] and
#     the two face states U[i] +- minmod(D[i], D[i+1]) / 2)
#   Roe flux per face (2D, returned as 2F): primitive states, Roe averages,
#     wave strengths and dissipation, central fluxes; each 1/x is 6 flops and
#     each 1/sqrt(x) 8 (hardware estimate plus one third-order correction),
#     3 of the latter and 1 of the former
#   cell update: residual of 4 faces x 4 variables (5 flops each) and the RK
#     combination (2, 5, 5 flops in stages 1, 2, 3), averaged over the stages
#   CFL wave speed of a cell: 1/rho, velocities, pressure, c, sum over axes
FLOPS_MUSCL_CELL_AXIS = 4 * 5
FLOPS_ROE_FACE_2D = 131
FLOPS_CELL_UPDATE_2D = 4 * (5 + 4)
FLOPS_CELL_LAMBDA = 31


def fused_stage_flops(spec):
    """Algorithmic FP64 flops of one fused stage launch, averaged over the three stages."""
    per_cell = 2 * (FLOPS_MUSCL_CELL_AXIS + FLOPS_ROE_FACE_2D) + FLOPS_CELL_UPDATE_2D + FLOPS_CELL_LAMBDA / 3.0
    return per_cell * spec.ncells
