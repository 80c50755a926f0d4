"""Sampled-patch checks of full-size 3D steps against the oracle.

The oracle cannot step a 256^3 grid within a test, but a cell's value after
s SSP-RK3 steps depends only on cells at most 6 s away (three stages, a
two-cell MUSCL stencil each). So the oracle steps a P^3 patch cut out of the
initial state (with transmissive faces of its own) and the inner
(P - 12 s)^3 cells of the patch are exact. Periodic axes wrap the cut; on a
transmissive axis the patch is clamped inside the grid, and where the patch
touches a true transmissive face its own transmissive face is that face.
"""
import numpy as np

from paper_2306_14011_amd import inputs


def sod_front_origins(n, normal, P, rng, count):
    """Patch origins whose centres lie on the tilted Sod plane (through the
    box centre, unit box, n cells per side), at seeded (y, z) positions."""
    out = []
    for _ in range(count):
        jc, kc = rng.integers(0, n, size=2)
        y = (jc + 0.5) / n
        z = (kc + 0.5) / n
        x = 0.5 - ((y - 0.5) * normal[1] + (z - 0.5) * normal[2]) / normal[0]
        ic = int(np.floor(x * n))
        out.append((ic - P // 2, int(jc) - P // 2, int(kc) - P // 2))
    return out


def cut(U, origin, P, n, periodic):
    """Patch of U (nvar, nz, ny, nx) at origin (i, j, k): periodic axes wrap,
    the others are clamped so the patch stays inside the grid."""
    idx = []
    o = list(origin)
    for a in range(3):
        if not periodic[a]:
            o[a] = min(max(o[a], 0), n[a] - P)
        idx.append((o[a] + np.arange(P)) % n[a])
    return U[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]], tuple(o)


def check_patches(got, U0, g, dts, origins, P, halo, tol=1e-12, min_change=None, what=""):
    """Steps each patch of U0 by len(dts) oracle steps at the given dt and
    compares the inner cells (halo cells away from every patch face) with
    `got`, per variable, with the scale of each variable over the inner
    reference. With min_change, a patch must also differ from its initial
    state by at least min_change times that scale (the check is not run on a
    flow at rest). Returns the number of patches and the largest error ratio."""
    import oracle
    n = [int(v) for v in g.n]
    periodic = [int(g.bc[a][0]) == 0 for a in range(3)]
    worst = 0.0
    nontrivial = 0
    for origin in origins:
        patch, o = cut(U0, origin, P, n, periodic)
        pg = inputs.grid3d(P, P, P, hi=tuple(P * (g.hi[a] - g.lo[a]) / n[a] for a in range(3)),
                           bc=((1, 1), (1, 1), (1, 1)))
        ref, _, _ = oracle.run(pg, patch, len(dts), dt_in=np.asarray(dts, dtype=np.float64))
        gp, _ = cut(got, o, P, n, periodic)
        sl = (slice(None),) + (slice(halo, P - halo),) * 3
        ref_in, got_in, u0_in = ref[sl], gp[sl], patch[sl]
        changed = False
        for v in range(ref.shape[0]):
            scale = max(np.abs(ref_in[v]).max(), 1e-300)
            err = np.abs(got_in[v] - ref_in[v]).max()
            assert err <= tol * scale, f"{what} patch {o} var {v}: err {err:.3e} scale {scale:.3e}"
            worst = max(worst, err / scale)
            if min_change is not None and np.abs(ref_in[v] - u0_in[v]).max() > min_change * scale:
                changed = True
        nontrivial += changed
    if min_change is not None:
        assert nontrivial == len(origins), f"{what}: {len(origins) - nontrivial} patches did not change"
    return len(origins), worst
