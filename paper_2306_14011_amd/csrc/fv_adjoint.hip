// Adjoint (transpose-Jacobian) of the residual and of the SSP-RK3 stage
// combinations, FP64, gfx950.
//
// One kernel per reverse Runge-Kutta stage. A workgroup of 256 threads owns a
// tile of cells (2D 32 x 8, 3D 16 x 4 x 4) and, axis by axis:
//   1. evaluates the reverse of every face whose stencil holds a cell of the
//      tile (the tile's faces along the axis and three more): the MUSCL face
//      states from the four stencil cells (ghost positions mapped by the face
//      kinds: periodic wrap, transmissive clamp, the mirror cell with the
//      normal momentum reversed behind a slip wall, the given state behind an
//      inflow face), the reverse of the Roe flux with the face adjoint
//      Fb = area (w_left - w_right), and the reverse of the reconstruction,
//      whose four contributions (to the stencil cells k-1 .. k+2) go to LDS;
//   2. each cell adds the contributions of its four faces along the axis
//      and, next to a non-periodic boundary, those that the faces gave the
//      ghost positions copying it (the transpose of the ghost rule; inflow
//      ghosts hold a fixed state and pass nothing on).
// mu = (dR/dU)^T w then enters the stage's adjoint recurrence in the same
// kernel, so no face array or mu array goes through HBM. On a periodic axis
// the faces beyond the grid's ends are evaluated on wrapped stencils: such a
// face is the face on the other side, and the four faces around every cell
// carry all of its contributions.
#include "fv_internal.h"

namespace fvk {

constexpr int ADJ_T = 256;  // threads per workgroup, one per tile cell

template <int NDIM>
struct AdjTile;
template <>
struct AdjTile<2> {
    static constexpr int X = 32, Y = 8, Z = 1;
};
template <>
struct AdjTile<3> {
    static constexpr int X = 16, Y = 4, Z = 4;
};

// Entries of the face block of axis AX: the tile's extent along the other
// axes times its extent plus three along AX.
template <int NDIM, int AX>
constexpr int adj_faces() {
    using T = AdjTile<NDIM>;
    return (T::X + (AX == 0 ? 3 : 0)) * (T::Y + (AX == 1 ? 3 : 0)) * (T::Z + (AX == 2 ? 3 : 0));
}

template <int NDIM>
constexpr int adj_faces_max() {
    constexpr int a = adj_faces<NDIM, 0>(), b = adj_faces<NDIM, 1>(), c = NDIM == 3 ? adj_faces<NDIM, 2>() : 0;
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

// Cell read at position p along an axis of n cells with face kinds lo / hi
// (0 periodic, 1 transmissive, 2 slip wall, 3 inflow): p itself inside the
// grid; a periodic wrap (any p); the end cell; the mirror cell, with flip set
// (the normal momentum changes sign); -1 behind an inflow face.
__device__ __forceinline__ int adj_src(int p, int n, int lo, int hi, bool& flip) {
    flip = false;
    if (p >= 0 && p < n) return p;
    const bool low = p < 0;
    const int kind = low ? lo : hi;
    if (kind == 0) {
        const int r = p % n;
        return r < 0 ? r + n : r;
    }
    if (kind == 3) return -1;
    if (kind == 2) {
        flip = true;
        return low ? -1 - p : 2 * n - 1 - p;
    }
    return low ? 0 : n - 1;
}

// Steps 1 and 2 above for the faces of axis AX; adds the axis's part of mu
// to acc. o: the tile's first cell, (lx, ly, lz): this thread's cell in
// the tile, own: whether that cell is inside the grid.
template <int NDIM, int AX>
__device__ __forceinline__ void adj_axis(const double* __restrict__ Us, const double* __restrict__ w, const Geo& g,
                                         const BcState& bcs, const int* o, int lx, int ly, int lz, bool own,
                                         double* C, double* acc) {
    constexpr int NV = NDIM + 2;
    using T = AdjTile<NDIM>;
    constexpr int EX = T::X + (AX == 0 ? 3 : 0), EY = T::Y + (AX == 1 ? 3 : 0), EZ = T::Z + (AX == 2 ? 3 : 0);
    constexpr int NF = EX * EY * EZ;
    const int n = g.n[AX];
    const int lo = g.bc[AX][0], hi = g.bc[AX][1];
    const bool periodic = lo == 0;
    const long long st = AX == 0 ? 1 : (AX == 1 ? g.sy : g.sz);
    const long long wst = AX == 0 ? 1 : (AX == 1 ? g.n[0] : (long long)g.n[0] * g.n[1]);
    // the inflow states of this axis's two faces, read with constant indices
    // and picked per stencil cell by a select (a run-time index into the
    // table would move it to scratch memory)
    double q_lo[NV], q_hi[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        q_lo[v] = bcs.q[AX][0][v];
        q_hi[v] = bcs.q[AX][1][v];
    }
    for (int fi = threadIdx.x; fi < NF; fi += ADJ_T) {
        int p[3];
        p[0] = o[0] + fi % EX;
        p[1] = o[1] + (fi / EX) % EY;
        p[2] = o[2] + fi / (EX * EY);
        p[AX] -= 1;  // the face between cells fpos - 1 and fpos along AX
        const int fpos = p[AX];
        bool live = periodic || (fpos >= 0 && fpos <= n);
#pragma unroll
        for (int d = 0; d < NDIM; ++d)
            if (d != AX) live = live && p[d] < g.n[d];
        double gq[4][NV];
        if (live) {
            p[AX] = 0;
            const long long line = g.off0 + p[0] + (long long)p[1] * g.sy + (long long)p[2] * g.sz;
            const long long wline = ((long long)p[2] * g.n[1] + p[1]) * g.n[0] + p[0];
            double q[4][NV];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int pos = fpos - 2 + s;
                bool flip;
                const int src = adj_src(pos, n, lo, hi, flip);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (src < 0) {
                        q[s][v] = pos < 0 ? q_lo[v] : q_hi[v];
                    } else {
                        const double x = Us[v * g.sv + line + src * st];
                        q[s][v] = (flip && v == 1 + AX) ? -x : x;
                    }
                }
            }
            // the face adds F A to its left cell's residual and -F A to its right cell's
            int cl = fpos - 1, cr = fpos;
            bool hl = cl >= 0, hr = cr < n;
            if (periodic) {
                bool f;
                cl = adj_src(cl, n, 0, 0, f);
                cr = adj_src(cr, n, 0, 0, f);
                hl = hr = true;
            }
            double qL[NV], qR[NV], Fb[NV], qLb[NV], qRb[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                muscl(q[0][v], q[1][v], q[2][v], q[3][v], g.scheme, qL[v], qR[v]);
                const double wl = hl ? w[v * (long long)g.ncell + wline + cl * wst] : 0.0;
                const double wr = hr ? w[v * (long long)g.ncell + wline + cr * wst] : 0.0;
                Fb[v] = g.area[AX] * (wl - wr);
            }
            roe_flux_vjp<NDIM, AX>(qL, qR, g.gm1, Fb, qLb, qRb);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                gq[0][v] = gq[1][v] = gq[2][v] = gq[3][v] = 0.0;
                muscl_vjp(q[0][v], q[1][v], q[2][v], q[3][v], g.scheme, qLb[v], qRb[v], gq[0][v], gq[1][v],
                          gq[2][v], gq[3][v]);
            }
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int v = 0; v < NV; ++v) gq[m][v] = 0.0;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int v = 0; v < NV; ++v) C[(m * NV + v) * NF + fi] = gq[m][v];
    }
    __syncthreads();
    if (own) {
        const int lp[3] = {lx, ly, lz};
        const int xa = o[AX] + lp[AX];
        // entry of the face block at local face position i along AX, at this cell's other coordinates
        auto fidx = [&](int i) {
            int q[3] = {lx, ly, lz};
            q[AX] = i;
            return q[0] + EX * (q[1] + EY * q[2]);
        };
        // face x + 2 - m (local position lp + 3 - m) holds this cell at stencil slot m
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = fidx(lp[AX] + 3 - m);
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += C[(m * NV + v) * NF + e];
        }
        if (!periodic && (xa < 2 || xa >= n - 2)) {
            // ghosts -2, -1, n, n + 1 that copy this cell
#pragma unroll
            for (int gi = 0; gi < 4; ++gi) {
                const int gp = gi < 2 ? gi - 2 : n + gi - 2;
                const int kind = gi < 2 ? lo : hi;
                if (kind == 3) continue;
                const int src = kind == 2 ? (gi < 2 ? -1 - gp : 2 * n - 1 - gp) : (gi < 2 ? 0 : n - 1);
                if (src != xa) continue;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int f = gp + 2 - m;  // face holding the ghost at slot m
                    const int i = f - o[AX] + 1;
                    if (f < 0 || f > n || i < 0 || i >= (AX == 0 ? EX : (AX == 1 ? EY : EZ))) continue;
                    const int e = fidx(i);
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const double c = C[(m * NV + v) * NF + e];
                        acc[v] += (kind == 2 && v == 1 + AX) ? -c : c;
                    }
                }
            }
        }
    }
    __syncthreads();  // the next axis reuses C
}

// Reverse of the SSP-RK3 stage combinations with L = -R/|Omega|, s = dt/|Omega|,
// mu = (dR/dU_stage)^T w:
//   MODE 3 (w = lam):  lamA = 2/3 lam - 2/3 s mu  (dJ/dU2),  lamB = 1/3 lam
//   MODE 2 (w = lamA): R = 1/4 lamA - 1/4 s mu    (dJ/dU1),  lamB += 3/4 lamA
//   MODE 1 (w = R):    lam = lamB + R - s mu      (dJ/dU^n)
// w is read at the neighbours of a cell, so no stage writes its own w.
template <int NDIM, int MODE>
__global__ void __launch_bounds__(ADJ_T) k_adj_stage(const double* __restrict__ Us, const double* __restrict__ w,
                                                     double* lam, double* lamA, double* lamB, double* R,
                                                     const double* __restrict__ dtp, Geo g, BcState bcs) {
    constexpr int NV = NDIM + 2;
    using T = AdjTile<NDIM>;
    __shared__ double C[4 * NV * adj_faces_max<NDIM>()];
    const int tiles_x = (g.n[0] + T::X - 1) / T::X, tiles_y = (g.n[1] + T::Y - 1) / T::Y;
    const int b = blockIdx.x;
    const int o[3] = {(b % tiles_x) * T::X, ((b / tiles_x) % tiles_y) * T::Y, (b / (tiles_x * tiles_y)) * T::Z};
    const int t = threadIdx.x;
    const int lx = t % T::X, ly = (t / T::X) % T::Y, lz = t / (T::X * T::Y);
    const int cx = o[0] + lx, cy = o[1] + ly, cz = o[2] + lz;
    const bool own = cx < g.n[0] && cy < g.n[1] && cz < g.n[2];
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    adj_axis<NDIM, 0>(Us, w, g, bcs, o, lx, ly, lz, own, C, acc);
    adj_axis<NDIM, 1>(Us, w, g, bcs, o, lx, ly, lz, own, C, acc);
    if constexpr (NDIM == 3) adj_axis<NDIM, 2>(Us, w, g, bcs, o, lx, ly, lz, own, C, acc);
    if (!own) return;
    const double s = *dtp * g.inv_vol;
    const long long e = ((long long)cz * g.n[1] + cy) * g.n[0] + cx;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const long long i = v * (long long)g.ncell + e;
        if (MODE == 3) {
            const double l = w[i];
            lamA[i] = (2.0 / 3.0) * l - (2.0 / 3.0) * s * acc[v];
            lamB[i] = (1.0 / 3.0) * l;
        } else if (MODE == 2) {
            const double a = w[i];
            R[i] = 0.25 * a - 0.25 * s * acc[v];
            lamB[i] += 0.75 * a;
        } else {
            lam[i] = lamB[i] + w[i] - s * acc[v];
        }
    }
}

// ---------------------------------------------------------------------------

template <int NDIM, int MODE>
static void launch_adj_stage_t(const double* Us, const double* w, double* lam, double* lamA, double* lamB, double* R,
                               const double* dt, const Geo& g, const BcState& bcs, hipStream_t s) {
    using T = AdjTile<NDIM>;
    const long long tiles = (long long)((g.n[0] + T::X - 1) / T::X) * ((g.n[1] + T::Y - 1) / T::Y) *
                            ((g.n[2] + T::Z - 1) / T::Z);
    hipLaunchKernelGGL((k_adj_stage<NDIM, MODE>), dim3((unsigned)tiles), dim3(ADJ_T), 0, s, Us, w, lam, lamA, lamB,
                       R, dt, g, bcs);
}

void launch_adj_stage(int mode, const double* Us, const double* w, double* lam, double* lamA, double* lamB, double* R,
                      const double* dt, const Geo& g, const BcState& bcs, hipStream_t s) {
    if (g.ndim == 2) {
        if (mode == 3) launch_adj_stage_t<2, 3>(Us, w, lam, lamA, lamB, R, dt, g, bcs, s);
        else if (mode == 2) launch_adj_stage_t<2, 2>(Us, w, lam, lamA, lamB, R, dt, g, bcs, s);
        else launch_adj_stage_t<2, 1>(Us, w, lam, lamA, lamB, R, dt, g, bcs, s);
    } else {
        if (mode == 3) launch_adj_stage_t<3, 3>(Us, w, lam, lamA, lamB, R, dt, g, bcs, s);
        else if (mode == 2) launch_adj_stage_t<3, 2>(Us, w, lam, lamA, lamB, R, dt, g, bcs, s);
        else launch_adj_stage_t<3, 1>(Us, w, lam, lamA, lamB, R, dt, g, bcs, s);
    }
}

}  // namespace fvk
