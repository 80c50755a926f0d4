// Primal kernels of the split step for gfx950 (FP64): ghost fill, MUSCL-Roe
// face fluxes per axis, residual assembly, SSP-RK3 stage update and the
// wave-speed max-reduction for the CFL time step.
//
// Every output element is computed by exactly one thread with an arithmetic
// sequence that does not depend on the launch shape, and the reduction is a
// max (exact and order-independent), so every valid launch configuration
// produces bitwise-identical results.
#include "fv_internal.h"

namespace fvk {

// ---------------------------------------------------------------------------
// Ghost fill. Element e enumerates, axis by axis, the 4 ghost layers
// (-2, -1, n, n+1) times the interior cross-section of that axis; layer is the
// fastest index. Periodic faces copy the opposite interior layers,
// transmissive faces copy the nearest interior cell (zero gradient), slip
// walls the mirror image across the face with the normal momentum reversed,
// inflow faces take their given state.
template <int NV>
__global__ void __launch_bounds__(1024) k_bc_fill(double* __restrict__ U, Geo g, BcState bcs, int total, int seg0,
                                                   int seg1, int stride_all) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride_all) {
        int ax, q, layer;
        if (e < seg0) {
            ax = 0;
            q = e >> 2;
        } else if (e < seg0 + seg1) {
            ax = 1;
            q = (e - seg0) >> 2;
        } else {
            ax = 2;
            q = (e - seg0 - seg1) >> 2;
        }
        layer = e & 3;
        int c[3];
        // cross-section coordinates, first remaining axis fastest
        if (ax == 0) {
            c[1] = q % g.n[1];
            c[2] = q / g.n[1];
        } else if (ax == 1) {
            c[0] = q % g.n[0];
            c[2] = q / g.n[0];
        } else {
            c[0] = q % g.n[0];
            c[1] = q / g.n[0];
        }
        const int n = g.n[ax];
        const int gpos = layer < 2 ? layer - 2 : n + layer - 2;  // -2, -1, n, n+1
        int src;
        const bool lo = layer < 2;
        const int kind = g.bc[ax][lo ? 0 : 1];
        if (kind == 0) {
            src = ((gpos % n) + n) % n;
        } else if (kind == 2) {
            src = lo ? -1 - gpos : 2 * n - 1 - gpos;
        } else if (kind == 3) {
            src = lo ? 0 : n - 1;  // not read: the ghost takes the given state
        } else {
            src = lo ? 0 : n - 1;
        }
        int cg[3] = {c[0], c[1], c[2]};
        int cs[3] = {c[0], c[1], c[2]};
        cg[ax] = gpos;
        cs[ax] = src;
        if (g.ndim == 2) {
            cg[2] = 0;
            cs[2] = 0;
        }
        const int og = g.off0 + cg[0] + cg[1] * g.sy + cg[2] * g.sz;
        const int os = g.off0 + cs[0] + cs[1] * g.sy + cs[2] * g.sz;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (kind == 3) {
                U[v * g.sv + og] = bcs.q[ax][lo ? 0 : 1][v];
            } else {
                const double q = U[v * g.sv + os];
                U[v * g.sv + og] = (kind == 2 && v == 1 + ax) ? -q : q;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Viscous face flux (Navier-Stokes): F_nu,n of Eq. (QF) on every face of axis
// AX, subtracted from the inviscid face flux in place (the residual sums
// F_i,n - F_nu,n). With w = (u, v, [w], T), T = p / rho (unit gas constant):
//   tau_{a,AX} = mu (dw_a/dx_AX + dw_AX/dx_a) - 2/3 mu delta_{a,AX} div(u),
//   Theta_AX  = sum_b ubar_b tau_{b,AX} + k dT/dx_AX,   k = mu gamma / ((gamma - 1) Pr),
// the normal derivative being the difference across the face over dx, each
// tangential derivative the mean of the central differences of the two cells
// across the face, and ubar the mean velocity of those two cells. Neighbour
// cells outside the grid (at most one cell out on the tangential axes, so
// edge and corner positions too) are mapped axis by axis: periodic wrap,
// transmissive clamp, slip-wall mirror with that axis's momentum reversed,
// or the given state of an inflow face.

// Velocity and temperature at interior-or-mapped position (i, j, k).
template <int NDIM>
__device__ __forceinline__ void visc_cell(const double* __restrict__ U, const Geo& g, const BcState& bcs, int i,
                                          int j, int k, double* w) {
    constexpr int NV = NDIM + 2;
    int p[3] = {i, j, k};
    double sg[NDIM];
#pragma unroll
    for (int d = 0; d < NDIM; ++d) sg[d] = 1.0;
    // the first inflow face crossed gives the state; its side is picked by a
    // select between constant indices (a run-time index into the table would
    // move it to scratch memory)
    bool fixed = false;
    double fq[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) fq[v] = 0.0;
#pragma unroll
    for (int a = 0; a < NDIM; ++a) {
        const int n = g.n[a];
        const int x = p[a];
        if (x < 0 || x >= n) {
            const int side = x < 0 ? 0 : 1;
            const int kind = g.bc[a][side];
            if (kind == 3 && !fixed) {
                fixed = true;
#pragma unroll
                for (int v = 0; v < NV; ++v) fq[v] = side ? bcs.q[a][1][v] : bcs.q[a][0][v];
            }
            if (kind == 0) p[a] = x < 0 ? x + n : x - n;
            else if (kind == 2) {
                p[a] = x < 0 ? -1 - x : 2 * n - 1 - x;
                sg[a] = -1.0;
            } else p[a] = x < 0 ? 0 : n - 1;
        }
    }
    double q[NV];
    if (fixed) {
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = fq[v];
    } else {
        const int o = g.off0 + p[0] + p[1] * g.sy + (NDIM == 3 ? p[2] * g.sz : 0);
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = U[v * g.sv + o];
#pragma unroll
        for (int d = 0; d < NDIM; ++d) q[1 + d] *= sg[d];
    }
    const double ir = 1.0 / q[0];
    double qq = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        w[d] = q[1 + d] * ir;
        qq += w[d] * w[d];
    }
    w[NDIM] = g.gm1 * (q[NDIM + 1] - 0.5 * q[0] * qq) * ir;
}

template <int NDIM, int AX>
__global__ void __launch_bounds__(256) k_visc(const double* __restrict__ U, double* __restrict__ F, Geo g,
                                              BcState bcs, int cols, int rows_j, int nfaces) {
    constexpr int NW = NDIM + 1;
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nfaces; f += gridDim.x * blockDim.x) {
        const int i = f % cols;
        const int r = f / cols;
        const int j = r % rows_j;
        const int k = r / rows_j;
        // face (i, j, k) lies between cell c = (i, j, k) - e_AX and (i, j, k)
        int c0[3] = {i, j, k};
        c0[AX] -= 1;
        double wa[NW], wb[NW];
        visc_cell<NDIM>(U, g, bcs, c0[0], c0[1], c0[2], wa);
        visc_cell<NDIM>(U, g, bcs, i, j, k, wb);
        double grad[NW][NDIM];
#pragma unroll
        for (int m = 0; m < NW; ++m) grad[m][AX] = (wb[m] - wa[m]) * g.inv_dx[AX];
#pragma unroll
        for (int t = 0; t < NDIM; ++t) {
            if (t == AX) continue;
            double wp0[NW], wm0[NW], wp1[NW], wm1[NW];
            int p[3] = {c0[0], c0[1], c0[2]};
            p[t] += 1;
            visc_cell<NDIM>(U, g, bcs, p[0], p[1], p[2], wp0);
            p[t] -= 2;
            visc_cell<NDIM>(U, g, bcs, p[0], p[1], p[2], wm0);
            int q[3] = {i, j, k};
            q[t] += 1;
            visc_cell<NDIM>(U, g, bcs, q[0], q[1], q[2], wp1);
            q[t] -= 2;
            visc_cell<NDIM>(U, g, bcs, q[0], q[1], q[2], wm1);
#pragma unroll
            for (int m = 0; m < NW; ++m) grad[m][t] = ((wp0[m] - wm0[m]) + (wp1[m] - wm1[m])) * (0.25 * g.inv_dx[t]);
        }
        double divu = 0.0;
#pragma unroll
        for (int d = 0; d < NDIM; ++d) divu += grad[d][d];
        double tau[NDIM];
#pragma unroll
        for (int a = 0; a < NDIM; ++a) {
            tau[a] = g.mu * (grad[a][AX] + grad[AX][a]);
            if (a == AX) tau[a] -= (2.0 / 3.0) * g.mu * divu;
        }
        double theta = g.kcond * grad[NDIM][AX];
#pragma unroll
        for (int b = 0; b < NDIM; ++b) theta += 0.5 * (wa[b] + wb[b]) * tau[b];
        const long long fo = (long long)f;
#pragma unroll
        for (int a = 0; a < NDIM; ++a) F[(1 + a) * g.fsv[AX] + fo] -= tau[a];
        F[(NDIM + 1) * g.fsv[AX] + fo] -= theta;
    }
}

// ---------------------------------------------------------------------------
// Face fluxes along axis AX. Face (i, j, k) lies between cells (i,j,k) - e_AX
// and (i,j,k); its flux is stored at F[v * fsv + (k * rows_j + j) * cols + i]
// with cols = nx (+1 on x) and rows_j = ny (+1 on y). Threads: x -> i,
// y -> j (grid-stride), blockIdx.z -> k.
template <int NDIM, int AX, int MAXT>
__global__ void __launch_bounds__(MAXT) k_flux(const double* __restrict__ U, double* __restrict__ F,
                                               Geo g) {
    constexpr int NV = NDIM + 2;
    const int cols = g.n[0] + (AX == 0 ? 1 : 0);
    const int rows_j = g.n[1] + (AX == 1 ? 1 : 0);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cols) return;
    const int k = blockIdx.z;
    const int st = AX == 0 ? 1 : (AX == 1 ? g.sy : g.sz);
    const long long fsv = g.fsv[AX];
    for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < rows_j; j += gridDim.y * blockDim.y) {
        const int c = g.off0 + i + j * g.sy + k * g.sz;  // right cell of the face
        double qL[NV], qR[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double* Uv = U + v * g.sv;
            const double q0 = Uv[c - 2 * st], q1 = Uv[c - st], q2 = Uv[c], q3 = Uv[c + st];
            muscl(q0, q1, q2, q3, g.scheme, qL[v], qR[v]);
        }
        double Fl[NV];
        roe_flux<NDIM, AX>(qL, qR, g.gm1, Fl);
        const long long f = (long long)(k * rows_j + j) * cols + i;
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v * fsv + f] = Fl[v];
    }
}

// Faces along y or z (AX = 1, 2): each thread walks a run of RUN consecutive
// faces of its column with a window of four cells in registers, so each cell
// is loaded once per run instead of four times. Same face arithmetic.
template <int NDIM, int AX, int MAXT, int RUN>
__global__ void __launch_bounds__(MAXT) k_flux_run(const double* __restrict__ U, double* __restrict__ F, Geo g) {
    constexpr int NV = NDIM + 2;
    static_assert(AX >= 1 && RUN % 4 == 0, "runs march along y or z in groups of four");
    const int cols = g.n[0];
    const int rows_j = g.n[1] + (AX == 1 ? 1 : 0);
    const int rows_k = NDIM == 3 ? g.n[2] + (AX == 2 ? 1 : 0) : 1;
    const int nax = AX == 1 ? rows_j : rows_k;   // faces along the axis
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cols) return;
    const int st = AX == 1 ? g.sy : g.sz;
    const long long fsv = g.fsv[AX];
    // the other (non-marching) index: k for AX = 1 (grid z), j for AX = 2 (grid y)
    const int other = AX == 1 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (AX == 2 && other >= rows_j) return;
    const int r0 = AX == 1 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : (int)blockIdx.z;
    const int rstride = AX == 1 ? (int)(gridDim.y * blockDim.y) : (int)gridDim.z;
    for (int run = r0; run * RUN < nax; run += rstride) {
        const int a0 = run * RUN;   // first face of the run
        const int j = AX == 1 ? a0 : other, k = AX == 1 ? other : a0;
        const int c0 = g.off0 + i + j * g.sy + k * g.sz;  // right cell of face a0
        double W[4][NV];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < NV; ++v) W[q][v] = U[v * g.sv + c0 + (q - 2) * st];
#pragma unroll
        for (int t = 0; t < RUN; ++t) {
            const int a = a0 + t;
            if (a >= nax) break;
            // face a: cells a-2 .. a+1 in slots t, t+1, t+2, t+3 (mod 4)
            double qL[NV], qR[NV], Fl[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                muscl(W[t & 3][v], W[(t + 1) & 3][v], W[(t + 2) & 3][v], W[(t + 3) & 3][v], g.scheme, qL[v],
                      qR[v]);
            roe_flux<NDIM, AX>(qL, qR, g.gm1, Fl);
            const int fj = AX == 1 ? a : j, fk = AX == 1 ? k : a;
            const long long f = (long long)(fk * rows_j + fj) * cols + i;
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v * fsv + f] = Fl[v];
            if (t + 1 < RUN && a + 1 < nax) {
#pragma unroll
                for (int v = 0; v < NV; ++v) W[t & 3][v] = U[v * g.sv + c0 + (t + 2) * st];  // cell a + 2
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Curvilinear 2D grids. The metric streams (layout in fv_device.h) are
// computed once from the node coordinates nodes[d][j][i] ((nx + 1) x
// (ny + 1) nodes, x then y): a face's area vector is its edge turned by a
// right angle towards the higher-index cell, its length the edge length, a
// cell's area half the cross product of its diagonals.
__global__ void __launch_bounds__(256) k_metrics(const double* __restrict__ nodes, double* __restrict__ met,
                                                 int nx, int ny) {
    const MetricOffsets mo = metric_offsets(nx, ny);
    const long long nn = (long long)(nx + 1) * (ny + 1);
    auto X = [&](int i, int j) { return nodes[(long long)j * (nx + 1) + i]; };
    auto Y = [&](int i, int j) { return nodes[nn + (long long)j * (nx + 1) + i]; };
    const long long total = mo.nfx + mo.nfy + mo.nc;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < mo.nfx) {
            // x face (i, j): edge from node (i, j) to (i, j + 1)
            const int i = (int)(e % (nx + 1)), j = (int)(e / (nx + 1));
            const double ex = X(i, j + 1) - X(i, j), ey = Y(i, j + 1) - Y(i, j);
            const double len = sqrt(ex * ex + ey * ey);
            met[mo.fx + e] = ey / len;
            met[mo.fx + mo.nfx + e] = -ex / len;
            met[mo.fx + 2 * mo.nfx + e] = len;
        } else if (e < mo.nfx + mo.nfy) {
            // y face (i, j): edge from node (i, j) to (i + 1, j)
            const long long q = e - mo.nfx;
            const int i = (int)(q % nx), j = (int)(q / nx);
            const double ex = X(i + 1, j) - X(i, j), ey = Y(i + 1, j) - Y(i, j);
            const double len = sqrt(ex * ex + ey * ey);
            met[mo.fy + q] = -ey / len;
            met[mo.fy + mo.nfy + q] = ex / len;
            met[mo.fy + 2 * mo.nfy + q] = len;
        } else {
            const long long q = e - mo.nfx - mo.nfy;
            const int i = (int)(q % nx), j = (int)(q / nx);
            const double d1x = X(i + 1, j + 1) - X(i, j), d1y = Y(i + 1, j + 1) - Y(i, j);
            const double d2x = X(i, j + 1) - X(i + 1, j), d2y = Y(i, j + 1) - Y(i + 1, j);
            const double area = 0.5 * (d1x * d2y - d1y * d2x);
            met[mo.cell + q] = area;
            met[mo.cell + mo.nc + q] = 1.0 / area;
        }
    }
}

// Face fluxes on a curvilinear 2D grid, times the face length, along AX.
// The same face indexing and launch shape as k_flux. The four stencil cells
// along the grid line are read through the boundary maps (no ghost layer is
// used): periodic wrap, transmissive clamp, the given state of an inflow
// face, or a slip wall's mirror cell with its velocity reflected about the
// wall face's unit normal, u - 2 (u.n) n.
template <int AX, int MAXT>
__global__ void __launch_bounds__(MAXT) k_flux_curv(const double* __restrict__ U, double* __restrict__ F, Geo g,
                                                    BcState bcs) {
    constexpr int NV = 4;
    const int nx = g.n[0], ny = g.n[1];
    const int cols = nx + (AX == 0 ? 1 : 0);
    const int rows_j = ny + (AX == 1 ? 1 : 0);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cols) return;
    const MetricOffsets mo = metric_offsets(nx, ny);
    const long long mbase = AX == 0 ? mo.fx : mo.fy;
    const long long mstride = AX == 0 ? mo.nfx : mo.nfy;
    const int n = g.n[AX];
    const long long fsv = g.fsv[AX];
    for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < rows_j; j += gridDim.y * blockDim.y) {
        const long long f = (long long)j * cols + i;
        const double fnx = g.met[mbase + f], fny = g.met[mbase + mstride + f], len = g.met[mbase + 2 * mstride + f];
        const int a0 = AX == 0 ? i : j;  // index of the face's right cell on AX
        double q[4][NV];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int pos = a0 - 2 + m;
            const bool lo = pos < 0, hi = pos >= n;
            const int kind = lo ? g.bc[AX][0] : (hi ? g.bc[AX][1] : -1);
            int p = pos;
            if (kind == 0) p = lo ? pos + n : pos - n;
            else if (kind == 2) p = lo ? -1 - pos : 2 * n - 1 - pos;
            else if (kind == 1 || kind == 3) p = lo ? 0 : n - 1;
            const int ci = AX == 0 ? p : i, cj = AX == 0 ? j : p;
            const int o = g.off0 + ci + cj * g.sy;
            if (kind == 3) {
#pragma unroll
                for (int v = 0; v < NV; ++v) q[m][v] = bcs.q[AX][lo ? 0 : 1][v];
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) q[m][v] = U[v * g.sv + o];
            }
            if (kind == 2) {
                // the wall face of this grid line: face 0 or face n on AX
                const long long wf = AX == 0 ? (long long)j * cols + (lo ? 0 : n) : (long long)(lo ? 0 : n) * cols + i;
                const double wx = g.met[mbase + wf], wy = g.met[mbase + mstride + wf];
                const double mn = q[m][1] * wx + q[m][2] * wy;
                q[m][1] -= 2.0 * mn * wx;
                q[m][2] -= 2.0 * mn * wy;
            }
        }
        double qL[NV], qR[NV], Fl[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) muscl(q[0][v], q[1][v], q[2][v], q[3][v], g.scheme, qL[v], qR[v]);
        roe_flux_n2(qL, qR, fnx, fny, g.gm1, Fl);
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v * fsv + f] = Fl[v] * len;
    }
}

// ---------------------------------------------------------------------------
// Interior cell e -> (i, j, k) and its offset in the ghosted layout.
__device__ __forceinline__ void decode_cell(int e, const Geo& g, int& i, int& j, int& k) {
    const uint32_t t = divq((uint32_t)e, g.dnx);
    i = e - (int)t * g.n[0];
    k = (int)divq(t, g.dny);
    j = (int)t - k * g.n[1];
}

// R[v][e] = sum_d (F_d[face e + e_d] - F_d[face e]) * area_d - |Omega| S[v][e]
// (the source term of the residual; S null for none).
template <int NDIM, int MAXT>
__global__ void __launch_bounds__(MAXT) k_residual(const double* __restrict__ Fx,
                                                   const double* __restrict__ Fy,
                                                   const double* __restrict__ Fz, const double* __restrict__ S,
                                                   double* __restrict__ R, Geo g, int stride_all) {
    constexpr int NV = NDIM + 2;
    const int nx = g.n[0], ny = g.n[1];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.ncell; e += stride_all) {
        int i, j, k;
        decode_cell(e, g, i, j, k);
        const long long fx = (long long)(k * ny + j) * (nx + 1) + i;
        const long long fy = (long long)(k * (ny + 1) + j) * nx + i;
        const long long fz = (long long)(k * ny + j) * nx + i;
        const long long zs = (long long)ny * nx;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double r = (Fx[v * g.fsv[0] + fx + 1] - Fx[v * g.fsv[0] + fx]) * g.area[0];
            r += (Fy[v * g.fsv[1] + fy + nx] - Fy[v * g.fsv[1] + fy]) * g.area[1];
            if (NDIM == 3) r += (Fz[v * g.fsv[2] + fz + zs] - Fz[v * g.fsv[2] + fz]) * g.area[2];
            if (S) r -= (g.met ? g.met[metric_offsets(nx, ny).cell + e] : g.vol) * S[(long long)v * g.ncell + e];
            R[(long long)v * g.ncell + e] = r;
        }
    }
}

// Residual norm: 256 blocks each sum R_v^2 over a grid-stride range of cells
// (partial[v * 256 + block]), then one block adds the 256 partial sums of each
// variable. Fixed block count and order, so the result does not depend on
// timing.
constexpr int NORM_BLOCKS = 256;

template <int NV>
__global__ void __launch_bounds__(256) k_sumsq(const double* __restrict__ R, int ncell,
                                               double* __restrict__ partial) {
    __shared__ double sm[NV][4];
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ncell; e += gridDim.x * blockDim.x)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double r = R[(long long)v * ncell + e];
            acc[v] = fma(r, r, acc[v]);
        }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double t = acc[v];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
        if ((threadIdx.x & 63) == 0) sm[v][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int v = threadIdx.x;
        partial[v * NORM_BLOCKS + blockIdx.x] = ((sm[v][0] + sm[v][1]) + sm[v][2]) + sm[v][3];
    }
}

template <int NV>
__global__ void __launch_bounds__(256) k_norm_final(const double* __restrict__ partial, int ncell,
                                                    double* __restrict__ norms) {
    __shared__ double sm[NV][4];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double t = partial[v * NORM_BLOCKS + threadIdx.x];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
        if ((threadIdx.x & 63) == 0) sm[v][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int v = threadIdx.x;
        norms[v] = sqrt((((sm[v][0] + sm[v][1]) + sm[v][2]) + sm[v][3]) / (double)ncell);
    }
}

// SSP-RK3 stage update with L = -R / |Omega| and dt read from device memory.
//   STAGE 0: Ud = Un + dt L
//   STAGE 1: Ud = 3/4 Un + 1/4 (Us + dt L)          (Ud may alias Us)
//   STAGE 2: Ud = 1/3 Un + 2/3 (Us + dt L)          (Ud may alias Un)
template <int NDIM, int STAGE, int MAXT>
__global__ void __launch_bounds__(MAXT) k_update(const double* Un, const double* Us, double* Ud,
                                                 const double* __restrict__ R,
                                                 const double* __restrict__ dtp, Geo g, int stride_all) {
    constexpr int NV = NDIM + 2;
    const double dt = *dtp;
    const double s0 = -dt * g.inv_vol;
    const long long inv_area = g.met ? metric_offsets(g.n[0], g.n[1]).cell + g.ncell : 0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.ncell; e += stride_all) {
        int i, j, k;
        decode_cell(e, g, i, j, k);
        const int o = g.off0 + i + j * g.sy + k * g.sz;
        const double s = g.met ? -dt * g.met[inv_area + e] : s0;  // -dt / |Omega| of this cell
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double Lr = R[(long long)v * g.ncell + e];
            const long long p = v * g.sv + o;
            double out;
            if (STAGE == 0) {
                out = Un[p] + s * Lr;
            } else if (STAGE == 1) {
                out = 0.75 * Un[p] + 0.25 * (Us[p] + s * Lr);
            } else {
                out = (1.0 / 3.0) * Un[p] + (2.0 / 3.0) * (Us[p] + s * Lr);
            }
            Ud[p] = out;
        }
    }
}

// ---------------------------------------------------------------------------
// Wave-speed reduction: lambda(cell) = sum_d (|u_d| + c) / dx_d, block max into
// partial[blockIdx.x]; NaN / rho <= 0 / p <= 0 set bits of the status word.
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Wave-speed bound of a cell of a curvilinear 2D grid: sum over the two grid
// directions of (|u.S| + c |S|) / area, S the mean of the cell's two face
// area vectors (unit normal times length) on that direction. (The flags come
// from cell_lambda, called first on the same state.)
__device__ __forceinline__ double curv_lambda(const double* q, const Geo& g, int i, int j) {
    const int nx = g.n[0], ny = g.n[1];
    const MetricOffsets mo = metric_offsets(nx, ny);
    const long long e = (long long)j * nx + i;
    double m[2][2][3];  // [axis][low, high face][normal x, normal y, length]
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        const long long base = ax == 0 ? mo.fx : mo.fy, st = ax == 0 ? mo.nfx : mo.nfy;
        const long long fa = ax == 0 ? (long long)j * (nx + 1) + i : e;
        const long long fb = ax == 0 ? fa + 1 : e + nx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            m[ax][0][c] = g.met[base + c * st + fa];
            m[ax][1][c] = g.met[base + c * st + fb];
        }
    }
    return curv_cell_lambda(q, g.gamma, g.gm1, m[0][0], m[0][1], m[1][0], m[1][1], g.met[mo.cell + e]);
}

template <int NDIM, int MAXT>
__global__ void __launch_bounds__(MAXT) k_cfl_partial(const double* __restrict__ U, double* __restrict__ partial,
                                                      uint32_t* __restrict__ status, Geo g, int stride_all) {
    __shared__ double sm[MAXT / 64];
    double lmax = 0.0;
    uint32_t fl = 0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.ncell; e += stride_all) {
        int i, j, k;
        decode_cell(e, g, i, j, k);
        const int o = g.off0 + i + j * g.sy + k * g.sz;
        double q[NDIM + 2];
#pragma unroll
        for (int v = 0; v < NDIM + 2; ++v) q[v] = U[v * g.sv + o];
        double lam = cell_lambda<NDIM>(q, g.gamma, g.gm1, g.inv_dx, fl);
        if (NDIM == 2 && g.met) lam = curv_lambda(q, g, i, j);
        if (g.mu > 0.0) {
            // explicit diffusion limit: 2 nu_eff sum_d 1/dx_d^2, nu_eff =
            // (mu / rho) max(4/3, gamma / Pr)
            double s2 = 0.0;
#pragma unroll
            for (int d = 0; d < NDIM; ++d) s2 += g.inv_dx[d] * g.inv_dx[d];
            lam += 2.0 * ((g.mu / q[0]) * g.nu_fac) * s2;
        }
        lmax = fmax(lmax, lam);
    }
    if (fl) atomicOr(status, fl);
    lmax = wave_max(lmax);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sm[w] = lmax;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int nw = blockDim.x >> 6;
        double v = threadIdx.x < nw ? sm[threadIdx.x] : 0.0;
        v = wave_max(v);
        if (threadIdx.x == 0) partial[blockIdx.x] = v;
    }
}

// One block: max over the partials, dt = cfl / max (or the frozen dt_in).
__global__ void __launch_bounds__(1024) k_cfl_final(const double* __restrict__ partial, int npart,
                                                    const double* __restrict__ dt_in, double* __restrict__ dt,
                                                    double* __restrict__ dt_out, uint32_t* __restrict__ status,
                                                    double cfl) {
    __shared__ double sm[16];
    double m = 0.0;
    for (int t = threadIdx.x; t < npart; t += blockDim.x) m = fmax(m, partial[t]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int nw = blockDim.x >> 6;
        double v = threadIdx.x < nw ? sm[threadIdx.x] : 0.0;
        v = wave_max(v);
        if (threadIdx.x == 0) {
            double d = dt_in ? *dt_in : cfl / v;
            if (!(v > 0.0) || !(d > 0.0) || isinf(d) || isnan(d)) atomicOr(status, 8u);
            *dt = d;
            if (dt_out) *dt_out = d;
        }
    }
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------------------
// Launchers.

static inline int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

// 1-D sites: gang 0 -> one thread per element; else a grid-stride loop.
static inline void grid1d(int64_t n, int gang, int threads, int& blocks, int& stride_all) {
    blocks = gang > 0 ? gang : blocks_for(n, threads);
    if (blocks < 1) blocks = 1;
    stride_all = blocks * threads;
}

#define FV_DISPATCH_THREADS(T, MACRO) \
    switch (T) {                      \
        case 64: MACRO(64); break;    \
        case 128: MACRO(128); break;  \
        case 256: MACRO(256); break;  \
        case 512: MACRO(512); break;  \
        default: MACRO(1024); break;  \
    }

void launch_bc_fill(double* U, const Geo& g, const BcState& bcs, int gang, int threads, hipStream_t s) {
    const int seg0 = 4 * g.n[1] * g.n[2];
    const int seg1 = 4 * g.n[0] * g.n[2];
    const int seg2 = g.ndim == 3 ? 4 * g.n[0] * g.n[1] : 0;
    const int total = seg0 + seg1 + seg2;
    int blocks, stride_all;
    grid1d(total, gang, threads, blocks, stride_all);
    if (g.ndim == 2)
        hipLaunchKernelGGL(k_bc_fill<4>, dim3(blocks), dim3(threads), 0, s, U, g, bcs, total, seg0, seg1, stride_all);
    else
        hipLaunchKernelGGL(k_bc_fill<5>, dim3(blocks), dim3(threads), 0, s, U, g, bcs, total, seg0, seg1, stride_all);
}

constexpr int FLUX_RUN = 8;  // faces per thread of the y / z flux kernels

template <int NDIM, int AX>
static void launch_flux_t(const double* U, double* F, const Geo& g, int bx, int threads, hipStream_t s) {
    const int by = threads / bx;
    const int cols = g.n[0] + (AX == 0 ? 1 : 0);
    const int rows_j = g.n[1] + (AX == 1 ? 1 : 0);
    const int rows_k = NDIM == 3 ? g.n[2] + (AX == 2 ? 1 : 0) : 1;
    // 3D blocks of 1024 threads leave 128 registers per lane, too few for the
    // five-variable window: those keep one face per thread
    if (AX == 0 || (NDIM == 3 && threads == 1024)) {
        int gy = blocks_for(rows_j, by);
        if (gy > 65535) gy = 65535;
        dim3 grid(blocks_for(cols, bx), gy, rows_k);
        dim3 block(bx, by);
#define FV_LF(T) hipLaunchKernelGGL((k_flux<NDIM, AX, T>), grid, block, 0, s, U, F, g)
        FV_DISPATCH_THREADS(threads, FV_LF)
#undef FV_LF
        return;
    }
    const int runs = AX == 1 ? blocks_for(rows_j, FLUX_RUN) : blocks_for(rows_k, FLUX_RUN);
    dim3 grid, block(bx, by);
    if (AX == 1) {
        int gy = blocks_for(runs, by);
        if (gy > 65535) gy = 65535;
        grid = dim3(blocks_for(cols, bx), gy, rows_k);
    } else {
        int gy = blocks_for(rows_j, by);
        if (gy > 65535) gy = 65535;  // rows_j <= 65535 * by for every valid grid
        grid = dim3(blocks_for(cols, bx), gy, runs);
    }
#define FV_LFR(T) hipLaunchKernelGGL((k_flux_run<NDIM, (AX > 0 ? AX : 1), T, FLUX_RUN>), grid, block, 0, s, U, F, g)
    FV_DISPATCH_THREADS(threads, FV_LFR)
#undef FV_LFR
}

void launch_metrics(const double* nodes, double* met, int nx, int ny, hipStream_t s) {
    const MetricOffsets mo = metric_offsets(nx, ny);
    const long long total = mo.nfx + mo.nfy + mo.nc;
    long long blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_metrics, dim3((unsigned)blocks), dim3(256), 0, s, nodes, met, nx, ny);
}

template <int AX>
static void launch_flux_curv_t(const double* U, double* F, const Geo& g, const BcState& bcs, int bx, int threads,
                               hipStream_t s) {
    const int by = threads / bx;
    const int cols = g.n[0] + (AX == 0 ? 1 : 0);
    const int rows_j = g.n[1] + (AX == 1 ? 1 : 0);
    int gy = blocks_for(rows_j, by);
    if (gy > 65535) gy = 65535;
    dim3 grid(blocks_for(cols, bx), gy, 1), block(bx, by);
#define FV_LFC(T) hipLaunchKernelGGL((k_flux_curv<AX, T>), grid, block, 0, s, U, F, g, bcs)
    FV_DISPATCH_THREADS(threads, FV_LFC)
#undef FV_LFC
}

void launch_flux_curv(int ax, const double* U, double* F, const Geo& g, const BcState& bcs, int bx, int threads,
                      hipStream_t s) {
    if (ax == 0) launch_flux_curv_t<0>(U, F, g, bcs, bx, threads, s);
    else launch_flux_curv_t<1>(U, F, g, bcs, bx, threads, s);
}

void launch_flux(int ax, const double* U, double* F, const Geo& g, int bx, int threads, hipStream_t s) {
    if (g.ndim == 2) {
        if (ax == 0) launch_flux_t<2, 0>(U, F, g, bx, threads, s);
        else launch_flux_t<2, 1>(U, F, g, bx, threads, s);
    } else {
        if (ax == 0) launch_flux_t<3, 0>(U, F, g, bx, threads, s);
        else if (ax == 1) launch_flux_t<3, 1>(U, F, g, bx, threads, s);
        else launch_flux_t<3, 2>(U, F, g, bx, threads, s);
    }
}

// Viscous fluxes of axis ax subtracted from its face fluxes F (one thread per
// face, a fixed launch shape: not a tuned site).
void launch_visc(int ax, const double* U, double* F, const Geo& g, const BcState& bcs, hipStream_t s) {
    const int cols = g.n[0] + (ax == 0 ? 1 : 0);
    const int rows_j = g.n[1] + (ax == 1 ? 1 : 0);
    const int rows_k = g.ndim == 3 ? g.n[2] + (ax == 2 ? 1 : 0) : 1;
    const int nfaces = cols * rows_j * rows_k;
    const int blocks = blocks_for(nfaces, 256);
    if (g.ndim == 2) {
        if (ax == 0) hipLaunchKernelGGL((k_visc<2, 0>), dim3(blocks), dim3(256), 0, s, U, F, g, bcs, cols, rows_j, nfaces);
        else hipLaunchKernelGGL((k_visc<2, 1>), dim3(blocks), dim3(256), 0, s, U, F, g, bcs, cols, rows_j, nfaces);
    } else {
        if (ax == 0) hipLaunchKernelGGL((k_visc<3, 0>), dim3(blocks), dim3(256), 0, s, U, F, g, bcs, cols, rows_j, nfaces);
        else if (ax == 1)
            hipLaunchKernelGGL((k_visc<3, 1>), dim3(blocks), dim3(256), 0, s, U, F, g, bcs, cols, rows_j, nfaces);
        else hipLaunchKernelGGL((k_visc<3, 2>), dim3(blocks), dim3(256), 0, s, U, F, g, bcs, cols, rows_j, nfaces);
    }
}

void launch_residual(const double* Fx, const double* Fy, const double* Fz, const double* S, double* R, const Geo& g,
                     int gang, int threads, hipStream_t s) {
    int blocks, stride_all;
    grid1d(g.ncell, gang, threads, blocks, stride_all);
#define FV_LR(T)                                                                                              \
    if (g.ndim == 2)                                                                                          \
        hipLaunchKernelGGL((k_residual<2, T>), dim3(blocks), dim3(T), 0, s, Fx, Fy, Fz, S, R, g, stride_all); \
    else                                                                                                      \
        hipLaunchKernelGGL((k_residual<3, T>), dim3(blocks), dim3(T), 0, s, Fx, Fy, Fz, S, R, g, stride_all);
    FV_DISPATCH_THREADS(threads, FV_LR)
#undef FV_LR
}

void launch_residual_norm(const double* R, double* partial, double* norms, const Geo& g, hipStream_t s) {
    if (g.ndim == 2) {
        hipLaunchKernelGGL(k_sumsq<4>, dim3(NORM_BLOCKS), dim3(256), 0, s, R, g.ncell, partial);
        hipLaunchKernelGGL(k_norm_final<4>, dim3(1), dim3(256), 0, s, partial, g.ncell, norms);
    } else {
        hipLaunchKernelGGL(k_sumsq<5>, dim3(NORM_BLOCKS), dim3(256), 0, s, R, g.ncell, partial);
        hipLaunchKernelGGL(k_norm_final<5>, dim3(1), dim3(256), 0, s, partial, g.ncell, norms);
    }
}

template <int STAGE>
static void launch_update_t(const double* Un, const double* Us, double* Ud, const double* R, const double* dt,
                            const Geo& g, int gang, int threads, hipStream_t s) {
    int blocks, stride_all;
    grid1d(g.ncell, gang, threads, blocks, stride_all);
#define FV_LU(T)                                                                                              \
    if (g.ndim == 2)                                                                                          \
        hipLaunchKernelGGL((k_update<2, STAGE, T>), dim3(blocks), dim3(T), 0, s, Un, Us, Ud, R, dt, g, stride_all); \
    else                                                                                                      \
        hipLaunchKernelGGL((k_update<3, STAGE, T>), dim3(blocks), dim3(T), 0, s, Un, Us, Ud, R, dt, g, stride_all);
    FV_DISPATCH_THREADS(threads, FV_LU)
#undef FV_LU
}

void launch_update(int stage, const double* Un, const double* Us, double* Ud, const double* R, const double* dt,
                   const Geo& g, int gang, int threads, hipStream_t s) {
    if (stage == 0) launch_update_t<0>(Un, Us, Ud, R, dt, g, gang, threads, s);
    else if (stage == 1) launch_update_t<1>(Un, Us, Ud, R, dt, g, gang, threads, s);
    else launch_update_t<2>(Un, Us, Ud, R, dt, g, gang, threads, s);
}

int cfl_blocks(const Geo& g, int gang, int threads) {
    int blocks, stride_all;
    grid1d(g.ncell, gang, threads, blocks, stride_all);
    return blocks;
}

void launch_cfl(const double* U, double* partial, uint32_t* status, const double* dt_in, double* dt,
                double* dt_out, const Geo& g, int gang, int threads, hipStream_t s) {
    int blocks, stride_all;
    grid1d(g.ncell, gang, threads, blocks, stride_all);
#define FV_LC(T)                                                                                             \
    if (g.ndim == 2)                                                                                         \
        hipLaunchKernelGGL((k_cfl_partial<2, T>), dim3(blocks), dim3(T), 0, s, U, partial, status, g, stride_all); \
    else                                                                                                     \
        hipLaunchKernelGGL((k_cfl_partial<3, T>), dim3(blocks), dim3(T), 0, s, U, partial, status, g, stride_all);
    FV_DISPATCH_THREADS(threads, FV_LC)
#undef FV_LC
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, s, partial, blocks, dt_in, dt, dt_out, status, g.cfl);
}

void launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, s, p, v);
}

}  // namespace fvk
