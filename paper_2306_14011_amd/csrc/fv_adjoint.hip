// Adjoint (transpose-Jacobian) of the residual and of the SSP-RK3 stage
// combinations, FP64, gfx950.
//
// mu = (dR/dU)^T w is formed in gather form, without atomics:
//   1. per axis, one thread per face recomputes the MUSCL face states and runs
//      the reverse of the Roe flux and of the limiter with the face adjoint
//      Fb = area * (w_left - w_right) (w = 0 outside the interior); the four
//      contributions to the stencil cells k-1, k, k+1, k+2 go to
//      G[m][v][face], m = stencil position;
//   2. one thread per interior cell sums, per axis, the entries of the faces
//      whose stencil holds it, plus those of the ghost cells that copy it
//      (the transpose of the ghost fill: periodic wrap or transmissive clamp).
#include "fv_internal.h"

namespace fvk {

template <int NDIM, int AX, int MAXT>
__global__ void __launch_bounds__(MAXT) k_adj_flux(const double* __restrict__ U, const double* __restrict__ w,
                                                   double* __restrict__ G, Geo g) {
    constexpr int NV = NDIM + 2;
    const int cols = g.n[0] + (AX == 0 ? 1 : 0);
    const int rows_j = g.n[1] + (AX == 1 ? 1 : 0);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cols) return;
    const int k = blockIdx.z;
    const int st = AX == 0 ? 1 : (AX == 1 ? g.sy : g.sz);
    const long long fsv = g.fsv[AX];
    const int nax = g.n[AX];
    for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < rows_j; j += gridDim.y * blockDim.y) {
        const int c = g.off0 + i + j * g.sy + k * g.sz;  // right cell of the face
        const int fpos = AX == 0 ? i : (AX == 1 ? j : k);  // face index along the axis
        double q[4][NV], qL[NV], qR[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double* Uv = U + v * g.sv;
            q[0][v] = Uv[c - 2 * st];
            q[1][v] = Uv[c - st];
            q[2][v] = Uv[c];
            q[3][v] = Uv[c + st];
            muscl(q[0][v], q[1][v], q[2][v], q[3][v], g.scheme, qL[v], qR[v]);
        }
        // face adjoint: the face adds F*A to its left cell and -F*A to its right cell
        const int e = (k * g.n[1] + j) * g.n[0] + i;  // interior index of (i, j, k) when inside
        const int estep = AX == 0 ? 1 : (AX == 1 ? g.n[0] : g.n[0] * g.n[1]);
        const bool has_left = fpos >= 1, has_right = fpos <= nax - 1;
        double Fb[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double wl = has_left ? w[(long long)v * g.ncell + e - estep] : 0.0;
            const double wr = has_right ? w[(long long)v * g.ncell + e] : 0.0;
            Fb[v] = g.area[AX] * (wl - wr);
        }
        double qLb[NV], qRb[NV];
        roe_flux_vjp<NDIM, AX>(qL, qR, g.gm1, Fb, qLb, qRb);
        const long long f = (long long)(k * rows_j + j) * cols + i;
        const long long ms = (long long)NV * fsv;  // stride between stencil slots
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
            muscl_vjp(q[0][v], q[1][v], q[2][v], q[3][v], g.scheme, qLb[v], qRb[v], g0, g1, g2, g3);
            G[0 * ms + v * fsv + f] = g0;
            G[1 * ms + v * fsv + f] = g1;
            G[2 * ms + v * fsv + f] = g2;
            G[3 * ms + v * fsv + f] = g3;
        }
    }
}

// Sum over the faces of axis `ax` whose stencil holds position x of the axis:
// face f has cells f-2, f-1, f, f+1 at slots 0..3, so position x is slot m of
// face x + 2 - m. Ghost positions -2, -1, n, n+1 add their slots to the
// interior cell they copy; behind a slip wall the copy is the mirror image,
// times wsign (-1 for the momentum normal to the wall, else 1); behind an
// inflow face the ghost holds a given state and copies no cell.
__device__ __forceinline__ double gather_axis(const double* __restrict__ Gv, long long ms, int x, int n, int lo_kind,
                                              int hi_kind, long long fbase, long long fstride, double wsign) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int f = x + 2 - m;
        if (f >= 0 && f <= n) acc += Gv[m * ms + fbase + f * fstride];
    }
    // ghosts that copy x
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
        const int gp = gi < 2 ? gi - 2 : n + gi - 2;  // -2, -1, n, n+1
        const bool lo = gi < 2;
        const int kind = lo ? lo_kind : hi_kind;
        const int src = kind == 0   ? ((gp % n) + n) % n
                        : kind == 2 ? (lo ? -1 - gp : 2 * n - 1 - gp)
                        : kind == 3 ? -1
                                    : (lo ? 0 : n - 1);
        if (src != x) continue;
        const double sg = kind == 2 ? wsign : 1.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int f = gp + 2 - m;
            if (f >= 0 && f <= n) acc += sg * Gv[m * ms + fbase + f * fstride];
        }
    }
    return acc;
}

template <int NDIM, int MAXT>
__global__ void __launch_bounds__(MAXT) k_adj_gather(const double* __restrict__ Gx, const double* __restrict__ Gy,
                                                     const double* __restrict__ Gz, double* __restrict__ mu, Geo g,
                                                     int stride_all) {
    constexpr int NV = NDIM + 2;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.ncell; e += stride_all) {
        int i, j, k;
        const uint32_t t = divq((uint32_t)e, g.dnx);
        i = e - (int)t * nx;
        k = (int)divq(t, g.dny);
        j = (int)t - k * ny;
        // face arrays: x faces (k*ny + j)*(nx+1) + f; y faces (k*(ny+1) + f)*nx + i; z faces (f*ny + j)*nx + i
        const long long bx = (long long)(k * ny + j) * (nx + 1);
        const long long by = (long long)k * (ny + 1) * nx + i;
        const long long bz = (long long)j * nx + i;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double acc = gather_axis(Gx + v * g.fsv[0], (long long)NV * g.fsv[0], i, nx, g.bc[0][0], g.bc[0][1], bx, 1,
                                     v == 1 ? -1.0 : 1.0);
            acc += gather_axis(Gy + v * g.fsv[1], (long long)NV * g.fsv[1], j, ny, g.bc[1][0], g.bc[1][1], by, nx,
                               v == 2 ? -1.0 : 1.0);
            if (NDIM == 3)
                acc += gather_axis(Gz + v * g.fsv[2], (long long)NV * g.fsv[2], k, nz, g.bc[2][0], g.bc[2][1], bz,
                                   (long long)nx * ny, v == 3 ? -1.0 : 1.0);
            mu[(long long)v * g.ncell + e] = acc;
        }
    }
}

// Reverse of the SSP-RK3 stage combinations with L = -R/|Omega|, s = dt/|Omega|:
//   MODE 3: lamA = 2/3 lam - 2/3 s mu      (dJ/dU2)    lamB = 1/3 lam
//   MODE 2: lam  = 1/4 lamA - 1/4 s mu     (dJ/dU1)    lamB += 3/4 lamA
//   MODE 1: lam  = lamB + lam - s mu       (dJ/dU^n)
template <int MODE>
__global__ void __launch_bounds__(256) k_adj_comb(double* __restrict__ lam, double* __restrict__ lamA,
                                                  double* __restrict__ lamB, const double* __restrict__ mu,
                                                  const double* __restrict__ dtp, double inv_vol, long long n) {
    const double s = *dtp * inv_vol;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        if (MODE == 3) {
            const double l = lam[e];
            lamA[e] = (2.0 / 3.0) * l - (2.0 / 3.0) * s * mu[e];
            lamB[e] = (1.0 / 3.0) * l;
        } else if (MODE == 2) {
            const double a = lamA[e];
            lam[e] = 0.25 * a - 0.25 * s * mu[e];
            lamB[e] += 0.75 * a;
        } else {
            lam[e] = lamB[e] + lam[e] - s * mu[e];
        }
    }
}

// ---------------------------------------------------------------------------

template <int NDIM, int AX>
static void launch_adj_flux_t(const double* U, const double* w, double* G, const Geo& g, hipStream_t s) {
    constexpr int BX = 64, BY = 4;
    const int cols = g.n[0] + (AX == 0 ? 1 : 0);
    const int rows_j = g.n[1] + (AX == 1 ? 1 : 0);
    const int rows_k = NDIM == 3 ? g.n[2] + (AX == 2 ? 1 : 0) : 1;
    int gy = (rows_j + BY - 1) / BY;
    if (gy > 65535) gy = 65535;
    dim3 grid((cols + BX - 1) / BX, gy, rows_k);
    hipLaunchKernelGGL((k_adj_flux<NDIM, AX, BX * BY>), grid, dim3(BX, BY), 0, s, U, w, G, g);
}

void launch_adj_flux(int ax, const double* U, const double* w, double* G, const Geo& g, hipStream_t s) {
    if (g.ndim == 2) {
        if (ax == 0) launch_adj_flux_t<2, 0>(U, w, G, g, s);
        else launch_adj_flux_t<2, 1>(U, w, G, g, s);
    } else {
        if (ax == 0) launch_adj_flux_t<3, 0>(U, w, G, g, s);
        else if (ax == 1) launch_adj_flux_t<3, 1>(U, w, G, g, s);
        else launch_adj_flux_t<3, 2>(U, w, G, g, s);
    }
}

void launch_adj_gather(const double* Gx, const double* Gy, const double* Gz, double* mu, const Geo& g,
                       hipStream_t s) {
    constexpr int T = 256;
    const int blocks = (g.ncell + T - 1) / T;
    if (g.ndim == 2)
        hipLaunchKernelGGL((k_adj_gather<2, T>), dim3(blocks), dim3(T), 0, s, Gx, Gy, Gz, mu, g, blocks * T);
    else
        hipLaunchKernelGGL((k_adj_gather<3, T>), dim3(blocks), dim3(T), 0, s, Gx, Gy, Gz, mu, g, blocks * T);
}

void launch_adj_comb(int mode, double* lam, double* lamA, double* lamB, const double* mu, const double* dt,
                     const Geo& g, hipStream_t s) {
    const long long n = (long long)g.nvar * g.ncell;
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (mode == 3)
        hipLaunchKernelGGL(k_adj_comb<3>, dim3((unsigned)blocks), dim3(256), 0, s, lam, lamA, lamB, mu, dt, g.inv_vol, n);
    else if (mode == 2)
        hipLaunchKernelGGL(k_adj_comb<2>, dim3((unsigned)blocks), dim3(256), 0, s, lam, lamA, lamB, mu, dt, g.inv_vol, n);
    else
        hipLaunchKernelGGL(k_adj_comb<1>, dim3((unsigned)blocks), dim3(256), 0, s, lam, lamA, lamB, mu, dt, g.inv_vol, n);
}

}  // namespace fvk
