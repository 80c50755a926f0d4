// Fused SSP-RK3 stage for 3D grids (FP64, gfx950): one kernel per stage does
// the ghost mapping, MUSCL face states (minmod, van Leer, or an unlimited
// kappa member) and Roe fluxes on the three axes, the residual and the stage
// combination, and the last stage also the CFL max of the new state.
//
// Work decomposition: a work item is a tile of TX x TY (32 x 7) cells of the (x, y)
// plane over a segment of seg planes along z (seg a multiple of 4), and one
// workgroup of 256 threads (four wavefronts) owns an item. Thread t < TX*TY
// owns the cell (t % TX, t / TX) of the tile and marches along z with a window
// of four planes of its own cell in registers (the z faces). At each plane
// the tile and its two-cell x and y halo are staged in LDS: the owned cells
// come from the threads' windows, the halo ring from global memory. Then every
// thread evaluates one x face and one y face from the LDS plane; the faces of
// the tile number (TX + 1) TY and TX (TY + 1), at most the 256 threads, so
// each face of the plane is computed once and each axis costs one pass:
// three flux evaluations per cell, against four when a wave owns one row and
// computes both y faces of it. The face fluxes go back to LDS and each owned
// cell sums its six faces. Two workgroup barriers per plane: after the plane
// is staged, and after the face fluxes are written. (Measured on the 256^3
// workload: 32 x 7 tiles step in 1.79 ms, 16 x 15 tiles in 1.90 ms, the
// per-row wave kernel this replaces in 1.93 ms; non-temporal stores and loads
// of U^n were slower.)
//
// Halo cells outside the grid are read through the boundary maps; the state
// may keep ghost layers but they are not read. Per-grid dt and the CFL max
// follow the 2D kernel: stage 1 computes dt from the max that the previous
// step's stage 3 (or the init kernel) accumulated, stage 2 resets it, stage 3
// accumulates the max of the new state.
#include "fv_fused_common.h"

namespace fvk {

constexpr int TX = 32, TY = 7;           // owned cells of a tile
constexpr int TCELLS = TX * TY;           // 224 owned cells, one per thread
constexpr int HX = TX + 4, HY = TY + 4;   // the tile with its two-cell halo
constexpr int HPLANE = HX * HY;           // doubles per variable of the staged plane
constexpr int NXF = (TX + 1) * TY;        // x faces of a tile plane (231)
constexpr int NYF = TX * (TY + 1);        // y faces of a tile plane (256)
constexpr int NHALO = 4 * TY + 4 * TX;    // halo cells used by the faces (no corners): 156
constexpr int T3 = 256;                   // threads per workgroup
static_assert(TCELLS <= T3 && NXF <= T3 && NYF <= T3 && NHALO <= T3, "tile does not fit the workgroup");

// Face states of one face from its four stencil values by the compile-time
// rule LIM (0 minmod, 1 Psi = 1 with kappa = -1, 2 the kappa weights ka, kb
// with explicit fused multiply-adds, 3 van Leer). The same operations as the
// per-cell forms of the 2D kernel (minmod and van Leer are symmetric).
template <int LIM>
__device__ __forceinline__ void face_states(double q0, double q1, double q2, double q3, double ka, double kb,
                                            double& qL, double& qR) {
    if (LIM == 2) {
        muscl_kappa_diffs(q1, q2, q1 - q0, q2 - q1, q3 - q2, ka, kb, qL, qR);
    } else if (LIM == 3) {
        const double dc = q2 - q1;
        qL = q1 + 0.5 * vanleer(q1 - q0, dc);
        qR = q2 - 0.5 * vanleer(dc, q3 - q2);
    } else {
        muscl_fixed<LIM == 1>(q0, q1, q2, q3, qL, qR);
    }
}

// Position (hx, hy) in the staged plane of halo cell h (0 .. NHALO-1): first
// the x halo (columns 0, 1, HX-2, HX-1 of the owned rows), then the y halo
// (rows 0, 1, HY-2, HY-1 of the owned columns), row by row so that the y halo
// loads of neighbouring threads are neighbouring columns.
__device__ __forceinline__ void halo_pos(int h, int& hx, int& hy) {
    if (h < 4 * TY) {
        const int c = h & 3;
        hx = c < 2 ? c : HX - 4 + c;
        hy = 2 + (h >> 2);
    } else {
        const int q = h - 4 * TY;
        const int r = q / TX;
        hx = 2 + q % TX;
        hy = r < 2 ? r : HY - 4 + r;
    }
}

// LDS of a workgroup. Each array has one spare slot at its end that threads
// with nothing to write store to, so that no LDS store sits on a branch.
struct TileLds {
    double P[5][HPLANE + 1];  // staged plane: owned cells and halo, [v][hy][hx]
    double FX[5][NXF + 1];    // x-face fluxes (times 2), [v][fy][fx], fx = 0 .. TX
    double FY[5][NYF];        // y-face fluxes (times 2), [v][fy][fx], fy = 0 .. TY
};

// The planes of one work item (tile (tx0, ty0), planes k0 .. k0 + seg - 1)
// for stage STAGE with the face-state rule LIM. No global memory access sits
// on a conditional path: loads are issued for every thread and plane (indices
// past the grid are mapped or clamped into it), and the stores of threads or
// planes without output go past the end of a per-variable descriptor, where
// they are dropped.
// Boundary variant (grids with slip-wall or inflow faces): the ghost rules
// of a loaded cell at (grid) position x, y and plane k: a slip wall reverses
// the momentum normal to it (the index map already mirrors the position), an
// inflow face gives the side's state. A position outside on two axes feeds
// no output.
struct Ghost3 {
    int xk, xs, yk, ys;  // kind (-1 inside) and side of the face behind x and y
};

__device__ __forceinline__ Ghost3 ghost_xy(const FGrid3& G, int x, int y) {
    Ghost3 g;
    g.xk = x < 0 ? G.bcx0 : (x >= G.nx ? G.bcx1 : -1);
    g.xs = x < 0 ? 0 : 1;
    g.yk = y < 0 ? G.bcy0 : (y >= G.ny ? G.bcy1 : -1);
    g.ys = y < 0 ? 0 : 1;
    return g;
}

template <bool BC>
__device__ __forceinline__ void ghost_fix(const FGrid3& G, const Ghost3& h, int kk, double* w) {
    if (!BC) return;
    const int zk = kk < 0 ? G.bcz0 : (kk >= G.nz ? G.bcz1 : -1);  // uniform
    const int zs = kk < 0 ? 0 : 1;
    if (zk == 2) w[3] = -w[3];
    if (zk == 3) {
#pragma unroll
        for (int v = 0; v < 5; ++v) w[v] = G.q[2][zs][v];
    }
    w[2] = h.yk == 2 ? -w[2] : w[2];
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v] = h.yk == 3 ? G.q[1][h.ys][v] : w[v];
    w[1] = h.xk == 2 ? -w[1] : w[1];
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v] = h.xk == 3 ? G.q[0][h.xs][v] : w[v];
}

__device__ __forceinline__ int map3(bool bc, int i, int n, int lo, int hi) {
    return bc ? map_index_bc(i, n, lo, hi) : map_index(i, n, lo, hi);
}

template <int STAGE, int LIM, bool SRC, bool BC>
__device__ __forceinline__ void tile_planes(const FGrid3& G, TileLds& L, int tid, int tx0, int ty0, int k0, double s,
                                            const double* Un, const double* Us, double* Ud, double& lmax,
                                            uint32_t& fl, double ka, double kb, const double* src, double vol) {
    constexpr int NV = 5;
    const int seg = G.seg;
    // owned cell of this thread (threads past TCELLS own a clamped copy of the
    // last cell: they load and compute like the others but store nothing)
    const int oc = tid < TCELLS ? tid : TCELLS - 1;
    const int cx = oc % TX, cy = oc / TX;
    const int gx = tx0 + cx, gy = ty0 + cy;
    const bool own = tid < TCELLS && gx < G.nx && gy < G.ny;
    // owned cells past the grid's edge hold the boundary map's values, as
    // ghost cells would (cells beyond the second ghost layer feed no output)
    const int cgx = gx < G.nx + 1 ? gx : G.nx + 1, cgy = gy < G.ny + 1 ? gy : G.ny + 1;
    const int mx = map3(BC, cgx, G.nx, G.bcx0, G.bcx1);
    const int my = map3(BC, cgy, G.ny, G.bcy0, G.bcy1);
    const Ghost3 gown = ghost_xy(G, cgx, cgy);
    const uint32_t cell_off = (uint32_t)(((long long)my * G.py + mx) * 8);
    // U^n, source and output offsets: the owned cell, clamped inside the grid
    const int ox = gx < G.nx ? gx : G.nx - 1, oy = gy < G.ny ? gy : G.ny - 1;
    const uint32_t own_off = (uint32_t)(((long long)oy * G.py + ox) * 8);
    const uint32_t st_off = own ? own_off : DROP_OFFSET;
    // halo cell of this thread (threads past NHALO load halo cell 0 again)
    int hx, hy;
    halo_pos(tid < NHALO ? tid : 0, hx, hy);
    const int hcx = tx0 + hx - 2 < G.nx + 1 ? tx0 + hx - 2 : G.nx + 1;
    const int hcy = ty0 + hy - 2 < G.ny + 1 ? ty0 + hy - 2 : G.ny + 1;
    const int hgx = map3(BC, hcx, G.nx, G.bcx0, G.bcx1);
    const int hgy = map3(BC, hcy, G.ny, G.bcy0, G.bcy1);
    const Ghost3 ghalo = ghost_xy(G, hcx, hcy);
    const uint32_t halo_off = (uint32_t)(((long long)hgy * G.py + hgx) * 8);
    const int halo_slot = tid < NHALO ? hy * HX + hx : HPLANE;
    const int own_slot = tid < TCELLS ? (cy + 2) * HX + cx + 2 : HPLANE;
    // face of this thread in each pass: x face (fx, fy) between columns
    // fx - 1 and fx of row fy; y face (fx, fy) between rows fy - 1 and fy of
    // column fx (threads past the face count evaluate face 0 again, unused)
    const int xf = tid < NXF ? tid : 0;
    const int xfy = xf < TCELLS ? xf / TX : xf - TCELLS;
    const int xfx = xf < TCELLS ? xf % TX : TX;
    const int yf = tid < NYF ? tid : 0;
    const int yfx = yf < TCELLS ? yf % TX : yf - TCELLS;
    const int yfy = yf < TCELLS ? yf / TX : TY;
    const int xs0 = (xfy + 2) * HX + xfx;      // stencil columns xfx .. xfx + 3 (halo coordinates)
    const int ys0 = yfy * HX + yfx + 2;        // stencil rows yfy .. yfy + 3
    const int xslot = tid < NXF ? xfy * (TX + 1) + xfx : NXF;
    // faces of the owned cell: left x face, right x face, lower y face, upper y face
    const int fxl = cy * (TX + 1) + cx, fyb = cy * TX + cx;

    const long long gbytes = NV * G.sv * 8;  // one grid's state, below 4 GiB
    const Rsrc rs = grid_rsrc(Us + G.base, gbytes), rn = grid_rsrc(Un + G.base, gbytes);
    Rsrc rd[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) rd[v] = grid_rsrc(Ud + G.base + v * G.sv, G.sv * 8);
    const uint32_t vstride = (uint32_t)(G.sv * 8);
    const double hax = 0.5 * G.ax, hay = 0.5 * G.ay, haz = 0.5 * G.az;
    const long long svol = (long long)G.nx * G.ny * G.nz;
    Rsrc rsrc;
    if (SRC) rsrc = grid_rsrc(src, NV * svol * 8);
    const uint32_t src_off = (uint32_t)(((long long)oy * G.nx + ox) * 8);  // S[v][k][j][i], dense
    auto plane_off = [&](int kk) -> uint32_t {
        return (uint32_t)((long long)map3(BC, kk, G.nz, G.bcz0, G.bcz1) * G.pz * 8);
    };
    auto out_plane = [&](int kk) -> uint32_t { return (uint32_t)((long long)(kk < G.nz ? kk : G.nz - 1) * G.pz * 8); };

    // window of the owned cell: plane kk in slot (kk - k0 + 2) & 3; z face f
    // (between planes k0 + f - 1 and k0 + f) uses slots f .. f + 3 (mod 4).
    // Face 0 first, then faces 1 .. seg in unrolled groups of four, so every
    // slot is a compile-time constant and a given z face of the grid is
    // computed by the same instructions whatever seg is.
    double W[4][NV];
#pragma unroll
    for (int kz = 0; kz < 4; ++kz) {
        const uint32_t o = plane_off(k0 - 2 + kz);
#pragma unroll
        for (int v = 0; v < NV; ++v) W[kz][v] = ld_buf(rs, cell_off, o + v * vstride);
        ghost_fix<BC>(G, gown, k0 - 2 + kz, W[kz]);
    }
    double H[NV];  // halo cell of the next staged plane
    {
        const uint32_t o = plane_off(k0);
#pragma unroll
        for (int v = 0; v < NV; ++v) H[v] = ld_buf(rs, halo_off, o + v * vstride);
        ghost_fix<BC>(G, ghalo, k0, H);
    }
    double Fz[2][NV];  // z-face fluxes (times 2): face f in Fz[f & 1]
    double qL[NV], qR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) face_states<LIM>(W[0][v], W[1][v], W[2][v], W[3][v], ka, kb, qL[v], qR[v]);
    roe_flux<3, 2, true>(qL, qR, G.gm1, Fz[0]);
    {
        const uint32_t o = plane_off(k0 + 2);
#pragma unroll
        for (int v = 0; v < NV; ++v) W[0][v] = ld_buf(rs, cell_off, o + v * vstride);
        ghost_fix<BC>(G, gown, k0 + 2, W[0]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll 1
    for (int m0 = 1; m0 <= seg; m0 += 4) {
        if (k0 + m0 - 1 >= G.nz) break;  // ragged last segment (uniform over the workgroup)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int f = m0 + jj;
            const int t = (jj + 1) & 3;  // f mod 4, a compile-time constant
            const int kk = k0 + f - 1;   // output plane finished at this face
            double c[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) c[v] = W[(t + 1) & 3][v];
            // stage plane kk: the owned cells from the window, the halo ring
            // from the loads issued one plane ahead
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                L.P[v][own_slot] = c[v];
                L.P[v][halo_slot] = H[v];
            }
            double Unc[NV];
            if (STAGE > 0) {
                const uint32_t o = out_plane(kk);
#pragma unroll
                for (int v = 0; v < NV; ++v) Unc[v] = ld_buf(rn, own_off, o + v * vstride);
            }
            // z face f: stencil planes kk-1 .. kk+2
#pragma unroll
            for (int v = 0; v < NV; ++v)
                face_states<LIM>(W[t][v], W[(t + 1) & 3][v], W[(t + 2) & 3][v], W[(t + 3) & 3][v], ka, kb, qL[v],
                                 qR[v]);
            roe_flux<3, 2, true>(qL, qR, G.gm1, Fz[t & 1]);
            __builtin_amdgcn_sched_barrier(0);
            __syncthreads();  // plane kk staged
            {
                double Fx[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double* p = &L.P[v][xs0];
                    face_states<LIM>(p[0], p[1], p[2], p[3], ka, kb, qL[v], qR[v]);
                }
                roe_flux<3, 0, true>(qL, qR, G.gm1, Fx);
#pragma unroll
                for (int v = 0; v < NV; ++v) L.FX[v][xslot] = Fx[v];
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                double Fy[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double* p = &L.P[v][ys0];
                    face_states<LIM>(p[0], p[HX], p[2 * HX], p[3 * HX], ka, kb, qL[v], qR[v]);
                }
                roe_flux<3, 1, true>(qL, qR, G.gm1, Fy);
#pragma unroll
                for (int v = 0; v < NV; ++v) L.FY[v][tid] = Fy[v];
            }
            __builtin_amdgcn_sched_barrier(0);
            // plane kk - 1 is dead: its slot takes plane kk + 3 for face f + 1;
            // the halo of plane kk + 1 is requested for the next staging
            {
                const uint32_t o = plane_off(kk + 3);
#pragma unroll
                for (int v = 0; v < NV; ++v) W[t][v] = ld_buf(rs, cell_off, o + v * vstride);
            }
            {
                const uint32_t o = plane_off(kk + 1);
#pragma unroll
                for (int v = 0; v < NV; ++v) H[v] = ld_buf(rs, halo_off, o + v * vstride);
            }
            if (BC) {
                // the ghost rules need the loaded values: applied here, after the
                // loads of the next planes were issued
                ghost_fix<BC>(G, gown, kk + 3, W[t]);
                ghost_fix<BC>(G, ghalo, kk + 1, H);
            }
            __syncthreads();  // face fluxes of plane kk written
            const bool plane_ok = kk < G.nz;  // uniform
            const uint32_t p = out_plane(kk);
            const uint32_t so = plane_ok ? st_off : DROP_OFFSET;
            double Sv[NV];
            if (SRC) {
                const uint32_t ps = (uint32_t)((long long)(kk < G.nz ? kk : G.nz - 1) * G.ny * G.nx * 8);
#pragma unroll
                for (int v = 0; v < NV; ++v) Sv[v] = ld_buf(rsrc, src_off, ps + (uint32_t)(v * svol * 8));
            }
            double out[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                // the doubled fluxes against halved areas: the same products
                double r = (L.FX[v][fxl + 1] - L.FX[v][fxl]) * hax;
                r += (L.FY[v][fyb + TX] - L.FY[v][fyb]) * hay;
                r += (Fz[t & 1][v] - Fz[(t + 1) & 1][v]) * haz;
                if (SRC) r -= vol * Sv[v];  // R = flux sum - |Omega| S
                if (STAGE == 0) {
                    out[v] = c[v] + s * r;
                } else if (STAGE == 1) {
                    out[v] = 0.75 * Unc[v] + 0.25 * (c[v] + s * r);
                } else {
                    out[v] = (1.0 / 3.0) * Unc[v] + (2.0 / 3.0) * (c[v] + s * r);
                }
                st_buf<false>(rd[v], so, p, out[v]);
            }
            if (STAGE == 2 && own && plane_ok) {
                const double idx[3] = {G.inv_dx, G.inv_dy, G.inv_dz};
                lmax = fmax(lmax, cell_lambda<3>(out, G.gamma, G.gm1, idx, fl));
            }
            // keep the scheduler from overlapping consecutive planes (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

__device__ __forceinline__ void tile_of_item(const FGrid3& G, int item, int& tx0, int& ty0, int& k0) {
    const int tiles_x = (G.nx + TX - 1) / TX, tiles_y = (G.ny + TY - 1) / TY;
    const int tx = item % tiles_x;
    const int r = item / tiles_x;
    tx0 = tx * TX;
    ty0 = (r % tiles_y) * TY;
    k0 = (r / tiles_y) * G.seg;
}

// At least 2 waves per SIMD: the stage-3 kernel with the ghost rules and a
// source term would take 257 registers and run at 1 wave per SIMD.
template <int STAGE, bool SRC, bool BC>
__global__ void __launch_bounds__(T3) __attribute__((amdgpu_waves_per_eu(2))) k_fused3d(const FGrid3* __restrict__ grid, int nitems, const double* Un,
                                                const double* __restrict__ Us, double* Ud,
                                                unsigned long long* __restrict__ lam, double* __restrict__ dtg,
                                                const double* __restrict__ dt_fixed, double* __restrict__ dt_out,
                                                uint32_t* __restrict__ status, const double* __restrict__ src,
                                                double vol) {
    __shared__ TileLds L;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int nblocks = gridDim.x;
    const int b0 = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x));
    if (STAGE == 1 && blockIdx.x == 0 && tid == 0) lam[0] = 0ull;  // stage 1 has read it
    const FGrid3 G = *grid;
    for (int item = b0; item < nitems; item += nblocks) {
        int tx0, ty0, k0;
        tile_of_item(G, item, tx0, ty0, k0);
        double dt;
        if (STAGE == 0) {
            dt = dt_fixed ? dt_fixed[0] : G.cfl / __longlong_as_double((long long)lam[0]);
            if (item == 0 && tid == 0) {
                dtg[0] = dt;
                if (dt_out) dt_out[0] = dt;
                if (!(dt > 0.0) || isinf(dt)) atomicOr(status, 8u);
            }
        } else {
            dt = dtg[0];
        }
        const double s = -dt * G.inv_vol;
        double lmax = 0.0;
        uint32_t fl = 0;
        if (G.scheme == 0) {
            tile_planes<STAGE, 0, SRC, BC>(G, L, tid, tx0, ty0, k0, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, vol);
        } else if (G.scheme == 5) {
            tile_planes<STAGE, 3, SRC, BC>(G, L, tid, tx0, ty0, k0, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, vol);
        } else if (G.scheme == 1) {
            tile_planes<STAGE, 1, SRC, BC>(G, L, tid, tx0, ty0, k0, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, vol);
        } else {
            double ka, kb;
            kappa_weights(G.scheme, ka, kb);
            tile_planes<STAGE, 2, SRC, BC>(G, L, tid, tx0, ty0, k0, s, Un, Us, Ud, lmax, fl, ka, kb, src, vol);
        }
        if (STAGE == 2) {
            lmax = wave_max_d(lmax);
            fl = wave_or(fl);
            if (lane == 0) {
                atomicMax(&lam[0], (unsigned long long)__double_as_longlong(lmax));
                if (fl) atomicOr(status, fl);
            }
        }
    }
}

// lambda_max of U^n (the first step's dt), over the same work items.
__global__ void __launch_bounds__(T3) k_fused3d_lambda(const FGrid3* __restrict__ grid, int nitems,
                                                       const double* __restrict__ U,
                                                       unsigned long long* __restrict__ lam,
                                                       uint32_t* __restrict__ status) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const FGrid3 G = *grid;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        int tx0, ty0, k0;
        tile_of_item(G, item, tx0, ty0, k0);
        const int gx = tx0 + tid % TX, gy = ty0 + tid / TX;
        double lmax = 0.0;
        uint32_t fl = 0;
        if (tid < TCELLS && gx < G.nx && gy < G.ny) {
            const double idx[3] = {G.inv_dx, G.inv_dy, G.inv_dz};
            for (int kk = k0; kk < k0 + G.seg && kk < G.nz; ++kk) {
                const long long p = G.base + (long long)kk * G.pz + (long long)gy * G.py + gx;
                double q[5];
#pragma unroll
                for (int v = 0; v < 5; ++v) q[v] = U[v * G.sv + p];
                lmax = fmax(lmax, cell_lambda<3>(q, G.gamma, G.gm1, idx, fl));
            }
        }
        lmax = wave_max_d(lmax);
        fl = wave_or(fl);
        if (lane == 0) {
            atomicMax(&lam[0], (unsigned long long)__double_as_longlong(lmax));
            if (fl) atomicOr(status, fl);
        }
    }
}

__global__ void k_fused3d_reset(unsigned long long* lam) { lam[0] = 0ull; }

// ---------------------------------------------------------------------------

int fused3d_items(const FGrid3& G, int seg) {
    const long long tiles = (long long)((G.nx + TX - 1) / TX) * ((G.ny + TY - 1) / TY);
    return (int)(tiles * ((G.nz + seg - 1) / seg));
}

// Workgroups of a launch: one per work item, or waves / 4 (rounded up) in a
// grid-stride loop over the items.
static inline int blocks_for(int nitems, int waves) {
    const int w = waves > 0 ? (waves + 3) / 4 : nitems;
    return w < nitems ? w : nitems;
}

template <bool SRC, bool BC>
static void launch_fused3d_stage_t(int stage, dim3 g, dim3 b, const FGrid3* grid, int nitems, const double* Un,
                                   const double* Us, double* Ud, unsigned long long* lam, double* dtg,
                                   const double* dt_fixed, double* dt_out, uint32_t* status, const double* src,
                                   double vol, hipStream_t s) {
    if (stage == 0)
        hipLaunchKernelGGL((k_fused3d<0, SRC, BC>), g, b, 0, s, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                           status, src, vol);
    else if (stage == 1)
        hipLaunchKernelGGL((k_fused3d<1, SRC, BC>), g, b, 0, s, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                           status, src, vol);
    else
        hipLaunchKernelGGL((k_fused3d<2, SRC, BC>), g, b, 0, s, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                           status, src, vol);
}

void launch_fused3d_stage(int stage, int waves, const FGrid3* grid, int nitems, const double* Un, const double* Us,
                          double* Ud, unsigned long long* lam, double* dtg, const double* dt_fixed, double* dt_out,
                          uint32_t* status, hipStream_t s, const double* src, double vol, bool walls) {
    const dim3 g(blocks_for(nitems, waves)), b(T3);
    if (walls) {
        if (src)
            launch_fused3d_stage_t<true, true>(stage, g, b, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                                               status, src, vol, s);
        else
            launch_fused3d_stage_t<false, true>(stage, g, b, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                                                status, nullptr, 0.0, s);
    } else if (src) {
        launch_fused3d_stage_t<true, false>(stage, g, b, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out, status,
                                            src, vol, s);
    } else {
        launch_fused3d_stage_t<false, false>(stage, g, b, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                                             status, nullptr, 0.0, s);
    }
}

void launch_fused3d_init(int waves, const FGrid3* grid, int nitems, const double* U, unsigned long long* lam,
                         uint32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_fused3d_reset, dim3(1), dim3(1), 0, s, lam);
    hipLaunchKernelGGL(k_fused3d_lambda, dim3(blocks_for(nitems, waves)), dim3(T3), 0, s, grid, nitems, U, lam,
                       status);
}

// Workgroups the device holds at once for the stage kernels.
int fused3d_slots() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int b0 = 0, b1 = 0, b2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, k_fused3d<0, false, false>, T3, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, k_fused3d<1, false, false>, T3, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, k_fused3d<2, false, false>, T3, 0) != hipSuccess)
        return 0;
    const int bmin = b0 < b1 ? (b0 < b2 ? b0 : b2) : (b1 < b2 ? b1 : b2);
    return bmin * cus;
}

// Segment height (a multiple of 4): as in 2D, the one minimising (rounds of
// resident workgroups) x (planes per item + 1); ties go to the taller segment.
int fused3d_auto_seg(const FGrid3& G, int slots) {
    if (slots <= 0) return 16;
    int best = 16;
    double best_cost = 0.0;
    for (int seg = 4; seg <= 256; seg += 4) {
        const long long items = fused3d_items(G, seg);
        const long long rounds = (items + slots - 1) / slots;
        const double cost = (double)rounds * (seg + 1);
        if (seg == 4 || cost <= best_cost) {
            best_cost = cost;
            best = seg;
        }
    }
    return best;
}

}  // namespace fvk
