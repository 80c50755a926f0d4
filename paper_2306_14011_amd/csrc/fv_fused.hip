// Fused SSP-RK3 stage for 2D grids (FP64, gfx950): one kernel per stage does
// the ghost mapping, MUSCL-minmod + Roe fluxes on both axes, the residual and
// the stage combination, and the last stage also the CFL max of the new state.
//
// Work decomposition: a work item is a 60-column strip x SEG-row segment of
// one grid; one wavefront (64 lanes) owns an item. Lane l holds column
// x0 + l, x0 = 60*strip - 2, so lanes 2..61 produce the 60 output columns and
// lanes 0, 1, 62, 63 carry the x halo. The wave marches up the segment one row
// at a time, keeping the last four rows in registers: that window gives the
// y-face flux, and the x-stencil and the right-face flux come from
// neighbouring lanes by wave shuffles. No LDS and no block barriers.
//
// Halo cells outside a grid are read through the boundary map (periodic
// wrap, transmissive clamp), so no ghost layers are needed. A grid table
// (FGrid) describes each grid's layout and constants; work items of grid g
// are [work0[g], work0[g+1]).
//
// Per-grid dt: stage 1 computes dt = cfl / lambda_max(U^n) from the max that
// the previous step's stage 3 (or the init kernel) accumulated; stage 2
// resets the accumulator; stage 3 accumulates lambda_max(U^{n+1}) with an
// atomic max on the bit pattern of the (non-negative) double.
#include "fv_internal.h"

namespace fvk {

constexpr int FW = 60;  // output columns per wave

__device__ __forceinline__ int map_index(int i, int n, int lo_kind, int hi_kind) {
    if (i < 0) return lo_kind == 0 ? ((i % n) + n) % n : 0;
    if (i >= n) return hi_kind == 0 ? i % n : n - 1;
    return i;
}

// Grid of the work item (uniform): largest g with work0 <= item.
__device__ __forceinline__ int find_grid(const FGrid* __restrict__ grids, int ngrids, int item) {
    int lo = 0, hi = ngrids - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (grids[mid].work0 <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off, 64);
    return v;
}

template <int STAGE, int SEG>
__global__ void __launch_bounds__(256) k_fused2d(const FGrid* __restrict__ grids, int ngrids, int nitems,
                                                 const double* Un, const double* __restrict__ Us, double* Ud,
                                                 unsigned long long* __restrict__ lam, double* __restrict__ dtg,
                                                 const double* __restrict__ dt_fixed, double* __restrict__ dt_out,
                                                 uint32_t* __restrict__ status, unsigned long long* __restrict__ clk) {
    constexpr int NV = 4;
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int wave0 = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (STAGE == 1 && blockIdx.x == 0)
        for (int g = threadIdx.x; g < ngrids; g += blockDim.x) lam[g] = 0ull;  // stage 1 has read it
    for (int item = wave0; item < nitems; item += nwaves) {
        unsigned long long t_start = 0;
        if (clk) t_start = wall_clock64();
        const int gi = find_grid(grids, ngrids, item);
        const FGrid G = grids[gi];
        const int local = item - G.work0;
        const int strip = local % G.strips;
        const int seg = local / G.strips;
        double dt;
        if (STAGE == 0) {
            dt = dt_fixed ? dt_fixed[G.gid] : G.cfl / __longlong_as_double((long long)lam[G.gid]);
            if (local == 0 && lane == 0) {
                dtg[G.gid] = dt;
                if (dt_out) dt_out[G.gid] = dt;
                if (!(dt > 0.0) || isinf(dt)) atomicOr(status, 8u);
            }
        } else {
            dt = dtg[G.gid];
        }
        const double s = -dt * G.inv_vol;
        const int col = FW * strip - 2 + lane;
        const int cmap = map_index(col < G.nx + 2 ? col : G.nx - 1, G.nx, G.bcx0, G.bcx1);
        const bool out_lane = lane >= 2 && lane < 2 + FW && col < G.nx;
        const int r0 = seg * SEG;
        const double* Usg = Us + G.base + cmap;
        double W[4][NV];
        double Fyb[NV];
        double lmax = 0.0;
        uint32_t fl = 0;
        // software pipeline: the next row of U_s and the U^n value of the next
        // finalised row are requested one iteration ahead of their use
        double Wn[NV], Unc[NV], Unn[NV];
        {
            const int rmap = map_index(r0 - 2, G.ny, G.bcy0, G.bcy1);
#pragma unroll
            for (int v = 0; v < NV; ++v) Wn[v] = Usg[v * G.sv + (long long)rmap * G.pitch];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) Unc[v] = Unn[v] = 0.0;
#pragma unroll 1
        for (int t = 0; t < SEG + 4; ++t) {
            const int row = r0 - 2 + t;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                W[0][v] = W[1][v];
                W[1][v] = W[2][v];
                W[2][v] = W[3][v];
                W[3][v] = Wn[v];
                Unc[v] = Unn[v];
            }
            if (t + 1 < SEG + 4) {
                const int nrow = row + 1;
                const int rmap = map_index(nrow < G.ny + 2 ? nrow : G.ny - 1, G.ny, G.bcy0, G.bcy1);
#pragma unroll
                for (int v = 0; v < NV; ++v) Wn[v] = Usg[v * G.sv + (long long)rmap * G.pitch];
            }
            if (STAGE > 0 && t >= 3 && t + 1 < SEG + 4) {
                // U^n of the row finalised in the next iteration (row - 1), clamped inside the grid
                const int fr = row - 1 < G.ny ? row - 1 : G.ny - 1;
                const long long pn = G.base + (long long)fr * G.pitch + (out_lane ? col : 0);
#pragma unroll
                for (int v = 0; v < NV; ++v) Unn[v] = Un[v * G.sv + pn];
            }
            if (t < 3) continue;
            // y face between rows row-2 and row-1 (stencil rows row-3 .. row)
            double qL[NV], qR[NV], Fyt[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) muscl(W[0][v], W[1][v], W[2][v], W[3][v], G.unlimited, qL[v], qR[v]);
            roe_flux<2, 1>(qL, qR, G.gm1, Fyt);
            if (t >= 4) {
                // finalise cell row rr = row - 2 (held in W[1])
                const int rr = row - 2;
                double Fxl[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double c1 = W[1][v];
                    const double a = __shfl_up(c1, 2, 64);
                    const double b = __shfl_up(c1, 1, 64);
                    const double d = __shfl_down(c1, 1, 64);
                    muscl(a, b, c1, d, G.unlimited, qL[v], qR[v]);
                }
                roe_flux<2, 0>(qL, qR, G.gm1, Fxl);
                double Fxr[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) Fxr[v] = __shfl_down(Fxl[v], 1, 64);
                if (out_lane && rr < G.ny) {
                    const long long p = G.base + (long long)rr * G.pitch + col;
                    double out[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        double r = (Fxr[v] - Fxl[v]) * G.ax;
                        r += (Fyt[v] - Fyb[v]) * G.ay;
                        if (STAGE == 0) {
                            out[v] = W[1][v] + s * r;
                        } else if (STAGE == 1) {
                            out[v] = 0.75 * Unc[v] + 0.25 * (W[1][v] + s * r);
                        } else {
                            out[v] = (1.0 / 3.0) * Unc[v] + (2.0 / 3.0) * (W[1][v] + s * r);
                        }
                        Ud[v * G.sv + p] = out[v];
                    }
                    if (STAGE == 2) {
                        const double idx[2] = {G.inv_dx, G.inv_dy};
                        lmax = fmax(lmax, cell_lambda<2>(out, G.gamma, G.gm1, idx, fl));
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) Fyb[v] = Fyt[v];
        }
        if (STAGE == 2) {
            lmax = wave_max_d(lmax);
            fl = wave_or(fl);
            if (lane == 0) {
                atomicMax(&lam[G.gid], (unsigned long long)__double_as_longlong(lmax));
                if (fl) atomicOr(status, fl);
            }
        }
        if (clk && lane == 0) {
            const unsigned long long t_end = wall_clock64();
            atomicMin(&clk[(G.gid * 3 + STAGE) * 2 + 0], t_start);
            atomicMax(&clk[(G.gid * 3 + STAGE) * 2 + 1], t_end);
        }
    }
}

// lambda_max of U^n per grid (the first step's dt), same work items.
template <int SEG>
__global__ void __launch_bounds__(256) k_fused_lambda(const FGrid* __restrict__ grids, int ngrids, int nitems,
                                                      const double* __restrict__ U, unsigned long long* __restrict__ lam,
                                                      uint32_t* __restrict__ status) {
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int wave0 = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    for (int item = wave0; item < nitems; item += nwaves) {
        const int gi = find_grid(grids, ngrids, item);
        const FGrid G = grids[gi];
        const int local = item - G.work0;
        const int strip = local % G.strips;
        const int seg = local / G.strips;
        const int col = FW * strip + lane;
        double lmax = 0.0;
        uint32_t fl = 0;
        if (lane < FW && col < G.nx) {
            const double idx[2] = {G.inv_dx, G.inv_dy};
            for (int rr = seg * SEG; rr < seg * SEG + SEG && rr < G.ny; ++rr) {
                const long long p = G.base + (long long)rr * G.pitch + col;
                double q[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) q[v] = U[v * G.sv + p];
                lmax = fmax(lmax, cell_lambda<2>(q, G.gamma, G.gm1, idx, fl));
            }
        }
        lmax = wave_max_d(lmax);
        fl = wave_or(fl);
        if (lane == 0) {
            atomicMax(&lam[G.gid], (unsigned long long)__double_as_longlong(lmax));
            if (fl) atomicOr(status, fl);
        }
    }
}

// Zero the lambda accumulators; clocks to (max, 0) when present.
__global__ void k_fused_reset(unsigned long long* lam, int ngrids, unsigned long long* clk) {
    for (int g = threadIdx.x; g < ngrids; g += blockDim.x) {
        lam[g] = 0ull;
        if (clk)
            for (int s = 0; s < 3; ++s) {
                clk[(g * 3 + s) * 2 + 0] = ~0ull;
                clk[(g * 3 + s) * 2 + 1] = 0ull;
            }
    }
}

// ---------------------------------------------------------------------------

int fused_items(const FGrid& G, int seg) { return G.strips * ((G.ny + seg - 1) / seg); }

int fused_strips(int nx) { return (nx + FW - 1) / FW; }

static inline int fused_blocks(int nitems, int waves) {
    const int w = waves > 0 ? (waves < nitems ? waves : nitems) : nitems;
    return (w + 3) / 4;
}

#define FV_SEG_DISPATCH(SEGV, MACRO)         \
    switch (SEGV) {                          \
        case 8: MACRO(8); break;             \
        case 32: MACRO(32); break;           \
        case 64: MACRO(64); break;           \
        default: MACRO(16); break;           \
    }

void launch_fused_stage(int stage, int seg, int waves, const FGrid* grids, int ngrids, int nitems, const double* Un,
                        const double* Us, double* Ud, unsigned long long* lam, double* dtg, const double* dt_fixed,
                        double* dt_out, uint32_t* status, unsigned long long* clk, hipStream_t s) {
    const dim3 grid(fused_blocks(nitems, waves)), block(256);
#define FV_LFS(SV)                                                                                               \
    if (stage == 0)                                                                                              \
        hipLaunchKernelGGL((k_fused2d<0, SV>), grid, block, 0, s, grids, ngrids, nitems, Un, Us, Ud, lam, dtg,   \
                           dt_fixed, dt_out, status, clk);                                                       \
    else if (stage == 1)                                                                                         \
        hipLaunchKernelGGL((k_fused2d<1, SV>), grid, block, 0, s, grids, ngrids, nitems, Un, Us, Ud, lam, dtg,   \
                           dt_fixed, dt_out, status, clk);                                                       \
    else                                                                                                         \
        hipLaunchKernelGGL((k_fused2d<2, SV>), grid, block, 0, s, grids, ngrids, nitems, Un, Us, Ud, lam, dtg,   \
                           dt_fixed, dt_out, status, clk);
    FV_SEG_DISPATCH(seg, FV_LFS)
#undef FV_LFS
}

void launch_fused_init(int seg, int waves, const FGrid* grids, int ngrids, int nitems, const double* U,
                       unsigned long long* lam, uint32_t* status, unsigned long long* clk, hipStream_t s) {
    hipLaunchKernelGGL(k_fused_reset, dim3(1), dim3(256), 0, s, lam, ngrids, clk);
    const dim3 grid(fused_blocks(nitems, waves)), block(256);
#define FV_LFL(SV) hipLaunchKernelGGL((k_fused_lambda<SV>), grid, block, 0, s, grids, ngrids, nitems, U, lam, status);
    FV_SEG_DISPATCH(seg, FV_LFL)
#undef FV_LFL
}

}  // namespace fvk
