// Fused SSP-RK3 stage for 2D grids: launches of the stage kernels of
// fv_fused2d.h (periodic and transmissive grids, the boundary variant, the
// viscous variant; the curvilinear variant is built in fv_fused_curv.hip),
// the initial wave-speed kernel, and the table helpers (work items, resident
// waves, the automatic segment height).
#include "fv_fused2d.h"

namespace fvk {

// lambda_max of U^n per grid (the first step's dt), same work items.
__global__ void __launch_bounds__(256) k_fused_lambda(const FGrid* __restrict__ grids, int ngrids, int nitems,
                                                      const double* __restrict__ U, unsigned long long* __restrict__ lam,
                                                      uint32_t* __restrict__ status, const double* __restrict__ met) {
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int wave0 = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    for (int item = wave0; item < nitems; item += nwaves) {
        const int gi = find_grid(grids, ngrids, item);
        const FGrid G = grids[gi];
        const int local = item - G.work0;
        const int strip = local % G.strips;
        const int sidx = local / G.strips;
        const int col = FW * strip + lane;
        double lmax = 0.0;
        uint32_t fl = 0;
        if (lane < FW && col < G.nx) {
            const double idx[2] = {G.inv_dx, G.inv_dy};
            for (int rr = sidx * G.seg; rr < sidx * G.seg + G.seg && rr < G.ny; ++rr) {
                const long long p = G.base + (long long)rr * G.pitch + col;
                double q[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) q[v] = U[v * G.sv + p];
                double lam = cell_lambda<2>(q, G.gamma, G.gm1, idx, fl);
                if (G.mu > 0.0) lam += 2.0 * ((G.mu / q[0]) * G.nu_fac) * (G.inv_dx * G.inv_dx + G.inv_dy * G.inv_dy);
                if (met) {
                    // curvilinear: the faces' unit normals and lengths, the cell's area
                    const MetricOffsets mo = metric_offsets(G.nx, G.ny);
                    const long long e = (long long)rr * G.nx + col;
                    const long long fx = (long long)rr * (G.nx + 1) + col;
                    double xa[3], xb[3], ya[3], yb[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        xa[k] = met[mo.fx + k * mo.nfx + fx];
                        xb[k] = met[mo.fx + k * mo.nfx + fx + 1];
                        ya[k] = met[mo.fy + k * mo.nfy + e];
                        yb[k] = met[mo.fy + k * mo.nfy + e + G.nx];
                    }
                    lam = curv_cell_lambda(q, G.gamma, G.gm1, xa, xb, ya, yb, met[mo.cell + e]);
                }
                lmax = fmax(lmax, lam);
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

// Zero the lambda accumulators.
__global__ void k_fused_reset(unsigned long long* lam, int ngrids) {
    for (int g = threadIdx.x; g < ngrids; g += blockDim.x) lam[g] = 0ull;
}

// ---------------------------------------------------------------------------

int fused_items(const FGrid& G, int seg) { return G.strips * ((G.ny + seg - 1) / seg); }

int fused_strips(int nx) { return (nx + FW - 1) / FW; }

// mode: 0 periodic and transmissive grids, 1 with slip walls or inflow
// faces too, 2 that and the viscous flux, 3 a curvilinear grid (any face
// kinds).
void launch_fused_stage(int stage, int waves, const FGrid* grids, int ngrids, int nitems, const double* Un,
                        const double* Us, double* Ud, unsigned long long* lam, double* dtg, const double* dt_fixed,
                        double* dt_out, uint32_t* status, unsigned long long* clk, hipStream_t s,
                        const double* src, int mode, const double* met) {
    const dim3 grid(fused_blocks(nitems, waves)), block(256);
#define FV_LFS(SRCB, M)                                                                                       \
    launch_fused_stage_t<SRCB, M>(stage, grid, block, grids, ngrids, nitems, Un, Us, Ud, lam, dtg, dt_fixed, \
                                  dt_out, status, clk, src, met, s)
    if (mode == 3) {
        launch_fused_stage_curv(stage, grid, block, grids, ngrids, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                                status, clk, src, met, s);
    } else if (src) {
        if (mode == 2) FV_LFS(true, 2);
        else if (mode == 1) FV_LFS(true, 1);
        else FV_LFS(true, 0);
    } else {
        if (mode == 2) FV_LFS(false, 2);
        else if (mode == 1) FV_LFS(false, 1);
        else FV_LFS(false, 0);
    }
#undef FV_LFS
}

void launch_fused_init(int waves, const FGrid* grids, int ngrids, int nitems, const double* U,
                       unsigned long long* lam, uint32_t* status, hipStream_t s, const double* met) {
    hipLaunchKernelGGL(k_fused_reset, dim3(1), dim3(256), 0, s, lam, ngrids);
    const dim3 grid(fused_blocks(nitems, waves)), block(256);
    hipLaunchKernelGGL(k_fused_lambda, grid, block, 0, s, grids, ngrids, nitems, U, lam, status, met);
}

// Waves of the stage kernels that are resident on the current device at once:
// blocks per CU (the least over the three stages) x 4 waves x CUs.
int fused_slots() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int b0 = 0, b1 = 0, b2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, k_fused2d<0, false, 0>, 256, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, k_fused2d<1, false, 0>, 256, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, k_fused2d<2, false, 0>, 256, 0) != hipSuccess)
        return 0;
    const int b = b0 < b1 ? (b0 < b2 ? b0 : b2) : (b1 < b2 ? b1 : b2);
    return b * 4 * cus;
}

// Segment height for a set of grids: the multiple of 4, at most 24 rows
// (16 when 24-row items fill the resident waves more than twice), that
// minimises (rounds of resident waves) x (rows per item + 1), the item's
// critical path in rows (one extra y face per item). Ties go to the taller
// segment, which re-reads fewer halo rows. Without the bound the rule picks
// tall segments for grids that take many rounds (96 rows at 4096^2, 124 at
// 8192^2), which measured slower: at 8192^2, 4.29 ms per step against 4.07
// with 16 rows; at 4096^2, 16 rows ran 4.5% faster than 24, and at 2048^2
// (one round of 24-row items) 24 rows ran 6% faster than 16. A likely
// reason: with short segments the waves resident at one time cover fewer
// rows, so the halo rows they share are more often still in L2.
int fused_auto_seg(const FGrid* grids, int ngrids, int slots) {
    if (slots <= 0) return 16;
    long long items24 = 0;
    for (int g = 0; g < ngrids; ++g) items24 += (long long)fused_items(grids[g], 24);
    const int max_seg = items24 > 2LL * slots ? 16 : 24;
    int best = 16;
    double best_cost = 0.0;
    for (int seg = 4; seg <= max_seg; seg += 4) {
        long long items = 0;
        for (int g = 0; g < ngrids; ++g) items += (long long)fused_items(grids[g], seg);
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
