// Fused SSP-RK3 stage for 3D grids (FP64, gfx950): one kernel per stage does
// the ghost mapping, MUSCL face states (minmod, or an unlimited kappa member)
// and Roe fluxes on the three axes, the residual and the stage combination,
// and the last stage also the CFL max of the new state.
//
// Work decomposition: a work item is a 60-column x strip of one grid row j
// over a segment of seg planes (seg a multiple of 4); one wavefront owns an
// item, lane l holding column 60*strip - 2 + l (lanes 2..61 produce outputs,
// lanes 0, 1, 62, 63 are the x halo). The wave marches along z with a window
// of four planes of its own row in registers, walking the segment's seg + 1
// z faces in unrolled groups of four so that every window slot is a
// compile-time constant (and each z face of the grid is computed by the same
// unrolled copy whatever seg is). At each plane it reads the rows j-2, j-1,
// j+1, j+2 of that plane and computes both y faces of its row; the x stencil
// comes from DPP lane shifts. A y face is thus computed by the two waves of
// the rows it separates (no block barriers, no LDS), which costs one flux in
// four extra against a shared-tile scheme.
//
// Halo cells outside the grid are read through the boundary maps; the state
// may keep ghost layers but they are not read. Per-grid dt and the CFL max
// follow the 2D kernel: stage 1 computes dt from the max that the previous
// step's stage 3 (or the init kernel) accumulated, stage 2 resets it, stage 3
// accumulates the max of the new state.
#include "fv_fused_common.h"

namespace fvk {

// Face states of one face from its four stencil cells, face-wise, by the
// compile-time rule LIM (0 minmod, 1 Psi = 1 with kappa = -1, 2 the kappa
// weights ka, kb with explicit fused multiply-adds, 3 van Leer).
template <int LIM>
__device__ __forceinline__ void zface_states(double q0, double q1, double q2, double q3, double ka, double kb,
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

// The planes of one work item (strip, row j, planes k0 .. k0 + seg - 1) for
// stage STAGE with the face-state rule fixed at compile time (LIM: 0 minmod,
// 1 Psi = 1 with kappa = -1, 2 Psi = 1 with kappa weights ka, kb, 3 van
// Leer). As in
// 2D, no memory access sits on a conditional path: loads are issued for
// every face (clamped indices), and stores of lanes or planes without output
// go past the end of a per-variable descriptor, where they are dropped.
template <int STAGE, int LIM, bool SRC>
__device__ __forceinline__ void fused3d_planes(const FGrid3& G, int lane, int strip, int j, int k0, double s,
                                               const double* Un, const double* Us, double* Ud, double& lmax,
                                               uint32_t& fl, double ka, double kb, const double* src, double vol) {
    constexpr bool UNL = LIM == 1;
    constexpr int NV = 5;
    const int col = FW * strip - 2 + lane;
    // lanes past the last halo column feed no output: they read that
    // column again (the same cache line) instead of wrapped or clamped data
    const int cmap = map_index(col < G.nx + 1 ? col : G.nx + 1, G.nx, G.bcx0, G.bcx1);
    const bool out_lane = lane >= 2 && lane < 2 + FW && col < G.nx;
    const int seg = G.seg;
    const long long gbytes = NV * G.sv * 8;  // one grid's state, below 4 GiB
    const Rsrc rs = grid_rsrc(Us + G.base, gbytes), rn = grid_rsrc(Un + G.base, gbytes);
    // one descriptor per output variable (a plane of the state is below
    // 1 GiB, so the drop offset plus any plane offset cannot wrap)
    Rsrc rd[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) rd[v] = grid_rsrc(Ud + G.base + v * G.sv, G.sv * 8);
    const uint32_t cboff = (uint32_t)cmap * 8u;                 // stencil column in bytes
    // U^n reads: lanes without output read a column of the strip's own
    // output range (the same cache lines), clamped inside the grid
    const int olast = FW * strip + FW - 1 < G.nx - 1 ? FW * strip + FW - 1 : G.nx - 1;
    const int ocol = col < FW * strip ? FW * strip : (col < olast ? col : olast);
    const uint32_t oboff = (uint32_t)ocol * 8u;
    const uint32_t sboff = out_lane ? (uint32_t)col * 8u : DROP_OFFSET;
    const uint32_t vstride = (uint32_t)(G.sv * 8);
    const uint32_t jo = (uint32_t)((long long)j * G.py * 8);
    const double hax = 0.5 * G.ax, hay = 0.5 * G.ay, haz = 0.5 * G.az;
    // source term S[v][k][j][i] (dense interior layout), read at the U^n
    // columns of row j; it is smaller than the grid's state (below 4 GiB)
    const long long svol = (long long)G.nx * G.ny * G.nz;
    Rsrc rsrc;
    if (SRC) rsrc = grid_rsrc(src, NV * svol * 8);
    // byte offsets of rows j-2 .. j+2 and of plane kk through the boundary maps
    uint32_t ro[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) ro[d] = (uint32_t)((long long)map_index(j - 2 + d, G.ny, G.bcy0, G.bcy1) * G.py * 8);
    auto plane_off = [&](int kk) -> uint32_t {
        return (uint32_t)((long long)map_index(kk, G.nz, G.bcz0, G.bcz1) * G.pz * 8);
    };
    auto out_plane = [&](int kk) -> uint32_t {
        return (uint32_t)((long long)(kk < G.nz ? kk : G.nz - 1) * G.pz * 8) + jo;
    };
    // window of the own row: plane kk in slot (kk - k0 + 2) & 3; z face f
    // (between planes k0 + f - 1 and k0 + f) uses slots f .. f + 3 (mod 4).
    // Face 0 first, then faces 1 .. seg in unrolled groups of four, so every
    // slot is a compile-time constant and a given z face of the grid is
    // computed by the same instructions whatever seg is.
    double W[4][NV];
#pragma unroll
    for (int kz = 0; kz < 4; ++kz) {
        const uint32_t o = plane_off(k0 - 2 + kz) + ro[2];
#pragma unroll
        for (int v = 0; v < NV; ++v) W[kz][v] = ld_buf(rs, cboff, o + v * vstride);
    }
    double Fz[2][NV];  // z-face fluxes (times 2): face f in Fz[f & 1]
    double qL[NV], qR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) zface_states<LIM>(W[0][v], W[1][v], W[2][v], W[3][v], ka, kb, qL[v], qR[v]);
    roe_flux<3, 2, true>(qL, qR, G.gm1, Fz[0]);
    {
        const uint32_t o = plane_off(k0 + 2) + ro[2];
#pragma unroll
        for (int v = 0; v < NV; ++v) W[0][v] = ld_buf(rs, cboff, o + v * vstride);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll 1
    for (int m0 = 1; m0 <= seg; m0 += 4) {
        if (k0 + m0 - 1 >= G.nz) break;  // ragged last segment (uniform)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int f = m0 + jj;
            const int t = (jj + 1) & 3;  // f mod 4, a compile-time constant
            const int kk = k0 + f - 1;   // output plane finished at this face
            // rows j-2, j-1, j+1, j+2 of plane kk, requested before the z face
            double Y[4][NV];
            double Unc[NV];
            {
                const uint32_t po = plane_off(kk);
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const uint32_t o = po + ro[d < 2 ? d : d + 1];
#pragma unroll
                    for (int v = 0; v < NV; ++v) Y[d][v] = ld_buf(rs, cboff, o + v * vstride);
                }
                if (STAGE > 0) {
                    const uint32_t o = out_plane(kk);
#pragma unroll
                    for (int v = 0; v < NV; ++v) Unc[v] = ld_buf(rn, oboff, o + v * vstride);
                }
            }
            // z face f: stencil planes kk-1 .. kk+2
#pragma unroll
            for (int v = 0; v < NV; ++v)
                zface_states<LIM>(W[t][v], W[(t + 1) & 3][v], W[(t + 2) & 3][v], W[(t + 3) & 3][v], ka, kb, qL[v],
                                  qR[v]);
            roe_flux<3, 2, true>(qL, qR, G.gm1, Fz[t & 1]);
            double c[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) c[v] = W[(t + 1) & 3][v];
            // plane kk - 1 is dead: its slot takes plane kk + 3 for face f + 1
            {
                const uint32_t o = plane_off(kk + 3) + ro[2];
#pragma unroll
                for (int v = 0; v < NV; ++v) W[t][v] = ld_buf(rs, cboff, o + v * vstride);
            }
            // y faces of row j at plane kk: below (rows j-2 .. j+1) and above
            // (rows j-1 .. j+2). With D[r] = U[r] - U[r-1], the own row's
            // limited slope lim(D[j], D[j+1]) serves both faces (minmod and van
            // Leer are symmetric).
            double Fyb[NV], Fyt[NV];  // times 2, like Fz
            double qLt[NV], qRt[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double d1 = Y[1][v] - Y[0][v], d2 = c[v] - Y[1][v];
                const double d3 = Y[2][v] - c[v], d4 = Y[3][v] - Y[2][v];
                if (LIM == 2) {
                    qL[v] = fma(ka, d1, fma(kb, d2, Y[1][v]));
                    qR[v] = fma(-kb, d2, fma(-ka, d3, c[v]));
                    qLt[v] = fma(ka, d2, fma(kb, d3, c[v]));
                    qRt[v] = fma(-kb, d3, fma(-ka, d4, Y[2][v]));
                } else {
                    const double m = UNL ? 0.0 : limited_slope<LIM>(d2, d3);
                    qL[v] = Y[1][v] + 0.5 * (UNL ? d1 : limited_slope<LIM>(d1, d2));
                    qR[v] = c[v] - 0.5 * (UNL ? d3 : m);
                    qLt[v] = c[v] + 0.5 * (UNL ? d2 : m);
                    qRt[v] = Y[2][v] - 0.5 * (UNL ? d4 : limited_slope<LIM>(d4, d3));
                }
            }
            roe_flux<3, 1, true>(qL, qR, G.gm1, Fyb);
            roe_flux<3, 1, true>(qLt, qRt, G.gm1, Fyt);
            // x faces: this lane computes its left face, its right face is the
            // lane above's left face; one difference and one slope per lane
            double Fxl[NV], Fxr[NV];  // times 2
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double d = c[v] - lane_shift1<true>(c[v]);  // D[i]
                const double dn = lane_shift1<false>(d);           // D[i+1]
                if (LIM == 2) {
                    qR[v] = fma(-kb, d, fma(-ka, dn, c[v]));
                    qL[v] = lane_shift1<true>(fma(ka, d, fma(kb, dn, c[v])));
                } else {
                    const double mr = UNL ? dn : limited_slope<LIM>(d, dn);
                    qR[v] = c[v] - 0.5 * mr;
                    qL[v] = lane_shift1<true>(c[v] + 0.5 * (UNL ? d : mr));
                }
            }
            roe_flux<3, 0, true>(qL, qR, G.gm1, Fxl);
#pragma unroll
            for (int v = 0; v < NV; ++v) Fxr[v] = lane_shift1<false>(Fxl[v]);
            const bool plane_ok = kk < G.nz;  // uniform
            const uint32_t p = out_plane(kk);
            const uint32_t so = plane_ok ? sboff : DROP_OFFSET;
            double Sv[NV];
            if (SRC) {
                const uint32_t ps =
                    (uint32_t)((((long long)(kk < G.nz ? kk : G.nz - 1)) * G.ny + j) * G.nx * 8);
#pragma unroll
                for (int v = 0; v < NV; ++v) Sv[v] = ld_buf(rsrc, oboff, ps + (uint32_t)(v * svol * 8));
            }
            double out[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                // the doubled fluxes against halved areas: the same products
                double r = (Fxr[v] - Fxl[v]) * hax;
                r += (Fyt[v] - Fyb[v]) * hay;
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
            if (STAGE == 2 && out_lane && plane_ok) {
                const double idx[3] = {G.inv_dx, G.inv_dy, G.inv_dz};
                lmax = fmax(lmax, cell_lambda<3>(out, G.gamma, G.gm1, idx, fl));
            }
            // keep the scheduler from overlapping consecutive planes (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int STAGE, bool SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_fused3d(const FGrid3* __restrict__ grid, int nitems, const double* Un,
                                                 const double* __restrict__ Us, double* Ud,
                                                 unsigned long long* __restrict__ lam, double* __restrict__ dtg,
                                                 const double* __restrict__ dt_fixed, double* __restrict__ dt_out,
                                                 uint32_t* __restrict__ status, const double* __restrict__ src,
                                                 double vol) {
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int wave0 = __builtin_amdgcn_readfirstlane(
        (int)((xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6));
    if (STAGE == 1 && blockIdx.x == 0 && threadIdx.x == 0) lam[0] = 0ull;  // stage 1 has read it
    const FGrid3 G = *grid;
    for (int item = wave0; item < nitems; item += nwaves) {
        const int strip = item % G.strips;
        const int t = item / G.strips;
        const int j = t % G.ny;
        const int zs = t / G.ny;
        double dt;
        if (STAGE == 0) {
            dt = dt_fixed ? dt_fixed[0] : G.cfl / __longlong_as_double((long long)lam[0]);
            if (item == 0 && lane == 0) {
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
            fused3d_planes<STAGE, 0, SRC>(G, lane, strip, j, zs * G.seg, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, vol);
        } else if (G.scheme == 5) {
            fused3d_planes<STAGE, 3, SRC>(G, lane, strip, j, zs * G.seg, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, vol);
        } else if (G.scheme == 1) {
            fused3d_planes<STAGE, 1, SRC>(G, lane, strip, j, zs * G.seg, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, vol);
        } else {
            double ka, kb;
            kappa_weights(G.scheme, ka, kb);
            fused3d_planes<STAGE, 2, SRC>(G, lane, strip, j, zs * G.seg, s, Un, Us, Ud, lmax, fl, ka, kb, src, vol);
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

// lambda_max of U^n (the first step's dt), same work items.
__global__ void __launch_bounds__(256) k_fused3d_lambda(const FGrid3* __restrict__ grid, int nitems,
                                                        const double* __restrict__ U,
                                                        unsigned long long* __restrict__ lam,
                                                        uint32_t* __restrict__ status) {
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int wave0 = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const FGrid3 G = *grid;
    for (int item = wave0; item < nitems; item += nwaves) {
        const int strip = item % G.strips;
        const int t = item / G.strips;
        const int j = t % G.ny;
        const int zs = t / G.ny;
        const int col = FW * strip + lane;
        double lmax = 0.0;
        uint32_t fl = 0;
        if (lane < FW && col < G.nx) {
            const double idx[3] = {G.inv_dx, G.inv_dy, G.inv_dz};
            for (int kk = zs * G.seg; kk < zs * G.seg + G.seg && kk < G.nz; ++kk) {
                const long long p = G.base + (long long)kk * G.pz + (long long)j * G.py + col;
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
    return fused_strips(G.nx) * G.ny * ((G.nz + seg - 1) / seg);
}

static inline int blocks_for(int nitems, int waves) {
    const int w = waves > 0 ? (waves < nitems ? waves : nitems) : nitems;
    return (w + 3) / 4;
}

template <bool SRC>
static void launch_fused3d_stage_t(int stage, dim3 g, dim3 b, const FGrid3* grid, int nitems, const double* Un,
                                   const double* Us, double* Ud, unsigned long long* lam, double* dtg,
                                   const double* dt_fixed, double* dt_out, uint32_t* status, const double* src,
                                   double vol, hipStream_t s) {
    if (stage == 0)
        hipLaunchKernelGGL((k_fused3d<0, SRC>), g, b, 0, s, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                           status, src, vol);
    else if (stage == 1)
        hipLaunchKernelGGL((k_fused3d<1, SRC>), g, b, 0, s, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                           status, src, vol);
    else
        hipLaunchKernelGGL((k_fused3d<2, SRC>), g, b, 0, s, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out,
                           status, src, vol);
}

void launch_fused3d_stage(int stage, int waves, const FGrid3* grid, int nitems, const double* Un, const double* Us,
                          double* Ud, unsigned long long* lam, double* dtg, const double* dt_fixed, double* dt_out,
                          uint32_t* status, hipStream_t s, const double* src, double vol) {
    const dim3 g(blocks_for(nitems, waves)), b(256);
    if (src)
        launch_fused3d_stage_t<true>(stage, g, b, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out, status, src,
                                     vol, s);
    else
        launch_fused3d_stage_t<false>(stage, g, b, grid, nitems, Un, Us, Ud, lam, dtg, dt_fixed, dt_out, status,
                                      nullptr, 0.0, s);
}

void launch_fused3d_init(int waves, const FGrid3* grid, int nitems, const double* U, unsigned long long* lam,
                         uint32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_fused3d_reset, dim3(1), dim3(1), 0, s, lam);
    hipLaunchKernelGGL(k_fused3d_lambda, dim3(blocks_for(nitems, waves)), dim3(256), 0, s, grid, nitems, U, lam,
                       status);
}

int fused3d_slots() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int b0 = 0, b1 = 0, b2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, k_fused3d<0, false>, 256, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, k_fused3d<1, false>, 256, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, k_fused3d<2, false>, 256, 0) != hipSuccess)
        return 0;
    const int bmin = b0 < b1 ? (b0 < b2 ? b0 : b2) : (b1 < b2 ? b1 : b2);
    return bmin * 4 * cus;
}

// Segment height (a multiple of 4): as in 2D, the one minimising (rounds of
// resident waves) x (planes per item + 1); ties go to the taller segment.
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
