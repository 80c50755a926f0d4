// Internal interface between the C ABI (fv_api.hip) and the kernel launchers.
#pragma once

#include "fv_device.h"

namespace fvk {

// One 2D grid of the fused path (device memory, read uniformly).
// Stage clock record of the batch (per grid and stage, earliest work-item
// start and latest end): each entry is spread over CLK_SLOTS slots, one
// 128-byte line apart, that work items pick by their index, so the per-item
// atomics do not all meet on one address; the slots are folded when the
// step's record is stored.
constexpr int CLK_SLOTS = 16;
constexpr int CLK_PAD = 16;  // unsigned long longs per slot (one 128-byte line)
__host__ __device__ inline int clk_index(int entry, int slot) { return (entry * CLK_SLOTS + slot) * CLK_PAD; }

struct FGrid {
    int nx, ny, pitch, strips, work0, scheme;  // scheme: FV_SCHEME_*
    int bcx0, bcx1, bcy0, bcy1, gid, seg;   // gid: the caller's grid index (slots of lam, dt, clocks);
                                            // seg: rows per work item (a multiple of 4)
    long long base;     // element offset of cell (0,0), variable 0
    long long sv;       // per-variable stride
    double ax, ay;      // face areas of x faces (dy) and y faces (dx)
    double inv_vol, inv_dx, inv_dy, cfl, gamma, gm1;
    double q[2][2][4];  // conserved ghost state of inflow faces per axis and side (the kernels'
                        // boundary variant only: grids with slip walls or inflow faces)
    double mu, kcond, nu_fac;  // viscosity, heat conductivity, max(4/3, gamma / Pr) (viscous variant)
};

// The 3D grid of the fused path (device memory, read uniformly).
struct FGrid3 {
    int nx, ny, nz, strips, seg, scheme;       // seg: planes per work item (a multiple of 4)
    int bcx0, bcx1, bcy0, bcy1, bcz0, bcz1;
    long long base;                                // element offset of cell (0,0,0), variable 0
    long long sv, py, pz;                          // strides: variable, row (y), plane (z)
    double ax, ay, az;                             // face areas: dy dz, dx dz, dx dy
    double inv_vol, inv_dx, inv_dy, inv_dz, cfl, gamma, gm1;
    double q[3][2][5];  // conserved ghost state of inflow faces per axis and side (boundary variant)
};

void launch_bc_fill(double* U, const Geo& g, const BcState& bcs, int gang, int threads, hipStream_t s);
void launch_flux(int ax, const double* U, double* F, const Geo& g, int bx, int threads, hipStream_t s);
void launch_metrics(const double* nodes, double* met, int nx, int ny, hipStream_t s);
void launch_flux_curv(int ax, const double* U, double* F, const Geo& g, const BcState& bcs, int bx, int threads,
                      hipStream_t s);
void launch_visc(int ax, const double* U, double* F, const Geo& g, const BcState& bcs, hipStream_t s);
void launch_residual(const double* Fx, const double* Fy, const double* Fz, const double* S, double* R, const Geo& g,
                     int gang, int threads, hipStream_t s);
// norms[v] = sqrt(sum_e R[v][e]^2 / ncell) with partial (256 * nvar doubles) as scratch.
void launch_residual_norm(const double* R, double* partial, double* norms, const Geo& g, hipStream_t s);
void launch_update(int stage, const double* Un, const double* Us, double* Ud, const double* R, const double* dt,
                   const Geo& g, int gang, int threads, hipStream_t s);
int cfl_blocks(const Geo& g, int gang, int threads);
void launch_cfl(const double* U, double* partial, uint32_t* status, const double* dt_in, double* dt,
                double* dt_out, const Geo& g, int gang, int threads, hipStream_t s);
void launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s);

// fused 2D stages
int fused_items(const FGrid& G, int seg);  // work items of G at segment height seg
int fused_strips(int nx);
void launch_fused_stage(int stage, int waves, const FGrid* grids, int ngrids, int nitems, const double* Un,
                        const double* Us, double* Ud, unsigned long long* lam, double* dtg, const double* dt_fixed,
                        double* dt_out, uint32_t* status, unsigned long long* clk, hipStream_t s,
                        const double* src = nullptr, int mode = 0, const double* met = nullptr);
void launch_fused_init(int waves, const FGrid* grids, int ngrids, int nitems, const double* U,
                       unsigned long long* lam, uint32_t* status, hipStream_t s, const double* met = nullptr);
int fused_slots();
int fused3d_items(const FGrid3& G, int seg);
void launch_fused3d_stage(int stage, int waves, const FGrid3* grid, int nitems, const double* Un, const double* Us,
                          double* Ud, unsigned long long* lam, double* dtg, const double* dt_fixed, double* dt_out,
                          uint32_t* status, hipStream_t s, const double* src = nullptr, double vol = 0.0,
                          bool walls = false);
void launch_fused3d_init(int waves, const FGrid3* grid, int nitems, const double* U, unsigned long long* lam,
                         uint32_t* status, hipStream_t s);
int fused3d_slots();
int fused3d_auto_seg(const FGrid3& G, int slots);
int fused_auto_seg(const FGrid* grids, int ngrids, int slots);

// adjoint: one reverse Runge-Kutta stage (mode 3, 2, 1 for stages 3, 2, 1)
void launch_adj_stage(int mode, const double* Us, const double* w, double* lam, double* lamA, double* lamB, double* R,
                      const double* dt, const Geo& g, const BcState& bcs, hipStream_t s);

}  // namespace fvk
