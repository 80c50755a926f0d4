// Internal interface between the C ABI (fv_api.hip) and the kernel launchers.
#pragma once

#include "fv_device.h"

namespace fvk {

void launch_bc_fill(double* U, const Geo& g, int gang, int threads, hipStream_t s);
void launch_flux(int ax, const double* U, double* F, const Geo& g, int bx, int threads, hipStream_t s);
void launch_residual(const double* Fx, const double* Fy, const double* Fz, double* R, const Geo& g, int gang,
                     int threads, hipStream_t s);
void launch_update(int stage, const double* Un, const double* Us, double* Ud, const double* R, const double* dt,
                   const Geo& g, int gang, int threads, hipStream_t s);
int cfl_blocks(const Geo& g, int gang, int threads);
void launch_cfl(const double* U, double* partial, uint32_t* status, const double* dt_in, double* dt,
                double* dt_out, const Geo& g, int gang, int threads, hipStream_t s);
void launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s);

// adjoint
void launch_adj_flux(int ax, const double* U, const double* w, double* G, const Geo& g, hipStream_t s);
void launch_adj_gather(const double* Gx, const double* Gy, const double* Gz, double* mu, const Geo& g,
                       hipStream_t s);
void launch_adj_comb(int mode, double* lam, double* lamA, double* lamB, const double* mu, const double* dt,
                     const Geo& g, hipStream_t s);

}  // namespace fvk
