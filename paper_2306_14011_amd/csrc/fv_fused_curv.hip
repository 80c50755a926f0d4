// The curvilinear variant of the 2D fused stage kernels (fv_fused2d.h), in a
// source of its own: it is built with multiply-add contraction limited to
// single expressions. The first y face of a work item is computed before the
// row loop and the others inside it; contracting across statements made the
// Roe flux along the face normal round differently in the two places, and the
// result then depended on the segment height.
#include "fv_fused2d.h"

namespace fvk {

void launch_fused_stage_curv(int stage, dim3 grid, dim3 block, const FGrid* grids, int ngrids, int nitems,
                             const double* Un, const double* Us, double* Ud, unsigned long long* lam, double* dtg,
                             const double* dt_fixed, double* dt_out, uint32_t* status, unsigned long long* clk,
                             const double* src, const double* met, hipStream_t s) {
    if (src)
        launch_fused_stage_t<true, 3>(stage, grid, block, grids, ngrids, nitems, Un, Us, Ud, lam, dtg, dt_fixed,
                                      dt_out, status, clk, src, met, s);
    else
        launch_fused_stage_t<false, 3>(stage, grid, block, grids, ngrids, nitems, Un, Us, Ud, lam, dtg, dt_fixed,
                                       dt_out, status, clk, src, met, s);
}

}  // namespace fvk
