// Fused SSP-RK3 stage for 2D grids (FP64, gfx950): one kernel per stage does
// the ghost mapping, MUSCL face states (minmod, or an unlimited kappa member)
// and Roe fluxes on both axes, the residual and the stage combination, and
// the last stage also the CFL max of the new state.
//
// Work decomposition: a work item is a 60-column strip x seg-row segment of
// one grid (seg a multiple of 4, per grid in the table); one wavefront (64
// lanes) owns an item. Lane l holds column
// x0 + l, x0 = 60*strip - 2, so lanes 2..61 produce the 60 output columns and
// lanes 0, 1, 62, 63 carry the x halo. The wave marches up the segment one row
// at a time, keeping the last four rows in registers: that window gives the
// y-face flux, and the x-stencil and the right-face flux come from
// neighbouring lanes by DPP lane shifts. No LDS and no block barriers. Loads
// and stores go through buffer descriptors of the grid's arrays, so one
// grid's state (4 variables) must stay below 4 GiB (checked on the host).
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
//
// The kernel template lives in this header so that the curvilinear variant
// can be instantiated in a source of its own, built with multiply-add
// contraction limited to single expressions (fv_fused_curv.hip); the other
// variants are instantiated in fv_fused.hip.
#pragma once

#include "fv_fused_common.h"

namespace fvk {

// The viscous variant's arithmetic contracts multiply-adds only within one
// source expression (the pragma in each viscous block): the first face of a
// work item is computed before the row loop and the others inside it, and
// contraction across statements could then differ between the two places,
// giving bits that depend on the segment height.

// Viscous variant: velocity and temperature w = (u, v, T = p / rho) of a cell.
__device__ __forceinline__ void visc_w2(const double* q, double gm1, double* w) {
#pragma clang fp contract(on)
    const double ir = 1.0 / q[0];
    w[0] = q[1] * ir;
    w[1] = q[2] * ir;
    w[2] = gm1 * (q[3] - 0.5 * q[0] * (w[0] * w[0] + w[1] * w[1])) * ir;
}

// Viscous flux F_nu,n (Eq. (QF), n = e_AX) through a face from w at its low
// (wa) and high (wb) cells, the tangential derivatives dt of (u, v, T) along
// the other axis, and 1 / dx_AX: tau_{a,AX} = mu (du_a/dx_AX + du_AX/dx_a) -
// 2/3 mu delta div(u), Theta = ubar . tau + k dT/dx_AX. F[0] = 0 is omitted.
template <int AX>
__device__ __forceinline__ void visc_flux2(const double* wa, const double* wb, const double* dt, double inv_dn,
                                           double mu, double kc, double* F) {
#pragma clang fp contract(on)
    double gn[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) gn[m] = (wb[m] - wa[m]) * inv_dn;
    // grad[m][d]: d w_m / d x_d
    const double dux = AX == 0 ? gn[0] : dt[0], duy = AX == 0 ? dt[0] : gn[0];
    const double dvx = AX == 0 ? gn[1] : dt[1], dvy = AX == 0 ? dt[1] : gn[1];
    const double divu = dux + dvy;
    double tau[2];
    if (AX == 0) {
        tau[0] = mu * (dux + dux) - (2.0 / 3.0) * mu * divu;
        tau[1] = mu * (dvx + duy);
    } else {
        tau[0] = mu * (duy + dvx);
        tau[1] = mu * (dvy + dvy) - (2.0 / 3.0) * mu * divu;
    }
    double th = kc * gn[2];
    th += 0.5 * (wa[0] + wb[0]) * tau[0];
    th += 0.5 * (wa[1] + wb[1]) * tau[1];
    F[0] = tau[0];
    F[1] = tau[1];
    F[2] = th;
}

// The rows of one work item (strip, rows r0 .. r0 + seg - 1) for stage STAGE
// with the face-state rule fixed at compile time (LIM: 0 minmod, 1 Psi = 1
// with kappa = -1, 2 Psi = 1 with the kappa weights ka, kb, 3 van Leer). The
// loop body has
// no branch around a memory access: every load is issued whatever the row
// (indices past the grid are clamped), and the stores of lanes or rows with
// no output go to an offset past the end of the buffer, where the hardware
// drops them. A conditional load or store would make the compiler's wait
// counting assume the shortest path and wait for every outstanding access
// (the prefetches included) at the top of each row.
template <int STAGE, int LIM, bool SRC, int MODE>
__device__ __forceinline__ void fused2d_rows(const FGrid& G, int lane, int strip, int r0, double s, const double* Un,
                                             const double* Us, double* Ud, double& lmax, uint32_t& fl, double ka,
                                             double kb, const double* src, const double* met) {
    constexpr bool BC = MODE >= 1;     // boundary variant: slip walls and inflow faces
    constexpr bool VISC = MODE == 2;   // and the viscous flux
    constexpr bool CURV = MODE == 3;   // or a curvilinear grid (metric streams)
    constexpr bool UNL = LIM == 1;
    constexpr int NV = 4;
    const int seg = G.seg;
    const int col = FW * strip - 2 + lane;
    // lanes past the last halo column feed no output: they read that
    // column again (the same cache line) instead of wrapped or clamped data
    const int ccl = col < G.nx + 1 ? col : G.nx + 1;
    const int cmap = BC ? map_index_bc(ccl, G.nx, G.bcx0, G.bcx1) : map_index(ccl, G.nx, G.bcx0, G.bcx1);
    // boundary variant: the kind of the face a ghost column lies behind
    // (slip wall: the mirror cell with its x momentum reversed; inflow: the
    // side's given state), per lane; -1 inside the grid
    const int xk = !BC ? -1 : (col < 0 ? G.bcx0 : (col >= G.nx ? G.bcx1 : -1));
    const int xside = col < 0 ? 0 : 1;
    // curvilinear variant: the metric streams (unit normal x, y and length of
    // the x faces, the same of the y faces, cell area and 1 / area) through
    // one descriptor per block, this lane's face and cell columns clamped
    // into the grid (lanes outside feed no output)
    Rsrc rmx, rmy, rmc;
    uint32_t sfx = 0, sfy = 0, scl = 0, xfo = 0, cfo = 0, xwo = 0;
    double wyn[2][2];  // unit normals of the y faces at this lane's column on the low and high y boundary
    if (CURV) {
        const MetricOffsets mo = metric_offsets(G.nx, G.ny);
        rmx = grid_rsrc(met + mo.fx, 3 * mo.nfx * 8);
        rmy = grid_rsrc(met + mo.fy, 3 * mo.nfy * 8);
        rmc = grid_rsrc(met + mo.cell, 2 * mo.nc * 8);
        sfx = (uint32_t)(mo.nfx * 8);
        sfy = (uint32_t)(mo.nfy * 8);
        scl = (uint32_t)(mo.nc * 8);
        xfo = (uint32_t)(col < 0 ? 0 : (col > G.nx ? G.nx : col)) * 8u;
        cfo = (uint32_t)(col < 0 ? 0 : (col > G.nx - 1 ? G.nx - 1 : col)) * 8u;
        xwo = (uint32_t)(xside ? G.nx : 0) * 8u;  // the x wall face of this lane's side
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const uint32_t yo = (uint32_t)((long long)(sd ? G.ny : 0) * G.nx * 8);
            wyn[sd][0] = ld_buf(rmy, cfo, yo);
            wyn[sd][1] = ld_buf(rmy, cfo, sfy + yo);
        }
    }
    // byte offsets of the metric rows: x faces and cells of row r, y faces of face row r (0 .. ny)
    auto mx_row = [&](int r) {
        return (uint32_t)((long long)(r < 0 ? 0 : (r > G.ny - 1 ? G.ny - 1 : r)) * (G.nx + 1) * 8);
    };
    auto my_row = [&](int r) { return (uint32_t)((long long)(r < 0 ? 0 : (r > G.ny ? G.ny : r)) * G.nx * 8); };
    auto mc_row = [&](int r) { return (uint32_t)((long long)(r < 0 ? 0 : (r > G.ny - 1 ? G.ny - 1 : r)) * G.nx * 8); };
    // a slip wall's mirror cell with its velocity reflected about the wall
    // face's unit normal (nx, ny): m - 2 (m . n) n
    auto reflect = [&](double* w, double nx, double ny) {
        const double mn = w[1] * nx + w[2] * ny;
        w[1] -= 2.0 * mn * nx;
        w[2] -= 2.0 * mn * ny;
    };
    // curvilinear variant: the unit normal of row r's x wall face on this lane's side
    auto wall_normal = [&](int r, double* wn) {
        if (!CURV) return;
        wn[0] = ld_buf(rmx, xwo, mx_row(r));
        wn[1] = ld_buf(rmx, xwo, sfx + mx_row(r));
    };
    // applies the ghost rules of row r (uniform) and of this lane's column to a
    // loaded cell (wn: the row's x wall normal, curvilinear variant)
    auto ghost = [&](double* w, int r, const double* wn) {
        if (!BC) return;
        const int yk = r < 0 ? G.bcy0 : (r >= G.ny ? G.bcy1 : -1);
        const int ys = r < 0 ? 0 : 1;
        // (the side indices select between constant indices: indexing the
        // kernel's local copy of the grid table, or a local array, with a
        // run-time index would move it to scratch memory)
        if (yk == 2) {
            if (CURV) reflect(w, ys ? wyn[1][0] : wyn[0][0], ys ? wyn[1][1] : wyn[0][1]);
            else w[2] = -w[2];
        }
        if (yk == 3) {
#pragma unroll
            for (int v = 0; v < NV; ++v) w[v] = ys ? G.q[1][1][v] : G.q[1][0][v];
        }
        if (CURV) {
            double m[NV] = {w[0], w[1], w[2], w[3]};
            reflect(m, wn[0], wn[1]);
            w[1] = xk == 2 ? m[1] : w[1];
            w[2] = xk == 2 ? m[2] : w[2];
        } else {
            w[1] = xk == 2 ? -w[1] : w[1];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = xk == 3 ? (xside ? G.q[0][1][v] : G.q[0][0][v]) : w[v];
    };
    const bool out_lane = lane >= 2 && lane < 2 + FW && col < G.nx;
    const long long gbytes = 4 * G.sv * 8;  // one grid's state, below 4 GiB
    const Rsrc rs = grid_rsrc(Us + G.base, gbytes), rn = grid_rsrc(Un + G.base, gbytes);
    // one descriptor per output variable: the plane is below 1 GiB, so the
    // drop offset plus any row offset stays past the end without wrapping
    Rsrc rd[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) rd[v] = grid_rsrc(Ud + G.base + v * G.sv, G.sv * 8);
    const uint32_t cboff = (uint32_t)cmap * 8u;                // this lane's (mapped) column in bytes
    // U^n reads: lanes without output read a column of the strip's own
    // output range (the same cache lines), clamped inside the grid
    const int olast = FW * strip + FW - 1 < G.nx - 1 ? FW * strip + FW - 1 : G.nx - 1;
    const int ocol = col < FW * strip ? FW * strip : (col < olast ? col : olast);
    const uint32_t oboff = (uint32_t)ocol * 8u;
    const uint32_t sboff = out_lane ? (uint32_t)col * 8u : DROP_OFFSET;
    // source term S[v][row][col] (dense interior layout), read at the U^n
    // columns; its plane and the grid's state are below 4 GiB
    const long long splane = (long long)G.nx * G.ny;
    Rsrc rsrc;
    if (SRC) rsrc = grid_rsrc(src, 4 * splane * 8);
    const double vol = G.ax * G.ay;
    const uint32_t vstride = (uint32_t)(G.sv * 8);
    const double hax = 0.5 * G.ax, hay = 0.5 * G.ay;
    // byte offset of U_s row r through the y boundary map (rows past the
    // last halo row are clamped inside the grid; they feed no output)
    auto row_off = [&](int r) -> uint32_t {
        const int m = BC ? map_index_bc(r, G.ny, G.bcy0, G.bcy1) : map_index(r, G.ny, G.bcy0, G.bcy1);
        return (uint32_t)((long long)m * G.pitch * 8);
    };
    auto out_row = [&](int r) -> uint32_t { return (uint32_t)((long long)(r < G.ny ? r : G.ny - 1) * G.pitch * 8); };
    // Circular window of four U_s rows: row r sits in slot (r - r0 + 2) & 3.
    // Face f of the segment (f = 0 .. seg) lies between rows r0 + f - 1 and
    // r0 + f. Face 0 is computed first; faces 1 .. seg follow in unrolled
    // groups of four, so each slot index is a compile-time constant and the
    // window never moves between registers.
    //
    // MUSCL per cell rather than per face: with D[r] = U[r] - U[r-1], the
    // left state of the face above row r is U[r] + lim(D[r], D[r+1]) / 2 and
    // the right state of the face below it U[r] - lim(D[r+1], D[r]) / 2 for a
    // symmetric limited slope lim (minmod, van Leer)
    // (unlimited: D[r] / 2 and D[r+1] / 2; other kappa: the weighted sums
    // ka D[r] + kb D[r+1] and kb D[r] + ka D[r+1]), so each row needs one new
    // difference and one minmod, and the face's left state is carried from
    // the previous face. The same values as the face-wise formula, operation
    // for operation (minmod is symmetric); since r0 is a multiple of 4, a
    // given face of the grid is computed by the same instructions whatever
    // the segment height.
    double W[4][NV];
    double wxp[2];  // curvilinear variant: x wall normal of the row loaded last
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t o = row_off(r0 - 2 + k);
#pragma unroll
        for (int v = 0; v < NV; ++v) W[k][v] = ld_buf(rs, cboff, o + v * vstride);
        double wn[2];
        wall_normal(r0 - 2 + k, wn);
        ghost(W[k], r0 - 2 + k, wn);
    }
    double Fy[2][NV];   // y-face fluxes (times 2): face f in Fy[f & 1]
    double Unb[2][NV];  // U^n of the output row of face f in Unb[f & 1], requested one face ahead
    double qL[NV], qR[NV];
    double qLy[NV], Dy[NV];  // left state of the next y face, and D of its upper row
    if (STAGE > 0) {
        const uint32_t pn = out_row(r0);
#pragma unroll
        for (int v = 0; v < NV; ++v) Unb[1][v] = ld_buf(rn, oboff, pn + v * vstride);
    }
    // face 0: rows r0-2 .. r0+1 in slots 0 .. 3
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double d0 = W[1][v] - W[0][v], d1 = W[2][v] - W[1][v], d2 = W[3][v] - W[2][v];
        if (LIM == 2) {
            qL[v] = fma(ka, d0, fma(kb, d1, W[1][v]));
            qR[v] = fma(-kb, d1, fma(-ka, d2, W[2][v]));
            qLy[v] = fma(ka, d1, fma(kb, d2, W[2][v]));
        } else {
            qL[v] = W[1][v] + 0.5 * (UNL ? d0 : limited_slope<LIM>(d0, d1));
            const double mr = UNL ? d2 : limited_slope<LIM>(d1, d2);
            qR[v] = W[2][v] - 0.5 * mr;
            qLy[v] = W[2][v] + 0.5 * (UNL ? d1 : mr);
        }
        Dy[v] = d2;
    }
    {
        const uint32_t o = row_off(r0 + 2);
#pragma unroll
        for (int v = 0; v < NV; ++v) W[0][v] = ld_buf(rs, cboff, o + v * vstride);
        wall_normal(r0 + 2, wxp);  // its ghost rules wait for the first row of the loop
    }
    // curvilinear variant: metrics of face f's row in slot f & 1 (x faces and
    // cells of row r0 + f - 1, y face between rows r0 + f - 1 and r0 + f),
    // requested one face ahead; Ylo: the y face below the output row (stage 3)
    double Mx[2][3], My[2][3], Mi[2], Ma[2], Ylo[3];
    auto load_metrics = [&](int slot, int f) {
        const int r = r0 + f - 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Mx[slot][k] = ld_buf(rmx, xfo, k * sfx + mx_row(r));
            My[slot][k] = ld_buf(rmy, cfo, k * sfy + my_row(r + 1));
        }
        Mi[slot] = ld_buf(rmc, cfo, scl + mc_row(r));
        if (SRC || STAGE == 2) Ma[slot] = ld_buf(rmc, cfo, mc_row(r));
    };
    if (CURV) {
#pragma unroll
        for (int k = 0; k < 3; ++k) My[0][k] = ld_buf(rmy, cfo, k * sfy + my_row(r0));
        load_metrics(1, 1);
        roe_flux_n2(qL, qR, My[0][0], My[0][1], G.gm1, Fy[0]);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fy[0][v] *= My[0][2];
#pragma unroll
        for (int k = 0; k < 3; ++k) Ylo[k] = My[0][k];
    } else {
        roe_flux<2, 1, true>(qL, qR, G.gm1, Fy[0]);
    }
    // viscous variant: w = (u, v, T) of row r in Wv[(r - r0 + 2) & 3], like the
    // window; the viscous y-face fluxes of face f in Vy[f & 1]
    double Wv[4][3], Vy[2][3];
    const double qdx = 0.25 * G.inv_dx, qdy = 0.25 * G.inv_dy;
    if (VISC) {
#pragma clang fp contract(on)
        visc_w2(W[1], G.gm1, Wv[1]);  // row r0 - 1
        visc_w2(W[2], G.gm1, Wv[2]);  // row r0
        double dt[3];
#pragma unroll
        for (int m = 0; m < 3; ++m)
            dt[m] = ((lane_shift1<false>(Wv[1][m]) - lane_shift1<true>(Wv[1][m])) +
                     (lane_shift1<false>(Wv[2][m]) - lane_shift1<true>(Wv[2][m]))) * qdx;
        visc_flux2<1>(Wv[1], Wv[2], dt, G.inv_dy, G.mu, G.kcond, Vy[0]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll 1
    for (int m0 = 1; m0 <= seg; m0 += 4) {
        if (r0 + m0 - 1 >= G.ny) break;  // ragged last segment (uniform)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int f = m0 + j;
            const int t = (j + 1) & 3;  // f mod 4, a compile-time constant
            const int rr = r0 + f - 1;  // output row finished at this face
            // rows rr-1 .. rr+2 sit in slots t .. t+3; row rr-1 is no longer
            // needed, so its slot takes row rr + 3 (for face f + 1) right away
            // row rr + 2, loaded one row ago, takes its ghost rules here, where
            // it is first used: applied at the load, they would make the row
            // wait for its own loads
            ghost(W[(t + 3) & 3], rr + 2, wxp);
            double c[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) c[v] = W[(t + 1) & 3][v];
            {
                const uint32_t o = row_off(rr + 3);
#pragma unroll
                for (int v = 0; v < NV; ++v) W[t][v] = ld_buf(rs, cboff, o + v * vstride);
                wall_normal(rr + 3, wxp);
            }
            if (STAGE > 0) {
                // U^n of row rr + 1, used at face f + 1
                const uint32_t pn = out_row(rr + 1);
#pragma unroll
                for (int v = 0; v < NV; ++v) Unb[(t + 1) & 1][v] = ld_buf(rn, oboff, pn + v * vstride);
            }
            if (CURV) load_metrics((t + 1) & 1, f + 1);
            // y face f between rows rr and rr+1
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double u1 = W[(t + 2) & 3][v];
                const double dn = W[(t + 3) & 3][v] - u1;  // D[rr+2]
                qL[v] = qLy[v];
                if (LIM == 2) {
                    qR[v] = fma(-kb, Dy[v], fma(-ka, dn, u1));
                    qLy[v] = fma(ka, Dy[v], fma(kb, dn, u1));
                } else {
                    const double mr = UNL ? dn : limited_slope<LIM>(Dy[v], dn);
                    qR[v] = u1 - 0.5 * mr;
                    qLy[v] = u1 + 0.5 * (UNL ? Dy[v] : mr);
                }
                Dy[v] = dn;
            }
            if (CURV) {
                roe_flux_n2(qL, qR, My[t & 1][0], My[t & 1][1], G.gm1, Fy[t & 1]);
#pragma unroll
                for (int v = 0; v < NV; ++v) Fy[t & 1][v] *= My[t & 1][2];
            } else {
                roe_flux<2, 1, true>(qL, qR, G.gm1, Fy[t & 1]);
            }
            // viscous y face f between rows rr and rr + 1; the neighbours'
            // w of rows rr and rr + 1 serve the x face below too
            double wl0[3], wl1[3];  // w of the lane below (column i - 1) in rows rr, rr + 1
            if (VISC) {
#pragma clang fp contract(on)
                visc_w2(W[(t + 2) & 3], G.gm1, Wv[(t + 2) & 3]);  // row rr + 1
                double dt[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    wl0[m] = lane_shift1<true>(Wv[(t + 1) & 3][m]);
                    wl1[m] = lane_shift1<true>(Wv[(t + 2) & 3][m]);
                    dt[m] = ((lane_shift1<false>(Wv[(t + 1) & 3][m]) - wl0[m]) +
                             (lane_shift1<false>(Wv[(t + 2) & 3][m]) - wl1[m])) * qdx;
                }
                visc_flux2<1>(Wv[(t + 1) & 3], Wv[(t + 2) & 3], dt, G.inv_dy, G.mu, G.kcond, Vy[t & 1]);
            }
            // x faces of row rr: this lane computes its left face; its right
            // face is the left face of the lane above. Each lane forms its
            // backward difference once and its slope once, and takes the
            // left state of its left face from the lane below.
            double Fxl[NV], Fxr[NV];  // times 2, like Fy
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
            if (CURV) {
                roe_flux_n2(qL, qR, Mx[t & 1][0], Mx[t & 1][1], G.gm1, Fxl);
#pragma unroll
                for (int v = 0; v < NV; ++v) Fxl[v] *= Mx[t & 1][2];
            } else {
                roe_flux<2, 0, true>(qL, qR, G.gm1, Fxl);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) Fxr[v] = lane_shift1<false>(Fxl[v]);
            // viscous x face left of this lane (columns i - 1 and i of row
            // rr), tangential derivative from rows rr - 1 and rr + 1
            double Vxl[3], Vxr[3];
            if (VISC) {
#pragma clang fp contract(on)
                double dt[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const double lo_m = lane_shift1<true>(Wv[t][m]);  // (i - 1, rr - 1)
                    dt[m] = ((wl1[m] - lo_m) + (Wv[(t + 2) & 3][m] - Wv[t][m])) * qdy;
                }
                visc_flux2<0>(wl0, Wv[(t + 1) & 3], dt, G.inv_dx, G.mu, G.kcond, Vxl);
#pragma unroll
                for (int m = 0; m < 3; ++m) Vxr[m] = lane_shift1<false>(Vxl[m]);
            }
            const bool row_ok = rr < G.ny;  // uniform
            const uint32_t p = out_row(rr);
            const uint32_t so = row_ok ? sboff : DROP_OFFSET;
            double Sv[NV];
            if (SRC) {
                const uint32_t ps = (uint32_t)((long long)(rr < G.ny ? rr : G.ny - 1) * G.nx * 8);
#pragma unroll
                for (int v = 0; v < NV; ++v) Sv[v] = ld_buf(rsrc, oboff, ps + (uint32_t)(v * splane * 8));
            }
            double out[NV];
            const double sc = CURV ? s * Mi[t & 1] : s;  // -dt / |Omega| of this cell
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                // the doubled fluxes against halved areas: the same products
                // (curvilinear: the fluxes already carry the face lengths)
                double r = CURV ? Fxr[v] - Fxl[v] : (Fxr[v] - Fxl[v]) * hax;
                if (CURV) r += Fy[t & 1][v] - Fy[(t + 1) & 1][v];
                else r += (Fy[t & 1][v] - Fy[(t + 1) & 1][v]) * hay;
                if (VISC && v > 0) {
                    // minus the viscous face fluxes (Eq. (residual): F_i,n - F_nu,n)
                    r -= (Vxr[v - 1] - Vxl[v - 1]) * G.ax;
                    r -= (Vy[t & 1][v - 1] - Vy[(t + 1) & 1][v - 1]) * G.ay;
                }
                if (SRC) r -= (CURV ? Ma[t & 1] : vol) * Sv[v];  // R = flux sum - |Omega| S
                if (STAGE == 0) {
                    out[v] = c[v] + sc * r;
                } else if (STAGE == 1) {
                    out[v] = 0.75 * Unb[t & 1][v] + 0.25 * (c[v] + sc * r);
                } else {
                    out[v] = (1.0 / 3.0) * Unb[t & 1][v] + (2.0 / 3.0) * (c[v] + sc * r);
                }
                st_buf<true>(rd[v], so, p, out[v]);
            }
            if (CURV && STAGE == 2) {
                // the x face right of this cell is the left face of the lane above
                double xr[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) xr[k] = lane_shift1<false>(Mx[t & 1][k]);
                if (out_lane && row_ok) {
                    const double lam =
                        curv_cell_lambda(out, G.gamma, G.gm1, Mx[t & 1], xr, Ylo, My[t & 1], Ma[t & 1], &fl);
                    lmax = fmax(lmax, lam);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) Ylo[k] = My[t & 1][k];
            } else if (STAGE == 2 && out_lane && row_ok) {
                const double idx[2] = {G.inv_dx, G.inv_dy};
                double lam = cell_lambda<2>(out, G.gamma, G.gm1, idx, fl);
                if (VISC) lam += 2.0 * ((G.mu / out[0]) * G.nu_fac) * (G.inv_dx * G.inv_dx + G.inv_dy * G.inv_dy);
                lmax = fmax(lmax, lam);
            }
            // keep the scheduler from overlapping consecutive rows, which
            // would raise the live register count
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// The viscous and curvilinear variants ask for two waves per SIMD (at most
// 256 VGPRs): their stage-3 kernels come out two registers above that
// otherwise, at one wave per SIMD. The curvilinear stage-1 kernel without a
// source asks for three (at most 168): it comes out at 170 otherwise, and at
// 168 it needs no spill and runs the curvilinear step 2.5% faster. The other
// variants keep the default.
template <int STAGE, bool SRC, int MODE>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu((MODE == 3 && STAGE == 0 && !SRC) ? 3 : (MODE >= 2 ? 2 : 1)))) k_fused2d(const FGrid* __restrict__ grids, int ngrids, int nitems,
                                                 const double* Un, const double* __restrict__ Us, double* Ud,
                                                 unsigned long long* __restrict__ lam, double* __restrict__ dtg,
                                                 const double* __restrict__ dt_fixed, double* __restrict__ dt_out,
                                                 uint32_t* __restrict__ status, unsigned long long* __restrict__ clk,
                                                 const double* __restrict__ src, const double* __restrict__ met) {
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int wave0 = __builtin_amdgcn_readfirstlane(
        (int)((xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6));
    if (STAGE == 1 && blockIdx.x == 0)
        for (int g = threadIdx.x; g < ngrids; g += blockDim.x) lam[g] = 0ull;  // stage 1 has read it
    for (int item = wave0; item < nitems; item += nwaves) {
        unsigned long long t_start = 0;
        if (clk) t_start = wall_clock64();
        const int gi = find_grid(grids, ngrids, item);
        const FGrid G = grids[gi];
        const int local = item - G.work0;
        const int strip = local % G.strips;
        const int sidx = local / G.strips;
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
        const double s = MODE == 3 ? -dt : -dt * G.inv_vol;  // curvilinear: times each cell's 1 / area
        double lmax = 0.0;
        uint32_t fl = 0;
        if (G.scheme == 0) {
            fused2d_rows<STAGE, 0, SRC, MODE>(G, lane, strip, sidx * G.seg, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, met);
        } else if (G.scheme == 5) {
            fused2d_rows<STAGE, 3, SRC, MODE>(G, lane, strip, sidx * G.seg, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, met);
        } else if (G.scheme == 1) {
            fused2d_rows<STAGE, 1, SRC, MODE>(G, lane, strip, sidx * G.seg, s, Un, Us, Ud, lmax, fl, 0.0, 0.0, src, met);
        } else {
            double ka, kb;
            kappa_weights(G.scheme, ka, kb);
            fused2d_rows<STAGE, 2, SRC, MODE>(G, lane, strip, sidx * G.seg, s, Un, Us, Ud, lmax, fl, ka, kb, src, met);
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
            const int slot = item & (CLK_SLOTS - 1);
            atomicMin(&clk[clk_index((G.gid * 3 + STAGE) * 2 + 0, slot)], t_start);
            atomicMax(&clk[clk_index((G.gid * 3 + STAGE) * 2 + 1, slot)], t_end);
        }
    }
}

static inline int fused_blocks(int nitems, int waves) {
    const int w = waves > 0 ? (waves < nitems ? waves : nitems) : nitems;
    return (w + 3) / 4;
}

template <bool SRC, int MODE>
static void launch_fused_stage_t(int stage, dim3 grid, dim3 block, const FGrid* grids, int ngrids, int nitems,
                                 const double* Un, const double* Us, double* Ud, unsigned long long* lam,
                                 double* dtg, const double* dt_fixed, double* dt_out, uint32_t* status,
                                 unsigned long long* clk, const double* src, const double* met, hipStream_t s) {
    if (stage == 0)
        hipLaunchKernelGGL((k_fused2d<0, SRC, MODE>), grid, block, 0, s, grids, ngrids, nitems, Un, Us, Ud, lam, dtg,
                           dt_fixed, dt_out, status, clk, src, met);
    else if (stage == 1)
        hipLaunchKernelGGL((k_fused2d<1, SRC, MODE>), grid, block, 0, s, grids, ngrids, nitems, Un, Us, Ud, lam, dtg,
                           dt_fixed, dt_out, status, clk, src, met);
    else
        hipLaunchKernelGGL((k_fused2d<2, SRC, MODE>), grid, block, 0, s, grids, ngrids, nitems, Un, Us, Ud, lam, dtg,
                           dt_fixed, dt_out, status, clk, src, met);
}

// The curvilinear variant's launches (fv_fused_curv.hip).
void launch_fused_stage_curv(int stage, dim3 grid, dim3 block, const FGrid* grids, int ngrids, int nitems,
                             const double* Un, const double* Us, double* Ud, unsigned long long* lam, double* dtg,
                             const double* dt_fixed, double* dt_out, uint32_t* status, unsigned long long* clk,
                             const double* src, const double* met, hipStream_t s);

}  // namespace fvk
