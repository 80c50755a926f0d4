// Device-side building blocks of the finite-volume step for gfx950:
// geometry of the ghosted SoA layout, integer division by an invariant,
// the minmod MUSCL face states and the Roe flux.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fvk {

constexpr int NG = 2;  // ghost layers per face (the 4-cell MUSCL stencil)

// Division by a run-time invariant d >= 1 for 0 <= n < 2^32, by multiply-high
// and shifts (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, unsigned case).
struct DivMod {
    uint32_t d, m, sh1, sh2;
};

inline DivMod make_divmod(uint32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;  // l = ceil(log2 d)
    DivMod r;
    r.d = d;
    r.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
    r.sh1 = l < 1 ? l : 1;
    r.sh2 = l > 0 ? l - 1 : 0;
    return r;
}

__host__ __device__ inline uint32_t divq(uint32_t n, const DivMod& dm) {
    uint32_t t = (uint32_t)(((uint64_t)dm.m * n) >> 32);
    return (t + ((n - t) >> dm.sh1)) >> dm.sh2;
}

// Geometry and constants of one grid, passed by value to every kernel.
// Ghost state of inflow faces, per axis and side (conserved variables).
struct BcState {
    double q[3][2][5];
};

struct Geo {
    int ndim, nvar;
    int n[3];           // interior cells per axis
    int sy, sz;         // state strides in elements (s_x = 1)
    int off0;           // offset of interior cell (0,0,0) inside one variable
    int ncell;          // n[0] * n[1] * n[2]
    long long sv;       // per-variable stride of the state
    long long fsv[3];   // per-variable stride of the face-flux array of each axis
    DivMod dnx, dny;    // division by n[0] and n[1]
    double inv_dx[3];   // 1 / dx_d
    double area[3];     // face area of axis d: product of the other widths
    double inv_vol;     // 1 / |Omega|
    double vol;         // |Omega|
    double gamma, gm1;  // gamma, gamma - 1
    double cfl;
    int bc[3][2];
    int scheme;         // 0 minmod; Psi = 1 with kappa = -1, 0, 1/3, 1 for 1 .. 4; 5 van Leer; 6 kappa = 1/2
    double mu;          // dynamic viscosity, 0 for the Euler equations
    double kcond;       // heat conductivity mu gamma / ((gamma - 1) Pr)
    double nu_fac;      // max(4/3, gamma / Pr): the larger diffusivity per unit kinematic viscosity
    // Curvilinear 2D grid (null for the uniform box): metric streams in the
    // workspace, SoA. x faces ((nx + 1) ny each, face (i, j) between cells
    // (i - 1, j) and (i, j)): unit normal x, unit normal y, length; then y
    // faces (nx (ny + 1) each, face (i, j) between (i, j - 1) and (i, j)): the
    // same three; then per cell: area and 1 / area.
    const double* met;
};

// Offsets of the metric streams of a curvilinear grid (elements).
struct MetricOffsets {
    long long fx, fy, cell;  // first element of the x-face, y-face and cell blocks
    long long nfx, nfy, nc;  // entries per stream of each block
};

__host__ __device__ inline MetricOffsets metric_offsets(int nx, int ny) {
    MetricOffsets m;
    m.nfx = (long long)(nx + 1) * ny;
    m.nfy = (long long)nx * (ny + 1);
    m.nc = (long long)nx * ny;
    m.fx = 0;
    m.fy = 3 * m.nfx;
    m.cell = m.fy + 3 * m.nfy;
    return m;
}

// 1/a and 1/sqrt(a) for the flux arithmetic: the hardware estimates
// (v_rcp_f64, v_rsq_f64, relative error about 5e-8) refined by one
// third-order correction each. With e the residual of the estimate y0,
//   1/a       = y0 / (1 - e)      = y0 (1 + e + e^2 + ...),        e = 1 - a y0,
//   1/sqrt(a) = y0 (1 - e)^(-1/2) = y0 (1 + e/2 + 3e^2/8 + ...),  e = 1 - a y0^2,
// and the series is cut after e^2, leaving an error of order e^3 (below
// 1e-21) plus the rounding of the last fma: within about one ulp of the
// correctly rounded result for the normal, positive arguments the Euler
// fluxes produce, in 3 (rcp) and 5 (rsqrt) operations after the estimate.
__host__ __device__ __forceinline__ double rcp_nr(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double x = __builtin_amdgcn_rcp(a);
    const double e = fma(-a, x, 1.0);
    return fma(x, fma(e, e, e), x);
#else
    return 1.0 / a;
#endif
}

__host__ __device__ __forceinline__ double rsqrt_nr(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(a);
    const double e = fma(-a * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
#else
    return 1.0 / sqrt(a);
#endif
}

// minmod(a, b): zero unless a and b share a strict sign, else the one of smaller
// magnitude, i.e. the median of a, b and 0, written as
// max(min(a, b), min(max(a, b), 0)): for two positive slopes the inner min
// with 0 gives 0 and the outer max the smaller slope, for two negative ones
// the inner min gives the one nearer 0, and for mixed signs or a zero the
// result is 0. No product, so tiny slopes do not underflow, and no compares
// or selects (four min/max).
__host__ __device__ __forceinline__ double minmod(double a, double b) {
    return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// van Leer's limited difference Psi(b/a) a with Psi(r) = (r + |r|)/(1 + |r|):
// 2ab/(a + b) for slopes of one sign, else 0. Symmetric in a and b, bit for
// bit (products and sums commute), so one value serves both faces of a cell.
__host__ __device__ __forceinline__ double vanleer(double a, double b) {
    const double ab = a * b;
    return ab > 0.0 ? 2.0 * ab * rcp_nr(a + b) : 0.0;
}

// MUSCL face states from the three differences of the stencil,
// dm = q1 - q0, dc = q2 - q1, dp = q3 - q2 (for callers that share them
// between neighbouring faces); UNL selects Psi = 1.
template <bool UNL>
__host__ __device__ __forceinline__ void muscl_from_diffs(double q1, double q2, double dm, double dc, double dp,
                                                         double& qL, double& qR) {
    if (UNL) {
        qL = q1 + 0.5 * dm;
        qR = q2 - 0.5 * dp;
    } else {
        qL = q1 + 0.5 * minmod(dm, dc);
        qR = q2 - 0.5 * minmod(dp, dc);
    }
}

// MUSCL face states (epsilon = 1, kappa = -1, minmod) at face k+1/2 of the
// cells q0 = k-1, q1 = k, q2 = k+1, q3 = k+2.
__host__ __device__ __forceinline__ void muscl_minmod(double q0, double q1, double q2, double q3,
                                             double& qL, double& qR) {
    muscl_from_diffs<false>(q1, q2, q1 - q0, q2 - q1, q3 - q2, qL, qR);
}

// The same with the choice fixed at compile time (UNL: Psi = 1), for loops
// that must stay free of branches.
template <bool UNL>
__host__ __device__ __forceinline__ void muscl_fixed(double q0, double q1, double q2, double q3, double& qL,
                                                    double& qR) {
    muscl_from_diffs<UNL>(q1, q2, q1 - q0, q2 - q1, q3 - q2, qL, qR);
}

// Weights of the unlimited (Psi = 1) kappa family of Eq. (flux) with
// epsilon = 1: Q^L = Q_k + a dQ_{k-1/2} + b dQ_{k+1/2} and
// Q^R = Q_{k+1} - b dQ_{k+1/2} - a dQ_{k+3/2}, a = (1 - kappa)/4,
// b = (1 + kappa)/4, for schemes 2 .. 4 (kappa = 0, 1/3, 1) and 6 (kappa = 1/2).
__host__ __device__ __forceinline__ void kappa_weights(int scheme, double& a, double& b) {
    const double kappa = scheme == 2 ? 0.0 : (scheme == 3 ? 1.0 / 3.0 : (scheme == 6 ? 0.5 : 1.0));
    a = 0.25 * (1.0 - kappa);
    b = 0.25 * (1.0 + kappa);
}

// Face states of the kappa family from the stencil's differences, with
// explicit fused multiply-adds: the same bits whether the differences are
// formed per face or shared per cell, whatever the compiler contracts.
__host__ __device__ __forceinline__ void muscl_kappa_diffs(double q1, double q2, double dm, double dc, double dp,
                                                          double a, double b, double& qL, double& qR) {
    qL = fma(a, dm, fma(b, dc, q1));
    qR = fma(-b, dc, fma(-a, dp, q2));
}

// The same with the scheme chosen at run time (uniform): 0 minmod, 1 Psi = 1
// with kappa = -1, 2 .. 4 and 6 the other kappa members, 5 van Leer.
__host__ __device__ __forceinline__ void muscl(double q0, double q1, double q2, double q3, int scheme,
                                              double& qL, double& qR) {
    if (scheme == 1) {
        qL = q1 + 0.5 * (q1 - q0);
        qR = q2 - 0.5 * (q3 - q2);
    } else if (scheme == 0) {
        muscl_minmod(q0, q1, q2, q3, qL, qR);
    } else if (scheme == 5) {
        const double dc = q2 - q1;
        qL = q1 + 0.5 * vanleer(q1 - q0, dc);
        qR = q2 - 0.5 * vanleer(dc, q3 - q2);
    } else {
        double a, b;
        kappa_weights(scheme, a, b);
        muscl_kappa_diffs(q1, q2, q1 - q0, q2 - q1, q3 - q2, a, b, qL, qR);
    }
}

// Roe flux along axis AX for NDIM dimensions, conserved face states in, flux out.
// F = (F(qL) + F(qR))/2 - sum_k |lambda_k| alpha_k r_k / 2, no entropy fix.
// TWICE returns 2F: callers that difference the fluxes fold the exact factor
// 1/2 into their face areas and save a multiply per component.
template <int NDIM, int AX, bool TWICE = false>
__host__ __device__ __forceinline__ void roe_flux(const double* qL, const double* qR, double gm1, double* F) {
    constexpr int IE = NDIM + 1;
    // left / right primitive states; rho^(-1/2) gives both sqrt(rho) and 1/rho
    const double rL = qL[0], rR = qR[0];
    const double rsL = rsqrt_nr(rL), rsR = rsqrt_nr(rR);
    const double irL = rsL * rsL, irR = rsR * rsR;
    double uL[NDIM], uR[NDIM];
    double qqL = 0.0, qqR = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        uL[d] = qL[1 + d] * irL;
        uR[d] = qR[1 + d] * irR;
        qqL += uL[d] * uL[d];
        qqR += uR[d] * uR[d];
    }
    const double pL = gm1 * (qL[IE] - 0.5 * rL * qqL);
    const double pR = gm1 * (qR[IE] - 0.5 * rR * qqR);
    const double HL = (qL[IE] + pL) * irL;
    const double HR = (qR[IE] + pR) * irR;
    const double vnL = uL[AX], vnR = uR[AX];

    // Roe averages with weights sqrt(rho) / (sqrt(rhoL) + sqrt(rhoR))
    const double sL = rL * rsL, sR = rR * rsR;
    const double iw = rcp_nr(sL + sR);
    const double wL = sL * iw, wR = sR * iw;
    double ut[NDIM];
    double qqt = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        ut[d] = wL * uL[d] + wR * uR[d];
        qqt += ut[d] * ut[d];
    }
    const double Ht = wL * HL + wR * HR;
    const double rt = sL * sR;
    const double c2 = gm1 * (Ht - 0.5 * qqt);
    const double rc = rsqrt_nr(c2);
    const double c = c2 * rc;
    const double ic2 = rc * rc;
    const double un = ut[AX];

    // wave strengths
    const double dp = pR - pL;
    const double dun = vnR - vnL;
    const double rcdu = rt * c * dun;
    const double hic2 = 0.5 * ic2;  // exact scaling: a1, a5 as (0.5 (dp -+ rcdu)) / c^2
    const double a1 = (dp - rcdu) * hic2;
    const double a2 = (rR - rL) - dp * ic2;
    const double a5 = (dp + rcdu) * hic2;
    // |lambda| times strength
    const double w1 = fabs(un - c) * a1;
    const double w2 = fabs(un) * a2;
    const double w5 = fabs(un + c) * a5;
    const double aun = fabs(un) * rt;  // |u_n| rho~ (shear waves)

    // dissipation D = sum_k |lambda_k| alpha_k r_k
    double D[NDIM + 2];
    const double w15 = w1 + w5;
    D[0] = w15 + w2;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        if (d == AX)
            D[1 + d] = w15 * ut[d] + (w5 - w1) * c + w2 * ut[d];
        else
            D[1 + d] = (w15 + w2) * ut[d] + aun * (uR[d] - uL[d]);
    }
    double De = w15 * Ht + (w5 - w1) * un * c + w2 * 0.5 * qqt;
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
        if (d != AX) De += aun * (uR[d] - uL[d]) * ut[d];
    D[IE] = De;

    // central part: physical fluxes of both sides (the mass flux rho u_n is
    // the normal momentum itself)
    const double mL = qL[1 + AX], mR = qR[1 + AX];
    constexpr double h = TWICE ? 1.0 : 0.5;
    F[0] = h * (mL + mR - D[0]);
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        double fl = mL * uL[d], fr = mR * uR[d];
        if (d == AX) {
            fl += pL;
            fr += pR;
        }
        F[1 + d] = h * (fl + fr - D[1 + d]);
    }
    F[IE] = h * ((qL[IE] + pL) * vnL + (qR[IE] + pR) * vnR - D[IE]);
}

// Roe flux through a 2D face of unit normal (nx, ny), conserved face states
// in, flux out: the momenta are turned into the face's frame (normal
// nx u + ny v, tangential -ny u + nx v), the flux of the x-axis form above is
// taken there, and its momentum part is turned back. The same flux as the
// normal form F = (F_n(QL) + F_n(QR))/2 - |A_n| dQ / 2 with V_n = n.u.
__host__ __device__ __forceinline__ void roe_flux_n2(const double* qL, const double* qR, double nx, double ny,
                                                     double gm1, double* F) {
    double a[4], b[4], G[4];
    a[0] = qL[0];
    a[1] = nx * qL[1] + ny * qL[2];
    a[2] = -ny * qL[1] + nx * qL[2];
    a[3] = qL[3];
    b[0] = qR[0];
    b[1] = nx * qR[1] + ny * qR[2];
    b[2] = -ny * qR[1] + nx * qR[2];
    b[3] = qR[3];
    roe_flux<2, 0>(a, b, gm1, G);
    F[0] = G[0];
    F[1] = nx * G[1] - ny * G[2];
    F[2] = ny * G[1] + nx * G[2];
    F[3] = G[3];
}

// Wave-speed bound of one cell, sum_d (|u_d| + c) * inv_dx[d], and the
// non-physical flags (1 NaN, 2 rho <= 0, 4 p <= 0) it raises.
template <int NDIM>
__host__ __device__ __forceinline__ double cell_lambda(const double* q, double gamma, double gm1, const double* inv_dx,
                                                       uint32_t& fl) {
    constexpr int IE = NDIM + 1;
    const double rho = q[0];
    const double ir = rcp_nr(rho);
    double u[NDIM];
    double qq = 0.0;
    for (int d = 0; d < NDIM; ++d) {
        u[d] = q[1 + d] * ir;
        qq += u[d] * u[d];
    }
    const double p = gm1 * (q[IE] - 0.5 * rho * qq);
    // c = sqrt(c^2) as c^2 * (c^2)^(-1/2); a negative c^2 gives NaN, as sqrt does
    const double c2 = gamma * p * ir;
    const double c = c2 * rsqrt_nr(c2);
    double lam = 0.0;
    for (int d = 0; d < NDIM; ++d) lam += (fabs(u[d]) + c) * inv_dx[d];
    if (isnan(lam) || isnan(rho) || isnan(p)) fl |= 1u;
    if (!(rho > 0.0)) fl |= 2u;
    if (!(p > 0.0)) fl |= 4u;
    return lam;
}

// Wave-speed bound of a cell of a curvilinear 2D grid from its conserved
// state, the unit normals and lengths (nx, ny, len) of its low and high x
// faces (xa, xb) and y faces (ya, yb), and its area: per grid direction, the
// mean of the two faces' area vectors S gives (|u . S| + c |S|) / area.
__host__ __device__ __forceinline__ double curv_cell_lambda(const double* q, double gamma, double gm1,
                                                            const double* xa, const double* xb, const double* ya,
                                                            const double* yb, double area, uint32_t* fl = nullptr) {
    const double ir = 1.0 / q[0];
    const double u = q[1] * ir, v = q[2] * ir;
    const double p = gm1 * (q[3] - 0.5 * q[0] * (u * u + v * v));
    const double c = sqrt(gamma * p * ir);
    double lam = 0.0;
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        const double* a = ax == 0 ? xa : ya;
        const double* b = ax == 0 ? xb : yb;
        const double sx = 0.5 * (a[0] * a[2] + b[0] * b[2]);
        const double sy = 0.5 * (a[1] * a[2] + b[1] * b[2]);
        lam += (fabs(u * sx + v * sy) + c * sqrt(sx * sx + sy * sy)) / area;
    }
    if (fl) {
        // the non-physical flags of cell_lambda: 1 NaN, 2 rho <= 0, 4 p <= 0
        if (isnan(lam) || isnan(q[0]) || isnan(p)) *fl |= 1u;
        if (!(q[0] > 0.0)) *fl |= 2u;
        if (!(p > 0.0)) *fl |= 4u;
    }
    return lam;
}

// ---------------------------------------------------------------------------
// Reverse (adjoint) of the face computation, hand-derived from the forward
// sequence above: given Fb = dJ/dF, accumulate dJ/dq of the four stencil
// cells. Branches (minmod selection, |lambda| signs) follow the forward
// evaluation; |x| has derivative 0 at x = 0.

// MUSCL-minmod reverse for one variable: qLb = dJ/dQL, qRb = dJ/dQR.
// g0..g3 receive dJ/dq of cells k-1, k, k+1, k+2 (accumulated).
__host__ __device__ __forceinline__ void muscl_minmod_vjp(double q0, double q1, double q2, double q3, double qLb,
                                                          double qRb, double& g0, double& g1, double& g2,
                                                          double& g3) {
    const double dm = q1 - q0, dc = q2 - q1, dp = q3 - q2;
    // QL = q1 + minmod(dm, dc) / 2 (Psi(dc/dm) dm: the dm branch at a tie)
    if (((dm > 0.0) & (dc > 0.0)) | ((dm < 0.0) & (dc < 0.0))) {
        if (fabs(dm) <= fabs(dc)) {  // q1 + (q1 - q0)/2
            g1 += 1.5 * qLb;
            g0 -= 0.5 * qLb;
        } else {  // (q1 + q2)/2
            g1 += 0.5 * qLb;
            g2 += 0.5 * qLb;
        }
    } else {
        g1 += qLb;
    }
    // QR = q2 - minmod(dp, dc) / 2; at a tie |dp| = |dc| both branches give the
    // same value, and the derivative follows the limiter written as
    // Psi(dp/dc) dc with Psi saturating at ratio >= 1, i.e. the dc branch
    if (((dp > 0.0) & (dc > 0.0)) | ((dp < 0.0) & (dc < 0.0))) {
        if (fabs(dp) < fabs(dc)) {  // 3/2 q2 - q3/2
            g2 += 1.5 * qRb;
            g3 -= 0.5 * qRb;
        } else {  // (q1 + q2)/2
            g1 += 0.5 * qRb;
            g2 += 0.5 * qRb;
        }
    } else {
        g2 += qRb;
    }
}

// Reverse of muscl(): the unlimited states are linear in the stencil,
// Q^L = (1 - b + a) q1 - a q0 + b q2 and Q^R = (1 - b + a) q2 + b q1 - a q3
// (a = 1/2, b = 0 for kappa = -1).
__host__ __device__ __forceinline__ void muscl_vjp(double q0, double q1, double q2, double q3, int scheme,
                                                   double qLb, double qRb, double& g0, double& g1, double& g2,
                                                   double& g3) {
    if (scheme == 1) {
        g1 += 1.5 * qLb;
        g0 -= 0.5 * qLb;
        g2 += 1.5 * qRb;
        g3 -= 0.5 * qRb;
    } else if (scheme == 0) {
        muscl_minmod_vjp(q0, q1, q2, q3, qLb, qRb, g0, g1, g2, g3);
    } else if (scheme == 5) {
        // d vl(a, b)/da = 2 b^2 / (a + b)^2 and symmetric, zero unless ab > 0
        const double dm = q1 - q0, dc = q2 - q1, dp = q3 - q2;
        double ga = 0.0, gb = 0.0, ha = 0.0, hb = 0.0;
        if (dm * dc > 0.0) {
            const double i2 = 2.0 / ((dm + dc) * (dm + dc));
            ga = i2 * dc * dc;
            gb = i2 * dm * dm;
        }
        if (dc * dp > 0.0) {
            const double i2 = 2.0 / ((dc + dp) * (dc + dp));
            ha = i2 * dp * dp;
            hb = i2 * dc * dc;
        }
        g0 -= 0.5 * ga * qLb;
        g1 += (1.0 + 0.5 * ga - 0.5 * gb) * qLb + 0.5 * ha * qRb;
        g2 += 0.5 * gb * qLb + (1.0 - 0.5 * ha + 0.5 * hb) * qRb;
        g3 -= 0.5 * hb * qRb;
    } else {
        double a, b;
        kappa_weights(scheme, a, b);
        const double c = 1.0 - b + a;
        g0 -= a * qLb;
        g1 += c * qLb + b * qRb;
        g2 += b * qLb + c * qRb;
        g3 -= a * qRb;
    }
}

__host__ __device__ __forceinline__ double sgn0(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// Reverse of roe_flux<NDIM, AX>: Fb[NV] in, qLb[NV] and qRb[NV] out (overwritten).
template <int NDIM, int AX>
__host__ __device__ __forceinline__ void roe_flux_vjp(const double* qL, const double* qR, double gm1, const double* Fb,
                                                      double* qLb, double* qRb) {
    constexpr int IE = NDIM + 1;
    // ---- forward recomputation (as in roe_flux) ----
    const double rL = qL[0], rR = qR[0];
    const double rsL = rsqrt_nr(rL), rsR = rsqrt_nr(rR);
    const double irL = rsL * rsL, irR = rsR * rsR;
    double uL[NDIM], uR[NDIM];
    double qqL = 0.0, qqR = 0.0;
    for (int d = 0; d < NDIM; ++d) {
        uL[d] = qL[1 + d] * irL;
        uR[d] = qR[1 + d] * irR;
        qqL += uL[d] * uL[d];
        qqR += uR[d] * uR[d];
    }
    const double EL = qL[IE], ER = qR[IE];
    const double pL = gm1 * (EL - 0.5 * rL * qqL);
    const double pR = gm1 * (ER - 0.5 * rR * qqR);
    const double HL = (EL + pL) * irL;
    const double HR = (ER + pR) * irR;
    const double vnL = uL[AX], vnR = uR[AX];
    const double sL = rL * rsL, sR = rR * rsR;
    const double iw = rcp_nr(sL + sR);
    const double wL = sL * iw, wR = sR * iw;
    double ut[NDIM];
    double qqt = 0.0;
    for (int d = 0; d < NDIM; ++d) {
        ut[d] = wL * uL[d] + wR * uR[d];
        qqt += ut[d] * ut[d];
    }
    const double Ht = wL * HL + wR * HR;
    const double rt = sL * sR;
    const double c2 = gm1 * (Ht - 0.5 * qqt);
    const double rc = rsqrt_nr(c2);
    const double c = c2 * rc;
    const double ic2 = rc * rc;
    const double un = ut[AX];
    const double dp = pR - pL;
    const double dun = vnR - vnL;
    const double rcdu = rt * c * dun;
    const double hic2 = 0.5 * ic2;  // exact scaling: a1, a5 as (0.5 (dp -+ rcdu)) / c^2
    const double a1 = (dp - rcdu) * hic2;
    const double a2 = (rR - rL) - dp * ic2;
    const double a5 = (dp + rcdu) * hic2;
    const double l1 = fabs(un - c), l2 = fabs(un), l5 = fabs(un + c);
    const double w1 = l1 * a1, w2 = l2 * a2, w5 = l5 * a5;
    const double aun = l2 * rt;
    const double w15 = w1 + w5;
    const double fmL = rL * vnL, fmR = rR * vnR;  // mass fluxes

    // ---- reverse ----
    double rLb = 0.0, rRb = 0.0, ELb = 0.0, ERb = 0.0, pLb = 0.0, pRb = 0.0;
    double vnLb = 0.0, vnRb = 0.0, fmLb = 0.0, fmRb = 0.0;
    double uLb[NDIM], uRb[NDIM], utb[NDIM];
    for (int d = 0; d < NDIM; ++d) uLb[d] = uRb[d] = utb[d] = 0.0;
    // F0 = (fmL + fmR - D0)/2; F[1+d] = (fmL uL + fmR uR + [d==AX](pL + pR) - D[1+d])/2;
    // F[IE] = ((EL + pL) vnL + (ER + pR) vnR - De)/2
    const double D0b = -0.5 * Fb[0];
    fmLb += 0.5 * Fb[0];
    fmRb += 0.5 * Fb[0];
    double Db[NDIM];
    for (int d = 0; d < NDIM; ++d) {
        const double f = 0.5 * Fb[1 + d];
        fmLb += f * uL[d];
        uLb[d] += f * fmL;
        fmRb += f * uR[d];
        uRb[d] += f * fmR;
        if (d == AX) {
            pLb += f;
            pRb += f;
        }
        Db[d] = -f;
    }
    {
        const double f = 0.5 * Fb[IE];
        ELb += f * vnL;
        pLb += f * vnL;
        vnLb += f * (EL + pL);
        ERb += f * vnR;
        pRb += f * vnR;
        vnRb += f * (ER + pR);
    }
    const double Deb = -0.5 * Fb[IE];
    // mass fluxes fm = r vn
    rLb += fmLb * vnL;
    vnLb += fmLb * rL;
    rRb += fmRb * vnR;
    vnRb += fmRb * rR;
    // De = w15 Ht + (w5 - w1) un c + w2 qqt/2 + sum_{d != AX} aun (uR - uL)_d ut_d
    double w15b = 0.0, w1b = 0.0, w2b = 0.0, w5b = 0.0, Htb = 0.0, unb = 0.0, cb = 0.0, qqtb = 0.0, aunb = 0.0;
    w15b += Deb * Ht;
    Htb += Deb * w15;
    w5b += Deb * un * c;
    w1b -= Deb * un * c;
    unb += Deb * (w5 - w1) * c;
    cb += Deb * (w5 - w1) * un;
    w2b += Deb * 0.5 * qqt;
    qqtb += Deb * 0.5 * w2;
    for (int d = 0; d < NDIM; ++d) {
        if (d == AX) continue;
        const double du = uR[d] - uL[d];
        aunb += Deb * du * ut[d];
        uRb[d] += Deb * aun * ut[d];
        uLb[d] -= Deb * aun * ut[d];
        utb[d] += Deb * aun * du;
    }
    // D[1+d]
    for (int d = 0; d < NDIM; ++d) {
        if (d == AX) {
            // w15 ut + (w5 - w1) c + w2 ut
            w15b += Db[d] * ut[d];
            w2b += Db[d] * ut[d];
            utb[d] += Db[d] * (w15 + w2);
            w5b += Db[d] * c;
            w1b -= Db[d] * c;
            cb += Db[d] * (w5 - w1);
        } else {
            // (w15 + w2) ut + aun (uR - uL)
            w15b += Db[d] * ut[d];
            w2b += Db[d] * ut[d];
            utb[d] += Db[d] * (w15 + w2);
            aunb += Db[d] * (uR[d] - uL[d]);
            uRb[d] += Db[d] * aun;
            uLb[d] -= Db[d] * aun;
        }
    }
    // D0 = w15 + w2
    w15b += D0b;
    w2b += D0b;
    // w15 = w1 + w5
    w1b += w15b;
    w5b += w15b;
    // aun = l2 rt; w_k = l_k a_k
    double l1b = w1b * a1, l2b = w2b * a2 + aunb * rt, l5b = w5b * a5;
    double rtb = aunb * l2;
    const double a1b = w1b * l1, a2b = w2b * l2, a5b = w5b * l5;
    // l1 = |un - c|, l2 = |un|, l5 = |un + c|
    {
        const double s1 = sgn0(un - c), s2 = sgn0(un), s5 = sgn0(un + c);
        unb += l1b * s1 + l2b * s2 + l5b * s5;
        cb += -l1b * s1 + l5b * s5;
    }
    // a5 = (dp + rcdu) ic2 / 2; a2 = dr - dp ic2; a1 = (dp - rcdu) ic2 / 2
    double dpb = 0.5 * a5b * ic2 + 0.5 * a1b * ic2 - a2b * ic2;
    const double rcdub = 0.5 * a5b * ic2 - 0.5 * a1b * ic2;
    double ic2b = a5b * 0.5 * (dp + rcdu) + a1b * 0.5 * (dp - rcdu) - a2b * dp;
    rRb += a2b;
    rLb -= a2b;
    // rcdu = rt c dun
    rtb += rcdub * c * dun;
    cb += rcdub * rt * dun;
    const double dunb = rcdub * rt * c;
    vnRb += dunb;
    vnLb -= dunb;
    pRb += dpb;
    pLb -= dpb;
    // ic2 = 1/c2; c = sqrt(c2); c2 = gm1 (Ht - qqt/2)
    double c2b = -ic2b * ic2 * ic2 + cb * 0.5 * rc;
    Htb += gm1 * c2b;
    qqtb -= 0.5 * gm1 * c2b;
    // rt = sL sR
    double sLb = rtb * sR, sRb = rtb * sL;
    // Ht = wL HL + wR HR
    double wLb = Htb * HL, wRb = Htb * HR;
    const double HLb = Htb * wL, HRb = Htb * wR;
    // un is ut[AX]; qqt = sum ut^2; ut = wL uL + wR uR
    utb[AX] += unb;
    for (int d = 0; d < NDIM; ++d) {
        utb[d] += 2.0 * ut[d] * qqtb;
        wLb += utb[d] * uL[d];
        uLb[d] += utb[d] * wL;
        wRb += utb[d] * uR[d];
        uRb[d] += utb[d] * wR;
    }
    // wL = sL iw, wR = sR iw, iw = 1/(sL + sR)
    const double iwb = wLb * sL + wRb * sR;
    sLb += wLb * iw;
    sRb += wRb * iw;
    const double sumb = -iwb * iw * iw;
    sLb += sumb;
    sRb += sumb;
    rLb += sLb * 0.5 * rsL;
    rRb += sRb * 0.5 * rsR;
    // per side: H = (E + p) ir; p = gm1 (E - r qq / 2); qq = sum u^2; u = m ir; ir = 1/r
    {
        double irb = HLb * (EL + pL);
        ELb += HLb * irL;
        pLb += HLb * irL;
        ELb += gm1 * pLb;
        rLb -= 0.5 * gm1 * qqL * pLb;
        const double qqb = -0.5 * gm1 * rL * pLb;
        uLb[AX] += vnLb;
        for (int d = 0; d < NDIM; ++d) {
            uLb[d] += 2.0 * uL[d] * qqb;
            qLb[1 + d] = uLb[d] * irL;
            irb += uLb[d] * qL[1 + d];
        }
        rLb -= irb * irL * irL;
        qLb[0] = rLb;
        qLb[IE] = ELb;
    }
    {
        double irb = HRb * (ER + pR);
        ERb += HRb * irR;
        pRb += HRb * irR;
        ERb += gm1 * pRb;
        rRb -= 0.5 * gm1 * qqR * pRb;
        const double qqb = -0.5 * gm1 * rR * pRb;
        uRb[AX] += vnRb;
        for (int d = 0; d < NDIM; ++d) {
            uRb[d] += 2.0 * uR[d] * qqb;
            qRb[1 + d] = uRb[d] * irR;
            irb += uRb[d] * qR[1 + d];
        }
        rRb -= irb * irR * irR;
        qRb[0] = rRb;
        qRb[IE] = ERb;
    }
}

}  // namespace fvk
