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
    double gamma, gm1;  // gamma, gamma - 1
    double cfl;
    int bc[3][2];
};

// minmod(a, b): zero unless a and b share a strict sign, else the one of smaller
// magnitude. Sign tests, not a*b > 0, so tiny slopes do not underflow to a tie.
__device__ __forceinline__ double minmod(double a, double b) {
    const bool pos = (a > 0.0) & (b > 0.0);
    const bool neg = (a < 0.0) & (b < 0.0);
    const double m = fabs(a) <= fabs(b) ? a : b;
    return (pos | neg) ? m : 0.0;
}

// MUSCL face states (epsilon = 1, kappa = -1, minmod) at face k+1/2 of the
// cells q0 = k-1, q1 = k, q2 = k+1, q3 = k+2.
__device__ __forceinline__ void muscl_minmod(double q0, double q1, double q2, double q3,
                                             double& qL, double& qR) {
    const double dm = q1 - q0, dc = q2 - q1, dp = q3 - q2;
    qL = q1 + 0.5 * minmod(dm, dc);
    qR = q2 - 0.5 * minmod(dp, dc);
}

// Roe flux along axis AX for NDIM dimensions, conserved face states in, flux out.
// F = (F(qL) + F(qR))/2 - sum_k |lambda_k| alpha_k r_k / 2, no entropy fix.
template <int NDIM, int AX>
__device__ __forceinline__ void roe_flux(const double* qL, const double* qR, double gm1, double* F) {
    constexpr int IE = NDIM + 1;
    // left / right primitive states
    const double rL = qL[0], rR = qR[0];
    const double irL = 1.0 / rL, irR = 1.0 / rR;
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
    const double sL = sqrt(rL), sR = sqrt(rR);
    const double iw = 1.0 / (sL + sR);
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
    const double c = sqrt(c2);
    const double ic2 = 1.0 / c2;
    const double un = ut[AX];

    // wave strengths
    const double dp = pR - pL;
    const double dun = vnR - vnL;
    const double rcdu = rt * c * dun;
    const double a1 = 0.5 * (dp - rcdu) * ic2;
    const double a2 = (rR - rL) - dp * ic2;
    const double a5 = 0.5 * (dp + rcdu) * ic2;
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

    // central part: physical fluxes of both sides
    const double mL = rL * vnL, mR = rR * vnR;
    F[0] = 0.5 * (mL + mR - D[0]);
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        double fl = mL * uL[d], fr = mR * uR[d];
        if (d == AX) {
            fl += pL;
            fr += pR;
        }
        F[1 + d] = 0.5 * (fl + fr - D[1 + d]);
    }
    F[IE] = 0.5 * ((qL[IE] + pL) * vnL + (qR[IE] + pR) * vnR - D[IE]);
}

}  // namespace fvk
