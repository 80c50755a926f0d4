// FP64 CPU oracle for the explicit finite-volume Euler step.
//
// TEST INFRASTRUCTURE ONLY. Nothing on the product path links, loads or calls
// this file; only the test suite, the smoke check and the CPU-baseline leg of
// the bench do. It shares no code, header or constant with the HIP library.
//
// What it computes, each part following the paper's description of SENSEI:
//   * cell-wise semi-discrete form |Omega_k| dU/dt + R = 0 (Eq. spatial_residual),
//   * residual R = sum over faces of the normal inviscid minus viscous flux
//     times face area, minus |Omega| times the cell-averaged source (Eq.
//     residual; the fluxes of Eq. QF; the viscous flux, with Stokes stresses
//     and Fourier heat conduction, only when a viscosity is given),
//   * face states by MUSCL extrapolation with epsilon = 1 and a limiter Psi
//     (Eq. flux); kappa is a parameter, -1 (fully upwind) on the measured path,
//   * an explicit Runge-Kutta march (Sec. "A Test Case"), here the three-stage
//     strong-stability-preserving scheme of Shu and Osher,
//   * a stability-limited time step (Sec. "The CFD Code Base" asks only that the
//     time march be stable): dt = CFL / max_cells sum_d (|u_d| + c) / dx_d,
//     plus the explicit diffusion limit when a viscosity is given.
// The paper names no limiter, flux function or Runge-Kutta order; this oracle
// uses the minmod limiter, Roe's approximate Riemann solver (Roe 1981; Toro,
// "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 11) and
// SSP-RK3, taken in the textbook form written out below.
//
// Layout: interior cells only, U[v][k][j][i], v over (rho, rho u, rho v,
// [rho w], E). Boundary conditions are index maps: a periodic face wraps the
// index, a transmissive face clamps it to the nearest interior cell (a
// zero-gradient ghost state), a slip wall reflects it across the face and
// reverses the momentum normal to the wall (the mirror image), and an inflow
// face holds a given state in its ghost cells (supersonic inflow: every
// characteristic enters). Two ghost layers are implied by the 4-cell MUSCL
// stencil.
//
// Every routine is a template over the scalar type so that the same code runs
// on std::complex<double> for complex-step derivatives (Squire & Trapp 1998):
// branches (limiter, |lambda|) are taken on the real part.
//
// Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (see oracle/build.py).

#include <omp.h>

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

typedef std::complex<double> cplx;

extern "C" {
// Grid description passed from Python (ctypes mirrors this struct).
struct OrGrid {
    int32_t ndim;       // 2 or 3
    int32_t limiter;    // 1 = minmod, 2 = van Leer, 0 = unlimited (Psi = 1)
    int64_t n[3];       // cells per axis (n[2] = 1 in 2D)
    double dx[3];       // cell widths
    int32_t bc[3][2];   // 0 = periodic, 1 = transmissive, 2 = slip wall, 3 = inflow, per axis and side
    double gamma;       // ratio of specific heats
    double cfl;         // CFL number for the stable time step
    double kappa;       // MUSCL kappa (-1 on the measured path)
    const double* source;  // cell-averaged source S[v][k][j][i], or null for S = 0
    double bc_state[3][2][5];  // conserved state of the ghost cells of an inflow face
    double mu;          // dynamic viscosity (constant); 0 for the Euler equations
    double prandtl;     // Prandtl number of the heat flux (used when mu > 0)
    const double* nodes;  // 2D curvilinear grid: node coordinates [2][ny+1][nx+1], or null for the
                          // uniform box given by dx
};
}

// Flag bits returned by the wave-speed reduction.
static const uint32_t OR_FLAG_NAN = 1u;
static const uint32_t OR_FLAG_RHO = 2u;
static const uint32_t OR_FLAG_P = 4u;

// Real part used for branch decisions. Under the complex step, products of
// imaginary parts shift real parts by O(h^2) (about 1e-60 for h = 1e-30); a real
// value that is exactly zero in the real evaluation (a state at rest, a flat
// stencil) would then take an arbitrary branch. Magnitudes below 1e-50 are read
// as zero so every branch matches the real evaluation. Real arithmetic is
// unaffected.
static inline double re(double x) { return x; }
static inline double re(const cplx& x) {
    const double r = x.real();
    return std::fabs(r) < 1e-50 ? 0.0 : r;
}

// |x| with the branch taken on the real part; the derivative at 0 is 0.
template <class T> static inline T absr(const T& x) {
    if (re(x) > 0.0) return x;
    if (re(x) < 0.0) return -x;
    return T(0.0);
}

// minmod limiter function Psi(r) = max(0, min(1, r)) (Roe / Sweby form).
template <class T> static inline T psi_minmod(const T& r) {
    if (!(re(r) > 0.0)) return T(0.0);
    if (re(r) < 1.0) return r;
    return T(1.0);
}

// van Leer's limiter function Psi(r) = (r + |r|) / (1 + |r|) (van Leer 1974),
// written for r > 0 as 2r / (1 + r); zero for r <= 0.
template <class T> static inline T psi_vanleer(const T& r) {
    if (!(re(r) > 0.0)) return T(0.0);
    return 2.0 * r / (1.0 + r);
}

// Limited difference Psi(num/den) * den, with Psi * 0 := 0.
// limiter: 0 Psi = 1, 1 minmod (this equals minmod(den, num)), 2 van Leer.
template <class T> static inline T limited(const T& num, const T& den, int limiter) {
    if (!limiter) return den;
    if (re(den) == 0.0) return T(0.0);
    if (limiter == 2) return psi_vanleer(num / den) * den;
    // the branch of Psi is taken on the ratio of the real parts
    const double rr = re(num) / re(den);
    if (!(rr > 0.0)) return T(0.0);
    if (rr < 1.0) return (num / den) * den;
    return den;
}

// MUSCL extrapolation to face k+1/2 from cells k-1, k, k+1, k+2 (Eq. flux):
//   QL = Q_k     + eps/4 [(1-kappa) Psi+_{k-1/2} (Q_k - Q_{k-1})
//                       + (1+kappa) Psi-_{k+1/2} (Q_{k+1} - Q_k)]
//   QR = Q_{k+1} - eps/4 [(1+kappa) Psi+_{k+1/2} (Q_{k+1} - Q_k)
//                       + (1-kappa) Psi-_{k+3/2} (Q_{k+2} - Q_{k+1})]
// with eps = 1 and the ratios r+_{j} = dQ_{j+1}/dQ_{j}, r-_{j} = dQ_{j-1}/dQ_{j}
// of consecutive differences dQ_{k-1/2}, dQ_{k+1/2}, dQ_{k+3/2}.
template <class T>
static inline void muscl(const T& qm1, const T& q0, const T& qp1, const T& qp2,
                         int limiter, double kappa, T& qL, T& qR) {
    const double eps = 1.0;
    T dm = q0 - qm1;   // dQ_{k-1/2}
    T d0 = qp1 - q0;   // dQ_{k+1/2}
    T dp = qp2 - qp1;  // dQ_{k+3/2}
    T lim_m_plus = limited(d0, dm, limiter);   // Psi+_{k-1/2} dQ_{k-1/2}
    T lim_0_minus = limited(dm, d0, limiter);  // Psi-_{k+1/2} dQ_{k+1/2}
    T lim_0_plus = limited(dp, d0, limiter);   // Psi+_{k+1/2} dQ_{k+1/2}
    T lim_p_minus = limited(d0, dp, limiter);  // Psi-_{k+3/2} dQ_{k+3/2}
    qL = q0 + (eps / 4.0) * ((1.0 - kappa) * lim_m_plus + (1.0 + kappa) * lim_0_minus);
    qR = qp1 - (eps / 4.0) * ((1.0 + kappa) * lim_0_plus + (1.0 - kappa) * lim_p_minus);
}

// Physical inviscid flux normal to axis `ax` (Eq. QF with n = e_ax).
template <class T>
static void phys_flux(int ndim, int ax, double gam, const T* Q, T* F) {
    const int ie = ndim + 1;
    T rho = Q[0];
    T u[3];
    T qq = T(0.0);
    for (int d = 0; d < ndim; ++d) {
        u[d] = Q[1 + d] / rho;
        qq = qq + u[d] * u[d];
    }
    T p = (gam - 1.0) * (Q[ie] - 0.5 * rho * qq);
    T vn = u[ax];
    F[0] = rho * vn;
    for (int d = 0; d < ndim; ++d) F[1 + d] = rho * u[d] * vn + (d == ax ? p : T(0.0));
    F[ie] = (Q[ie] + p) * vn;  // rho h_t V_n with h_t = (E + p)/rho
}

// Roe flux normal to axis `ax`: F = (F(QL) + F(QR))/2 - sum_k |lambda_k| alpha_k r_k / 2.
template <class T>
static void roe_flux(int ndim, int ax, double gam, const T* QL, const T* QR, T* F) {
    const int nv = ndim + 2;
    const int ie = ndim + 1;
    T FL[5], FR[5];
    phys_flux(ndim, ax, gam, QL, FL);
    phys_flux(ndim, ax, gam, QR, FR);

    T rL = QL[0], rR = QR[0];
    T uL[3], uR[3];
    T qqL = T(0.0), qqR = T(0.0);
    for (int d = 0; d < ndim; ++d) {
        uL[d] = QL[1 + d] / rL;
        uR[d] = QR[1 + d] / rR;
        qqL = qqL + uL[d] * uL[d];
        qqR = qqR + uR[d] * uR[d];
    }
    T pL = (gam - 1.0) * (QL[ie] - 0.5 * rL * qqL);
    T pR = (gam - 1.0) * (QR[ie] - 0.5 * rR * qqR);
    T HL = (QL[ie] + pL) / rL;
    T HR = (QR[ie] + pR) / rR;

    // Roe-averaged state.
    T sL = std::sqrt(rL), sR = std::sqrt(rR);
    T ut[3];
    T qqt = T(0.0);
    for (int d = 0; d < ndim; ++d) {
        ut[d] = (sL * uL[d] + sR * uR[d]) / (sL + sR);
        qqt = qqt + ut[d] * ut[d];
    }
    T Ht = (sL * HL + sR * HR) / (sL + sR);
    T rt = sL * sR;
    T c2 = (gam - 1.0) * (Ht - 0.5 * qqt);
    T c = std::sqrt(c2);
    T un = ut[ax];

    // Wave strengths.
    T drho = rR - rL;
    T dpr = pR - pL;
    T du[3];
    for (int d = 0; d < ndim; ++d) du[d] = uR[d] - uL[d];
    T a1 = (dpr - rt * c * du[ax]) / (2.0 * c2);
    T a2 = drho - dpr / c2;
    T a5 = (dpr + rt * c * du[ax]) / (2.0 * c2);

    // Wave speeds.
    T l1 = absr(un - c), l2 = absr(un), l5 = absr(un + c);

    // Sum of |lambda_k| alpha_k r_k, eigenvector by eigenvector.
    T D[5];
    for (int v = 0; v < nv; ++v) D[v] = T(0.0);
    // acoustic wave u_n - c: r1 = (1, u - c e_ax, H - u_n c)
    D[0] = D[0] + l1 * a1;
    for (int d = 0; d < ndim; ++d) D[1 + d] = D[1 + d] + l1 * a1 * (ut[d] - (d == ax ? c : T(0.0)));
    D[ie] = D[ie] + l1 * a1 * (Ht - un * c);
    // entropy wave u_n: r2 = (1, u, |u|^2/2)
    D[0] = D[0] + l2 * a2;
    for (int d = 0; d < ndim; ++d) D[1 + d] = D[1 + d] + l2 * a2 * ut[d];
    D[ie] = D[ie] + l2 * a2 * (0.5 * qqt);
    // shear waves u_n, one per tangential axis t: r_t = (0, e_t, u_t), alpha_t = rho du_t
    for (int t = 0; t < ndim; ++t) {
        if (t == ax) continue;
        T at = rt * du[t];
        D[1 + t] = D[1 + t] + l2 * at;
        D[ie] = D[ie] + l2 * at * ut[t];
    }
    // acoustic wave u_n + c: r5 = (1, u + c e_ax, H + u_n c)
    D[0] = D[0] + l5 * a5;
    for (int d = 0; d < ndim; ++d) D[1 + d] = D[1 + d] + l5 * a5 * (ut[d] + (d == ax ? c : T(0.0)));
    D[ie] = D[ie] + l5 * a5 * (Ht + un * c);

    for (int v = 0; v < nv; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * D[v];
}

// Ghost-index map of one axis: periodic wraps, transmissive clamps.
static inline int64_t bc_index(int64_t i, int64_t n, int lo_kind, int hi_kind) {
    if (i < 0) {
        if (lo_kind == 0) return ((i % n) + n) % n;
        if (lo_kind == 2) return -1 - i;  // mirror image across the face
        return 0;
    }
    if (i >= n) {
        if (hi_kind == 0) return i % n;
        if (hi_kind == 2) return 2 * n - 1 - i;
        return n - 1;
    }
    return i;
}

// The given state when position i lies behind an inflow face (else null).
static inline const double* bc_fixed(const OrGrid* g, int ax, int64_t i) {
    const int64_t n = g->n[ax];
    if (i < 0 && g->bc[ax][0] == 3) return g->bc_state[ax][0];
    if (i >= n && g->bc[ax][1] == 3) return g->bc_state[ax][1];
    return nullptr;
}

// -1 for the normal momentum of a ghost position behind a slip wall (the
// mirror image's velocity normal to the wall is reversed), else +1.
static inline double bc_sign(int64_t i, int64_t n, int lo_kind, int hi_kind, int v, int ax) {
    if (v != 1 + ax) return 1.0;
    if ((i < 0 && lo_kind == 2) || (i >= n && hi_kind == 2)) return -1.0;
    return 1.0;
}

static inline int64_t cell_offset(const OrGrid* g, int64_t i, int64_t j, int64_t k) {
    return (k * g->n[1] + j) * g->n[0] + i;
}

// Flux through the face between cell c and cell c + e_ax (c given by i, j, k).
template <class T>
static void face_flux(const OrGrid* g, const T* U, int ax, int64_t i, int64_t j, int64_t k, T* F) {
    const int nv = g->ndim + 2;
    const int64_t ncell = g->n[0] * g->n[1] * g->n[2];
    int64_t idx[3] = {i, j, k};
    int64_t off[4], pos[4];
    for (int m = 0; m < 4; ++m) {
        int64_t c[3] = {idx[0], idx[1], idx[2]};
        pos[m] = idx[ax] - 1 + m;  // cells k-1, k, k+1, k+2 along the axis
        c[ax] = bc_index(pos[m], g->n[ax], g->bc[ax][0], g->bc[ax][1]);
        off[m] = cell_offset(g, c[0], c[1], c[2]);
    }
    T QL[5], QR[5];
    for (int v = 0; v < nv; ++v) {
        const T* Uv = U + v * ncell;
        T q[4];
        for (int m = 0; m < 4; ++m) {
            const double* fixed = bc_fixed(g, ax, pos[m]);
            q[m] = fixed ? T(fixed[v]) : Uv[off[m]] * bc_sign(pos[m], g->n[ax], g->bc[ax][0], g->bc[ax][1], v, ax);
        }
        muscl(q[0], q[1], q[2], q[3], g->limiter, g->kappa, QL[v], QR[v]);
    }
    roe_flux(g->ndim, ax, g->gamma, QL, QR, F);
}

// Conserved state at cell position p (each axis index in [-2, n + 1]) through
// the boundary maps of every axis it lies outside of: the index is mapped
// axis by axis, a slip wall reverses that axis's momentum, and a position
// behind an inflow face takes the face's given state. A corner position (out
// of range on two axes) composes the maps of both.
template <class T>
static void cell_state(const OrGrid* g, const T* U, const int64_t p[3], T* q) {
    const int nv = g->ndim + 2;
    const int64_t ncell = g->n[0] * g->n[1] * g->n[2];
    int64_t c[3];
    double sgn[5] = {1.0, 1.0, 1.0, 1.0, 1.0};
    for (int ax = 0; ax < 3; ++ax) {
        if (ax < g->ndim) {
            const double* fixed = bc_fixed(g, ax, p[ax]);
            if (fixed) {
                for (int v = 0; v < nv; ++v) q[v] = T(fixed[v]);
                return;
            }
            for (int v = 0; v < nv; ++v) sgn[v] *= bc_sign(p[ax], g->n[ax], g->bc[ax][0], g->bc[ax][1], v, ax);
            c[ax] = bc_index(p[ax], g->n[ax], g->bc[ax][0], g->bc[ax][1]);
        } else {
            c[ax] = 0;
        }
    }
    const int64_t off = cell_offset(g, c[0], c[1], c[2]);
    for (int v = 0; v < nv; ++v) q[v] = U[v * ncell + off] * sgn[v];
}

// Velocity and temperature of a conserved state: T = p / rho, the ideal gas
// with unit gas constant of the nondimensional states used here.
template <class T>
static void velocity_temperature(int ndim, double gam, const T* q, T* w) {
    const T rho = q[0];
    T qq = T(0.0);
    for (int d = 0; d < ndim; ++d) {
        w[d] = q[1 + d] / rho;
        qq = qq + w[d] * w[d];
    }
    const T p = (gam - 1.0) * (q[ndim + 1] - 0.5 * rho * qq);
    w[ndim] = p / rho;
}

// Viscous flux normal to axis `ax` through the face between cell c and
// c + e_ax (F_nu,n of Eq. QF with n = e_ax):
//   (0, tau_{x,ax}, tau_{y,ax}, [tau_{z,ax}], Theta_ax),
//   tau_ab = mu (du_a/dx_b + du_b/dx_a) - 2/3 mu delta_ab div(u)   (Stokes),
//   Theta_ax = sum_b u_b tau_{b,ax} + k dT/dx_ax,   k = mu c_p / Pr,
//   c_p = gamma / (gamma - 1) (unit gas constant).
// Face gradients, second order on the uniform grid: the normal derivative is
// the difference of the two cells across the face over dx_ax; a tangential
// derivative along t is the mean of the central differences of those two
// cells, (w(c+e_t) - w(c-e_t) + w(c+e_ax+e_t) - w(c+e_ax-e_t)) / (4 dx_t);
// the velocity in Theta is the mean of the two cells.
template <class T>
static void visc_face_flux(const OrGrid* g, const T* U, int ax, int64_t i, int64_t j, int64_t k, T* F) {
    const int ndim = g->ndim, nv = ndim + 2;
    const double mu = g->mu;
    const double kc = mu * (g->gamma / (g->gamma - 1.0)) / g->prandtl;
    const int64_t c0[3] = {i, j, k};
    // w = (u, v, [w], T) at the two cells across the face
    T q[5], wa[4], wb[4];
    int64_t p[3] = {c0[0], c0[1], c0[2]};
    cell_state(g, U, p, q);
    velocity_temperature(ndim, g->gamma, q, wa);
    p[ax] += 1;
    cell_state(g, U, p, q);
    velocity_temperature(ndim, g->gamma, q, wb);
    // grad[m][d] = d w_m / d x_d at the face
    T grad[4][3];
    for (int m = 0; m <= ndim; ++m) grad[m][ax] = (wb[m] - wa[m]) / g->dx[ax];
    for (int t = 0; t < ndim; ++t) {
        if (t == ax) continue;
        T wp[2][4], wm[2][4];
        for (int side = 0; side < 2; ++side) {
            int64_t pp[3] = {c0[0], c0[1], c0[2]};
            pp[ax] += side;
            pp[t] += 1;
            cell_state(g, U, pp, q);
            velocity_temperature(ndim, g->gamma, q, wp[side]);
            pp[t] -= 2;
            cell_state(g, U, pp, q);
            velocity_temperature(ndim, g->gamma, q, wm[side]);
        }
        for (int m = 0; m <= ndim; ++m)
            grad[m][t] = ((wp[0][m] - wm[0][m]) + (wp[1][m] - wm[1][m])) / (4.0 * g->dx[t]);
    }
    T divu = T(0.0);
    for (int d = 0; d < ndim; ++d) divu = divu + grad[d][d];
    // tau_{a,ax} for every a, then Theta_ax
    T tau[3];
    for (int a = 0; a < ndim; ++a) {
        tau[a] = mu * (grad[a][ax] + grad[ax][a]);
        if (a == ax) tau[a] = tau[a] - (2.0 / 3.0) * mu * divu;
    }
    T theta = kc * grad[ndim][ax];
    for (int b = 0; b < ndim; ++b) theta = theta + 0.5 * (wa[b] + wb[b]) * tau[b];
    F[0] = T(0.0);
    for (int a = 0; a < ndim; ++a) F[1 + a] = tau[a];
    F[nv - 1] = theta;
}

// ---------------------------------------------------------------------------
// Curvilinear grids (2D): the cells are the quadrilaterals of a structured
// node array; the fluxes of Eq. (QF) are taken normal to each face, V_n = n.u,
// and scaled by the face's length (its area per unit depth); the residual is
// divided by each cell's own area.

static inline double node(const OrGrid* g, int d, int64_t i, int64_t j) {
    return g->nodes[(int64_t)d * (g->n[0] + 1) * (g->n[1] + 1) + j * (g->n[0] + 1) + i];
}

// Area vector S (length times unit normal, pointing from cell c to c + e_ax)
// of the face between cell c = (i, j) and c + e_ax; the face runs along node
// column i + 1 (ax = 0) or node row j + 1 (ax = 1), so c may be -1 on ax.
static void face_vector(const OrGrid* g, int ax, int64_t i, int64_t j, double S[2]) {
    double ax0, ay0, ax1, ay1;
    if (ax == 0) {
        ax0 = node(g, 0, i + 1, j), ay0 = node(g, 1, i + 1, j);
        ax1 = node(g, 0, i + 1, j + 1), ay1 = node(g, 1, i + 1, j + 1);
        S[0] = ay1 - ay0;
        S[1] = -(ax1 - ax0);
    } else {
        ax0 = node(g, 0, i, j + 1), ay0 = node(g, 1, i, j + 1);
        ax1 = node(g, 0, i + 1, j + 1), ay1 = node(g, 1, i + 1, j + 1);
        S[0] = -(ay1 - ay0);
        S[1] = ax1 - ax0;
    }
}

// Area of quadrilateral cell (i, j): half the cross product of its diagonals.
static double cell_area(const OrGrid* g, int64_t i, int64_t j) {
    const double d1x = node(g, 0, i + 1, j + 1) - node(g, 0, i, j), d1y = node(g, 1, i + 1, j + 1) - node(g, 1, i, j);
    const double d2x = node(g, 0, i, j + 1) - node(g, 0, i + 1, j), d2y = node(g, 1, i, j + 1) - node(g, 1, i + 1, j);
    return 0.5 * (d1x * d2y - d1y * d2x);
}

// Roe flux along a unit normal n (Roe 1981; the normal form of Blazek,
// "Computational Fluid Dynamics: Principles and Applications", sec. 4.3.3):
//   F = (F_n(QL) + F_n(QR))/2 - 1/2 [ |V - c| (dp - rho c dV)/(2c^2) (1, u - c n, H - V c)
//       + |V| ((drho - dp/c^2) (1, u, |u|^2/2) + rho (0, du - dV n, u.du - V dV))
//       + |V + c| (dp + rho c dV)/(2c^2) (1, u + c n, H + V c) ],
// V = n.u, Roe-averaged quantities without subscripts.
template <class T>
static void roe_flux_n(int ndim, const double* n, double gam, const T* QL, const T* QR, T* F) {
    const int ie = ndim + 1;
    T rL = QL[0], rR = QR[0];
    T uL[3], uR[3];
    T qqL = T(0.0), qqR = T(0.0), VL = T(0.0), VR = T(0.0);
    for (int d = 0; d < ndim; ++d) {
        uL[d] = QL[1 + d] / rL;
        uR[d] = QR[1 + d] / rR;
        qqL = qqL + uL[d] * uL[d];
        qqR = qqR + uR[d] * uR[d];
        VL = VL + n[d] * uL[d];
        VR = VR + n[d] * uR[d];
    }
    T pL = (gam - 1.0) * (QL[ie] - 0.5 * rL * qqL);
    T pR = (gam - 1.0) * (QR[ie] - 0.5 * rR * qqR);
    T HL = (QL[ie] + pL) / rL, HR = (QR[ie] + pR) / rR;
    // physical normal fluxes (Eq. QF)
    T FL[5], FR[5];
    FL[0] = rL * VL;
    FR[0] = rR * VR;
    for (int d = 0; d < ndim; ++d) {
        FL[1 + d] = QL[1 + d] * VL + n[d] * pL;
        FR[1 + d] = QR[1 + d] * VR + n[d] * pR;
    }
    FL[ie] = rL * HL * VL;
    FR[ie] = rR * HR * VR;
    // Roe averages
    T sL = std::sqrt(rL), sR = std::sqrt(rR);
    T u[3], qq = T(0.0), V = T(0.0);
    for (int d = 0; d < ndim; ++d) {
        u[d] = (sL * uL[d] + sR * uR[d]) / (sL + sR);
        qq = qq + u[d] * u[d];
        V = V + n[d] * u[d];
    }
    T H = (sL * HL + sR * HR) / (sL + sR);
    T rho = sL * sR;
    T c = std::sqrt((gam - 1.0) * (H - 0.5 * qq));
    T dp = pR - pL, drho = rR - rL, dV = VR - VL;
    T du[3], udu = T(0.0);
    for (int d = 0; d < ndim; ++d) {
        du[d] = uR[d] - uL[d];
        udu = udu + u[d] * du[d];
    }
    T l1 = absr(V - c), l2 = absr(V), l5 = absr(V + c);
    T a1 = (dp - rho * c * dV) / (2.0 * c * c);
    T a5 = (dp + rho * c * dV) / (2.0 * c * c);
    T a2 = drho - dp / (c * c);
    T D[5];
    D[0] = l1 * a1 + l2 * a2 + l5 * a5;
    for (int d = 0; d < ndim; ++d)
        D[1 + d] = l1 * a1 * (u[d] - c * n[d]) + l2 * (a2 * u[d] + rho * (du[d] - dV * n[d])) +
                   l5 * a5 * (u[d] + c * n[d]);
    D[ie] = l1 * a1 * (H - V * c) + l2 * (a2 * 0.5 * qq + rho * (udu - V * dV)) + l5 * a5 * (H + V * c);
    for (int v = 0; v < ndim + 2; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * D[v];
}

// Flux through the face between cell (i, j) and its neighbour along ax on a
// curvilinear 2D grid, times the face length. The four stencil cells along
// the grid line are mapped as on the uniform grid; behind a slip wall the
// mirror cell's velocity is reflected about the wall face's unit normal
// (u - 2 (u.n) n), which on a Cartesian face reverses the normal momentum.
template <class T>
static void face_flux_curv(const OrGrid* g, const T* U, int ax, int64_t i, int64_t j, T* F) {
    const int nv = 4;
    const int64_t ncell = g->n[0] * g->n[1];
    const int64_t n = g->n[ax];
    int64_t idx[2] = {i, j};
    double S[2];
    face_vector(g, ax, i, j, S);
    const double len = std::sqrt(S[0] * S[0] + S[1] * S[1]);
    const double nrm[3] = {S[0] / len, S[1] / len, 0.0};
    T q[4][4];
    for (int m = 0; m < 4; ++m) {
        int64_t c[2] = {idx[0], idx[1]};
        const int64_t pos = idx[ax] - 1 + m;
        c[ax] = bc_index(pos, n, g->bc[ax][0], g->bc[ax][1]);
        const double* fixed = bc_fixed(g, ax, pos);
        if (fixed) {
            for (int v = 0; v < nv; ++v) q[m][v] = T(fixed[v]);
            continue;
        }
        const int64_t off = c[1] * g->n[0] + c[0];
        for (int v = 0; v < nv; ++v) q[m][v] = U[v * ncell + off];
        const bool wall = (pos < 0 && g->bc[ax][0] == 2) || (pos >= n && g->bc[ax][1] == 2);
        if (wall) {
            // unit normal of the wall face of this grid line
            int64_t w[2] = {idx[0], idx[1]};
            w[ax] = pos < 0 ? -1 : n - 1;
            double Sw[2];
            face_vector(g, ax, w[0], w[1], Sw);
            const double lw = std::sqrt(Sw[0] * Sw[0] + Sw[1] * Sw[1]);
            const double nw[2] = {Sw[0] / lw, Sw[1] / lw};
            T mn = q[m][1] * nw[0] + q[m][2] * nw[1];
            q[m][1] = q[m][1] - 2.0 * mn * nw[0];
            q[m][2] = q[m][2] - 2.0 * mn * nw[1];
        }
    }
    T QL[4], QR[4];
    for (int v = 0; v < nv; ++v) muscl(q[0][v], q[1][v], q[2][v], q[3][v], g->limiter, g->kappa, QL[v], QR[v]);
    roe_flux_n(2, nrm, g->gamma, QL, QR, F);
    for (int v = 0; v < nv; ++v) F[v] = F[v] * len;
}

template <class T>
static void residual_curv(const OrGrid* g, const T* U, T* R) {
    const int64_t nx = g->n[0], ny = g->n[1];
    const int64_t ncell = nx * ny;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncell; ++c) {
        int64_t i = c % nx, j = c / nx;
        T acc[4];
        for (int v = 0; v < 4; ++v) acc[v] = T(0.0);
        for (int ax = 0; ax < 2; ++ax) {
            T Fp[4], Fm[4];
            face_flux_curv(g, U, ax, i, j, Fp);
            face_flux_curv(g, U, ax, ax == 0 ? i - 1 : i, ax == 1 ? j - 1 : j, Fm);
            for (int v = 0; v < 4; ++v) acc[v] = acc[v] + (Fp[v] - Fm[v]);
        }
        if (g->source) {
            const double vol = cell_area(g, i, j);
            for (int v = 0; v < 4; ++v) acc[v] = acc[v] - vol * g->source[v * ncell + c];
        }
        for (int v = 0; v < 4; ++v) R[v * ncell + c] = acc[v];
    }
}

// Volume of cell c (flattened index): the uniform box's, or the
// quadrilateral's area on a curvilinear grid.
static inline double cell_vol(const OrGrid* g, int64_t c);

static inline double face_area(const OrGrid* g, int ax) {
    double a = 1.0;
    for (int d = 0; d < g->ndim; ++d)
        if (d != ax) a *= g->dx[d];
    return a;
}

static inline double cell_volume(const OrGrid* g) {
    double v = 1.0;
    for (int d = 0; d < g->ndim; ++d) v *= g->dx[d];
    return v;
}

static inline double cell_vol(const OrGrid* g, int64_t c) {
    if (!g->nodes) return cell_volume(g);
    return cell_area(g, c % g->n[0], c / g->n[0]);
}

// R_c = sum_ax (F_{c+1/2} - F_{c-1/2}) * A_ax - |Omega| S_c   (Eq. residual;
// S_c is the cell average of the source, zero when none is given).
template <class T>
static void residual(const OrGrid* g, const T* U, T* R) {
    if (g->nodes) {
        residual_curv(g, U, R);
        return;
    }
    const int nv = g->ndim + 2;
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t ncell = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncell; ++c) {
        int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        T acc[5];
        for (int v = 0; v < nv; ++v) acc[v] = T(0.0);
        for (int ax = 0; ax < g->ndim; ++ax) {
            int64_t im[3] = {i, j, k};
            im[ax] -= 1;  // the cell on the low side of face c-1/2
            T Fp[5], Fm[5];
            face_flux(g, U, ax, i, j, k, Fp);
            face_flux(g, U, ax, im[0], im[1], im[2], Fm);
            if (g->mu > 0.0) {
                // F_i,n - F_nu,n on each face (Eq. residual)
                T Vp[5], Vm[5];
                visc_face_flux(g, U, ax, i, j, k, Vp);
                visc_face_flux(g, U, ax, im[0], im[1], im[2], Vm);
                for (int v = 0; v < nv; ++v) {
                    Fp[v] = Fp[v] - Vp[v];
                    Fm[v] = Fm[v] - Vm[v];
                }
            }
            double A = face_area(g, ax);
            for (int v = 0; v < nv; ++v) acc[v] = acc[v] + (Fp[v] - Fm[v]) * A;
        }
        if (g->source) {
            const double vol = cell_volume(g);
            for (int v = 0; v < nv; ++v) acc[v] = acc[v] - vol * g->source[v * ncell + c];
        }
        for (int v = 0; v < nv; ++v) R[v * ncell + c] = acc[v];
    }
}

// One SSP-RK3 step (Shu-Osher form) with L(U) = -R(U)/|Omega|:
//   U1 = U + dt L(U);  U2 = 3/4 U + 1/4 (U1 + dt L(U1));  U' = 1/3 U + 2/3 (U2 + dt L(U2)).
template <class T>
static void rk3_step(const OrGrid* g, T* U, double dt) {
    const int nv = g->ndim + 2;
    const int64_t ncell = g->n[0] * g->n[1] * g->n[2];
    const int64_t N = nv * ncell;
    std::vector<double> vol(ncell);
    for (int64_t c = 0; c < ncell; ++c) vol[c] = cell_vol(g, c);
    std::vector<T> R(N), U1(N), U2(N);
    residual(g, U, R.data());
    for (int64_t e = 0; e < N; ++e) U1[e] = U[e] + dt * (-R[e] / vol[e % ncell]);
    residual(g, U1.data(), R.data());
    for (int64_t e = 0; e < N; ++e) U2[e] = 0.75 * U[e] + 0.25 * (U1[e] + dt * (-R[e] / vol[e % ncell]));
    residual(g, U2.data(), R.data());
    for (int64_t e = 0; e < N; ++e)
        U[e] = (1.0 / 3.0) * U[e] + (2.0 / 3.0) * (U2[e] + dt * (-R[e] / vol[e % ncell]));
}

extern "C" {

// Threads of the OpenMP loops (for timing the oracle on one core and on all).
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_max_threads() { return omp_get_max_threads(); }

double or_psi_minmod(double r) { return psi_minmod(r); }

double or_psi_vanleer(double r) { return psi_vanleer(r); }

double or_limited(double num, double den, int limiter) { return limited(num, den, limiter); }

void or_muscl(double qm1, double q0, double qp1, double qp2, int limiter, double kappa,
              double* qL, double* qR) {
    muscl(qm1, q0, qp1, qp2, limiter, kappa, *qL, *qR);
}

void or_phys_flux(int ndim, int ax, double gam, const double* Q, double* F) {
    phys_flux(ndim, ax, gam, Q, F);
}

void or_roe_flux(int ndim, int ax, double gam, const double* QL, const double* QR, double* F) {
    roe_flux(ndim, ax, gam, QL, QR, F);
}

void or_residual(const OrGrid* g, const double* U, double* R) { residual(g, U, R); }

// Directional derivative of R along V by the complex step: R(U + i h V) = R + i h dR.
void or_residual_cs(const OrGrid* g, const double* U, const double* V, double h, double* R, double* dR) {
    const int64_t N = (int64_t)(g->ndim + 2) * g->n[0] * g->n[1] * g->n[2];
    std::vector<cplx> Uc(N), Rc(N);
    for (int64_t e = 0; e < N; ++e) Uc[e] = cplx(U[e], h * V[e]);
    residual(g, Uc.data(), Rc.data());
    for (int64_t e = 0; e < N; ++e) {
        R[e] = Rc[e].real();
        dR[e] = Rc[e].imag() / h;
    }
}

// max over cells of sum_d (|u_d| + c)/dx_d, with flags for NaN, rho <= 0, p <= 0.
double or_max_wavespeed(const OrGrid* g, const double* U, uint32_t* flags) {
    const int ndim = g->ndim, ie = ndim + 1;
    const int64_t ncell = g->n[0] * g->n[1] * g->n[2];
    double lmax = 0.0;
    uint32_t fl = 0;
#pragma omp parallel for reduction(max : lmax) reduction(| : fl) schedule(static)
    for (int64_t c = 0; c < ncell; ++c) {
        double rho = U[c];
        double u[3], qq = 0.0;
        for (int d = 0; d < ndim; ++d) {
            u[d] = U[(1 + d) * ncell + c] / rho;
            qq += u[d] * u[d];
        }
        double p = (g->gamma - 1.0) * (U[ie * ncell + c] - 0.5 * rho * qq);
        double cs = std::sqrt(g->gamma * p / rho);
        double lam = 0.0;
        if (g->nodes) {
            // curvilinear: sum over the grid directions of (|u.S| + c |S|) / area,
            // S the mean of the cell's two face area vectors on that direction
            const int64_t i = c % g->n[0], j = c / g->n[0];
            const double area = cell_area(g, i, j);
            for (int ax = 0; ax < 2; ++ax) {
                double Sa[2], Sb[2];
                face_vector(g, ax, ax == 0 ? i - 1 : i, ax == 1 ? j - 1 : j, Sa);
                face_vector(g, ax, i, j, Sb);
                const double Sx = 0.5 * (Sa[0] + Sb[0]), Sy = 0.5 * (Sa[1] + Sb[1]);
                lam += (std::fabs(u[0] * Sx + u[1] * Sy) + cs * std::sqrt(Sx * Sx + Sy * Sy)) / area;
            }
        } else {
            for (int d = 0; d < ndim; ++d) lam += (std::fabs(u[d]) + cs) / g->dx[d];
        }
        if (g->mu > 0.0) {
            // explicit diffusion limit: 2 nu_eff sum_d 1/dx_d^2 with the larger
            // of the momentum (4/3 mu / rho) and heat (gamma mu / (Pr rho))
            // diffusivities
            const double nu = (g->mu / rho) * std::fmax(4.0 / 3.0, g->gamma / g->prandtl);
            double s2 = 0.0;
            for (int d = 0; d < ndim; ++d) s2 += 1.0 / (g->dx[d] * g->dx[d]);
            lam += 2.0 * nu * s2;
        }
        if (std::isnan(lam) || std::isnan(rho) || std::isnan(p)) fl |= OR_FLAG_NAN;
        if (!(rho > 0.0)) fl |= OR_FLAG_RHO;
        if (!(p > 0.0)) fl |= OR_FLAG_P;
        if (lam > lmax) lmax = lam;
    }
    if (flags) *flags |= fl;
    return lmax;
}

void or_visc_face_flux(const OrGrid* g, const double* U, int ax, int64_t i, int64_t j, int64_t k, double* F) {
    visc_face_flux(g, U, ax, i, j, k, F);
}

double or_dt(const OrGrid* g, const double* U, uint32_t* flags) {
    return g->cfl / or_max_wavespeed(g, U, flags);
}

void or_rk3_step(const OrGrid* g, double* U, double dt) { rk3_step(g, U, dt); }

// mu = (dR/dU)^T w. Each face of each axis contributes F*A to the residual of
// its low-side cell and -F*A to its high-side cell (when those are interior),
// so its flux adjoint is A (w_low - w_high). The face flux depends on its four
// stencil cells (ghosts mapped to the interior cell they copy); its Jacobian
// columns are taken one input at a time by the complex step, which is exact to
// roundoff, and the transposed products are added to those cells.
void or_residual_vjp(const OrGrid* g, const double* U, const double* w, double* mu) {
    const int nv = g->ndim + 2;
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t ncell = nx * ny * nz;
    const double h = 1e-30;
    for (int64_t e = 0; e < nv * ncell; ++e) mu[e] = 0.0;
    std::vector<cplx> Uc((size_t)nv * ncell);
    for (int64_t e = 0; e < nv * ncell; ++e) Uc[e] = cplx(U[e], 0.0);
    for (int ax = 0; ax < g->ndim; ++ax) {
        const double A = face_area(g, ax);
        const int64_t n = g->n[ax];
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t idx[3] = {i, j, k};
                    // faces with low-side cell index -1 .. n-1 along ax; visit each
                    // once, through the cell on its high side (index 0 .. n) or, for
                    // the last face, through the last cell
                    const int64_t a = idx[ax];
                    int64_t lows[2];
                    int nl = 0;
                    lows[nl++] = a - 1;            // face between a-1 and a
                    if (a == n - 1) lows[nl++] = a; // face between n-1 and n
                    for (int q = 0; q < nl; ++q) {
                        const int64_t lo = lows[q];
                        int64_t cc[3] = {i, j, k};
                        cc[ax] = lo;  // face_flux takes the low-side cell
                        double Fb[5];
                        for (int v = 0; v < nv; ++v) {
                            double wl = 0.0, wh = 0.0;
                            if (lo >= 0) {
                                int64_t c2[3] = {i, j, k};
                                c2[ax] = lo;
                                wl = w[v * ncell + cell_offset(g, c2[0], c2[1], c2[2])];
                            }
                            if (lo + 1 <= n - 1) {
                                int64_t c2[3] = {i, j, k};
                                c2[ax] = lo + 1;
                                wh = w[v * ncell + cell_offset(g, c2[0], c2[1], c2[2])];
                            }
                            Fb[v] = A * (wl - wh);
                        }
                        // stencil cells lo-1 .. lo+2, mapped to the interior
                        int64_t off[4];
                        for (int m = 0; m < 4; ++m) {
                            int64_t c2[3] = {i, j, k};
                            c2[ax] = bc_index(lo - 1 + m, n, g->bc[ax][0], g->bc[ax][1]);
                            off[m] = cell_offset(g, c2[0], c2[1], c2[2]);
                        }
                        // slot value = sign * cell value (the wall's mirror reverses the
                        // normal momentum), so the cell's derivative is sign * the slot's
                        auto sgn = [&](int m, int v) {
                            return bc_sign(lo - 1 + m, n, g->bc[ax][0], g->bc[ax][1], v, ax);
                        };
                        // perturb one stencil entry (slot m, variable v) at a time
                        for (int m = 0; m < 4; ++m)
                            for (int v = 0; v < nv; ++v) {
                                // a ghost slot that maps to the same cell as another slot is
                                // still its own input of the face flux; perturb the slot, not the cell
                                cplx Q[4][5];
                                for (int mm = 0; mm < 4; ++mm) {
                                    const double* fixed = bc_fixed(g, ax, lo - 1 + mm);
                                    for (int vv = 0; vv < nv; ++vv)
                                        Q[mm][vv] = fixed ? cplx(fixed[vv], 0.0) : Uc[vv * ncell + off[mm]] * sgn(mm, vv);
                                }
                                // a slot behind an inflow face depends on no cell
                                if (bc_fixed(g, ax, lo - 1 + m)) continue;
                                Q[m][v] += cplx(0.0, h);
                                cplx QL[5], QR[5], F[5];
                                for (int vv = 0; vv < nv; ++vv)
                                    muscl(Q[0][vv], Q[1][vv], Q[2][vv], Q[3][vv], g->limiter, g->kappa, QL[vv], QR[vv]);
                                roe_flux(g->ndim, ax, g->gamma, QL, QR, F);
                                double dot = 0.0;
                                for (int vv = 0; vv < nv; ++vv) dot += F[vv].imag() / h * Fb[vv];
                                mu[v * ncell + off[m]] += sgn(m, v) * dot;
                            }
                    }
                }
    }
}

// Reverse of one SSP-RK3 step at frozen dt: lam holds dJ/dU^{n+1} on entry and
// dJ/dU^n on return. With L = -R/|Omega| and the stages
//   U1 = U + dt L(U), U2 = 3/4 U + 1/4 (U1 + dt L(U1)), U' = 1/3 U + 2/3 (U2 + dt L(U2)),
// the chain rule gives
//   l2 = 2/3 lam + 2/3 dt J(U2)^T lam,  l1 = 1/4 l2 + 1/4 dt J(U1)^T l2,
//   dJ/dU = 1/3 lam + 3/4 l2 + l1 + dt J(U)^T l1,   J = dL/dU = -(dR/dU)/|Omega|.
void or_rk3_step_vjp(const OrGrid* g, const double* U, double dt, double* lam) {
    const int nv = g->ndim + 2;
    const int64_t N = (int64_t)nv * g->n[0] * g->n[1] * g->n[2];
    const double vol = cell_volume(g);
    std::vector<double> R(N), U1(N), U2(N), mu(N), l2(N), l1(N);
    residual(g, U, R.data());
    for (int64_t e = 0; e < N; ++e) U1[e] = U[e] + dt * (-R[e] / vol);
    residual(g, U1.data(), R.data());
    for (int64_t e = 0; e < N; ++e) U2[e] = 0.75 * U[e] + 0.25 * (U1[e] + dt * (-R[e] / vol));
    or_residual_vjp(g, U2.data(), lam, mu.data());
    for (int64_t e = 0; e < N; ++e) l2[e] = (2.0 / 3.0) * lam[e] + (2.0 / 3.0) * dt * (-mu[e] / vol);
    or_residual_vjp(g, U1.data(), l2.data(), mu.data());
    for (int64_t e = 0; e < N; ++e) l1[e] = 0.25 * l2[e] + 0.25 * dt * (-mu[e] / vol);
    or_residual_vjp(g, U, l1.data(), mu.data());
    for (int64_t e = 0; e < N; ++e)
        lam[e] = (1.0 / 3.0) * lam[e] + 0.75 * l2[e] + l1[e] + dt * (-mu[e] / vol);
}

// Complex-step directional derivative of one RK3 step (dt frozen) along V.
void or_rk3_step_cs(const OrGrid* g, const double* U, const double* V, double h, double dt,
                    double* Unew, double* dUnew) {
    const int64_t N = (int64_t)(g->ndim + 2) * g->n[0] * g->n[1] * g->n[2];
    std::vector<cplx> Uc(N);
    for (int64_t e = 0; e < N; ++e) Uc[e] = cplx(U[e], h * V[e]);
    rk3_step(g, Uc.data(), dt);
    for (int64_t e = 0; e < N; ++e) {
        Unew[e] = Uc[e].real();
        dUnew[e] = Uc[e].imag() / h;
    }
}

// nsteps SSP-RK3 steps. dt per step is dt_in[s] if dt_in is given, else
// CFL / max wave speed of the state at the start of the step.
void or_run(const OrGrid* g, double* U, int32_t nsteps, const double* dt_in, double* dt_out,
            uint32_t* flags) {
    for (int32_t s = 0; s < nsteps; ++s) {
        double dt = dt_in ? dt_in[s] : or_dt(g, U, flags);
        if (dt_out) dt_out[s] = dt;
        rk3_step(g, U, dt);
    }
}

}  // extern "C"
