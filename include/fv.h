/*
 * fv.h - C ABI of libfv.so, an explicit finite-volume solver for the
 * compressible Euler equations on uniform Cartesian grids, FP64, for AMD
 * Instinct MI355X (gfx950).
 *
 * The method is the cell-centred finite-volume scheme of the paper's
 * Sec. "The CFD Code Base": conserved variables and inviscid normal flux of
 * Eq. (QF), the semi-discrete cell form of Eq. (spatial_residual), the face-sum
 * residual of Eq. (residual) with a zero source term, and face states by MUSCL
 * extrapolation, Eq. (flux), with epsilon = 1, kappa = -1 and the minmod
 * limiter. Face fluxes are Roe's approximate Riemann solver; the explicit
 * Runge-Kutta march is the three-stage SSP scheme of Shu and Osher; the time
 * step is the CFL limit dt = cfl / max_cells sum_d (|u_d| + c) / dx_d.
 *
 * The launch parameters of the seven kernels that make up a step are exposed
 * as 14 integers, two per kernel, mirroring the seven gang/vector pairs of the
 * paper's Table "Tuning Parameters" (Sec. "Tuning Parameters").
 *
 * Conventions shared by every entry point:
 *  - Memory: every pointer argument of type double* or void* workspace is a
 *    DEVICE pointer, owned by the caller, which must keep it valid until the
 *    work enqueued on the context's stream has completed. The library never
 *    allocates device memory: scratch comes from the caller's workspace (or,
 *    for fv_mlp_sweep_static, from a static device array of the library).
 *  - State layout ("ghosted SoA"): FP64, variables outermost, x fastest:
 *      U[v * s_v + (k + g3) * s_z + (j + 2) * s_y + (i + 2)]
 *    for interior cell (i, j, k), v in (rho, rho u, rho v, [rho w], E),
 *    g3 = 2 in 3D and 0 in 2D. Two ghost layers per face along each active
 *    axis. The strides come from fv_query. Ghost cells are overwritten by the
 *    library; only interior cells are read as input.
 *  - Residual layout ("dense interior"): R[v * ncell + (k * ny + j) * nx + i].
 *  - Asynchrony: calls enqueue work on the context's HIP stream and return
 *    without waiting, except fv_status, which synchronises that stream.
 *  - Errors: the return value is FV_OK or a negative FV_E* code for argument,
 *    workspace and launch errors; no state is changed when a call returns
 *    FV_EINVAL. Non-physical states (NaN, rho <= 0, p <= 0) are recorded in a
 *    device status word read by fv_status. fv_last_error gives a message.
 *  - Threading: a context is used from one host thread at a time.
 */
#ifndef FV_H
#define FV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FV_OK = 0,
    FV_EINVAL = -1,      /* bad argument: no state changed */
    FV_EDEVICE = -2,     /* a HIP call or kernel launch failed */
    FV_ENONPHYS = -3,    /* the status word holds a non-physical flag */
    FV_ENOTSUP = -4,     /* configuration not supported */
    FV_EWORKSPACE = -5   /* workspace missing, too small or misaligned */
};

/* Boundary kinds per axis side. FV_BC_WALL is an inviscid slip wall (the
 * reading for the solid boundaries of the supersonic inlet of Sec. "A Test
 * Case"): the ghost cells
 * are the mirror image of the interior across the face with the velocity
 * normal to the wall reversed, so no mass or energy crosses it. It needs at
 * least 2 cells on its axis. It runs on the split path (fv_residual,
 * fv_step, fv_adjoint_step) and on the fused path (a boundary variant of the
 * stage kernels maps ghost rows, columns and planes to the mirror cells),
 * and in batches. */
/* FV_BC_INFLOW holds the given conserved state fv_grid_desc.bc_state[axis]
 * [side] in the ghost cells (supersonic inflow: every characteristic enters
 * through the face; the supersonic inlet of Sec. "A Test Case" takes in its
 * free stream), with the same path support as the wall. Its state must have
 * a positive density and pressure. FV_BC_TRANSMISSIVE serves as the
 * supersonic outflow. */
enum { FV_BC_PERIODIC = 0, FV_BC_TRANSMISSIVE = 1, FV_BC_WALL = 2, FV_BC_INFLOW = 3 };

/* Status-word bits (set by the time-step reduction over the state). */
enum { FV_FLAG_NAN = 1u, FV_FLAG_RHO = 2u, FV_FLAG_P = 4u, FV_FLAG_DT = 8u };

/* Launch sites: the kernels of one step. Slot 2*s holds the first and slot
 * 2*s+1 the second parameter of site s. */
enum {
    FV_SITE_FLUX_X = 0,   /* MUSCL + Roe flux on x faces (paper: xi limiter/flux) */
    FV_SITE_FLUX_Y = 1,   /* the same on y faces (paper: eta limiter/flux)        */
    FV_SITE_FLUX_Z = 2,   /* the same on z faces (3D only; inert in 2D)           */
    FV_SITE_RESIDUAL = 3, /* face-flux differences times areas (paper: RHS)       */
    FV_SITE_UPDATE = 4,   /* Runge-Kutta stage update (paper: update solution)    */
    FV_SITE_BC = 5,       /* ghost-layer fill                                     */
    FV_SITE_CFL = 6,      /* wave-speed max-reduction for dt                      */
    FV_NSITES = 7
};

/* Scheme of fv_grid_desc.scheme: the MUSCL face states of Eq. (flux) with
 * epsilon = 1. With a symmetric limiter (minmod, van Leer) the kappa terms
 * collapse (Psi+ and Psi- give the same limited difference) and every kappa
 * gives Q^L = Q_k + Psi dQ / 2. With Psi = 1, kappa selects the member of
 * the family. */
enum {
    FV_SCHEME_MINMOD = 0,      /* minmod limiter (the default)                          */
    FV_SCHEME_UNLIMITED = 1,   /* Psi = 1, kappa = -1: fully upwind                     */
    FV_SCHEME_FROMM = 2,       /* Psi = 1, kappa = 0: Fromm's upwind-biased scheme      */
    FV_SCHEME_THIRD = 3,       /* Psi = 1, kappa = 1/3: third-order upwind-biased       */
    FV_SCHEME_CENTRAL = 4,     /* Psi = 1, kappa = 1: central                            */
    FV_SCHEME_VANLEER = 5,     /* van Leer's limiter, Psi(r) = (r + |r|)/(1 + |r|) (symmetric,
                                  so kappa drops out as with minmod)                      */
    FV_SCHEME_QUICK = 6        /* Psi = 1, kappa = 1/2: Leonard's QUICK (quadratic upstream
                                  interpolation, exact for quadratic point values)        */
};

/* Grid description. ndim is 2 or 3; n[2] must be 1 in 2D. The box is
 * [lo, hi] per axis with n cells each. bc[d][0] / bc[d][1] is the low / high
 * face kind of axis d; periodic must be set on both faces of an axis. */
typedef struct fv_grid_desc {
    int32_t ndim;
    int32_t scheme;     /* FV_SCHEME_* */
    int64_t n[3];
    double lo[3];
    double hi[3];
    int32_t bc[3][2];
    double gamma;       /* ratio of specific heats, > 1 */
    double cfl;         /* CFL number, > 0 */
    double bc_state[3][2][5];  /* conserved ghost state of FV_BC_INFLOW faces (rho, rho u, rho v, [rho w], E) */
    double mu;          /* dynamic viscosity, >= 0: 0 gives the Euler equations; > 0 adds the
                           viscous flux of Eq. (QF) (Navier-Stokes), see below */
    double prandtl;     /* Prandtl number of the heat flux, > 0 when mu > 0 */
    const double* nodes;  /* curvilinear 2D grid (see below): DEVICE pointer to the node
                             coordinates, or NULL for the uniform box [lo, hi] */
} fv_grid_desc;

/* Curvilinear grids (nodes != NULL, 2D only): the structured cells are the
 * quadrilaterals of a node array of (nx + 1) x (ny + 1) points,
 * nodes[d * (nx + 1) * (ny + 1) + j * (nx + 1) + i] for d = 0 (x), 1 (y),
 * i increasing along the first grid direction and j along the second (a
 * right-handed, non-degenerate grid: every cell's area is positive). The
 * inviscid flux of Eq. (QF) is taken along each face's unit normal,
 * V_n = n . u, times the face's length, and the residual is divided by each
 * cell's area; MUSCL works along the grid lines as on the box; a slip wall's
 * mirror cell has its velocity reflected about the wall face's normal. The
 * metric streams (unit normal and length per face, area per cell) are
 * computed on the device by fv_create into the context's workspace; the
 * node array is read there only (the caller may free it once the stream has
 * passed fv_create's work). lo and hi are not used. Curvilinear grids run on
 * the split path (fv_residual, fv_step, fv_residual_norm) and on the fused
 * path (a curvilinear variant of the 2D stage kernels that reads the metric
 * streams, every boundary kind); the viscous flux (mu > 0) is FV_EINVAL with
 * them, fv_adjoint_step returns FV_ENOTSUP, and batches refuse them. */

/* Viscous flux (mu > 0): the residual of Eq. (residual) sums F_i,n - F_nu,n
 * over the faces, with F_nu,n = (0, tau . n, Theta . n) of Eq. (QF): Stokes
 * stresses tau_ab = mu (du_a/dx_b + du_b/dx_a) - 2/3 mu delta_ab div(u) and
 * Theta = u . tau + k grad T, T = p / rho (unit gas constant),
 * k = mu gamma / ((gamma - 1) prandtl). Face gradients are second order: the
 * difference across the face for the normal derivative, the mean of the two
 * cells' central differences for tangential ones; edge and corner neighbours
 * outside the grid go through the boundary maps of each axis. The time step
 * adds the explicit diffusion limit: the wave-speed sum of each cell gains
 * 2 (mu / rho) max(4/3, gamma / prandtl) sum_d 1 / dx_d^2. Viscous grids run
 * on the split path (fv_residual, fv_step, fv_residual_norm) and, in 2D, on
 * the fused path (a viscous variant of the stage kernels), also in batches;
 * fv_set_path (FV_PATH_FUSED) on 3D viscous grids and fv_adjoint_step
 * return FV_ENOTSUP. */

/* Launch parameters, two per site (FV_SITE_* order).
 *  Stencil sites (flux x/y/z): p[2s] = block width along x, a power of two in
 *    [1, 1024]; p[2s+1] = threads per block, a power of two in [64, 1024],
 *    >= p[2s]. The block height is p[2s+1] / p[2s].
 *  One-dimensional sites (residual, update, bc, cfl): p[2s] = number of blocks
 *    ("gang"), 0 for one thread per element or a power of two in [1, 65536]
 *    for a grid-stride loop; p[2s+1] = threads per block, a power of two in
 *    [64, 1024].
 * Every valid vector yields bitwise-identical results. */
typedef struct fv_launch {
    int32_t p[14];
} fv_launch;

typedef struct fv_ctx fv_ctx;   /* opaque, library-owned host object */

/* Writes the defaults: stencil sites (64, 256), one-dimensional sites (0, 256). */
void fv_default_launch(fv_launch* out);

/* Validates g and reports the ghosted state strides (elements):
 * strides_out = {s_x = 1, s_y, s_z, s_v}, the state size is nvar * s_v
 * doubles, and *workspace_bytes the scratch a context needs. Either output
 * may be NULL. Returns FV_EINVAL for an invalid description. */
int fv_query(const fv_grid_desc* g, int64_t strides_out[4], size_t* workspace_bytes);

/* Creates a context for grid g on the current HIP device. workspace is a
 * device buffer of at least the queried size, 256-byte aligned, owned by the
 * caller and used exclusively by this context until fv_destroy. stream is a
 * hipStream_t (NULL = the default stream). The launch table starts at the
 * defaults and the status word at 0. On grids the fused path takes, it also
 * uploads the fused path's per-stage tables at the library's choice (used
 * by fv_adjoint_step's forward recomputation whichever path is selected) and
 * synchronises the stream once to do so: create contexts outside stream
 * capture. */
int fv_create(const fv_grid_desc* g, void* workspace, size_t workspace_bytes, void* stream,
              fv_ctx** out);

/* Releases the host object; does not touch the caller's device memory. */
int fv_destroy(fv_ctx* ctx);

/* Rebinds the context to another HIP stream (NULL = the default stream). */
int fv_set_stream(fv_ctx* ctx, void* stream);

/* Spatial residual of Eq. (residual): R = sum over the 2*ndim faces of the
 * Roe flux of the MUSCL face states times the face area, minus |Omega| S
 * when a source is set (fv_set_source; S = 0 otherwise). Fills the ghost
 * layers of U (the interior is not changed) and writes R in the dense
 * interior layout (nvar * ncell doubles). */
int fv_residual(fv_ctx* ctx, double* U, double* R);

/* Per-variable L2 norm of the residual of U, the convergence monitor behind
 * the relative residual history of Sec. "A Test Case" (Fig. inlet-resid):
 * norms[v] = sqrt(sum over cells of R_v^2 / ncell), R as fv_residual
 * computes it (source included). norms is a device pointer to nvar doubles;
 * the residual itself goes to the context's scratch. Fills the ghost layers
 * of U. The sums run in a fixed order: the same U gives the same bits. */
int fv_residual_norm(fv_ctx* ctx, double* U, double* norms);

/* Sets the cell-averaged source term S_h of Eq. (residual) (a body force, a
 * manufactured solution's source): S is a device pointer to nvar * ncell
 * doubles in the dense interior layout of fv_residual's R (variable, then
 * cell with x fastest), or NULL to remove it. The caller keeps S allocated
 * and unchanged while it is set: fv_residual, fv_step (both paths) and
 * fv_adjoint_step read it on the device. The source does not depend on U, so
 * the adjoint's transposed Jacobian is unchanged; its recomputed stage states
 * include it. The fused stage kernels (2D and 3D) read S with the state, in
 * kernel instantiations of their own, so the source-free kernels are
 * unchanged. Only a null context is rejected. */
int fv_set_source(fv_ctx* ctx, const double* S);

/* Advances U (ghosted layout, in place) by nsteps SSP-RK3 steps:
 *   U1 = U + dt L(U), U2 = 3/4 U + 1/4 (U1 + dt L(U1)),
 *   U <- 1/3 U + 2/3 (U2 + dt L(U2)),  L = -R / |Omega|,
 * ghosts refilled before every stage. dt of step s is dt_in[s] when dt_in
 * (device, nsteps doubles) is non-NULL, else cfl / max wave speed of U at the
 * start of the step. dt_out (device, nsteps doubles, may be NULL) receives the
 * dt used by each step. The status word collects the flags of every step. */
int fv_step(fv_ctx* ctx, double* U, int32_t nsteps, const double* dt_in, double* dt_out);

/* Reverse (adjoint) of one SSP-RK3 step with the step size frozen at *dt
 * (device scalar): on entry lam (dense interior layout) holds dJ/dU^{n+1};
 * on return it holds dJ/dU^n, where U^{n+1} = step(U_n, dt). U_n (ghosted
 * layout) is the state at the start of the step; its interior is not changed
 * (its ghosts may be). The stage states U1, U2 are recomputed internally
 * (the fused stage kernels, two launches; the split kernels on grids the
 * fused path refuses). Each reverse stage is one kernel: mu = (dR/dU)^T w of
 * Eq. (residual) by the reverse of the Roe flux and the MUSCL states of every
 * face, gathered per cell (the transposed ghost rules included) and combined
 * with the stage's recurrence, with no face array in the workspace. Viscous
 * and curvilinear grids return FV_ENOTSUP. */
int fv_adjoint_step(fv_ctx* ctx, double* U_n, const double* dt, double* lam);

/* Sets / reads the 14 launch parameters. An invalid vector returns FV_EINVAL
 * and leaves the previous one in place. */
int fv_set_launch(fv_ctx* ctx, const fv_launch* launch);
int fv_get_launch(const fv_ctx* ctx, fv_launch* out);

/* Synchronises the context's stream and reads the status word (FV_FLAG_*).
 * Returns FV_ENONPHYS when any flag is set, FV_OK otherwise. */
int fv_status(fv_ctx* ctx, uint32_t* flags);

/* Enqueues a reset of the status word to 0. */
int fv_clear_status(fv_ctx* ctx);

/* Step paths. FV_PATH_SPLIT runs the seven tunable kernels (the launch
 * table applies). FV_PATH_FUSED runs one kernel per Runge-Kutta stage that
 * does the ghost mapping, the fluxes of every axis, the residual and the
 * stage update, and the last stage also the CFL max of the new state; the
 * state then moves through HBM 8 times per step instead of ~33 (2D) or ~42
 * (3D). `seg` is the segment height of a work item (rows in 2D, planes in
 * 3D), a multiple of 4 in [4, 1024], or 0 to let the library choose it from
 * the grid and the number of wavefronts the device holds at once (in 2D a work
 * item is a 60-column strip of a segment, one wavefront; in 3D a 32 x 7-cell
 * tile of the plane over a segment of planes, one workgroup of four
 * wavefronts); `waves` is the
 * number of wavefronts launched (0 = one per work item, else a grid-stride
 * loop over the items). Every segment height and wave count gives bitwise the
 * same result. Both paths compute the same cell arithmetic; fv_residual always
 * uses the split kernels, and fv_adjoint_step recomputes its stage states with
 * the fused stage kernels of the current table (the library's choice until a
 * table is set) on every grid the fused path takes. Returns FV_ENOTSUP for states
 * of 4 GiB or more (the fused kernels address a grid through 32-bit buffer
 * offsets) and for 3D viscous grids, and FV_EINVAL for other seg values. The
 * fused path takes every boundary kind and curvilinear 2D grids. */
enum { FV_PATH_SPLIT = 0, FV_PATH_FUSED = 1 };
int fv_set_path(fv_ctx* ctx, int path, int32_t seg, int32_t waves);

/* Launch table of the fused path, one entry per Runge-Kutta stage: seg[s]
 * is the segment height of stage s's work items (0 = the library's choice, or
 * a multiple of 4 in [4, 1024]) and waves[s] the wavefronts its launch holds
 * (0 = one per work item, else a grid-stride loop; in 3D rounded up to whole
 * workgroups of four). fv_set_path(FV_PATH_FUSED, seg, waves) gives all three
 * stages the same pair. Every table gives bitwise the same result: the table
 * changes only how the work is cut, the launch surface the autotuner searches
 * for the fused path. fv_set_fused_launch needs the fused path selected
 * (FV_EINVAL otherwise, and for an invalid entry, leaving the table as it
 * was); fv_get_fused_launch reads the table in use (with the library's
 * choices filled in). */
typedef struct fv_fused_launch {
    int32_t seg[3];
    int32_t waves[3];
} fv_fused_launch;
int fv_set_fused_launch(fv_ctx* ctx, const fv_fused_launch* launch);
int fv_get_fused_launch(const fv_ctx* ctx, fv_fused_launch* out);

/* Wavefronts of the fused stage kernels of ctx's dimension that the current
 * device holds at once (from its compute-unit count and the kernels'
 * occupancy), the scale of fv_fused_launch.waves. */
int fv_fused_slots(const fv_ctx* ctx, int32_t* waves);

/* Reads back the path, the segment height in use by the first stage (the
 * library's choice when fv_set_path was given 0; 0 on the split path) and its
 * wave count. Outputs may be NULL. */
int fv_get_path(const fv_ctx* ctx, int32_t* path, int32_t* seg, int32_t* waves);

/* Per-site kernel timing, a diagnostic for profiling and the autotuner's
 * measurements. When enabled, every kernel launch of fv_step / fv_residual /
 * fv_adjoint_step is bracketed by two HIP events on the context's stream and
 * each call waits for its last event, so enabling it serialises the host with
 * the stream; kernel durations themselves are unaffected. fv_get_timing
 * writes, per timer (FV_SITE_* and FV_TIMER_FUSED for the fused stages), the
 * accumulated milliseconds and number of launches since the last read, then
 * resets them. Either output may be NULL. */
enum { FV_TIMER_FUSED = 7, FV_NTIMERS = 8 };
int fv_set_timing(fv_ctx* ctx, int enable);
int fv_get_timing(fv_ctx* ctx, double ms_out[8], int64_t launches_out[8]);

/* Message of the last failing call on ctx (or of fv_query / fv_create when
 * ctx is NULL). Never NULL. */
const char* fv_last_error(const fv_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batches of uneven 2D grids advanced together by the fused stage kernels.
 *
 * Grid g of a batch is stored dense, variables outermost:
 *   U[offsets[g] + v * nx_g * ny_g + j * nx_g + i],
 * grids back to back (offsets from fv_batch_query). Every grid has its own
 * CFL dt. A step is three fused stage launches that cover all work items of
 * all grids (a work item is a 60-column x seg-row piece of one grid, one
 * wavefront each); the three launches are captured once in a HIP graph and
 * replayed per step on the caller's stream.
 * ------------------------------------------------------------------------ */
typedef struct fv_batch fv_batch;

enum { FV_ORDER_GIVEN = 0, FV_ORDER_LARGEST_FIRST = 1 };

/* Validates the grids (2D each, each state below 4 GiB, i.e. under 2^27
 * cells; every boundary kind and the viscous flux are taken, curvilinear
 * grids are refused) and reports the element offsets of every grid
 * (offsets[0..ngrids], host array, may be NULL) and the workspace size. A
 * batch runs one variant of the stage kernels for all its grids: the viscous
 * one if any grid is viscous, else the boundary one if any grid has a slip
 * wall or an inflow face, else the plain one. */
int fv_batch_query(int32_t ngrids, const fv_grid_desc* grids, int64_t* offsets, size_t* workspace_bytes);

/* Creates a batch. seg: segment height of every grid, a multiple of 4 in
 * [4, 1024], or 0 for the library's choice over all grids of the batch
 * (fv_batch_set_schedule sets one per grid); waves: wavefronts per stage
 * launch (0 = one per work item, else a grid-stride loop); order: FV_ORDER_*
 * of the grids in the work list. The workspace (queried size, 256-byte
 * aligned) is owned by the caller. */
int fv_batch_create(int32_t ngrids, const fv_grid_desc* grids, int32_t seg, int32_t waves, int32_t order,
                    void* workspace, size_t workspace_bytes, void* stream, fv_batch** out);

/* Advances every grid of the batch state U (device) by nsteps steps, each
 * grid with its own CFL dt. The steps are replayed from HIP graphs captured
 * at the first call for U (one of 8 steps, one of 1 step for the rest). */
int fv_batch_step(fv_batch* b, double* U, int32_t nsteps);

/* Device-clock record of each step: when history (device, max_steps *
 * ngrids * 6 uint64) is non-NULL, step n of the following fv_batch_step calls
 * writes, per grid and stage, the earliest work-item start and the latest
 * work-item end (wall_clock64 ticks) to history[((n * ngrids + g) * 3 + stage) * 2 + {0,1}]
 * for n < max_steps. NULL turns recording off. *ticks_per_us receives the
 * clock rate. */
int fv_batch_set_timing(fv_batch* b, uint64_t* history, int32_t max_steps, double* ticks_per_us);

/* Copies the dt of the last step of every grid to dt (device, ngrids doubles). */
int fv_batch_dt(fv_batch* b, double* dt);

/* Synchronises the stream and reads the batch status word (FV_FLAG_*). */
int fv_batch_status(fv_batch* b, uint32_t* flags);

/* Sets the schedule: the segment height of every grid (segs[g] for the
 * caller's grid g, each a multiple of 4 in [4, 1024]; NULL keeps the current
 * ones) and the work-list order (FV_ORDER_*). Results are bitwise the same
 * under every schedule; the step's graph is rebuilt on the next
 * fv_batch_step. Synchronises the batch's stream. */
int fv_batch_set_schedule(fv_batch* b, const int32_t* segs, int32_t order);

/* The schedule in use: segment height per grid (segs, ngrids entries), the
 * work-list order and the number of work items of one stage launch. Outputs
 * may be NULL. */
int fv_batch_info(const fv_batch* b, int32_t* segs, int32_t* order, int32_t* nitems);

/* Message of the last failing call on b (or of fv_batch_query /
 * fv_batch_create when b is NULL). Never NULL. */
const char* fv_batch_last_error(const fv_batch* b);

int fv_batch_destroy(fv_batch* b);

/* ------------------------------------------------------------------------
 * Launch-parameter autotuner: the paper's runtime-regression network
 * (Sec. "Hyperparameters", Table para-setting; Sec. "Feature Centering and
 * Scaling"), trained and evaluated by FP32 kernels.
 *
 * Network: n_in -> 64 -> 64 -> 64 -> 1, ReLU hidden layers, identity
 * output, where n_in is FV_MLP_IN (the paper's network: the 14 launch
 * features) or FV_MLP_IN_SIZED (a problem-size-conditioned network, the
 * extension proposed in Sec. "Broader Impact": the 14 launch features followed
 * by FV_MLP_MAX_EXTRA problem features, here the standardised log2 of the
 * grid's cell count and its dimension, so that one network serves grids of
 * several sizes). Parameters are one flat FP32 array of
 * FV_MLP_NPARAM_FOR(n_in) floats:
 *   W1[64][n_in], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[1][64], b4[1]
 * (W[out][in]); an n_in other than the two widths is FV_EINVAL. Rows of X
 * hold n_in features. Loss of a minibatch of B rows:
 *   L = sum_r (yhat_r - y_r)^2 / (2B) + alpha / (2B) * sum of squared weights
 * (biases not penalised). Adam (Kingma & Ba, efficient form):
 *   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 *   theta -= lr sqrt(1-b2^t) / (1-b1^t) * m / (sqrt(v) + eps).
 * All pointers below are device pointers unless stated; every call enqueues
 * on `stream` and returns without waiting.
 * ------------------------------------------------------------------------ */
#define FV_MLP_IN 14
#define FV_MLP_MAX_EXTRA 2
#define FV_MLP_IN_SIZED 16
#define FV_MLP_HID 64
#define FV_MLP_NPARAM_FOR(n_in) (64 * (n_in) + 8449)
#define FV_MLP_NPARAM 9345
#define FV_MLP_NPARAM_SIZED 9473

typedef struct fv_mlp_hparams {
    float lr;              /* learning rate (constant) */
    float beta1, beta2;    /* moment decay factors */
    float eps;             /* numerical stability factor */
    float alpha;           /* L2 penalty */
    float tol;             /* improvement tolerance of the epoch loss */
    int32_t batch;         /* minibatch size (rows beyond n are not used) */
    int32_t max_epochs;
    int32_t n_iter_no_change; /* stop after this many epochs without an improvement of tol */
    int32_t reserved;
} fv_mlp_hparams;

/* Bytes of device scratch the MLP calls need for n rows (at most 65536). */
int fv_mlp_workspace(int32_t n, size_t* bytes);

/* Loss L and its gradient (FV_MLP_NPARAM_FOR(n_in) floats) over all n rows
 * of X ([n][n_in], row-major) and y ([n]) at `params`, with penalty alpha.
 * loss is one device float. */
int fv_mlp_loss_grad(const float* params, int32_t n_in, const float* X, const float* y, int32_t n, float alpha,
                     float* grad, float* loss, void* workspace, size_t ws_bytes, void* stream);

/* Predictions out[n] for the rows of X ([n][n_in]). */
int fv_mlp_predict(const float* params, int32_t n_in, const float* X, int32_t n, float* out, void* stream);

/* Trains params (n_in inputs) in place with Adam from the moments adam_m /
 * adam_v (FV_MLP_NPARAM_FOR(n_in) floats each, zero for a fresh start) and step counter
 * *adam_t (device int32, 0 for a fresh start). Epoch e visits the rows in
 * the order order[e * n .. e * n + n - 1] (a permutation of 0..n-1 per epoch,
 * drawn by the caller), in minibatches of hp->batch rows. epoch_loss[e]
 * receives sum over minibatches of L_b * B_b / n; *epochs_run (device int32)
 * the number of epochs done. Training stops early once the epoch loss has
 * failed to improve on the best so far by hp->tol for more than
 * hp->n_iter_no_change consecutive epochs. One workgroup does all the work. */
int fv_mlp_train(float* params, int32_t n_in, float* adam_m, float* adam_v, int32_t* adam_t, const float* X,
                 const float* y, int32_t n, const int32_t* order, const fv_mlp_hparams* hp, float* epoch_loss,
                 int32_t* epochs_run, void* workspace, size_t ws_bytes, void* stream);

/* Search space of launch vectors: site s has radix[s] choices (1 = pinned);
 * choice c gives parameters (p1[s][c], p2[s][c]) and the network features
 * (f1[s][c], f2[s][c]), already standardised. Index decoding is mixed radix
 * with site 0 fastest: c_s = (idx / prod_{t<s} radix[t]) % radix[s].
 * n_extra is 0 (the network has FV_MLP_IN inputs) or FV_MLP_MAX_EXTRA (it has
 * FV_MLP_IN_SIZED inputs, the last n_extra of which are extra[0..n_extra-1],
 * standardised, the same for every index: the problem being tuned). */
#define FV_SPACE_MAXC 32
typedef struct fv_tune_space {
    int32_t radix[FV_NSITES];
    int32_t p1[FV_NSITES][FV_SPACE_MAXC];
    int32_t p2[FV_NSITES][FV_SPACE_MAXC];
    float f1[FV_NSITES][FV_SPACE_MAXC];
    float f2[FV_NSITES][FV_SPACE_MAXC];
    int32_t n_extra;
    float extra[FV_MLP_MAX_EXTRA];
} fv_tune_space;

/* Predicts every index in [begin, begin + count) of the space (host
 * pointer) with the network of 2 * FV_NSITES + space->n_extra inputs and returns the k (1..8) lowest predictions, ascending, ties to
 * the lower index: top_idx[k] (device int64) and top_val[k] (device float). */
int fv_mlp_sweep(const float* params, const fv_tune_space* space, int64_t begin, int64_t count, int32_t k,
                 int64_t* top_idx, float* top_val, void* workspace, size_t ws_bytes, void* stream);

/* Bytes of device scratch fv_mlp_sweep needs. */
int fv_mlp_sweep_workspace(size_t* bytes);

/* fv_mlp_sweep without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * re-tune in place, harnesses that forbid hipMalloc): the per-block top-k
 * lists go to a static device array of the library (384 KiB per device,
 * held until the process ends; its device address is looked up once per
 * device on the first call made with that device current). The call itself
 * allocates nothing. Arguments, results and error codes are those of
 * fv_mlp_sweep; k above 8 is FV_EINVAL, and a count of any size fits (the
 * sweep's block count is capped at the array's capacity). FV_EDEVICE when
 * the array's address cannot be obtained. Every call on a device shares that
 * device's array: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller. No entry of the array
 * needs to start at zero: each call writes every entry it reads. */
int fv_mlp_sweep_static(const float* params, const fv_tune_space* space, int64_t begin, int64_t count, int32_t k,
                        int64_t* top_idx, float* top_val, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FV_H */
