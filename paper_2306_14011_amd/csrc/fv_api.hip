// C ABI of libfv.so: context, workspace carving, launch-table validation and
// the orchestration of a step out of the kernels in fv_kernels.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "../../include/fv.h"
#include "fv_internal.h"

using fvk::Geo;

struct fv_ctx {
    fv_grid_desc desc;
    Geo g;
    hipStream_t stream;
    fv_launch launch;
    int device;
    // carved from the caller's workspace
    uint32_t* status;
    double* dt;
    double* partial;
    int max_partial;
    double* U1;
    double* U2;
    double* F[3];
    double* R;
    double* lamA;
    double* lamB;
    // fused path
    int path, fseg[3], fwaves[3], fitems[3];   // per Runge-Kutta stage
    fvk::FGrid* fgrid[3];  // the fused path's grid description per stage (an FGrid3 in 3D); they differ in seg
    unsigned long long* flam;
    double* fdt;
    bool fused_ready;   // the per-stage tables are set (also used by the adjoint's forward recomputation)
    const double* src;  // caller's cell-averaged source S[v][cell], or null
    fvk::BcState bcs;   // ghost states of inflow faces
    // per-site event timing (diagnostic)
    static const int kMaxEv = 64;
    bool timing;
    bool ev_ready;
    hipEvent_t ev[2 * kMaxEv];
    int ev_site[kMaxEv];
    int nev;
    double acc_ms[FV_NTIMERS];
    int64_t acc_n[FV_NTIMERS];
    char err[256];
};

static char g_err[256] = "";

static int fail(fv_ctx* c, int code, const char* fmt, const char* detail = "") {
    char* dst = c ? c->err : g_err;
    snprintf(dst, 256, fmt, detail);
    return code;
}

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

namespace {

struct Layout {
    int nvar;
    int64_t pitch, sy, sz, sv;
    int64_t faces[3];
    int64_t ncell;
    int max_partial;
    size_t off_status, off_dt, off_fused, off_partial, off_U1, off_U2, off_F[3], off_R, off_lamA, off_lamB, off_met,
        total;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int validate(const fv_grid_desc* g, Layout* L, char* why) {
    if (!g) {
        snprintf(why, 256, "null grid description");
        return FV_EINVAL;
    }
    if (g->ndim != 2 && g->ndim != 3) {
        snprintf(why, 256, "ndim must be 2 or 3");
        return FV_EINVAL;
    }
    if (g->scheme < FV_SCHEME_MINMOD || g->scheme > FV_SCHEME_QUICK) {
        snprintf(why, 256, "unknown scheme");
        return FV_EINVAL;
    }
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 1 || g->n[d] > 65534) {
            snprintf(why, 256, "cell counts must be in [1, 65534]");
            return FV_EINVAL;
        }
    }
    if (g->ndim == 2 && g->n[2] != 1) {
        snprintf(why, 256, "n[2] must be 1 in 2D");
        return FV_EINVAL;
    }
    for (int d = 0; d < g->ndim; ++d) {
        if (!(g->hi[d] > g->lo[d])) {
            snprintf(why, 256, "hi must exceed lo on every axis");
            return FV_EINVAL;
        }
        for (int s = 0; s < 2; ++s) {
            if (g->bc[d][s] != FV_BC_PERIODIC && g->bc[d][s] != FV_BC_TRANSMISSIVE && g->bc[d][s] != FV_BC_WALL &&
                g->bc[d][s] != FV_BC_INFLOW) {
                snprintf(why, 256, "unknown boundary kind");
                return FV_EINVAL;
            }
            if (g->bc[d][s] == FV_BC_INFLOW) {
                const double* q = g->bc_state[d][s];
                const int nv = g->ndim + 2;
                double m2 = 0.0;
                for (int a = 0; a < g->ndim; ++a) m2 += q[1 + a] * q[1 + a];
                const double p = (g->gamma - 1.0) * (q[nv - 1] - 0.5 * m2 / q[0]);
                if (!(q[0] > 0.0) || !(p > 0.0) || !isfinite(p)) {
                    snprintf(why, 256, "an inflow state needs a positive density and pressure");
                    return FV_EINVAL;
                }
            }
            if (g->bc[d][s] == FV_BC_WALL && g->n[d] < 2) {
                snprintf(why, 256, "a slip wall needs at least 2 cells on its axis");
                return FV_EINVAL;
            }
        }
        if ((g->bc[d][0] == FV_BC_PERIODIC) != (g->bc[d][1] == FV_BC_PERIODIC)) {
            snprintf(why, 256, "periodic must be set on both faces of an axis");
            return FV_EINVAL;
        }
    }
    if (!(g->gamma > 1.0) || !(g->cfl > 0.0)) {
        snprintf(why, 256, "gamma must exceed 1 and cfl must be positive");
        return FV_EINVAL;
    }
    if (!(g->mu >= 0.0) || !isfinite(g->mu) || (g->mu > 0.0 && (!(g->prandtl > 0.0) || !isfinite(g->prandtl)))) {
        snprintf(why, 256, "viscosity must be finite and >= 0, with a positive Prandtl number when > 0");
        return FV_EINVAL;
    }
    if (g->nodes && g->ndim != 2) {
        snprintf(why, 256, "curvilinear grids (nodes) are 2D only");
        return FV_EINVAL;
    }
    if (g->nodes && g->mu > 0.0) {
        snprintf(why, 256, "the viscous flux is taken on uniform grids only");
        return FV_EINVAL;
    }
    const int nd = g->ndim;
    L->nvar = nd + 2;
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    // row pitch padded to a multiple of 8 doubles (64 B)
    L->pitch = ((nx + 2 * fvk::NG) + 7) / 8 * 8;
    L->sy = L->pitch;
    L->sz = L->sy * (ny + 2 * fvk::NG);
    L->sv = L->sz * (nd == 3 ? nz + 2 * fvk::NG : 1);
    if (L->sv >= (int64_t)1 << 31) {
        snprintf(why, 256, "grid too large: one variable must hold fewer than 2^31 doubles");
        return FV_EINVAL;
    }
    L->ncell = nx * ny * nz;
    L->faces[0] = (nx + 1) * ny * nz;
    L->faces[1] = nx * (ny + 1) * nz;
    L->faces[2] = nd == 3 ? nx * ny * (nz + 1) : 0;
    const int64_t maxp = (L->ncell + 63) / 64;
    L->max_partial = (int)(maxp > 65536 ? maxp : 65536);
    size_t o = 0;
    L->off_status = o;
    o += 256;
    L->off_dt = o;
    o += 256;
    L->off_fused = o;   // 3 x 512 B: an FGrid or FGrid3 per stage; lambda at +1536, dt at +1544
    o += 2048;
    L->off_partial = o;
    o = align256(o + (size_t)L->max_partial * 8);
    const size_t state = (size_t)L->nvar * L->sv * 8;
    const size_t dense = (size_t)L->nvar * L->ncell * 8;
    L->off_U1 = o;
    o = align256(o + state);
    L->off_U2 = o;
    o = align256(o + state);
    for (int d = 0; d < 3; ++d) {
        L->off_F[d] = o;
        o = align256(o + (size_t)L->nvar * L->faces[d] * 8);
    }
    L->off_R = o;
    o = align256(o + dense);
    L->off_lamA = o;
    o = align256(o + dense);
    L->off_lamB = o;
    o = align256(o + dense);
    L->off_met = o;
    if (g->nodes) {
        const fvk::MetricOffsets mo = fvk::metric_offsets((int)nx, (int)ny);
        o = align256(o + (size_t)(mo.cell + 2 * mo.nc) * 8);
    }
    L->total = o;
    return FV_OK;
}

int validate_launch(const fv_launch* l, int ndim, char* why) {
    for (int s = 0; s < FV_NSITES; ++s) {
        const int a = l->p[2 * s], b = l->p[2 * s + 1];
        if (s <= FV_SITE_FLUX_Z) {
            if (s == FV_SITE_FLUX_Z && ndim == 2 && a == 0 && b == 0) continue;
            if (!is_pow2(a) || a > 1024 || !is_pow2(b) || b < 64 || b > 1024 || a > b) {
                snprintf(why, 256, "site %d: block width must be a power of two <= threads, threads in [64, 1024]", s);
                return FV_EINVAL;
            }
        } else {
            if (!(a == 0 || (is_pow2(a) && a <= 65536)) || !is_pow2(b) || b < 64 || b > 1024) {
                snprintf(why, 256, "site %d: gang must be 0 or a power of two <= 65536, threads in [64, 1024]", s);
                return FV_EINVAL;
            }
        }
    }
    return FV_OK;
}

Geo make_geo(const fv_grid_desc* d, const Layout& L) {
    Geo g;
    memset(&g, 0, sizeof(g));
    g.ndim = d->ndim;
    g.nvar = L.nvar;
    for (int a = 0; a < 3; ++a) g.n[a] = (int)d->n[a];
    g.sy = (int)L.sy;
    g.sz = (int)L.sz;
    g.sv = L.sv;
    g.off0 = (int)(fvk::NG + fvk::NG * L.sy + (d->ndim == 3 ? fvk::NG * L.sz : 0));
    g.ncell = (int)L.ncell;
    for (int a = 0; a < 3; ++a) g.fsv[a] = L.faces[a];
    g.dnx = fvk::make_divmod((uint32_t)d->n[0]);
    g.dny = fvk::make_divmod((uint32_t)d->n[1]);
    double dx[3];
    for (int a = 0; a < 3; ++a) dx[a] = a < d->ndim ? (d->hi[a] - d->lo[a]) / (double)d->n[a] : 1.0;
    double vol = 1.0;
    for (int a = 0; a < d->ndim; ++a) vol *= dx[a];
    for (int a = 0; a < 3; ++a) {
        g.inv_dx[a] = 1.0 / dx[a];
        double ar = 1.0;
        for (int b = 0; b < d->ndim; ++b)
            if (b != a) ar *= dx[b];
        g.area[a] = ar;
    }
    g.inv_vol = 1.0 / vol;
    g.vol = vol;
    g.gamma = d->gamma;
    g.gm1 = d->gamma - 1.0;
    g.cfl = d->cfl;
    for (int a = 0; a < 3; ++a) {
        g.bc[a][0] = d->bc[a][0];
        g.bc[a][1] = d->bc[a][1];
    }
    g.scheme = d->scheme;
    g.met = nullptr;  // set by fv_create for curvilinear grids
    if (d->nodes)
        for (int a = 0; a < 3; ++a) g.area[a] = 1.0;  // the face fluxes carry their lengths
    g.mu = d->mu;
    if (d->mu > 0.0) {
        g.kcond = d->mu * d->gamma / ((d->gamma - 1.0) * d->prandtl);
        const double hf = d->gamma / d->prandtl;
        g.nu_fac = hf > 4.0 / 3.0 ? hf : 4.0 / 3.0;
    }
    return g;
}

int check_launch_error(fv_ctx* c) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, FV_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return FV_OK;
}

inline int P(const fv_ctx* c, int site, int k) { return c->launch.p[2 * site + k]; }

// Event bracket around one site's launch when timing is enabled.
struct SiteTimer {
    fv_ctx* c;
    int slot;
    SiteTimer(fv_ctx* ctx, int site) : c(ctx), slot(-1) {
        if (c->timing && c->nev < fv_ctx::kMaxEv) {
            slot = c->nev++;
            c->ev_site[slot] = site;
            (void)hipEventRecord(c->ev[2 * slot], c->stream);
        }
    }
    ~SiteTimer() {
        if (slot >= 0) (void)hipEventRecord(c->ev[2 * slot + 1], c->stream);
    }
};

// Waits for the recorded events and accumulates their durations per site.
int drain_timing(fv_ctx* c) {
    if (!c->timing || c->nev == 0) return FV_OK;
    hipError_t e = hipEventSynchronize(c->ev[2 * (c->nev - 1) + 1]);
    if (e != hipSuccess) return fail(c, FV_EDEVICE, "event wait failed: %s", hipGetErrorString(e));
    for (int i = 0; i < c->nev; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) == hipSuccess) {
            c->acc_ms[c->ev_site[i]] += ms;
            c->acc_n[c->ev_site[i]] += 1;
        }
    }
    c->nev = 0;
    return FV_OK;
}

void enqueue_bc(fv_ctx* c, double* U) {
    SiteTimer t(c, FV_SITE_BC);
    fvk::launch_bc_fill(U, c->g, c->bcs, P(c, FV_SITE_BC, 0), P(c, FV_SITE_BC, 1), c->stream);
}

void enqueue_fluxes(fv_ctx* c, const double* U) {
    for (int ax = 0; ax < c->g.ndim; ++ax) {
        SiteTimer t(c, FV_SITE_FLUX_X + ax);
        if (c->g.met)
            fvk::launch_flux_curv(ax, U, c->F[ax], c->g, c->bcs, P(c, FV_SITE_FLUX_X + ax, 0),
                                  P(c, FV_SITE_FLUX_X + ax, 1), c->stream);
        else
            fvk::launch_flux(ax, U, c->F[ax], c->g, P(c, FV_SITE_FLUX_X + ax, 0), P(c, FV_SITE_FLUX_X + ax, 1),
                             c->stream);
        if (c->g.mu > 0.0) fvk::launch_visc(ax, U, c->F[ax], c->g, c->bcs, c->stream);
    }
}

void enqueue_residual(fv_ctx* c, double* R) {
    SiteTimer t(c, FV_SITE_RESIDUAL);
    fvk::launch_residual(c->F[0], c->F[1], c->F[2], c->src, R, c->g, P(c, FV_SITE_RESIDUAL, 0),
                         P(c, FV_SITE_RESIDUAL, 1), c->stream);
}

void enqueue_update(fv_ctx* c, int stage, const double* Un, const double* Us, double* Ud,
                    const double* dtp = nullptr) {
    SiteTimer t(c, FV_SITE_UPDATE);
    fvk::launch_update(stage, Un, Us, Ud, c->R, dtp ? dtp : c->dt, c->g, P(c, FV_SITE_UPDATE, 0),
                       P(c, FV_SITE_UPDATE, 1), c->stream);
}

void enqueue_cfl(fv_ctx* c, const double* U, const double* dt_in, double* dt_out) {
    SiteTimer t(c, FV_SITE_CFL);
    fvk::launch_cfl(U, c->partial, c->status, dt_in, c->dt, dt_out, c->g, P(c, FV_SITE_CFL, 0), P(c, FV_SITE_CFL, 1),
                    c->stream);
}

// L(Us) into c->R, then the stage combination into Ud.
void enqueue_stage(fv_ctx* c, int stage, const double* Un, double* Us, double* Ud) {
    enqueue_bc(c, Us);
    enqueue_fluxes(c, Us);
    enqueue_residual(c, c->R);
    enqueue_update(c, stage, Un, Us, Ud);
}

}  // namespace

extern "C" {

void fv_default_launch(fv_launch* out) {
    if (!out) return;
    for (int s = 0; s < FV_NSITES; ++s) {
        if (s <= FV_SITE_FLUX_Z) {
            out->p[2 * s] = 64;
            out->p[2 * s + 1] = 256;
        } else {
            out->p[2 * s] = 0;
            out->p[2 * s + 1] = 256;
        }
    }
}

int fv_query(const fv_grid_desc* g, int64_t strides_out[4], size_t* workspace_bytes) {
    Layout L;
    int rc = validate(g, &L, g_err);
    if (rc != FV_OK) return rc;
    if (strides_out) {
        strides_out[0] = 1;
        strides_out[1] = L.sy;
        strides_out[2] = L.sz;
        strides_out[3] = L.sv;
    }
    if (workspace_bytes) *workspace_bytes = L.total;
    return FV_OK;
}

static int set_fused_stage(fv_ctx* c, int st, int32_t seg, int32_t waves);

// Whether the fused stage kernels can run this grid: not 3D viscous, a state
// below 4 GiB (their buffer offsets are 32-bit; a curvilinear grid's metric
// blocks are then below 4 GiB too).
static int fused_refusal(const fv_ctx* c, const char** why) {
    if (c->g.mu > 0.0 && c->g.ndim == 3) {
        *why = "3D viscous grids run on the split path only%s";
        return FV_ENOTSUP;
    }
    if ((long long)c->g.nvar * c->g.sv * 8 >= (1ll << 32)) {
        *why = "the fused path needs a state below 4 GiB (buffer offsets are 32-bit)%s";
        return FV_ENOTSUP;
    }
    return FV_OK;
}

int fv_create(const fv_grid_desc* g, void* workspace, size_t workspace_bytes, void* stream, fv_ctx** out) {
    if (!out) return fail(nullptr, FV_EINVAL, "null output pointer%s");
    *out = nullptr;
    Layout L;
    int rc = validate(g, &L, g_err);
    if (rc != FV_OK) return rc;
    if (!workspace) return fail(nullptr, FV_EWORKSPACE, "null workspace%s");
    if (((uintptr_t)workspace & 255) != 0) return fail(nullptr, FV_EWORKSPACE, "workspace must be 256-byte aligned%s");
    if (workspace_bytes < L.total) return fail(nullptr, FV_EWORKSPACE, "workspace too small%s");
    fv_ctx* c = new (std::nothrow) fv_ctx;
    if (!c) return fail(nullptr, FV_EDEVICE, "host allocation failed%s");
    memset(c, 0, sizeof(*c));
    c->desc = *g;
    c->g = make_geo(g, L);
    memcpy(c->bcs.q, g->bc_state, sizeof(c->bcs.q));
    c->stream = (hipStream_t)stream;
    fv_default_launch(&c->launch);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, FV_EDEVICE, "hipGetDevice failed%s");
    }
    char* base = (char*)workspace;
    c->status = (uint32_t*)(base + L.off_status);
    c->dt = (double*)(base + L.off_dt);
    c->partial = (double*)(base + L.off_partial);
    c->max_partial = L.max_partial;
    c->U1 = (double*)(base + L.off_U1);
    c->U2 = (double*)(base + L.off_U2);
    for (int d = 0; d < 3; ++d) c->F[d] = (double*)(base + L.off_F[d]);
    c->R = (double*)(base + L.off_R);
    c->lamA = (double*)(base + L.off_lamA);
    c->lamB = (double*)(base + L.off_lamB);
    for (int st = 0; st < 3; ++st) c->fgrid[st] = (fvk::FGrid*)(base + L.off_fused + 512 * st);
    c->flam = (unsigned long long*)(base + L.off_fused + 1536);
    c->fdt = (double*)(base + L.off_fused + 1544);
    c->path = FV_PATH_SPLIT;
    if (g->nodes) {
        double* met = (double*)(base + L.off_met);
        fvk::launch_metrics(g->nodes, met, (int)g->n[0], (int)g->n[1], c->stream);
        c->g.met = met;
    }
    fvk::launch_set_u32(c->status, 0u, c->stream);
    if (check_launch_error(c) != FV_OK) {
        snprintf(g_err, 256, "%s", c->err);
        delete c;
        return FV_EDEVICE;
    }
    // the fused stage tables at the library's choice: fv_adjoint_step
    // recomputes its stage states with the fused stage kernels
    const char* why;
    if (fused_refusal(c, &why) == FV_OK) {
        for (int st = 0; st < 3; ++st) {
            if (set_fused_stage(c, st, 0, 0) != FV_OK) {
                snprintf(g_err, 256, "%s", c->err);
                delete c;
                return FV_EDEVICE;
            }
        }
        c->fused_ready = true;
    }
    *out = c;
    return FV_OK;
}

int fv_destroy(fv_ctx* c) {
    if (!c) return FV_EINVAL;
    if (c->ev_ready)
        for (int i = 0; i < 2 * fv_ctx::kMaxEv; ++i) (void)hipEventDestroy(c->ev[i]);
    delete c;
    return FV_OK;
}

int fv_set_stream(fv_ctx* c, void* stream) {
    if (!c) return FV_EINVAL;
    c->stream = (hipStream_t)stream;
    return FV_OK;
}

int fv_residual(fv_ctx* c, double* U, double* R) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    if (!U || !R) return fail(c, FV_EINVAL, "null state or residual pointer%s");
    enqueue_bc(c, U);
    enqueue_fluxes(c, U);
    enqueue_residual(c, R);
    int rc = check_launch_error(c);
    if (rc != FV_OK) return rc;
    return drain_timing(c);
}

static_assert(sizeof(fvk::FGrid) <= 512 && sizeof(fvk::FGrid3) <= 512, "fused grid slot is 512 bytes");

// Whether a grid has a slip-wall or inflow face (the fused kernels' boundary variant).
static bool has_walls(const fv_ctx* c) {
    for (int d = 0; d < c->g.ndim; ++d)
        for (int s = 0; s < 2; ++s)
            if (c->g.bc[d][s] == FV_BC_WALL || c->g.bc[d][s] == FV_BC_INFLOW) return true;
    return false;
}

static int fused_step3(fv_ctx* c, double* U, int32_t nsteps, const double* dt_in, double* dt_out) {
    const fvk::FGrid3* const* G = (const fvk::FGrid3* const*)c->fgrid;
    const bool walls = has_walls(c);
    fvk::launch_fused3d_init(c->fwaves[0], G[0], c->fitems[0], U, c->flam, c->status, c->stream);
    for (int32_t s = 0; s < nsteps; ++s) {
        {
            SiteTimer t(c, FV_TIMER_FUSED);
            fvk::launch_fused3d_stage(0, c->fwaves[0], G[0], c->fitems[0], U, U, c->U1, c->flam, c->fdt,
                                      dt_in ? dt_in + s : nullptr, dt_out ? dt_out + s : nullptr, c->status,
                                      c->stream, c->src, c->g.vol, walls);
        }
        {
            SiteTimer t(c, FV_TIMER_FUSED);
            fvk::launch_fused3d_stage(1, c->fwaves[1], G[1], c->fitems[1], U, c->U1, c->U2, c->flam, c->fdt,
                                      nullptr, nullptr, c->status, c->stream, c->src, c->g.vol, walls);
        }
        {
            SiteTimer t(c, FV_TIMER_FUSED);
            fvk::launch_fused3d_stage(2, c->fwaves[2], G[2], c->fitems[2], U, c->U2, U, c->flam, c->fdt, nullptr,
                                      nullptr, c->status, c->stream, c->src, c->g.vol, walls);
        }
        int rc = check_launch_error(c);
        if (rc != FV_OK) return rc;
        rc = drain_timing(c);
        if (rc != FV_OK) return rc;
    }
    return FV_OK;
}

static int fused_step(fv_ctx* c, double* U, int32_t nsteps, const double* dt_in, double* dt_out) {
    if (nsteps == 0) return FV_OK;
    if (c->g.ndim == 3) return fused_step3(c, U, nsteps, dt_in, dt_out);
    const int walls = c->g.met ? 3 : (c->g.mu > 0.0 ? 2 : (has_walls(c) ? 1 : 0));
    fvk::launch_fused_init(c->fwaves[0], c->fgrid[0], 1, c->fitems[0], U, c->flam, c->status, c->stream, c->g.met);
    for (int32_t s = 0; s < nsteps; ++s) {
        {
            SiteTimer t(c, FV_TIMER_FUSED);
            fvk::launch_fused_stage(0, c->fwaves[0], c->fgrid[0], 1, c->fitems[0], U, U, c->U1, c->flam, c->fdt,
                                    dt_in ? dt_in + s : nullptr, dt_out ? dt_out + s : nullptr, c->status, nullptr,
                                    c->stream, c->src, walls, c->g.met);
        }
        {
            SiteTimer t(c, FV_TIMER_FUSED);
            fvk::launch_fused_stage(1, c->fwaves[1], c->fgrid[1], 1, c->fitems[1], U, c->U1, c->U2, c->flam, c->fdt,
                                    nullptr, nullptr, c->status, nullptr, c->stream, c->src, walls, c->g.met);
        }
        {
            SiteTimer t(c, FV_TIMER_FUSED);
            fvk::launch_fused_stage(2, c->fwaves[2], c->fgrid[2], 1, c->fitems[2], U, c->U2, U, c->flam, c->fdt,
                                    nullptr, nullptr, c->status, nullptr, c->stream, c->src, walls, c->g.met);
        }
        int rc = check_launch_error(c);
        if (rc != FV_OK) return rc;
        rc = drain_timing(c);
        if (rc != FV_OK) return rc;
    }
    return FV_OK;
}

// Builds the fused grid description of stage `st` with segment height seg
// (0: the library's choice) and wave count waves, uploads it to the stage's
// slot and records the stage's work items.
static int set_fused_stage(fv_ctx* c, int st, int32_t seg, int32_t waves) {
    hipError_t e;
    if (c->g.ndim == 3) {
        fvk::FGrid3 G;
        memset(&G, 0, sizeof(G));
        G.nx = c->g.n[0];
        G.ny = c->g.n[1];
        G.nz = c->g.n[2];
        G.strips = fvk::fused_strips(G.nx);
        G.scheme = c->g.scheme;
        G.bcx0 = c->g.bc[0][0];
        G.bcx1 = c->g.bc[0][1];
        G.bcy0 = c->g.bc[1][0];
        G.bcy1 = c->g.bc[1][1];
        G.bcz0 = c->g.bc[2][0];
        G.bcz1 = c->g.bc[2][1];
        G.base = c->g.off0;
        G.sv = c->g.sv;
        G.py = c->g.sy;
        G.pz = c->g.sz;
        G.ax = c->g.area[0];
        G.ay = c->g.area[1];
        G.az = c->g.area[2];
        G.inv_vol = c->g.inv_vol;
        G.inv_dx = c->g.inv_dx[0];
        G.inv_dy = c->g.inv_dx[1];
        G.inv_dz = c->g.inv_dx[2];
        G.cfl = c->g.cfl;
        G.gamma = c->g.gamma;
        G.gm1 = c->g.gm1;
        memcpy(G.q, c->bcs.q, sizeof(G.q));
        if (seg == 0) seg = fvk::fused3d_auto_seg(G, fvk::fused3d_slots());
        G.seg = seg;
        e = hipMemcpyAsync(c->fgrid[st], &G, sizeof(G), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        c->fitems[st] = fvk::fused3d_items(G, seg);
    } else {
        fvk::FGrid G;
        memset(&G, 0, sizeof(G));
        G.nx = c->g.n[0];
        G.ny = c->g.n[1];
        G.pitch = c->g.sy;
        G.strips = fvk::fused_strips(G.nx);
        G.work0 = 0;
        G.scheme = c->g.scheme;
        G.bcx0 = c->g.bc[0][0];
        G.bcx1 = c->g.bc[0][1];
        G.bcy0 = c->g.bc[1][0];
        G.bcy1 = c->g.bc[1][1];
        G.base = c->g.off0;
        G.sv = c->g.sv;
        G.ax = c->g.area[0];
        G.ay = c->g.area[1];
        G.inv_vol = c->g.inv_vol;
        G.inv_dx = c->g.inv_dx[0];
        G.inv_dy = c->g.inv_dx[1];
        G.cfl = c->g.cfl;
        G.gamma = c->g.gamma;
        G.gm1 = c->g.gm1;
        for (int a = 0; a < 2; ++a)
            for (int sd = 0; sd < 2; ++sd)
                for (int v = 0; v < 4; ++v) G.q[a][sd][v] = c->bcs.q[a][sd][v];
        G.mu = c->g.mu;
        G.kcond = c->g.kcond;
        G.nu_fac = c->g.nu_fac;
        if (seg == 0) seg = fvk::fused_auto_seg(&G, 1, fvk::fused_slots());
        G.seg = seg;
        e = hipMemcpyAsync(c->fgrid[st], &G, sizeof(G), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        c->fitems[st] = fvk::fused_items(G, seg);
    }
    if (e != hipSuccess) return fail(c, FV_EDEVICE, "grid table upload failed: %s", hipGetErrorString(e));
    c->fseg[st] = seg;
    c->fwaves[st] = waves;
    return FV_OK;
}

static bool valid_fused_seg(int32_t seg) { return seg == 0 || (seg >= 4 && seg <= 1024 && seg % 4 == 0); }

int fv_set_path(fv_ctx* c, int path, int32_t seg, int32_t waves) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    if (path == FV_PATH_SPLIT) {
        c->path = FV_PATH_SPLIT;
        return FV_OK;
    }
    if (path != FV_PATH_FUSED) return fail(c, FV_EINVAL, "unknown path%s");
    const char* why;
    const int refused = fused_refusal(c, &why);
    if (refused != FV_OK) return fail(c, refused, why);
    if (!valid_fused_seg(seg))
        return fail(c, FV_EINVAL, "seg must be 0 (automatic) or a multiple of 4 in [4, 1024]%s");
    if (waves < 0) return fail(c, FV_EINVAL, "negative wave count%s");
    for (int st = 0; st < 3; ++st) {
        const int rc = set_fused_stage(c, st, seg, waves);
        if (rc != FV_OK) return rc;
    }
    c->path = FV_PATH_FUSED;
    return FV_OK;
}

int fv_set_fused_launch(fv_ctx* c, const fv_fused_launch* l) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    if (!l) return fail(c, FV_EINVAL, "null launch table%s");
    if (c->path != FV_PATH_FUSED) return fail(c, FV_EINVAL, "select the fused path first (fv_set_path)%s");
    for (int st = 0; st < 3; ++st) {
        if (!valid_fused_seg(l->seg[st]))
            return fail(c, FV_EINVAL, "seg must be 0 (automatic) or a multiple of 4 in [4, 1024]%s");
        if (l->waves[st] < 0) return fail(c, FV_EINVAL, "negative wave count%s");
    }
    for (int st = 0; st < 3; ++st) {
        const int rc = set_fused_stage(c, st, l->seg[st], l->waves[st]);
        if (rc != FV_OK) return rc;
    }
    return FV_OK;
}

int fv_fused_slots(const fv_ctx* c, int32_t* waves) {
    if (!c || !waves) return FV_EINVAL;
    const int w = c->g.ndim == 3 ? 4 * fvk::fused3d_slots() : fvk::fused_slots();
    if (w <= 0) return FV_EDEVICE;
    *waves = w;
    return FV_OK;
}

int fv_get_fused_launch(const fv_ctx* c, fv_fused_launch* out) {
    if (!c || !out) return FV_EINVAL;
    if (c->path != FV_PATH_FUSED) return FV_EINVAL;
    for (int st = 0; st < 3; ++st) {
        out->seg[st] = c->fseg[st];
        out->waves[st] = c->fwaves[st];
    }
    return FV_OK;
}

int fv_get_path(const fv_ctx* c, int32_t* path, int32_t* seg, int32_t* waves) {
    if (!c) return FV_EINVAL;
    if (path) *path = c->path;
    if (seg) *seg = c->path == FV_PATH_FUSED ? c->fseg[0] : 0;
    if (waves) *waves = c->path == FV_PATH_FUSED ? c->fwaves[0] : 0;
    return FV_OK;
}

int fv_step(fv_ctx* c, double* U, int32_t nsteps, const double* dt_in, double* dt_out) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    if (!U) return fail(c, FV_EINVAL, "null state pointer%s");
    if (nsteps < 0) return fail(c, FV_EINVAL, "negative step count%s");
    if (c->path == FV_PATH_FUSED) return fused_step(c, U, nsteps, dt_in, dt_out);
    for (int32_t s = 0; s < nsteps; ++s) {
        enqueue_bc(c, U);
        enqueue_cfl(c, U, dt_in ? dt_in + s : nullptr, dt_out ? dt_out + s : nullptr);
        // stage 1: U1 = U + dt L(U)   (ghosts of U already filled)
        enqueue_fluxes(c, U);
        enqueue_residual(c, c->R);
        enqueue_update(c, 0, U, U, c->U1);
        // stage 2: U2 = 3/4 U + 1/4 (U1 + dt L(U1)), in place over U1
        enqueue_stage(c, 1, U, c->U1, c->U1);
        // stage 3: U = 1/3 U + 2/3 (U2 + dt L(U2)), in place over U
        enqueue_stage(c, 2, U, c->U1, U);
        int rc = check_launch_error(c);
        if (rc != FV_OK) return rc;
        rc = drain_timing(c);
        if (rc != FV_OK) return rc;
    }
    return FV_OK;
}

int fv_residual_norm(fv_ctx* c, double* U, double* norms) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    if (!U || !norms) return fail(c, FV_EINVAL, "null state or norms pointer%s");
    enqueue_bc(c, U);
    enqueue_fluxes(c, U);
    enqueue_residual(c, c->R);
    fvk::launch_residual_norm(c->R, c->partial, norms, c->g, c->stream);
    int rc = check_launch_error(c);
    if (rc != FV_OK) return rc;
    return drain_timing(c);
}

int fv_set_source(fv_ctx* c, const double* S) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    c->src = S;
    return FV_OK;
}

int fv_adjoint_step(fv_ctx* c, double* U_n, const double* dt, double* lam) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    if (!U_n || !dt || !lam) return fail(c, FV_EINVAL, "null state, dt or adjoint pointer%s");
    if (c->g.mu > 0.0) return fail(c, FV_ENOTSUP, "the adjoint step covers the inviscid residual only%s");
    if (c->g.met) return fail(c, FV_ENOTSUP, "the adjoint step covers uniform grids only%s");
    // recompute the stage states with the frozen dt: U1 = U + dt L(U), U2 = 3/4 U + 1/4 (U1 + dt L(U1))
    if (c->fused_ready) {
        const bool walls = has_walls(c);
        if (c->g.ndim == 3) {
            const fvk::FGrid3* const* G = (const fvk::FGrid3* const*)c->fgrid;
            fvk::launch_fused3d_stage(0, c->fwaves[0], G[0], c->fitems[0], U_n, U_n, c->U1, c->flam, c->fdt, dt,
                                      nullptr, c->status, c->stream, c->src, c->g.vol, walls);
            fvk::launch_fused3d_stage(1, c->fwaves[1], G[1], c->fitems[1], U_n, c->U1, c->U2, c->flam, c->fdt,
                                      nullptr, nullptr, c->status, c->stream, c->src, c->g.vol, walls);
        } else {
            fvk::launch_fused_stage(0, c->fwaves[0], c->fgrid[0], 1, c->fitems[0], U_n, U_n, c->U1, c->flam, c->fdt,
                                    dt, nullptr, c->status, nullptr, c->stream, c->src, walls ? 1 : 0);
            fvk::launch_fused_stage(1, c->fwaves[1], c->fgrid[1], 1, c->fitems[1], U_n, c->U1, c->U2, c->flam,
                                    c->fdt, nullptr, nullptr, c->status, nullptr, c->stream, c->src, walls ? 1 : 0);
        }
    } else {
        enqueue_bc(c, U_n);
        enqueue_fluxes(c, U_n);
        enqueue_residual(c, c->R);
        enqueue_update(c, 0, U_n, U_n, c->U1, dt);
        enqueue_bc(c, c->U1);
        enqueue_fluxes(c, c->U1);
        enqueue_residual(c, c->R);
        enqueue_update(c, 1, U_n, c->U1, c->U2, dt);
    }
    // reverse stages 3, 2, 1 (the kernels map the ghost positions themselves)
    fvk::launch_adj_stage(3, c->U2, lam, lam, c->lamA, c->lamB, c->R, dt, c->g, c->bcs, c->stream);
    fvk::launch_adj_stage(2, c->U1, c->lamA, lam, c->lamA, c->lamB, c->R, dt, c->g, c->bcs, c->stream);
    fvk::launch_adj_stage(1, U_n, c->R, lam, c->lamA, c->lamB, c->R, dt, c->g, c->bcs, c->stream);
    int rc = check_launch_error(c);
    if (rc != FV_OK) return rc;
    return drain_timing(c);
}

int fv_set_launch(fv_ctx* c, const fv_launch* l) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    if (!l) return fail(c, FV_EINVAL, "null launch table%s");
    char why[256];
    if (validate_launch(l, c->g.ndim, why) != FV_OK) return fail(c, FV_EINVAL, "%s", why);
    const int cb = fvk::cfl_blocks(c->g, l->p[2 * FV_SITE_CFL], l->p[2 * FV_SITE_CFL + 1]);
    if (cb > c->max_partial) return fail(c, FV_EINVAL, "cfl gang exceeds the partial buffer%s");
    c->launch = *l;
    if (c->g.ndim == 2) {
        // the z-flux pair is inert in 2D: keep a valid placeholder
        c->launch.p[2 * FV_SITE_FLUX_Z] = l->p[2 * FV_SITE_FLUX_Z] ? l->p[2 * FV_SITE_FLUX_Z] : 64;
        c->launch.p[2 * FV_SITE_FLUX_Z + 1] = l->p[2 * FV_SITE_FLUX_Z + 1] ? l->p[2 * FV_SITE_FLUX_Z + 1] : 256;
    }
    return FV_OK;
}

int fv_get_launch(const fv_ctx* c, fv_launch* out) {
    if (!c || !out) return FV_EINVAL;
    *out = c->launch;
    return FV_OK;
}

int fv_status(fv_ctx* c, uint32_t* flags) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    uint32_t h = 0;
    hipError_t e = hipMemcpyAsync(&h, c->status, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, FV_EDEVICE, "status read failed: %s", hipGetErrorString(e));
    if (flags) *flags = h;
    return h ? FV_ENONPHYS : FV_OK;
}

int fv_clear_status(fv_ctx* c) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    fvk::launch_set_u32(c->status, 0u, c->stream);
    return check_launch_error(c);
}

int fv_set_timing(fv_ctx* c, int enable) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    if (enable && !c->ev_ready) {
        for (int i = 0; i < 2 * fv_ctx::kMaxEv; ++i) {
            hipError_t e = hipEventCreate(&c->ev[i]);
            if (e != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->ev[j]);
                return fail(c, FV_EDEVICE, "event creation failed: %s", hipGetErrorString(e));
            }
        }
        c->ev_ready = true;
    }
    c->timing = enable != 0;
    c->nev = 0;
    return FV_OK;
}

int fv_get_timing(fv_ctx* c, double ms_out[8], int64_t launches_out[8]) {
    if (!c) return fail(nullptr, FV_EINVAL, "null context%s");
    int rc = drain_timing(c);
    if (rc != FV_OK) return rc;
    for (int s = 0; s < FV_NTIMERS; ++s) {
        if (ms_out) ms_out[s] = c->acc_ms[s];
        if (launches_out) launches_out[s] = c->acc_n[s];
        c->acc_ms[s] = 0.0;
        c->acc_n[s] = 0;
    }
    return FV_OK;
}

const char* fv_last_error(const fv_ctx* c) { return c ? c->err : g_err; }

}  // extern "C"
