// C ABI of the batched fused step: many uneven 2D grids advanced together by
// three fused stage launches per step, captured once in a HIP graph (a
// one-step graph and a graph of GRAPH_STEPS steps, so that a long run pays one
// graph launch per GRAPH_STEPS steps).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/fv.h"
#include "fv_internal.h"

namespace {

// Clock record of one step: n entries (even: earliest start, odd: latest
// end), each over fvk::CLK_SLOTS slots.
__global__ void k_clk_reset(unsigned long long* clk, int n) {
    for (int i = threadIdx.x; i < n * fvk::CLK_SLOTS; i += blockDim.x)
        clk[fvk::clk_index(i / fvk::CLK_SLOTS, i % fvk::CLK_SLOTS)] = ((i / fvk::CLK_SLOTS) & 1) ? 0ull : ~0ull;
}

// Folds the slots of this step's clock record into history[counter] and
// advances the counter.
__global__ void k_clk_store(const unsigned long long* clk, int n, unsigned long long* history, int max_steps,
                            int* counter) {
    const int step = *counter;
    if (step < max_steps)
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            unsigned long long v = clk[fvk::clk_index(i, 0)];
            for (int k = 1; k < fvk::CLK_SLOTS; ++k) {
                const unsigned long long w = clk[fvk::clk_index(i, k)];
                v = (i & 1) ? (w > v ? w : v) : (w < v ? w : v);
            }
            history[(long long)step * n + i] = v;
        }
    __syncthreads();
    if (threadIdx.x == 0) *counter = step + 1;
}

__global__ void k_copy_dt(const double* src, double* dst, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BLayout {
    std::vector<int64_t> offsets;
    size_t off_fgrid, off_lam, off_dt, off_status, off_clk, off_counter, off_U1, off_U2, total;
};

int validate_batch(int32_t ngrids, const fv_grid_desc* grids, BLayout* L, char* why) {
    if (ngrids < 1 || ngrids > 65536 || !grids) {
        snprintf(why, 256, "ngrids must be in [1, 65536] with a grid array");
        return FV_EINVAL;
    }
    L->offsets.assign(ngrids + 1, 0);
    for (int g = 0; g < ngrids; ++g) {
        const fv_grid_desc& d = grids[g];
        if (d.ndim != 2 || d.n[2] != 1) {
            snprintf(why, 256, "grid %d: batches hold 2D grids only", g);
            return FV_ENOTSUP;
        }
        if (d.n[0] < 1 || d.n[1] < 1 || d.n[0] > 65534 || d.n[1] > 65534) {
            snprintf(why, 256, "grid %d: cell counts must be in [1, 65534]", g);
            return FV_EINVAL;
        }
        if ((int64_t)d.n[0] * d.n[1] * 4 * 8 >= ((int64_t)1 << 32)) {
            snprintf(why, 256, "grid %d: a state of 4 GiB or more (buffer offsets are 32-bit)", g);
            return FV_EINVAL;
        }
        if (d.scheme < FV_SCHEME_MINMOD || d.scheme > FV_SCHEME_QUICK) {
            snprintf(why, 256, "grid %d: unknown scheme", g);
            return FV_EINVAL;
        }
        for (int a = 0; a < 2; ++a) {
            if (!(d.hi[a] > d.lo[a])) {
                snprintf(why, 256, "grid %d: hi must exceed lo", g);
                return FV_EINVAL;
            }
            for (int s = 0; s < 2; ++s) {
                const int kind = d.bc[a][s];
                if (kind != FV_BC_PERIODIC && kind != FV_BC_TRANSMISSIVE && kind != FV_BC_WALL &&
                    kind != FV_BC_INFLOW) {
                    snprintf(why, 256, "grid %d: unknown boundary kind", g);
                    return FV_EINVAL;
                }
                if (kind == FV_BC_WALL && d.n[a] < 2) {
                    snprintf(why, 256, "grid %d: a slip wall needs at least 2 cells on its axis", g);
                    return FV_EINVAL;
                }
                if (kind == FV_BC_INFLOW) {
                    const double* q = d.bc_state[a][s];
                    const double p = (d.gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
                    if (!(q[0] > 0.0) || !(p > 0.0) || !isfinite(p)) {
                        snprintf(why, 256, "grid %d: an inflow state needs a positive density and pressure", g);
                        return FV_EINVAL;
                    }
                }
            }
            if ((d.bc[a][0] == FV_BC_PERIODIC) != (d.bc[a][1] == FV_BC_PERIODIC)) {
                snprintf(why, 256, "grid %d: periodic must be set on both faces", g);
                return FV_EINVAL;
            }
        }
        if (!(d.gamma > 1.0) || !(d.cfl > 0.0)) {
            snprintf(why, 256, "grid %d: gamma must exceed 1 and cfl be positive", g);
            return FV_EINVAL;
        }
        if (!(d.mu >= 0.0) || !isfinite(d.mu) || (d.mu > 0.0 && (!(d.prandtl > 0.0) || !isfinite(d.prandtl)))) {
            snprintf(why, 256, "grid %d: viscosity must be finite and >= 0, with a positive Prandtl number", g);
            return FV_EINVAL;
        }
        if (d.nodes) {
            snprintf(why, 256, "grid %d: batches take uniform grids only (no nodes)", g);
            return FV_EINVAL;
        }
        L->offsets[g + 1] = L->offsets[g] + 4 * d.n[0] * d.n[1];
    }
    const size_t total_el = (size_t)L->offsets[ngrids];
    size_t o = 0;
    L->off_fgrid = o;
    o = a256(o + sizeof(fvk::FGrid) * ngrids);
    L->off_lam = o;
    o = a256(o + 8 * (size_t)ngrids);
    L->off_dt = o;
    o = a256(o + 8 * (size_t)ngrids);
    L->off_status = o;
    o = a256(o + 4);
    L->off_clk = o;
    o = a256(o + 6 * sizeof(unsigned long long) * fvk::CLK_SLOTS * fvk::CLK_PAD * (size_t)ngrids);
    L->off_counter = o;
    o = a256(o + 4);
    L->off_U1 = o;
    o = a256(o + 8 * total_el);
    L->off_U2 = o;
    o = a256(o + 8 * total_el);
    L->total = o;
    return FV_OK;
}

}  // namespace

struct fv_batch {
    int ngrids, waves, nitems, order;
    int mode;  // stage-kernel variant: 0 periodic / transmissive, 1 walls or inflow faces, 2 viscous
    hipStream_t stream, cap;
    fvk::FGrid* grids;
    unsigned long long* lam;
    double* dt;
    uint32_t* status;
    unsigned long long* clk;
    int* counter;
    double* U1;
    double* U2;
    std::vector<fvk::FGrid> by_grid;     // table entry of each grid, in the caller's order
    std::vector<fvk::FGrid> host_grids;  // the uploaded table, in work-list order
    hipGraph_t graph, graph_many;  // one step; GRAPH_STEPS steps
    hipGraphExec_t exec, exec_many;
    double* graph_U;
    bool graph_timed;
    unsigned long long* graph_history;  // history buffer baked into the captured graph
    unsigned long long* history;
    int max_steps;
    char err[256];
};

static char g_berr[256] = "";

static int bfail(fv_batch* b, int code, const char* msg) {
    snprintf(b ? b->err : g_berr, 256, "%s", msg);
    return code;
}

constexpr int GRAPH_STEPS = 8;

static void drop_graph(fv_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->exec_many) (void)hipGraphExecDestroy(b->exec_many);
    if (b->graph_many) (void)hipGraphDestroy(b->graph_many);
    b->exec = nullptr;
    b->graph = nullptr;
    b->exec_many = nullptr;
    b->graph_many = nullptr;
    b->graph_U = nullptr;
    b->graph_history = nullptr;
}

// Enqueues one step (three stages, plus the clock record when timing) on s.
static void enqueue_step(fv_batch* b, double* U, hipStream_t s) {
    const int nclk = 6 * b->ngrids;
    unsigned long long* clk = b->history ? b->clk : nullptr;
    if (clk) hipLaunchKernelGGL(k_clk_reset, dim3(1), dim3(256), 0, s, b->clk, nclk);
    fvk::launch_fused_stage(0, b->waves, b->grids, b->ngrids, b->nitems, U, U, b->U1, b->lam, b->dt, nullptr,
                            nullptr, b->status, clk, s, nullptr, b->mode);
    fvk::launch_fused_stage(1, b->waves, b->grids, b->ngrids, b->nitems, U, b->U1, b->U2, b->lam, b->dt,
                            nullptr, nullptr, b->status, clk, s, nullptr, b->mode);
    fvk::launch_fused_stage(2, b->waves, b->grids, b->ngrids, b->nitems, U, b->U2, U, b->lam, b->dt, nullptr,
                            nullptr, b->status, clk, s, nullptr, b->mode);
    if (clk) hipLaunchKernelGGL(k_clk_store, dim3(1), dim3(256), 0, s, b->clk, nclk, b->history, b->max_steps, b->counter);
}

static bool valid_seg(int32_t seg) { return seg >= 4 && seg <= 1024 && seg % 4 == 0; }

// Orders the table by the work-list order, assigns each grid its segment
// height and first work item, and uploads it. Work items of a grid are
// contiguous; the step's graph is rebuilt on the next step.
static int apply_schedule(fv_batch* b, int32_t order) {
    const int n = b->ngrids;
    std::vector<int> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    if (order == FV_ORDER_LARGEST_FIRST)
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) {
            return (long long)b->by_grid[a].nx * b->by_grid[a].ny > (long long)b->by_grid[c].nx * b->by_grid[c].ny;
        });
    b->host_grids.resize(n);
    long long work = 0;
    for (int q = 0; q < n; ++q) {
        fvk::FGrid G = b->by_grid[perm[q]];
        G.work0 = (int)work;
        work += fvk::fused_items(G, G.seg);
        b->host_grids[q] = G;
    }
    if (work > 0x7fffffff) return bfail(b, FV_EINVAL, "too many work items");
    b->nitems = (int)work;
    b->order = order;
    hipError_t e = hipMemcpyAsync(b->grids, b->host_grids.data(), sizeof(fvk::FGrid) * n, hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, FV_EDEVICE, "grid table upload failed");
    drop_graph(b);
    return FV_OK;
}

extern "C" {

int fv_batch_query(int32_t ngrids, const fv_grid_desc* grids, int64_t* offsets, size_t* workspace_bytes) {
    BLayout L;
    int rc = validate_batch(ngrids, grids, &L, g_berr);
    if (rc != FV_OK) return rc;
    if (offsets)
        for (int g = 0; g <= ngrids; ++g) offsets[g] = L.offsets[g];
    if (workspace_bytes) *workspace_bytes = L.total;
    return FV_OK;
}

int fv_batch_create(int32_t ngrids, const fv_grid_desc* grids, int32_t seg, int32_t waves, int32_t order,
                    void* workspace, size_t workspace_bytes, void* stream, fv_batch** out) {
    if (!out) return bfail(nullptr, FV_EINVAL, "null output pointer");
    *out = nullptr;
    BLayout L;
    int rc = validate_batch(ngrids, grids, &L, g_berr);
    if (rc != FV_OK) return rc;
    if (seg != 0 && !valid_seg(seg))
        return bfail(nullptr, FV_EINVAL, "seg must be 0 (automatic) or a multiple of 4 in [4, 1024]");
    if (waves < 0) return bfail(nullptr, FV_EINVAL, "negative wave count");
    if (order != FV_ORDER_GIVEN && order != FV_ORDER_LARGEST_FIRST) return bfail(nullptr, FV_EINVAL, "unknown order");
    if (!workspace || ((uintptr_t)workspace & 255)) return bfail(nullptr, FV_EWORKSPACE, "workspace missing or misaligned");
    if (workspace_bytes < L.total) return bfail(nullptr, FV_EWORKSPACE, "workspace too small");
    fv_batch* b = new (std::nothrow) fv_batch();
    if (!b) return bfail(nullptr, FV_EDEVICE, "host allocation failed");
    b->ngrids = ngrids;
    b->waves = waves;
    b->stream = (hipStream_t)stream;
    char* base = (char*)workspace;
    b->grids = (fvk::FGrid*)(base + L.off_fgrid);
    b->lam = (unsigned long long*)(base + L.off_lam);
    b->dt = (double*)(base + L.off_dt);
    b->status = (uint32_t*)(base + L.off_status);
    b->clk = (unsigned long long*)(base + L.off_clk);
    b->counter = (int*)(base + L.off_counter);
    b->U1 = (double*)(base + L.off_U1);
    b->U2 = (double*)(base + L.off_U2);
    // table entries by grid; each keeps the element offset of its own slot of the state
    b->by_grid.resize(ngrids);
    for (int g = 0; g < ngrids; ++g) {
        const fv_grid_desc& d = grids[g];
        fvk::FGrid& G = b->by_grid[g];
        memset(&G, 0, sizeof(G));
        G.nx = (int)d.n[0];
        G.ny = (int)d.n[1];
        G.pitch = G.nx;
        G.strips = fvk::fused_strips(G.nx);
        G.scheme = d.scheme;
        G.bcx0 = d.bc[0][0];
        G.bcx1 = d.bc[0][1];
        G.bcy0 = d.bc[1][0];
        G.bcy1 = d.bc[1][1];
        G.gid = g;
        G.base = L.offsets[g];
        G.sv = (long long)G.nx * G.ny;
        const double dx = (d.hi[0] - d.lo[0]) / (double)d.n[0];
        const double dy = (d.hi[1] - d.lo[1]) / (double)d.n[1];
        G.ax = dy;
        G.ay = dx;
        G.inv_vol = 1.0 / (dx * dy);
        G.inv_dx = 1.0 / dx;
        G.inv_dy = 1.0 / dy;
        G.cfl = d.cfl;
        G.gamma = d.gamma;
        G.gm1 = d.gamma - 1.0;
        for (int a = 0; a < 2; ++a)
            for (int sd = 0; sd < 2; ++sd)
                for (int v = 0; v < 4; ++v) G.q[a][sd][v] = d.bc_state[a][sd][v];
        G.mu = d.mu;
        if (d.mu > 0.0) {
            G.kcond = d.mu * d.gamma / ((d.gamma - 1.0) * d.prandtl);
            const double hf = d.gamma / d.prandtl;
            G.nu_fac = hf > 4.0 / 3.0 ? hf : 4.0 / 3.0;
        }
        // the stage kernels' variant: viscous if any grid is, else the
        // boundary variant if any grid has a slip wall or an inflow face
        for (int a = 0; a < 2; ++a)
            for (int sd = 0; sd < 2; ++sd)
                if ((d.bc[a][sd] == FV_BC_WALL || d.bc[a][sd] == FV_BC_INFLOW) && b->mode < 1) b->mode = 1;
        if (d.mu > 0.0) b->mode = 2;
    }
    if (seg == 0) seg = fvk::fused_auto_seg(b->by_grid.data(), ngrids, fvk::fused_slots());
    for (int g = 0; g < ngrids; ++g) b->by_grid[g].seg = seg;
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        snprintf(g_berr, 256, "batch set-up failed: %s", hipGetErrorString(e));
        delete b;
        return FV_EDEVICE;
    }
    rc = apply_schedule(b, order);
    if (rc != FV_OK) {
        snprintf(g_berr, 256, "%s", b->err);
        (void)hipStreamDestroy(b->cap);
        delete b;
        return rc;
    }
    fvk::launch_set_u32(b->status, 0u, b->stream);
    *out = b;
    return FV_OK;
}

int fv_batch_step(fv_batch* b, double* U, int32_t nsteps) {
    if (!b) return bfail(nullptr, FV_EINVAL, "null batch");
    if (!U || nsteps < 0) return bfail(b, FV_EINVAL, "null state or negative step count");
    if (nsteps == 0) return FV_OK;
    const bool timed = b->history != nullptr;
    if (b->graph_U != U || !b->exec || b->graph_timed != timed || b->graph_history != b->history) {
        drop_graph(b);
        hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            enqueue_step(b, U, b->cap);
            e = hipStreamEndCapture(b->cap, &b->graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            for (int s = 0; s < GRAPH_STEPS; ++s) enqueue_step(b, U, b->cap);
            e = hipStreamEndCapture(b->cap, &b->graph_many);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec_many, b->graph_many, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return bfail(b, FV_EDEVICE, "graph capture failed");
        }
        b->graph_U = U;
        b->graph_timed = timed;
        b->graph_history = b->history;
    }
    fvk::launch_fused_init(b->waves, b->grids, b->ngrids, b->nitems, U, b->lam, b->status, b->stream);
    for (int32_t s = 0; s < nsteps;) {
        const bool many = nsteps - s >= GRAPH_STEPS;
        hipError_t e = hipGraphLaunch(many ? b->exec_many : b->exec, b->stream);
        if (e != hipSuccess) return bfail(b, FV_EDEVICE, "graph launch failed");
        s += many ? GRAPH_STEPS : 1;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, FV_EDEVICE, hipGetErrorString(e));
    return FV_OK;
}

int fv_batch_set_timing(fv_batch* b, uint64_t* history, int32_t max_steps, double* ticks_per_us) {
    if (!b) return bfail(nullptr, FV_EINVAL, "null batch");
    if (history && max_steps < 1) return bfail(b, FV_EINVAL, "max_steps must be positive");
    b->history = (unsigned long long*)history;
    b->max_steps = history ? max_steps : 0;
    fvk::launch_set_u32((uint32_t*)b->counter, 0u, b->stream);
    if (ticks_per_us) {
        int dev = 0, khz = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) khz = 0;
        *ticks_per_us = khz / 1000.0;
    }
    return FV_OK;
}

int fv_batch_dt(fv_batch* b, double* dt) {
    if (!b || !dt) return bfail(b, FV_EINVAL, "null argument");
    hipLaunchKernelGGL(k_copy_dt, dim3(1), dim3(256), 0, b->stream, b->dt, dt, b->ngrids);
    return hipGetLastError() == hipSuccess ? FV_OK : FV_EDEVICE;
}

int fv_batch_status(fv_batch* b, uint32_t* flags) {
    if (!b) return bfail(nullptr, FV_EINVAL, "null batch");
    uint32_t h = 0;
    hipError_t e = hipMemcpyAsync(&h, b->status, sizeof(h), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, FV_EDEVICE, "status read failed");
    if (flags) *flags = h;
    return h ? FV_ENONPHYS : FV_OK;
}

int fv_batch_set_schedule(fv_batch* b, const int32_t* segs, int32_t order) {
    if (!b) return bfail(nullptr, FV_EINVAL, "null batch");
    if (order != FV_ORDER_GIVEN && order != FV_ORDER_LARGEST_FIRST) return bfail(b, FV_EINVAL, "unknown order");
    if (segs)
        for (int g = 0; g < b->ngrids; ++g)
            if (!valid_seg(segs[g])) return bfail(b, FV_EINVAL, "seg must be a multiple of 4 in [4, 1024]");
    if (segs)
        for (int g = 0; g < b->ngrids; ++g) b->by_grid[g].seg = segs[g];
    return apply_schedule(b, order);
}

int fv_batch_info(const fv_batch* b, int32_t* segs, int32_t* order, int32_t* nitems) {
    if (!b) return FV_EINVAL;
    if (segs)
        for (int g = 0; g < b->ngrids; ++g) segs[g] = b->by_grid[g].seg;
    if (order) *order = b->order;
    if (nitems) *nitems = b->nitems;
    return FV_OK;
}

const char* fv_batch_last_error(const fv_batch* b) { return b ? b->err : g_berr; }

int fv_batch_destroy(fv_batch* b) {
    if (!b) return FV_EINVAL;
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return FV_OK;
}

}  // extern "C"
