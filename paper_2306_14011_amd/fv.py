"""Thin ctypes binding of ``libfv.so`` (declared in ``include/fv.h``).

The functions carry the C names and only marshal arguments: every step of
the method runs in the library's HIP kernels. PyTorch provides device memory
and streams. There is no fallback: when the library is missing, loading it
raises.

``Solver`` is a convenience that owns the torch buffers of one grid (ghosted
state, workspace) and converts between the dense ``(nvar, nz, ny, nx)``
interior layout and the library's ghosted layout.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfv.so")

FV_OK = 0
FV_EINVAL = -1
FV_EDEVICE = -2
FV_ENONPHYS = -3
FV_ENOTSUP = -4
FV_EWORKSPACE = -5

FV_SCHEME_MINMOD = 0
FV_SCHEME_UNLIMITED = 1
FV_SCHEME_FROMM = 2
FV_SCHEME_THIRD = 3
FV_SCHEME_CENTRAL = 4
FV_SCHEME_VANLEER = 5
FV_SCHEME_QUICK = 6
# kappa of the unlimited (Psi = 1) members of the MUSCL family
_SCHEME_OF_KAPPA = ((-1.0, FV_SCHEME_UNLIMITED), (0.0, FV_SCHEME_FROMM), (1.0 / 3.0, FV_SCHEME_THIRD),
                    (0.5, FV_SCHEME_QUICK), (1.0, FV_SCHEME_CENTRAL))


def scheme_of(spec):
    """FV_SCHEME_* of a grid spec: spec.limiter True (or "minmod") gives minmod,
    "vanleer" van Leer, False the unlimited member for spec.kappa (-1 by
    default; 0, 1/3, 1/2 and 1 also exist)."""
    lim = getattr(spec, "limiter", True)
    if lim == "vanleer":
        return FV_SCHEME_VANLEER
    if lim is True or lim == "minmod":
        return FV_SCHEME_MINMOD
    if lim is not False and lim is not None:
        raise ValueError(f"unknown limiter {lim!r}")
    kappa = float(getattr(spec, "kappa", -1.0))
    for k, code in _SCHEME_OF_KAPPA:
        if abs(kappa - k) <= 1e-12:
            return code
    raise ValueError(f"unlimited MUSCL supports kappa in (-1, 0, 1/3, 1/2, 1), got {kappa}")

FV_BC_PERIODIC = 0
FV_BC_TRANSMISSIVE = 1
FV_BC_WALL = 2
FV_BC_INFLOW = 3

FV_FLAG_NAN = 1
FV_FLAG_RHO = 2
FV_FLAG_P = 4
FV_FLAG_DT = 8

SITES = ("flux_x", "flux_y", "flux_z", "residual", "update", "bc", "cfl")
NSITES = 7
TIMERS = SITES + ("fused",)
NTIMERS = 8
FV_PATH_SPLIT = 0
FV_PATH_FUSED = 1


class fv_grid_desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("bc_state", ((ctypes.c_double * 5) * 2) * 3),
        ("mu", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("nodes", ctypes.c_void_p),
    ]


class fv_launch(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32 * 14)]


class fv_fused_launch(ctypes.Structure):
    _fields_ = [("seg", ctypes.c_int32 * 3), ("waves", ctypes.c_int32 * 3)]


FV_MLP_IN = 14
FV_MLP_MAX_EXTRA = 2
FV_MLP_IN_SIZED = 16
FV_MLP_HID = 64
FV_MLP_NPARAM = 9345
FV_MLP_NPARAM_SIZED = 9473


def fv_mlp_nparam(n_in):
    return 64 * int(n_in) + 8449
FV_SPACE_MAXC = 32


class fv_mlp_hparams(ctypes.Structure):
    _fields_ = [
        ("lr", ctypes.c_float),
        ("beta1", ctypes.c_float),
        ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("alpha", ctypes.c_float),
        ("tol", ctypes.c_float),
        ("batch", ctypes.c_int32),
        ("max_epochs", ctypes.c_int32),
        ("n_iter_no_change", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class fv_tune_space(ctypes.Structure):
    _fields_ = [
        ("radix", ctypes.c_int32 * NSITES),
        ("p1", (ctypes.c_int32 * FV_SPACE_MAXC) * NSITES),
        ("p2", (ctypes.c_int32 * FV_SPACE_MAXC) * NSITES),
        ("f1", (ctypes.c_float * FV_SPACE_MAXC) * NSITES),
        ("f2", (ctypes.c_float * FV_SPACE_MAXC) * NSITES),
        ("n_extra", ctypes.c_int32),
        ("extra", ctypes.c_float * FV_MLP_MAX_EXTRA),
    ]


class FvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fv error {code}: {msg}")
        self.code = code


_lib = None

_vp = ctypes.c_void_p


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2306_14011_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        L.fv_default_launch.argtypes = [ctypes.POINTER(fv_launch)]
        L.fv_default_launch.restype = None
        L.fv_query.argtypes = [ctypes.POINTER(fv_grid_desc), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_size_t)]
        L.fv_create.argtypes = [ctypes.POINTER(fv_grid_desc), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
        L.fv_destroy.argtypes = [_vp]
        L.fv_set_stream.argtypes = [_vp, _vp]
        L.fv_residual.argtypes = [_vp, _vp, _vp]
        L.fv_step.argtypes = [_vp, _vp, ctypes.c_int32, _vp, _vp]
        L.fv_adjoint_step.argtypes = [_vp, _vp, _vp, _vp]
        L.fv_set_source.argtypes = [_vp, _vp]
        L.fv_residual_norm.argtypes = [_vp, _vp, _vp]
        L.fv_set_launch.argtypes = [_vp, ctypes.POINTER(fv_launch)]
        L.fv_get_launch.argtypes = [_vp, ctypes.POINTER(fv_launch)]
        L.fv_status.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint32)]
        L.fv_clear_status.argtypes = [_vp]
        L.fv_set_timing.argtypes = [_vp, ctypes.c_int]
        L.fv_set_path.argtypes = [_vp, ctypes.c_int, ctypes.c_int32, ctypes.c_int32]
        L.fv_get_path.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)]
        L.fv_set_fused_launch.argtypes = [_vp, ctypes.POINTER(fv_fused_launch)]
        L.fv_get_fused_launch.argtypes = [_vp, ctypes.POINTER(fv_fused_launch)]
        L.fv_fused_slots.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32)]
        L.fv_get_timing.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.fv_last_error.argtypes = [_vp]
        L.fv_last_error.restype = ctypes.c_char_p
        L.fv_batch_query.argtypes = [ctypes.c_int32, ctypes.POINTER(fv_grid_desc), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_size_t)]
        L.fv_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(fv_grid_desc), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
        L.fv_batch_step.argtypes = [_vp, _vp, ctypes.c_int32]
        L.fv_batch_set_timing.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.fv_batch_dt.argtypes = [_vp, _vp]
        L.fv_batch_status.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint32)]
        L.fv_batch_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]
        L.fv_batch_set_schedule.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
        L.fv_batch_destroy.argtypes = [_vp]
        L.fv_batch_last_error.argtypes = [_vp]
        L.fv_batch_last_error.restype = ctypes.c_char_p
        L.fv_mlp_workspace.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.fv_mlp_sweep_workspace.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
        L.fv_mlp_loss_grad.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32, ctypes.c_float, _vp, _vp,
                                       _vp, ctypes.c_size_t, _vp]
        L.fv_mlp_predict.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp]
        L.fv_mlp_train.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp,
                                   ctypes.POINTER(fv_mlp_hparams), _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.fv_mlp_sweep.argtypes = [_vp, ctypes.POINTER(fv_tune_space), ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.fv_mlp_sweep_static.argtypes = [_vp, ctypes.POINTER(fv_tune_space), ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int32, _vp, _vp, _vp]
        for name in ("fv_query", "fv_create", "fv_destroy", "fv_set_stream", "fv_residual", "fv_step",
                     "fv_adjoint_step", "fv_set_source", "fv_residual_norm", "fv_set_launch", "fv_get_launch", "fv_status", "fv_clear_status",
                     "fv_set_timing", "fv_get_timing", "fv_set_path", "fv_get_path", "fv_set_fused_launch",
                     "fv_get_fused_launch", "fv_fused_slots", "fv_batch_query", "fv_batch_create",
                     "fv_batch_step", "fv_batch_set_timing", "fv_batch_dt", "fv_batch_status", "fv_batch_info", "fv_batch_set_schedule", "fv_batch_destroy",
                     "fv_mlp_workspace", "fv_mlp_sweep_workspace",
                     "fv_mlp_loss_grad", "fv_mlp_predict", "fv_mlp_train", "fv_mlp_sweep", "fv_mlp_sweep_static"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != FV_OK:
        msg = lib().fv_last_error(ctx).decode()
        raise FvError(rc, msg)
    return rc


def make_desc(spec, nodes_ptr=None) -> fv_grid_desc:
    """fv_grid_desc from any object with ndim, n, lo, hi, bc, gamma, cfl (and
    optionally limiter: False selects the unlimited scheme of kappa, see
    scheme_of; mu and prandtl for the viscous flux, bc_state for inflow faces,
    nodes for a curvilinear grid, whose device copy nodes_ptr points to)."""
    if getattr(spec, "nodes", None) is not None and nodes_ptr is None:
        raise ValueError("a curvilinear grid needs the device pointer of its nodes (Solver uploads them)")
    d = fv_grid_desc()
    d.nodes = nodes_ptr
    d.ndim = spec.ndim
    d.scheme = scheme_of(spec)
    for a in range(3):
        d.n[a] = int(spec.n[a])
        d.lo[a] = float(spec.lo[a])
        d.hi[a] = float(spec.hi[a])
        d.bc[a][0] = int(spec.bc[a][0])
        d.bc[a][1] = int(spec.bc[a][1])
    d.gamma = float(spec.gamma)
    d.cfl = float(spec.cfl)
    d.mu = float(getattr(spec, "mu", 0.0))
    d.prandtl = float(getattr(spec, "prandtl", 0.72))
    st = getattr(spec, "bc_state", None)
    if st is not None:
        st = np.asarray(st, dtype=np.float64)
        for a in range(3):
            for sd in range(2):
                for v in range(min(5, st.shape[2])):
                    d.bc_state[a][sd][v] = float(st[a, sd, v])
    return d


# --- C-named functions -------------------------------------------------------

def fv_default_launch():
    out = fv_launch()
    lib().fv_default_launch(ctypes.byref(out))
    return list(out.p)


def fv_query(desc):
    strides = (ctypes.c_int64 * 4)()
    ws = ctypes.c_size_t()
    _check(lib().fv_query(ctypes.byref(desc), strides, ctypes.byref(ws)))
    return list(strides), ws.value


def fv_create(desc, workspace_ptr, workspace_bytes, stream_ptr):
    out = _vp()
    _check(lib().fv_create(ctypes.byref(desc), _vp(workspace_ptr), workspace_bytes, _vp(stream_ptr),
                           ctypes.byref(out)))
    return out.value


def fv_destroy(ctx):
    return _check(lib().fv_destroy(_vp(ctx)))


def fv_set_stream(ctx, stream_ptr):
    return _check(lib().fv_set_stream(_vp(ctx), _vp(stream_ptr)), ctx)


def fv_residual(ctx, U_ptr, R_ptr):
    return _check(lib().fv_residual(_vp(ctx), _vp(U_ptr), _vp(R_ptr)), ctx)


def fv_step(ctx, U_ptr, nsteps, dt_in_ptr=None, dt_out_ptr=None):
    return _check(lib().fv_step(_vp(ctx), _vp(U_ptr), int(nsteps), _vp(dt_in_ptr), _vp(dt_out_ptr)), ctx)


def fv_residual_norm(ctx, U_ptr, norms_ptr):
    return _check(lib().fv_residual_norm(_vp(ctx), _vp(U_ptr), _vp(norms_ptr)), ctx)


def fv_set_source(ctx, S_ptr):
    return _check(lib().fv_set_source(_vp(ctx), _vp(S_ptr)), ctx)


def fv_adjoint_step(ctx, U_ptr, dt_ptr, lam_ptr):
    return _check(lib().fv_adjoint_step(_vp(ctx), _vp(U_ptr), _vp(dt_ptr), _vp(lam_ptr)), ctx)


def fv_set_launch(ctx, params):
    l = fv_launch()
    for i, v in enumerate(params):
        l.p[i] = int(v)
    return _check(lib().fv_set_launch(_vp(ctx), ctypes.byref(l)), ctx)


def fv_get_launch(ctx):
    l = fv_launch()
    _check(lib().fv_get_launch(_vp(ctx), ctypes.byref(l)), ctx)
    return list(l.p)


def fv_status(ctx):
    """(return code, flags); syncs the context's stream."""
    fl = ctypes.c_uint32()
    rc = lib().fv_status(_vp(ctx), ctypes.byref(fl))
    if rc not in (FV_OK, FV_ENONPHYS):
        _check(rc, ctx)
    return rc, fl.value


def fv_clear_status(ctx):
    return _check(lib().fv_clear_status(_vp(ctx)), ctx)


def fv_set_path(ctx, path, seg=0, waves=0):
    return _check(lib().fv_set_path(_vp(ctx), int(path), int(seg), int(waves)), ctx)


def fv_get_path(ctx):
    """(path, segment height in use, waves)."""
    p, sg, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().fv_get_path(_vp(ctx), ctypes.byref(p), ctypes.byref(sg), ctypes.byref(w)), ctx)
    return p.value, sg.value, w.value


def fv_set_fused_launch(ctx, seg, waves):
    """Per-stage fused launch table: seg and waves are 3-sequences."""
    l = fv_fused_launch()
    for st in range(3):
        l.seg[st] = int(seg[st])
        l.waves[st] = int(waves[st])
    return _check(lib().fv_set_fused_launch(_vp(ctx), ctypes.byref(l)), ctx)


def fv_get_fused_launch(ctx):
    """(seg[3], waves[3]) of the fused path in use."""
    l = fv_fused_launch()
    _check(lib().fv_get_fused_launch(_vp(ctx), ctypes.byref(l)), ctx)
    return list(l.seg), list(l.waves)


def fv_fused_table(vec):
    """(seg[3], waves[3]) of a fused-space launch vector (stage s in slots 2s, 2s + 1)."""
    return [int(vec[0]), int(vec[2]), int(vec[4])], [int(vec[1]), int(vec[3]), int(vec[5])]


def fv_fused_slots(ctx):
    """Wave slots the device holds at once for the fused stage kernels."""
    w = ctypes.c_int32()
    _check(lib().fv_fused_slots(_vp(ctx), ctypes.byref(w)), ctx)
    return w.value


def fv_set_timing(ctx, enable):
    return _check(lib().fv_set_timing(_vp(ctx), 1 if enable else 0), ctx)


def fv_get_timing(ctx):
    """(ms per timer, launches per timer) accumulated since the last read; timers
    are the seven sites then the fused stage."""
    ms = (ctypes.c_double * NTIMERS)()
    n = (ctypes.c_int64 * NTIMERS)()
    _check(lib().fv_get_timing(_vp(ctx), ms, n), ctx)
    return list(ms), list(n)


def fv_last_error(ctx=None):
    return lib().fv_last_error(_vp(ctx)).decode()


FV_ORDER_GIVEN = 0
FV_ORDER_LARGEST_FIRST = 1


def _desc_array(specs):
    arr = (fv_grid_desc * len(specs))()
    for i, s in enumerate(specs):
        arr[i] = make_desc(s)
    return arr


def fv_batch_query(specs):
    arr = _desc_array(specs)
    offs = (ctypes.c_int64 * (len(specs) + 1))()
    ws = ctypes.c_size_t()
    _batch_check(lib().fv_batch_query(len(specs), arr, offs, ctypes.byref(ws)))
    return list(offs), ws.value


def _batch_check(rc, b=None):
    if rc != FV_OK:
        raise FvError(rc, lib().fv_batch_last_error(b).decode())
    return rc


def fv_batch_create(specs, seg, waves, order, ws_ptr, ws_bytes, stream_ptr):
    arr = _desc_array(specs)
    out = _vp()
    _batch_check(lib().fv_batch_create(len(specs), arr, int(seg), int(waves), int(order), _vp(ws_ptr), ws_bytes,
                                       _vp(stream_ptr), ctypes.byref(out)))
    return out.value


def fv_batch_step(b, U_ptr, nsteps):
    return _batch_check(lib().fv_batch_step(_vp(b), _vp(U_ptr), int(nsteps)), b)


def fv_batch_set_timing(b, history_ptr, max_steps):
    tpu = ctypes.c_double()
    _batch_check(lib().fv_batch_set_timing(_vp(b), _vp(history_ptr), int(max_steps), ctypes.byref(tpu)), b)
    return tpu.value


def fv_batch_dt(b, dt_ptr):
    return _batch_check(lib().fv_batch_dt(_vp(b), _vp(dt_ptr)), b)


def fv_batch_status(b):
    fl = ctypes.c_uint32()
    rc = lib().fv_batch_status(_vp(b), ctypes.byref(fl))
    if rc not in (FV_OK, FV_ENONPHYS):
        _batch_check(rc, b)
    return rc, fl.value


def fv_batch_info(b, ngrids):
    """(segment height per grid, work-list order, work items per stage launch)."""
    segs = (ctypes.c_int32 * ngrids)()
    order, n = ctypes.c_int32(), ctypes.c_int32()
    _batch_check(lib().fv_batch_info(_vp(b), segs, ctypes.byref(order), ctypes.byref(n)), b)
    return list(segs), order.value, n.value


def fv_batch_set_schedule(b, segs, order):
    arr = None
    if segs is not None:
        arr = (ctypes.c_int32 * len(segs))(*[int(x) for x in segs])
    _batch_check(lib().fv_batch_set_schedule(_vp(b), arr, int(order)), b)


def fv_batch_destroy(b):
    return _batch_check(lib().fv_batch_destroy(_vp(b)))


def fv_mlp_workspace(n):
    b = ctypes.c_size_t()
    _check(lib().fv_mlp_workspace(int(n), ctypes.byref(b)))
    return b.value


def fv_mlp_sweep_workspace():
    b = ctypes.c_size_t()
    _check(lib().fv_mlp_sweep_workspace(ctypes.byref(b)))
    return b.value


def _mlp_check(rc, what):
    if rc != FV_OK:
        raise FvError(rc, what)
    return rc


def fv_mlp_loss_grad(params_ptr, n_in, X_ptr, y_ptr, n, alpha, grad_ptr, loss_ptr, ws_ptr, ws_bytes, stream_ptr):
    return _mlp_check(lib().fv_mlp_loss_grad(_vp(params_ptr), int(n_in), _vp(X_ptr), _vp(y_ptr), int(n),
                                             float(alpha), _vp(grad_ptr), _vp(loss_ptr), _vp(ws_ptr), ws_bytes,
                                             _vp(stream_ptr)), "fv_mlp_loss_grad")


def fv_mlp_predict(params_ptr, n_in, X_ptr, n, out_ptr, stream_ptr):
    return _mlp_check(lib().fv_mlp_predict(_vp(params_ptr), int(n_in), _vp(X_ptr), int(n), _vp(out_ptr),
                                           _vp(stream_ptr)), "fv_mlp_predict")


def fv_mlp_train(params_ptr, n_in, m_ptr, v_ptr, t_ptr, X_ptr, y_ptr, n, order_ptr, hp, loss_ptr, epochs_ptr,
                 ws_ptr, ws_bytes, stream_ptr):
    return _mlp_check(lib().fv_mlp_train(_vp(params_ptr), int(n_in), _vp(m_ptr), _vp(v_ptr), _vp(t_ptr),
                                         _vp(X_ptr), _vp(y_ptr), int(n), _vp(order_ptr), ctypes.byref(hp),
                                         _vp(loss_ptr), _vp(epochs_ptr), _vp(ws_ptr), ws_bytes, _vp(stream_ptr)),
                      "fv_mlp_train")


def fv_mlp_sweep(params_ptr, space, begin, count, k, top_idx_ptr, top_val_ptr, ws_ptr, ws_bytes, stream_ptr):
    return _mlp_check(lib().fv_mlp_sweep(_vp(params_ptr), ctypes.byref(space), int(begin), int(count), int(k),
                                         _vp(top_idx_ptr), _vp(top_val_ptr), _vp(ws_ptr), ws_bytes,
                                         _vp(stream_ptr)), "fv_mlp_sweep")


def fv_mlp_sweep_static(params_ptr, space, begin, count, k, top_idx_ptr, top_val_ptr, stream_ptr):
    return _mlp_check(lib().fv_mlp_sweep_static(_vp(params_ptr), ctypes.byref(space), int(begin), int(count), int(k),
                                                _vp(top_idx_ptr), _vp(top_val_ptr), _vp(stream_ptr)),
                      "fv_mlp_sweep_static")


# --- torch-side convenience ----------------------------------------------------

def _torch():
    import torch
    return torch


def current_stream_ptr(device=None):
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


class Solver:
    """One grid's device buffers and context.

    ``U`` is the ghosted state (a flat float64 tensor of nvar * s_v elements);
    ``interior()`` is a strided view of its interior cells, shape
    ``(nvar, nz, ny, nx)``.
    """

    def __init__(self, spec, device="cuda", stream=None):
        torch = _torch()
        self.spec = spec
        self.device = torch.device(device)
        self.nodes = None
        nodes = getattr(spec, "nodes", None)
        if nodes is not None:
            nx, ny = int(spec.n[0]), int(spec.n[1])
            self.nodes = torch.as_tensor(np.ascontiguousarray(nodes, dtype=np.float64)).to(self.device)
            if spec.ndim != 2 or tuple(self.nodes.shape) != (2, ny + 1, nx + 1):
                raise ValueError("curvilinear nodes must have shape (2, ny + 1, nx + 1) on a 2D grid")
        self.desc = make_desc(spec, self.nodes.data_ptr() if self.nodes is not None else None)
        self.strides, self.ws_bytes = fv_query(self.desc)
        self.nvar = spec.ndim + 2
        sx, sy, sz, sv = self.strides
        self.U = torch.zeros(self.nvar * sv, dtype=torch.float64, device=self.device)
        # workspace: torch's allocator returns blocks aligned to at least 256 B
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        assert self.workspace.data_ptr() % 256 == 0
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = fv_create(self.desc, self.workspace.data_ptr(), self.ws_bytes, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None):
            fv_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _view(self, flat):
        torch = _torch()
        sx, sy, sz, sv = self.strides
        nx, ny, nz = (int(v) for v in self.spec.n)
        g3 = 2 if self.spec.ndim == 3 else 0
        off = 2 + 2 * sy + g3 * sz
        return torch.as_strided(flat, (self.nvar, nz, ny, nx), (sv, sz, sy, 1), off)

    def interior(self):
        return self._view(self.U)

    def set_state(self, U_dense):
        torch = _torch()
        src = torch.as_tensor(np.ascontiguousarray(U_dense), dtype=torch.float64)
        self.interior().copy_(src.to(self.device))

    def get_state(self):
        return self.interior().detach().cpu().numpy().copy()

    def dense_zeros(self):
        torch = _torch()
        return torch.zeros(self.spec.shape, dtype=torch.float64, device=self.device)

    def residual(self):
        R = self.dense_zeros()
        fv_residual(self.ctx, self.U.data_ptr(), R.data_ptr())
        return R

    def residual_norm(self):
        """Per-variable L2 norm of the residual of the current state (numpy)."""
        torch = _torch()
        out = torch.zeros(self.nvar, dtype=torch.float64, device=self.device)
        fv_residual_norm(self.ctx, self.U.data_ptr(), out.data_ptr())
        return out.cpu().numpy()

    def set_source(self, S_dense):
        """Cell-averaged source of Eq. (residual), shape (nvar, nz, ny, nx) or
        any shape of nvar * ncell values in that order; None removes it. The
        device copy is held by the solver while set."""
        torch = _torch()
        if S_dense is None:
            fv_set_source(self.ctx, None)
            self._source = None
            return
        S = torch.as_tensor(np.ascontiguousarray(S_dense) if not torch.is_tensor(S_dense) else S_dense,
                            dtype=torch.float64).to(self.device).contiguous()
        if S.numel() != self.nvar * int(np.prod([int(v) for v in self.spec.n])):
            raise ValueError("source has the wrong number of cells or variables")
        fv_set_source(self.ctx, S.data_ptr())
        self._source = S

    def step(self, nsteps, dt_in=None, dt_out=None):
        fv_step(self.ctx, self.U.data_ptr(), nsteps,
                dt_in.data_ptr() if dt_in is not None else None,
                dt_out.data_ptr() if dt_out is not None else None)

    def set_launch(self, params):
        fv_set_launch(self.ctx, params)

    def get_launch(self):
        return fv_get_launch(self.ctx)

    def status(self):
        return fv_status(self.ctx)

    def set_path(self, path, seg=0, waves=0):
        """seg 0 lets the library choose the segment height (see get_path)."""
        fv_set_path(self.ctx, path, seg, waves)

    def get_path(self):
        return fv_get_path(self.ctx)

    def set_fused_launch(self, seg, waves):
        """Per-stage segment heights and wave counts of the fused path (selected first)."""
        fv_set_fused_launch(self.ctx, seg, waves)

    def get_fused_launch(self):
        return fv_get_fused_launch(self.ctx)

    def set_timing(self, enable):
        fv_set_timing(self.ctx, enable)

    def get_timing(self):
        return fv_get_timing(self.ctx)

    def clear_status(self):
        fv_clear_status(self.ctx)


class Batch:
    """Device buffers of a batch of 2D grids advanced by the fused stage kernels.

    ``U`` holds grid g's dense (4, ny, nx) state at [offsets[g], offsets[g+1]).
    """

    def __init__(self, specs, seg=0, waves=0, order=FV_ORDER_GIVEN, device="cuda"):
        torch = _torch()
        self.specs = list(specs)
        self.device = torch.device(device)
        self.offsets, self.ws_bytes = fv_batch_query(self.specs)
        self.U = torch.zeros(self.offsets[-1], dtype=torch.float64, device=self.device)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.b = fv_batch_create(self.specs, seg, waves, order, self.workspace.data_ptr(), self.ws_bytes,
                                 self.stream.cuda_stream)
        self.history = None

    def view(self, g):
        s = self.specs[g]
        return self.U[self.offsets[g]:self.offsets[g + 1]].view(4, 1, int(s.n[1]), int(s.n[0]))

    def set_states(self, states):
        torch = _torch()
        for g, st in enumerate(states):
            self.view(g).copy_(torch.as_tensor(np.ascontiguousarray(st), dtype=torch.float64))

    def get_states(self):
        return [self.view(g).cpu().numpy().copy() for g in range(len(self.specs))]

    def step(self, nsteps):
        fv_batch_step(self.b, self.U.data_ptr(), nsteps)

    def set_timing(self, max_steps):
        """Record per-step device clocks; returns ticks per microsecond."""
        torch = _torch()
        if max_steps <= 0:
            self.history = None
            return fv_batch_set_timing(self.b, None, 0)
        self.history = torch.zeros(max_steps * len(self.specs) * 6, dtype=torch.int64, device=self.device)
        return fv_batch_set_timing(self.b, self.history.data_ptr(), max_steps)

    def clocks(self):
        """(steps, grids, 3 stages, 2) int64 array of (first start, last end)."""
        h = self.history.cpu().numpy()
        return h.reshape(-1, len(self.specs), 3, 2)

    def dt(self):
        torch = _torch()
        out = torch.zeros(len(self.specs), dtype=torch.float64, device=self.device)
        fv_batch_dt(self.b, out.data_ptr())
        return out.cpu().numpy()

    def info(self):
        """(segment height per grid, work-list order, work items per stage launch)."""
        return fv_batch_info(self.b, len(self.specs))

    def set_schedule(self, segs=None, order=FV_ORDER_GIVEN):
        """Segment height per grid (None keeps them) and work-list order."""
        if segs is not None and len(segs) != len(self.specs):
            raise ValueError("one segment height per grid")
        fv_batch_set_schedule(self.b, segs, order)

    def status(self):
        return fv_batch_status(self.b)

    def close(self):
        if getattr(self, "b", None):
            fv_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
