"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/*.h declares, and validates descriptions and launch tables
without touching a GPU. Also checks that the oracle and the product path
share no code."""
import ctypes
import glob
import os
import re

import pytest

from paper_2306_14011_amd import fv, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(fv_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("fv_query", "fv_create", "fv_destroy", "fv_residual", "fv_step",
                     "fv_adjoint_step", "fv_set_launch", "fv_get_launch", "fv_status"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(fv.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_query_strides_and_workspace():
    g = inputs.grid2d(64, 64)
    strides, ws = fv.fv_query(fv.make_desc(g))
    sx, sy, sz, sv = strides
    assert sx == 1 and sy >= 64 + 4 and sy % 8 == 0
    assert sz == sy * (64 + 4) and sv == sz
    assert ws > 0
    g3 = inputs.grid3d(10, 12, 14)
    sx, sy, sz, sv = fv.fv_query(fv.make_desc(g3))[0]
    assert sy >= 14 and sz == sy * 16 and sv == sz * 18


@pytest.mark.parametrize("mutate", [
    lambda d: setattr(d, "ndim", 4),
    lambda d: d.n.__setitem__(0, 0),
    lambda d: d.n.__setitem__(2, 3),            # 2D with nz != 1
    lambda d: d.bc[0].__setitem__(0, 1),        # periodic on one face only
    lambda d: d.bc[1].__setitem__(1, 7),        # unknown kind
    lambda d: setattr(d, "gamma", 1.0),
    lambda d: setattr(d, "cfl", 0.0),
    lambda d: setattr(d, "scheme", 7),
    lambda d: setattr(d, "scheme", -1),
    lambda d: d.hi.__setitem__(0, d.lo[0]),
])
def test_query_rejects_invalid_descriptions(mutate):
    d = fv.make_desc(inputs.grid2d(16, 16))
    mutate(d)
    with pytest.raises(fv.FvError) as e:
        fv.fv_query(d)
    assert e.value.code == fv.FV_EINVAL
    assert fv.fv_last_error()


def test_schemes_of_the_muscl_family():
    """Every FV_SCHEME_* is accepted; a spec maps to the scheme of its limiter
    and kappa (with the limiter on, kappa does not matter: minmod collapses
    the kappa terms), and kappas outside the family are refused on the host."""
    g = inputs.grid2d(16, 16)
    for code in (fv.FV_SCHEME_MINMOD, fv.FV_SCHEME_UNLIMITED, fv.FV_SCHEME_FROMM, fv.FV_SCHEME_THIRD,
                 fv.FV_SCHEME_CENTRAL, fv.FV_SCHEME_VANLEER, fv.FV_SCHEME_QUICK):
        d = fv.make_desc(g)
        d.scheme = code
        fv.fv_query(d)
    assert fv.scheme_of(g) == fv.FV_SCHEME_MINMOD
    for kappa, code in ((-1.0, fv.FV_SCHEME_UNLIMITED), (0.0, fv.FV_SCHEME_FROMM), (1.0 / 3.0, fv.FV_SCHEME_THIRD),
                        (0.5, fv.FV_SCHEME_QUICK), (1.0, fv.FV_SCHEME_CENTRAL)):
        g.limiter, g.kappa = False, kappa
        assert fv.scheme_of(g) == code
        g.limiter = True
        assert fv.scheme_of(g) == fv.FV_SCHEME_MINMOD
    g.limiter, g.kappa = "vanleer", 1.0
    assert fv.scheme_of(g) == fv.FV_SCHEME_VANLEER
    g.limiter, g.kappa = False, 0.25
    with pytest.raises(ValueError):
        fv.make_desc(g)
    for code in (-1, fv.FV_SCHEME_QUICK + 1):
        d = fv.make_desc(inputs.grid2d(16, 16))
        d.scheme = code
        with pytest.raises(fv.FvError):
            fv.fv_query(d)
    g.limiter = "superbee"
    with pytest.raises(ValueError):
        fv.make_desc(g)


def test_query_rejects_oversized_grid():
    d = fv.make_desc(inputs.grid3d(1400, 1400, 1400))
    with pytest.raises(fv.FvError):
        fv.fv_query(d)


def test_default_launch():
    p = fv.fv_default_launch()
    assert p[:6] == [64, 256] * 3
    assert p[6:] == [0, 256] * 4


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(fv, "_lib", None)
    monkeypatch.setattr(fv, "LIB_PATH", "/nonexistent/libfv.so")
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        fv.lib()


def _sources(pattern):
    return [p for p in glob.glob(os.path.join(ROOT, pattern), recursive=True)]


def test_oracle_and_product_share_nothing():
    for path in _sources("oracle/**/*.py") + _sources("oracle/**/*.cpp"):
        text = open(path).read()
        assert not re.search(r"^\s*(from|import)\s+paper_2306_14011_amd", text, re.M), path
        assert "fv.h" not in text and "csrc" not in text, path
    for path in _sources("paper_2306_14011_amd/**/*.py") + _sources("paper_2306_14011_amd/csrc/*"):
        text = open(path).read()
        assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), path
        assert "liboracle" not in text and "fv_oracle" not in text, path


def test_batch_query_offsets_and_validation():
    grids = [inputs.grid2d(30, 20), inputs.grid2d(7, 1, bc=((1, 1), (0, 0))), inputs.grid2d(128, 64)]
    offs, ws = fv.fv_batch_query(grids)
    assert offs == [0, 4 * 600, 4 * 600 + 4 * 7, 4 * 600 + 28 + 4 * 128 * 64]
    assert ws > 2 * 8 * offs[-1]   # two stage states plus tables
    with pytest.raises(fv.FvError) as e:
        fv.fv_batch_query([inputs.grid2d(8, 8), inputs.grid3d(4, 4, 4)])
    assert e.value.code == fv.FV_ENOTSUP
    bad = inputs.grid2d(8, 8)
    bad.cfl = -1.0
    with pytest.raises(fv.FvError) as e:
        fv.fv_batch_query([bad])
    assert e.value.code == fv.FV_EINVAL
    # one grid's state must stay below 4 GiB: 2^27 cells is the first size refused
    fv.fv_batch_query([inputs.grid2d(8192, 16383)])
    with pytest.raises(fv.FvError) as e:
        fv.fv_batch_query([inputs.grid2d(8192, 16384)])
    assert e.value.code == fv.FV_EINVAL and "4 GiB" in str(e.value)   # the library's own message
    # slip walls, inflow faces and viscosity are taken, curvilinear grids are not
    walled = inputs.grid2d(8, 8, bc=((2, 2), (2, 1)))
    visc = inputs.grid2d(8, 8)
    visc.mu, visc.prandtl = 0.01, 0.72
    fv.fv_batch_query([walled, visc])
    for mutate in (lambda d: setattr(d, "prandtl", 0.0), lambda d: setattr(d, "mu", -1.0)):
        v2 = inputs.grid2d(8, 8)
        v2.mu, v2.prandtl = 0.01, 0.72
        mutate(v2)
        with pytest.raises(fv.FvError):
            fv.fv_batch_query([v2])
    thin = inputs.grid2d(8, 1, bc=((0, 0), (2, 2)))   # a wall on an axis of one cell
    with pytest.raises(fv.FvError):
        fv.fv_batch_query([thin])
    inflow = inputs.grid2d(8, 8, bc=((3, 1), (0, 0)))   # an inflow face without a physical state
    with pytest.raises(fv.FvError):
        fv.fv_batch_query([inflow])



def test_mlp_entry_points_reject_other_input_widths():
    # validated before any device work: non-null dummy pointers are never touched
    L = fv.lib()
    p = 256
    for n_in in (0, 13, 15, 17):
        assert L.fv_mlp_predict(p, n_in, p, 10, p, None) == fv.FV_EINVAL
        assert L.fv_mlp_loss_grad(p, n_in, p, p, 10, 0.0, p, p, p, 1 << 30, None) == fv.FV_EINVAL
        hp = fv.fv_mlp_hparams(1e-3, 0.9, 0.9, 1e-8, 0.0, 0.0, 10, 1, 1, 0)
        assert L.fv_mlp_train(p, n_in, p, p, p, p, p, 10, p, hp, p, p, p, 1 << 30, None) == fv.FV_EINVAL
    sp = fv.fv_tune_space()
    for s in range(fv.NSITES):
        sp.radix[s] = 1
    for n_extra in (1, 3, -1):
        sp.n_extra = n_extra
        assert L.fv_mlp_sweep(p, sp, 0, 1, 1, p, p, p, 1 << 30, None) == fv.FV_EINVAL
    assert fv.fv_mlp_nparam(fv.FV_MLP_IN) == fv.FV_MLP_NPARAM
    assert fv.fv_mlp_nparam(fv.FV_MLP_IN_SIZED) == fv.FV_MLP_NPARAM_SIZED


def test_slip_walls_accepted_with_two_cells_or_more():
    W = fv.FV_BC_WALL
    fv.fv_query(fv.make_desc(inputs.grid2d(16, 2, bc=((W, W), (W, W)))))
    fv.fv_query(fv.make_desc(inputs.grid2d(16, 9, bc=((W, fv.FV_BC_TRANSMISSIVE), (0, 0)))))
    for g in (inputs.grid2d(16, 1, bc=((0, 0), (W, W))), inputs.grid2d(16, 9, bc=((3, W), (0, 0)))):
        with pytest.raises(fv.FvError) as e:
            fv.fv_query(fv.make_desc(g))
        assert e.value.code == fv.FV_EINVAL


def test_inflow_state_must_be_physical():
    import dataclasses

    import numpy as np
    I = fv.FV_BC_INFLOW
    st = np.zeros((3, 2, 4))
    st[0, 0] = [1.0, 2.0, 0.1, 5.0]           # p = 0.4 * (5 - 0.5 * 4.01) > 0
    g = dataclasses.replace(inputs.grid2d(16, 9, bc=((I, 1), (0, 0))), bc_state=st)
    fv.fv_query(fv.make_desc(g))
    for bad in ([0.0, 2.0, 0.1, 5.0], [1.0, 2.0, 0.1, 1.0]):   # no density; negative pressure
        st2 = st.copy()
        st2[0, 0] = bad
        with pytest.raises(fv.FvError) as e:
            fv.fv_query(fv.make_desc(dataclasses.replace(g, bc_state=st2)))
        assert e.value.code == fv.FV_EINVAL
