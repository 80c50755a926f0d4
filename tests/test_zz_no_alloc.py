"""fv_mlp_sweep_static (the sweep without a workspace, its scratch in a static
device array) against fv_mlp_sweep with a caller workspace: the same top-k
indices and values, bit for bit, on two calls in a row, the second over a
smaller range of the space, with both network widths."""
import numpy as np
import pytest

from paper_2306_14011_amd import fv
from paper_2306_14011_amd.autotune import Network
from paper_2306_14011_amd.tune_space import LaunchSpace

pytestmark = pytest.mark.gpu


def sweep_both(N, sp, begin, count, k):
    import torch
    ws_bytes = fv.fv_mlp_sweep_workspace()
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = []
    for static in (False, True):
        ti = torch.full((k,), -1, dtype=torch.int64, device="cuda")
        tv = torch.full((k,), float("nan"), dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        if static:
            fv.fv_mlp_sweep_static(N.params.data_ptr(), sp, begin, count, k, ti.data_ptr(), tv.data_ptr(), stream)
        else:
            fv.fv_mlp_sweep(N.params.data_ptr(), sp, begin, count, k, ti.data_ptr(), tv.data_ptr(), ws.data_ptr(),
                            ws_bytes, stream)
        torch.cuda.synchronize()
        out.append((ti.cpu().numpy(), tv.cpu().numpy()))
    return out


@pytest.mark.parametrize("sized", [False, True])
def test_static_sweep_matches_workspace_sweep(sized):
    sp = LaunchSpace(2)
    n_in = fv.FV_MLP_IN_SIZED if sized else fv.FV_MLP_IN
    N = Network(21, n_in=n_in)
    F = sp.features(sp.sample(500, 3))
    mean, std = F.mean(axis=0), F.std(axis=0)
    std = np.where(std == 0.0, 1.0, std)
    if sized:
        st = sp.struct(np.concatenate([mean, [14.0, 2.5]]), np.concatenate([std, [2.0, 0.5]]), [16.0, 2.0])
    else:
        st = sp.struct(mean, std)
    # a large range first (the block count at the scratch's capacity), then a
    # smaller one that leaves most of the first call's lists in the array
    for begin, count, k in ((0, sp.size, 8), (12345, 70_000, 5)):
        (i0, v0), (i1, v1) = sweep_both(N, st, begin, count, k)
        assert np.array_equal(i0, i1), (begin, count, i0, i1)
        assert np.array_equal(v0.view(np.uint32), v1.view(np.uint32)), (begin, count, v0, v1)
        assert ((i0 >= begin) & (i0 < begin + count)).all()
        assert np.all(np.diff(v0) >= 0)


def test_static_sweep_rejects_what_the_workspace_sweep_rejects():
    import torch
    sp = LaunchSpace(2)
    N = Network(22)
    st = sp.struct(np.zeros(14), np.ones(14))
    ti = torch.zeros(9, dtype=torch.int64, device="cuda")
    tv = torch.zeros(9, dtype=torch.float32, device="cuda")
    L = fv.lib()
    s = torch.cuda.current_stream().cuda_stream
    p = N.params.data_ptr()
    import ctypes
    assert L.fv_mlp_sweep_static(ctypes.c_void_p(p), ctypes.byref(st), 0, 100, 9, ctypes.c_void_p(ti.data_ptr()),
                                 ctypes.c_void_p(tv.data_ptr()), ctypes.c_void_p(s)) == fv.FV_EINVAL
    assert L.fv_mlp_sweep_static(ctypes.c_void_p(p), ctypes.byref(st), sp.size - 10, 100, 8,
                                 ctypes.c_void_p(ti.data_ptr()), ctypes.c_void_p(tv.data_ptr()),
                                 ctypes.c_void_p(s)) == fv.FV_EINVAL
