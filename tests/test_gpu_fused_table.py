"""The fused path's per-stage launch table (segment height and wave count of
each Runge-Kutta stage): every table gives the same bits in 2D and 3D, bad
entries are refused without changing the table, and the paper's tuning loop
runs end to end on it (FusedAutotuner: timed samples, network, sweep, the
fastest of default / network pick / best random sample shipped)."""
import numpy as np
import pytest

import oracle
from paper_2306_14011_amd import inputs

pytestmark = pytest.mark.gpu


def run_table(g, U0, steps, seg, waves):
    import torch
    from paper_2306_14011_amd import fv
    s = fv.Solver(g)
    s.set_path(fv.FV_PATH_FUSED, 0, 0)
    if seg is not None:
        s.set_fused_launch(seg, waves)
    s.set_state(U0)
    dts = torch.zeros(steps, dtype=torch.float64, device="cuda")
    s.step(steps, dt_out=dts)
    rc, flags = s.status()
    table = s.get_fused_launch()
    out = s.get_state()
    s.close()
    assert flags == 0
    return out, dts.cpu().numpy(), table


def test_stage_tables_bitwise_equal_2d():
    g, U0 = inputs.vortex_bumps_case(197, seed=4)
    base, dts, table = run_table(g, U0, 3, None, None)
    assert len(table[0]) == 3 and all(sg > 0 for sg in table[0])
    for seg, waves in (([4, 8, 12], [0, 0, 0]), ([24, 8, 40], [7, 0, 300]), ([64, 64, 4], [1, 2, 3]),
                       ([0, 16, 0], [0, 50, 0])):
        got, d2, tab = run_table(g, U0, 3, seg, waves)
        assert np.array_equal(got, base) and np.array_equal(d2, dts), (seg, waves)
        assert tab[1] == waves and all(a == b for a, b in zip(tab[0], seg) if b)
    ref, rdts, _ = oracle.run(g, U0, 3)
    for v in range(4):
        assert np.abs(base[v] - ref[v]).max() <= 1e-11 * np.abs(ref[v]).max()


def test_stage_tables_bitwise_equal_3d():
    g = inputs.grid3d(37, 20, 13)
    U0 = inputs.sod_state(g, inputs.sod_rotated_normal(5), (0.5, 0.5, 0.5))
    base, dts, _ = run_table(g, U0, 2, None, None)
    for seg, waves in (([4, 8, 12], [0, 0, 0]), ([16, 4, 8], [5, 9, 0]), ([0, 0, 4], [4, 0, 12])):
        got, d2, _ = run_table(g, U0, 2, seg, waves)
        assert np.array_equal(got, base) and np.array_equal(d2, dts), (seg, waves)


def test_bad_tables_are_refused():
    from paper_2306_14011_amd import fv
    g, U0 = inputs.vortex_case(64, seed=0)
    s = fv.Solver(g)
    with pytest.raises(fv.FvError):           # the fused path is not selected
        s.set_fused_launch([8, 8, 8], [0, 0, 0])
    s.set_path(fv.FV_PATH_FUSED, 0, 0)
    s.set_fused_launch([8, 12, 16], [0, 64, 128])
    for seg, waves in (([8, 6, 16], [0, 0, 0]), ([8, 8, 2048], [0, 0, 0]), ([8, 8, 8], [0, -1, 0])):
        with pytest.raises(fv.FvError):
            s.set_fused_launch(seg, waves)
        assert s.get_fused_launch() == ([8, 12, 16], [0, 64, 128])
    assert fv.fv_fused_slots(s.ctx) >= 4 * 256
    s.close()


def test_fused_tuning_loop_end_to_end():
    from paper_2306_14011_amd.autotune import FusedAutotuner
    from paper_2306_14011_amd.tune_space import FUSED_SEGS
    g, U0 = inputs.vortex_bumps_case(512, seed=1)
    at = FusedAutotuner(g, U0, seed=3, repeats=1, warmup=1, min_ms=5.0, check_steps=1)
    res = at.run(count=48, k=4, rounds=2)
    at.close()
    assert res["n_samples"] == 48 and res["n_valid"] == 48   # every table gives the default's bits
    assert res["space_size"] == 32 ** 3
    assert res["shipped_from"] in ("default", "network", "best_random")
    assert res["tuned_ms"] == min(res["default_ms"], res["network_ms"], res["best_random_ms"])
    net = res["network_launch"]
    assert all(net[2 * st] in FUSED_SEGS for st in range(3))


def _auto_seg_rule(nx, ny, slots):
    # the library's choice of the 2D segment height, restated: the multiple
    # of 4 up to 24 rows (16 when 24-row items fill the resident waves more
    # than twice) that minimises rounds x (rows + 1), ties to the taller
    strips = -(-nx // 60)

    def items(seg):
        return strips * (-(-ny // seg))

    max_seg = 16 if items(24) > 2 * slots else 24
    best, best_cost = 16, None
    for seg in range(4, max_seg + 1, 4):
        cost = (-(-items(seg) // slots)) * (seg + 1)
        if best_cost is None or cost <= best_cost:
            best, best_cost = seg, cost
    return best


def test_automatic_segment_height():
    from paper_2306_14011_amd import fv
    got = {}
    for nx, ny in ((64, 64), (300, 70), (2048, 2048), (4096, 4096)):
        s = fv.Solver(inputs.grid2d(nx, ny))
        s.set_path(fv.FV_PATH_FUSED, 0, 0)
        slots = fv.fv_fused_slots(s.ctx)
        got[nx] = s.get_path()[1]
        s.close()
        assert got[nx] == _auto_seg_rule(nx, ny, slots), (nx, ny, slots, got[nx])
    # on a full MI355X (3072 wave slots): 24 rows at 2048^2, 16 at 4096^2
    if slots == 3072:
        assert got[2048] == 24 and got[4096] == 16
