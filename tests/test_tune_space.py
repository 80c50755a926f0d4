"""Host-side checks of the 14-parameter launch space."""
import math

import numpy as np
import pytest

from oracle import mlp
from paper_2306_14011_amd import inputs
from paper_2306_14011_amd.tune_space import STENCIL_PAIRS, LaunchSpace, gang_for, site_elements


def test_pair_counts_and_space_sizes():
    assert len(STENCIL_PAIRS) == 22
    assert all(w <= t for w, t in STENCIL_PAIRS)
    assert LaunchSpace(2).size == 22 ** 2 * 25 ** 4 == 189_062_500
    assert LaunchSpace(3).size == 22 ** 3 * 25 ** 4 == 4_159_375_000


def test_gang_is_relative_to_the_problem_size():
    # about e elements per thread: gang * threads * e ~ N, rounded to a power of two
    assert gang_for(2048 * 2048, 256, 1) == 0
    assert gang_for(2048 * 2048, 256, 4) == 4096
    assert gang_for(256 ** 3, 1024, 2) == 8192
    assert gang_for(10, 1024, 16) == 1
    assert gang_for(1 << 30, 64, 2) == 65536
    g = inputs.grid3d(256, 256, 256)
    counts = site_elements(g)
    assert counts[3] == 256 ** 3 and counts[5] == 3 * 4 * 256 * 256
    sp = LaunchSpace.for_grid(g)
    for s in (3, 4, 5, 6):
        for (gang, t), (le, lt) in zip(sp.choices[s], sp.feats[s]):
            assert 2 ** lt == t
            if le == 0:
                assert gang == 0
            else:
                assert 0.5 <= counts[s] / (gang * t * 2 ** le) <= 2.0 or gang in (1, 65536)


def test_default_launch_is_in_the_space():
    from paper_2306_14011_amd import fv
    d = fv.fv_default_launch()
    for nd in (2, 3):
        sp = LaunchSpace(nd)
        assert sp.decode(sp.encode(d)) == d


@pytest.mark.parametrize("ndim", [2, 3])
def test_decode_encode_round_trip(ndim):
    sp = LaunchSpace(ndim)
    rng = np.random.default_rng(0)
    for idx in [0, 1, sp.size - 1] + [int(i) for i in rng.integers(0, sp.size, 300)]:
        v = sp.decode(idx)
        assert len(v) == 14 and sp.encode(v) == idx
        # digits agree with an independent mixed-radix decode
        d = mlp.decode(idx, sp.radix)
        for s in range(7):
            assert tuple(v[2 * s:2 * s + 2]) == sp.choices[s][d[s]]
    with pytest.raises(ValueError):
        sp.decode(sp.size)


def test_feature_tables_match_direct_features():
    sp = LaunchSpace(2)
    rng = np.random.default_rng(1)
    idx = [int(i) for i in rng.integers(0, sp.size, 200)]
    # raw features are log2 of (width, threads) / (elements per thread, threads)
    F = sp.features(idx)
    raw = []
    for i in idx:
        d = mlp.decode(i, sp.radix)
        row = []
        for s in range(7):
            a, b = sp.choices[s][d[s]]
            if s >= 3:
                e = 2 ** sp.feats[s][d[s]][0]
                row += [e, b]
            else:
                row += [a, b]
        raw.append(row)
    mean, std = mlp.standard_scaler(F)
    f1, f2 = sp.tables(mean, std)
    direct = mlp.features(raw, mean, std)
    for row, i in zip(direct, idx):
        d = mlp.decode(i, sp.radix)
        tab = []
        for s in range(7):
            tab += [f1[s][d[s]], f2[s][d[s]]]
        assert np.allclose(row, tab, rtol=0, atol=1e-12)


def test_sampling_is_distinct_and_seeded():
    sp = LaunchSpace(2)
    a = sp.sample(300, 5)
    assert len(set(a)) == 300 and a == sp.sample(300, 5) and a != sp.sample(300, 6)


def test_target_scaler():
    from paper_2306_14011_amd.autotune import target_scaler
    m, s = target_scaler([1.0, 2.0, 3.0, 4.0])
    assert m == 2.5 and abs(s - math.sqrt(1.25)) < 1e-15   # population sigma
    assert target_scaler([2.0, 2.0]) == (2.0, 1.0)           # zero spread leaves the target centred only


def test_batch_space_buckets_and_schedules():
    from paper_2306_14011_amd.tune_space import BATCH_SEGS, BatchSpace, batch_bucket
    g = [inputs.grid2d(n, n) for n in (128, 351, 352, 575, 576, 799, 800, 1024)]
    assert [batch_bucket(x) for x in g] == [0, 0, 1, 1, 2, 2, 3, 3]
    sp = BatchSpace(g)
    assert sp.radix == [len(BATCH_SEGS)] * 4 + [2, 1, 1] and sp.size == len(BATCH_SEGS) ** 4 * 2
    rng = np.random.default_rng(0)
    for idx in rng.integers(0, sp.size, 50):
        segs, order = sp.schedule(int(idx))
        d = sp.digits(int(idx))
        assert segs == [BATCH_SEGS[d[b]] for b in sp.bucket] and order == d[4]
    # buckets without a grid are pinned
    sp2 = BatchSpace([inputs.grid2d(200, 200), inputs.grid2d(900, 900)])
    assert sp2.radix == [len(BATCH_SEGS), 1, 1, len(BATCH_SEGS), 2, 1, 1]
    X = sp2.features(sp2.sample(20, 1))
    assert X.shape == (20, 14) and np.all(X[:, 1::2] == 0.0)


def test_problem_features():
    from paper_2306_14011_amd.tune_space import problem_features
    g2, _ = inputs.vortex_bumps_case(256, seed=0)
    assert problem_features(g2) == [16.0, 2.0]
    g3 = inputs.sod3d_case(32, seed=0)[0]
    assert problem_features(g3) == [15.0, 3.0]


def test_struct_appends_standardised_problem_features():
    from paper_2306_14011_amd.fv import FV_MLP_MAX_EXTRA
    sp = LaunchSpace(2)
    F = sp.features(sp.sample(50, 1))
    E = np.tile([18.0, 2.0], (50, 1))
    E[::2] = [22.0, 2.0]
    mean, std = mlp.standard_scaler(np.hstack([F, E]))
    s = sp.struct(mean, std, [22.0, 2.0])
    assert s.n_extra == FV_MLP_MAX_EXTRA == 2
    assert abs(s.extra[0] - 1.0) < 1e-6 and s.extra[1] == 0.0     # (22 - 20) / 2; zero spread -> 0
    s14 = sp.struct(mean[:14], std[:14])
    assert s14.n_extra == 0
    for a, b in zip(s.f1[2], s14.f1[2]):
        assert a == b
    with pytest.raises(ValueError):
        sp.struct(mean[:14], std[:14], [22.0, 2.0])


def test_grid_relative_target():
    from paper_2306_14011_amd.autotune import grid_relative_target
    # two grids 8x apart in runtime; the same relative launch effects on both
    t = np.array([1.0, 2.0, 4.0, 8.0, 16.0, 32.0])
    gid = [0, 0, 0, 1, 1, 1]
    tr = np.arange(6)
    y, (m, s), off = grid_relative_target(t, gid, tr)
    assert abs(off[0] - math.log(2.0)) < 1e-15 and abs(off[1] - math.log(16.0)) < 1e-15
    assert np.allclose(y[:3], y[3:], rtol=0, atol=1e-15)           # the size factor is gone
    assert abs(y[tr].mean()) < 1e-15 and abs(y[tr].std() - 1.0) < 1e-14
    # offsets come from the training rows only
    y2, _, off2 = grid_relative_target(t, gid, np.array([0, 1, 3, 4]))
    assert abs(off2[0] - 0.5 * math.log(2.0)) < 1e-15 and abs(off2[1] - 0.5 * math.log(128.0)) < 1e-15


def test_fused_space_tables_and_features():
    from paper_2306_14011_amd.tune_space import FUSED_SEGS, FusedSpace, fused_items
    g = inputs.grid2d(2048, 2048)
    sp = FusedSpace(g, 3072)
    assert sp.size == 32 ** 3 and sp.radix[:3] == [32, 32, 32] and sp.radix[3:] == [1, 1, 1, 1]
    # 2048^2 at segment 24: 35 strips x 86 row segments
    assert fused_items(g, 24) == 35 * 86
    for idx in sp.sample(50, 3):
        vec = sp.decode(idx)
        seg, waves = FusedSpace.table(vec)
        assert all(sg in FUSED_SEGS for sg in seg)
        assert all(w in (0, 1536, 3072, 6144) for w in waves)
        assert sp.encode(vec) == idx
    F = sp.features(sp.sample(20, 4))
    assert np.isfinite(F).all() and (F[:, 6:] == 0).all()
    # the launched waves never exceed one per item
    g3 = inputs.grid3d(256, 256, 256)
    sp3 = FusedSpace(g3, 2048)
    for c, (sg, w) in enumerate(sp3.choices[0]):
        per_item = 4 * fused_items(g3, sg)
        assert 2 ** sp3.feats[0][c][1] <= per_item + 1e-9
