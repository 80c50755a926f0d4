"""Host-side checks of the 14-parameter launch space."""
import numpy as np
import pytest

from oracle import mlp
from paper_2306_14011_amd.tune_space import GANG_PAIRS, STENCIL_PAIRS, LaunchSpace


def test_pair_counts_and_space_sizes():
    assert len(STENCIL_PAIRS) == 22 and len(GANG_PAIRS) == 25
    assert all(w <= t for w, t in STENCIL_PAIRS)
    assert LaunchSpace(2).size == 22 ** 2 * 25 ** 4 == 189_062_500
    assert LaunchSpace(3).size == 22 ** 3 * 25 ** 4 == 4_159_375_000


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
    vecs = [sp.decode(i) for i in idx]
    # gang 0 (one thread per element) is encoded as 2^17 before the log
    enc = np.asarray(vecs, dtype=float)
    enc[enc == 0] = 2.0 ** 17
    mean, std = mlp.standard_scaler(np.log2(enc))
    f1, f2 = sp.tables(mean, std)
    direct = mlp.features(enc, mean, std)
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
