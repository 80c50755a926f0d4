"""The network kernels (FP32, through the C ABI) against the FP64 oracle, and
the tuning method on a synthetic cost with a known optimum."""
import math

import numpy as np
import pytest

from oracle import mlp
from paper_2306_14011_amd import inputs
from paper_2306_14011_amd.autotune import target_scaler
from paper_2306_14011_amd.tune_space import LaunchSpace

pytestmark = pytest.mark.gpu


def problem(n=225, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 14)).astype(np.float32).astype(np.float64)
    y = 1.0 + 0.3 * np.sin(X[:, 0]) + 0.2 * X[:, 3] * X[:, 5] + 0.05 * rng.standard_normal(n)
    return X, y


def net(seed):
    from paper_2306_14011_amd.autotune import Network
    return Network(seed)


def f32(theta):
    return theta.astype(np.float32).astype(np.float64)


def test_loss_and_gradient_match_oracle():
    X, y = problem()
    N = net(3)
    theta = N.params.cpu().numpy().astype(np.float64)
    assert np.array_equal(theta, f32(inputs.mlp_init(3)))
    for alpha in (0.0, 1e-4, 0.5):
        L, g = N.loss_grad(X, y, alpha)
        Lr, gr = mlp.loss_grad(theta, X, y, alpha)
        assert abs(L - Lr) <= 1e-5 * abs(Lr)
        assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
        assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max()


def test_predict_matches_oracle():
    X, _ = problem(1000, 1)
    N = net(4)
    theta = N.params.cpu().numpy().astype(np.float64)
    out = N.predict(X)
    ref = mlp.predict(theta, X)
    assert np.abs(out - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def test_first_adam_step_closed_form():
    X, y = problem(150, 2)
    N = net(5)
    theta = N.params.cpu().numpy().astype(np.float64)
    _, gr = mlp.loss_grad(theta, X, y, 1e-4)
    N.train(X, y, order=inputs.epoch_orders(150, 1, 0), max_epochs=1, batch=200)
    step = N.params.cpu().numpy().astype(np.float64) - theta
    expect = -9e-4 * gr / (np.abs(gr) + 1e-9 / math.sqrt(1 - 0.90))
    big = np.abs(gr) > 1e-3 * np.abs(gr).max()   # sign of tiny gradients is FP32 noise
    assert big.sum() > 1000
    assert np.allclose(step[big], expect[big], rtol=2e-3, atol=1e-9)
    assert int(N.t.item()) == 1


def test_training_tracks_oracle():
    X, y = problem(225, 3)
    order = inputs.epoch_orders(225, 30, 7)
    N = net(6)
    theta0 = N.params.cpu().numpy().astype(np.float64)
    losses = N.train(X, y, order=order, max_epochs=30)
    th_ref, lref, ne, _, _, _ = mlp.train(theta0, X, y, order, max_epochs=30)
    assert len(losses) == ne == 30
    assert np.allclose(losses, lref, rtol=2e-3, atol=0)
    pred = N.predict(X)
    assert np.abs(pred - mlp.predict(th_ref, X)).max() <= 1e-2 * np.abs(y).max()


def test_sweep_topk_matches_brute_force():
    sp = LaunchSpace(2)
    rng = np.random.default_rng(8)
    train_idx = sp.sample(200, 3)
    F = sp.features(train_idx)
    mean, std = mlp.standard_scaler(F)
    N = net(9)
    theta = N.params.cpu().numpy().astype(np.float64)
    begin, count = 1_234_567, 100_000
    ti, tv = N.sweep(sp.struct(mean, std), begin, count, 8)
    # oracle: FP64 predictions of every index of the window
    idx = np.arange(begin, begin + count)
    d = []
    rem = idx.copy()
    for r in sp.radix:
        d.append(rem % r)
        rem //= r
    f1, f2 = sp.tables(mean, std)
    Xw = np.zeros((count, 14))
    for s in range(7):
        Xw[:, 2 * s] = np.asarray(f1[s], dtype=np.float32)[d[s]]
        Xw[:, 2 * s + 1] = np.asarray(f2[s], dtype=np.float32)[d[s]]
    pred = mlp.predict(theta, Xw)
    order = np.argsort(pred, kind="stable")
    scale = np.abs(pred).max()
    assert all(begin <= i < begin + count for i in ti)
    assert list(tv) == sorted(tv)
    # values agree with the 8 lowest oracle predictions; each returned index is
    # within FP32 roundoff of the oracle's prediction for it
    assert np.allclose(tv, pred[order[:8]], rtol=0, atol=2e-5 * scale)
    for i, v in zip(ti, tv):
        assert abs(pred[i - begin] - v) <= 2e-5 * scale
    assert abs(pred[ti[0] - begin] - pred[order[0]]) <= 2e-5 * scale


def synthetic_cost(sp, idx, rng=None, noise=0.02):
    """Separable quadratic in the raw features plus two pairwise terms (sites 3-4 and 5-6)."""
    L = sp.features(idx)
    opt = np.array([5, 8, 6, 8, 6, 8, 1, 9, 2, 7, 0, 8, 3, 9], dtype=float)
    w = np.array([0.3, 0.2, 0.25, 0.15, 0.0, 0.0, 0.1, 0.2, 0.15, 0.1, 0.05, 0.05, 0.1, 0.1])
    c = 1.0 + (w * (L - opt) ** 2).sum(axis=1)
    c += 0.05 * (L[:, 6] - L[:, 8]) ** 2 + 0.04 * (L[:, 11] - L[:, 13]) ** 2
    if rng is not None:
        c *= 1.0 + noise * rng.standard_normal(len(c))
    return c


def synthetic_optimum(sp):
    """Exact minimum of synthetic_cost over the space: sites 0 and 1 are
    independent, sites (3, 4) and (5, 6) are coupled pairwise and searched
    jointly, site 2 is pinned."""
    def index_of(choice):
        idx_ = 0
        mul = 1
        for s in range(7):
            idx_ += choice[s] * mul
            mul *= sp.radix[s]
        return idx_
    choice = [0] * 7
    for s in (0, 1):
        cs = [synthetic_cost(sp, [index_of(choice[:s] + [c] + choice[s + 1:])])[0] for c in range(sp.radix[s])]
        choice[s] = int(np.argmin(cs))
    for s1, s2 in ((3, 4), (5, 6)):
        best_c, best_v = None, np.inf
        for c1 in range(sp.radix[s1]):
            for c2 in range(sp.radix[s2]):
                ch = list(choice)
                ch[s1], ch[s2] = c1, c2
                v = synthetic_cost(sp, [index_of(ch)])[0]
                if v < best_v:
                    best_c, best_v = (c1, c2), v
        choice[s1], choice[s2] = best_c
    return synthetic_cost(sp, [index_of(choice)])[0]


def test_tuner_at_300_samples_ranks_unseen_configurations():
    # 300 timed samples (225 training rows) is the budget the measured tuner
    # runs with. On this 14-D synthetic cost the fit is then partial (the FP64
    # network trained on the same rows reaches R^2 0.64): good enough to rank
    # unseen configurations, so its pick from a pool of 4e5 unseen random ones
    # beats the best of the 300 samples, but not to trust its minimum over all
    # 1.9e8 points, where its extrapolation errors dominate. The exhaustive
    # sweep is checked at the paper's budget in the next test.
    sp = LaunchSpace(2)
    rng = np.random.default_rng(11)
    idx = sp.sample(300, 21)
    t = synthetic_cost(sp, idx, rng)
    tr = np.arange(225)
    F = sp.features(idx)
    mean, std = mlp.standard_scaler(F[tr])
    t_mean, t_std = target_scaler(t[tr])
    X = (F - mean) / std
    y = (t - t_mean) / t_std
    N = net(12)
    N.train(X[tr], y[tr])
    from paper_2306_14011_amd.autotune import r2_score
    r2 = r2_score(y[225:], N.predict(X[225:]))
    pool = sp.sample(400_000, 5)
    pool_cost = synthetic_cost(sp, pool)
    pred = N.predict((sp.features(pool) - mean) / std)
    top = np.argsort(pred, kind="stable")[:8]
    best_tuned = pool_cost[top].min()
    best_random = synthetic_cost(sp, idx).min()
    share_tuned = float((pool_cost < best_tuned).mean())
    share_random = float((pool_cost < best_random).mean())
    info = dict(r2=r2, best_tuned=best_tuned, best_random=best_random, share_tuned=share_tuned,
                share_random=share_random)
    print(info)
    assert r2 > 0.55, info
    assert best_tuned < best_random, info
    assert share_tuned * 4 <= share_random, info


@pytest.mark.xfail(strict=True, reason="the known-optimum target (within 5% at 300 samples) is not met by the "
                   "paper's training budget: measured 2.42x the optimum, best random sample 2.28x")
def test_tuner_at_300_samples_against_the_known_optimum():
    """The known-optimum pin at the measured budget: 300 timed samples (225
    training rows), the whole 1.9e8-point space swept, the best of the 8
    lowest predictions, asserted against the target of landing within 5% of
    the optimum. The target is NOT met: with the paper's minibatch of 200 and
    at most 200 epochs, 225 rows give at most 400 Adam steps at lr 9e-4, the
    fit stays partial (R^2 about 0.6) and the exhaustive minimum lands among
    the network's extrapolation errors (measured 2.42x the optimum, against
    2.28x for the best of the 300 random samples). The test is a strict
    expected failure: it records the miss and fails if the method starts
    meeting the target without the record being updated."""
    sp = LaunchSpace(2)
    rng = np.random.default_rng(11)
    idx = sp.sample(300, 21)
    t = synthetic_cost(sp, idx, rng)
    tr = np.arange(225)
    F = sp.features(idx)
    mean, std = mlp.standard_scaler(F[tr])
    t_mean, t_std = target_scaler(t[tr])
    X = (F - mean) / std
    y = (t - t_mean) / t_std
    N = net(12)
    N.train(X[tr], y[tr])
    ti, _ = N.sweep(sp.struct(mean, std), 0, sp.size, 8)
    best_tuned = synthetic_cost(sp, ti).min()
    best_random = synthetic_cost(sp, idx).min()
    optimum = synthetic_optimum(sp)
    info = dict(tuned_over_optimum=best_tuned / optimum, random_over_optimum=best_random / optimum)
    print(info)
    assert best_tuned <= 1.05 * optimum, info


def test_tuner_with_the_papers_sample_budget_lands_near_the_optimum():
    # The paper trains on 7500 of 10000 samples (Sec. "Results"). The synthetic
    # cost is free to evaluate, so that budget is affordable here: with it the
    # fit is close (R^2 0.98 for the FP64 network on the same rows) and
    # the best of the 8 predicted configurations lies within 15% of the true
    # optimum (the FP64 network's exhaustive argmin lands at 1.10x).
    sp = LaunchSpace(2)
    rng = np.random.default_rng(11)
    idx = sp.sample(10_000, 21)
    t = synthetic_cost(sp, idx, rng)
    tr = np.arange(7500)
    F = sp.features(idx)
    mean, std = mlp.standard_scaler(F[tr])
    t_mean, t_std = target_scaler(t[tr])
    X = (F - mean) / std
    y = (t - t_mean) / t_std
    N = net(12)
    N.train(X[tr], y[tr])
    from paper_2306_14011_amd.autotune import r2_score
    r2 = r2_score(y[7500:], N.predict(X[7500:]))
    ti, _ = N.sweep(sp.struct(mean, std), 0, sp.size, 8)
    best_tuned = synthetic_cost(sp, ti).min()
    best_random = synthetic_cost(sp, idx).min()
    optimum = synthetic_optimum(sp)
    info = dict(r2=r2, best_tuned=best_tuned, best_random=best_random)
    print(info)
    assert r2 > 0.95, info
    assert best_tuned <= 1.15 * optimum, info
    assert best_tuned < best_random, info


def test_end_to_end_tuning_on_a_small_grid():
    # the whole loop on a 256^2 vortex with a reduced budget: every sampled
    # launch is bitwise valid, the network is trained and the sweep covers the space
    from paper_2306_14011_amd.autotune import Autotuner
    g, U0 = inputs.vortex_bumps_case(256, seed=1)
    at = Autotuner(g, U0, seed=2, repeats=1, warmup=1, min_ms=2.0)
    res = at.run(count=40, k=4, rounds=1)
    at.close()
    assert res["n_samples"] == 40 and res["n_valid"] == 40
    assert res["n_train"] == 30 and res["n_test"] == 10
    assert res["space_size"] == 189_062_500
    assert res["tuned_ms"] > 0 and res["default_ms"] > 0


def test_batch_schedule_tuning_end_to_end():
    # the same loop on a batch schedule: every sampled schedule is bitwise valid,
    # the space is the segment height per populated size bucket times the order
    from paper_2306_14011_amd.autotune import BatchAutotuner
    from paper_2306_14011_amd.tune_space import BATCH_SEGS, BatchSpace
    spec = inputs.batch_case(count=12, seed=2, smin=128, smax=1024)
    sp = BatchSpace(spec.grids)
    populated = len(set(sp.bucket))
    assert sp.size == len(BATCH_SEGS) ** populated * 2
    at = BatchAutotuner(spec.grids, spec.states, seed=1, steps=3, warmup=1)
    res = at.run(count=40, k=4, rounds=1)
    at.close()
    assert res["n_samples"] == 40 and res["n_valid"] == 40
    assert res["tuned_ms"] > 0 and res["default_ms"] > 0
    segs, order = res["tuned"]
    assert len(segs) == len(spec.grids) and order in (0, 1)
    # the shipped schedule is the fastest of the default, the network's pick and
    # the best random sample under the interleaved timing
    assert res["shipped_from"] in ("default", "network", "best_random")
    assert res["tuned_ms"] == min(res["default_ms"], res["network_ms"], res["best_random_ms"])
    if res["shipped_from"] != "default":
        assert all(sg in BATCH_SEGS for sg in segs)
    net_segs, _ = res["network_schedule"]["seg_per_bucket"], res["network_schedule"]["order"]
    assert all(sg in BATCH_SEGS for sg in net_segs.values())
