"""Machine-learning autotuning of the step's launch parameters (the paper's method).

Following Sec. "Data Collection" and "Results" of the paper:
  1. draw launch vectors at random from the 14-parameter space,
  2. time the solver with each (solver time only, excluding launch set-up and
     host-device copies) and keep the valid ones,
  3. split 75 % / 25 % into training and test sets,
  4. standardise the features (mean removal, unit variance),
  5. train a fully connected ReLU network on runtime with Adam
     (Table para-setting), report R^2 (Eq. R_square) on the test set,
  6. use the network to find the configurations with the lowest predicted
     runtime; here the whole space is predicted on the GPU and the best k
     are measured again, and the fastest measured one is kept.
The network is trained and evaluated by the library's FP32 kernels
(fv_mlp_train / fv_mlp_predict / fv_mlp_sweep). This module is host-side
orchestration only. Autotuner tunes the 14 launch parameters of the split
step; BatchAutotuner applies the same loop to the schedule of a batch of
grids (segment height per grid-size bucket and work-list order);
SizedAutotuner trains one problem-size-conditioned network on the samples of
several grids and tunes each of them, and grids it was not trained on.

A sample is valid when its launch produced a state bitwise equal to the
default launch's (every launch of the split step computes identical
arithmetic) and no device flag was raised; a launch the library rejects is
recorded as invalid and left out of the training data.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import fv, inputs
from .tune_space import LaunchSpace, problem_features

# Table para-setting of the paper.
PAPER_HPARAMS = dict(lr=9e-4, beta1=0.95, beta2=0.90, eps=1e-9, alpha=1e-4, tol=1e-6, batch=200,
                     max_epochs=200, n_iter_no_change=10)


def r2_score(y, yhat):
    y = np.asarray(y, dtype=np.float64)
    yhat = np.asarray(yhat, dtype=np.float64)
    return float(1.0 - np.sum((y - yhat) ** 2) / np.sum((y - y.mean()) ** 2))


def target_scaler(t_train):
    """(mean, population sigma) of the training runtimes; the target is
    centred and scaled like the features. Measured runtimes spread by only
    10-30% around their mean, and unscaled that spread is smaller than what
    the network resolves with the paper's learning rate (on the measured 2D
    and 3D samples, test R^2 of 0.86 / 0.66 scaled against -2.6 / -3.1 for
    runtimes divided by their median, means over six splits)."""
    t_train = np.asarray(t_train, dtype=np.float64)
    sd = float(t_train.std())
    return float(t_train.mean()), (sd if sd > 0.0 else 1.0)


def grid_relative_target(t, gid, train):
    """Target of the pooled, size-conditioned fit: the log of each runtime
    relative to the geometric mean of its grid's training runtimes, then
    standardised over the training rows. Runtimes of different grids differ
    many times over while a launch moves a grid's runtime by tens of percent;
    relative to its grid, a launch's effect is the same quantity on every grid
    and the fit is spent on it rather than on the grids' sizes. Returns
    (y, (mean, sigma) of the standardisation, {grid: log offset})."""
    z = np.log(np.asarray(t, dtype=np.float64))
    gid = np.asarray(gid)
    offset = {}
    for g in sorted(set(gid.tolist())):
        rows = train[gid[train] == g]
        offset[g] = float(z[rows].mean()) if len(rows) else float(z[gid == g].mean())
        z[gid == g] -= offset[g]
    z_mean, z_std = target_scaler(z[train])
    return (z - z_mean) / z_std, (z_mean, z_std), offset


def split_indices(n: int, seed: int, train_frac=0.75):
    rng = np.random.default_rng(seed + 17)
    perm = rng.permutation(n)
    k = int(round(train_frac * n))
    return perm[:k], perm[k:]


class Network:
    """FP32 network parameters and Adam state in device memory; n_in is
    fv.FV_MLP_IN (launch features) or fv.FV_MLP_IN_SIZED (launch features and
    the two problem-size features)."""

    def __init__(self, seed: int, device="cuda", n_in: int = fv.FV_MLP_IN):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.n_in = int(n_in)
        self.params = torch.as_tensor(inputs.mlp_init(seed, self.n_in), dtype=torch.float32).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.seed = seed

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _check_rows(self, X, y=None):
        # the kernels read n_in floats per row of X and one per entry of y
        if X.dim() != 2 or X.shape[1] != self.n_in:
            raise ValueError(f"X must have shape (n, {self.n_in}), got {tuple(X.shape)}")
        if y is not None and (y.dim() != 1 or y.shape[0] != X.shape[0]):
            raise ValueError(f"y must have shape ({X.shape[0]},), got {tuple(y.shape)}")

    def train(self, X, y, order=None, **hp):
        torch = self.torch
        h = dict(PAPER_HPARAMS)
        h.update(hp)
        X = torch.as_tensor(np.ascontiguousarray(X), dtype=torch.float32).to(self.device)
        y = torch.as_tensor(np.ascontiguousarray(y), dtype=torch.float32).to(self.device)
        self._check_rows(X, y)
        n = X.shape[0]
        if order is None:
            order = inputs.epoch_orders(n, h["max_epochs"], self.seed)
        order_t = torch.as_tensor(np.ascontiguousarray(order), dtype=torch.int32).to(self.device)
        hpc = fv.fv_mlp_hparams(h["lr"], h["beta1"], h["beta2"], h["eps"], h["alpha"], h["tol"], h["batch"],
                                h["max_epochs"], h["n_iter_no_change"], 0)
        ws_bytes = fv.fv_mlp_workspace(min(h["batch"], n))
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        losses = torch.zeros(max(h["max_epochs"], 1), dtype=torch.float32, device=self.device)
        ne = torch.zeros(1, dtype=torch.int32, device=self.device)
        fv.fv_mlp_train(self.params.data_ptr(), self.n_in, self.m.data_ptr(), self.v.data_ptr(), self.t.data_ptr(),
                        X.data_ptr(), y.data_ptr(), n, order_t.data_ptr(), hpc, losses.data_ptr(), ne.data_ptr(),
                        ws.data_ptr(), ws_bytes, self._stream())
        nrun = int(ne.item())
        return losses.cpu().numpy()[:nrun]

    def loss_grad(self, X, y, alpha):
        torch = self.torch
        X = torch.as_tensor(np.ascontiguousarray(X), dtype=torch.float32).to(self.device)
        y = torch.as_tensor(np.ascontiguousarray(y), dtype=torch.float32).to(self.device)
        self._check_rows(X, y)
        n = X.shape[0]
        ws_bytes = fv.fv_mlp_workspace(n)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        g = torch.zeros_like(self.params)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        fv.fv_mlp_loss_grad(self.params.data_ptr(), self.n_in, X.data_ptr(), y.data_ptr(), n, alpha, g.data_ptr(),
                            loss.data_ptr(), ws.data_ptr(), ws_bytes, self._stream())
        return float(loss.item()), g.cpu().numpy()

    def predict(self, X):
        torch = self.torch
        X = torch.as_tensor(np.ascontiguousarray(X), dtype=torch.float32).to(self.device)
        self._check_rows(X)
        n = X.shape[0]
        out = torch.zeros(n, dtype=torch.float32, device=self.device)
        fv.fv_mlp_predict(self.params.data_ptr(), self.n_in, X.data_ptr(), n, out.data_ptr(), self._stream())
        return out.cpu().numpy()

    def sweep(self, space_struct, begin, count, k):
        torch = self.torch
        if 2 * fv.NSITES + space_struct.n_extra != self.n_in:
            raise ValueError(f"the space has {space_struct.n_extra} extra features, the network {self.n_in} inputs")
        ws_bytes = fv.fv_mlp_sweep_workspace()
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        ti = torch.zeros(k, dtype=torch.int64, device=self.device)
        tv = torch.zeros(k, dtype=torch.float32, device=self.device)
        fv.fv_mlp_sweep(self.params.data_ptr(), space_struct, begin, count, k, ti.data_ptr(), tv.data_ptr(),
                        ws.data_ptr(), ws_bytes, self._stream())
        return ti.cpu().numpy().tolist(), tv.cpu().numpy().tolist()


def fit_samples(space, samples, seed):
    """Steps 3-5 on the valid samples: 75/25 split, standardised features and
    target, network training on the GPU, R^2 on both sets."""
    good = [s for s in samples if s.valid and np.isfinite(s.ms)]
    tr, te = split_indices(len(good), seed)
    F = space.features([s.index for s in good])
    t = np.array([s.ms for s in good])
    t_mean, t_std = target_scaler(t[tr])
    y = (t - t_mean) / t_std
    mean = F[tr].mean(axis=0)
    std = F[tr].std(axis=0)
    std = np.where(std == 0.0, 1.0, std)
    X = (F - mean) / std
    net = Network(seed)
    losses = net.train(X[tr], y[tr])
    r2_test = r2_score(y[te], net.predict(X[te]))
    r2_train = r2_score(y[tr], net.predict(X[tr]))
    return dict(net=net, mean=mean, std=std, t_mean=t_mean, t_std=t_std, r2_test=r2_test, r2_train=r2_train,
                losses=losses, n_train=len(tr), n_test=len(te), good=good)


def sweep_space(space, model, k=8):
    """Step 6: the k lowest predicted indices of the whole space (GPU sweep)."""
    import torch
    sp = space.struct(model["mean"], model["std"])
    t0 = time.perf_counter()
    idx, val = model["net"].sweep(sp, 0, space.size, k)
    torch.cuda.synchronize()
    return idx, val, time.perf_counter() - t0


def shipped(final_ms, options, names=("default", "network", "best_random")):
    """The option to ship and its name: the fastest under the interleaved
    timing `final_ms` of `options` (default first, ties to the earlier
    option), so that a network pick slower than the default or the best
    random sample is reported but not shipped."""
    i = min(range(len(options)), key=lambda q: (final_ms[q], q))
    return options[i], names[i]


@dataclass
class Sample:
    index: int
    launch: list
    ms: float          # median per-step time
    valid: bool
    reps: list = field(default_factory=list)


class Autotuner:
    """Runs the paper's tuning loop on one grid through the split step."""

    def __init__(self, spec, U0, seed=0, repeats=3, warmup=3, min_ms=20.0, check_steps=2, log_path=None):
        import torch
        self.torch = torch
        self.spec = spec
        self.solver = fv.Solver(spec)
        self.space = self.make_space()
        self.U0 = U0
        self.seed = seed
        self.repeats = repeats
        self.warmup = warmup
        self.min_ms = min_ms
        self.check_steps = check_steps
        self.log_path = log_path
        self.solver.set_state(U0)
        self.U_start = self.solver.U.clone()
        self.default = self.default_launch()
        self.ref = self._reference_state(self.default)
        self.steps = 1
        t = self._time(self.default, 1, 1)
        self.steps = max(1, int(math.ceil(self.min_ms / max(t, 1e-3))))

    def make_space(self):
        return LaunchSpace.for_grid(self.spec)

    def default_launch(self):
        return fv.fv_default_launch()

    def apply_launch(self, launch):
        """Sets a launch vector of the space on the solver."""
        self.solver.set_launch(launch)

    def _reference_state(self, launch):
        s = self.solver
        self.apply_launch(launch)
        s.U.copy_(self.U_start)
        s.step(self.check_steps)
        return s.U.clone()

    def _time(self, launch, steps, repeats):
        torch = self.torch
        s = self.solver
        self.apply_launch(launch)
        stream = torch.cuda.current_stream()
        s.step(self.warmup)
        reps = []
        for _ in range(repeats):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.step(steps)
            e1.record(stream)
            e1.synchronize()
            reps.append(e0.elapsed_time(e1) / steps)
        self._last_reps = reps
        return float(np.median(reps))

    def measure(self, launch):
        """(median ms per step, valid) for one launch vector."""
        torch = self.torch
        s = self.solver
        try:
            self.apply_launch(launch)
        except fv.FvError:
            return float("nan"), False
        s.U.copy_(self.U_start)
        s.step(self.check_steps)
        valid = bool(torch.equal(s.U, self.ref))
        rc, flags = s.status()
        if flags:
            s.clear_status()
            valid = False
        s.U.copy_(self.U_start)
        ms = self._time(launch, self.steps, self.repeats)
        return ms, valid

    def collect(self, count, budget_s=None):
        """Times up to `count` seeded samples; with a time budget (seconds)
        sampling stops once it is spent and self.budget_hit records it."""
        t0 = time.perf_counter()
        self.budget_hit = False
        samples = []
        done = {}
        if self.log_path and os.path.exists(self.log_path):
            for line in open(self.log_path):
                r = json.loads(line)
                done[r["index"]] = Sample(r["index"], r["launch"], r["ms"], r["valid"], r.get("reps", []))
        for idx in self.space.sample(count, self.seed):
            if budget_s is not None and time.perf_counter() - t0 > budget_s:
                self.budget_hit = True
                break
            if idx in done:
                samples.append(done[idx])
                continue
            launch = self.space.decode(idx)
            ms, valid = self.measure(launch)
            smp = Sample(idx, launch, ms, valid, list(self._last_reps))
            samples.append(smp)
            if self.log_path:
                with open(self.log_path, "a") as f:
                    f.write(json.dumps(smp.__dict__) + "\n")
        return samples

    def fit(self, samples):
        return fit_samples(self.space, samples, self.seed)

    def sweep(self, model, k=8):
        return sweep_space(self.space, model, k)

    def interleaved(self, launches, rounds=5, steps=None):
        """Median per-step ms of each launch, timed A/B/A/B... over `rounds`."""
        steps = steps or self.steps
        res = [[] for _ in launches]
        for _ in range(rounds):
            for i, l in enumerate(launches):
                res[i].append(self._time(l, steps, 1))
        return [float(np.median(r)) for r in res]

    def run(self, count=300, k=8, rounds=5, final_steps=None, budget_s=None):
        t0 = time.perf_counter()
        samples = self.collect(count, budget_s)
        t_collect = time.perf_counter() - t0
        model = self.fit(samples)
        top_idx, top_val, t_sweep = self.sweep(model, k)
        cands = [self.space.decode(i) for i in top_idx]
        cand_ms = [self.measure(l) for l in cands]
        ok = [(ms, i) for i, (ms, v) in enumerate(cand_ms) if v]
        best = cands[min(ok)[1]] if ok else self.default
        good = model["good"]
        best_random = min(good, key=lambda s: s.ms).launch
        final = self.interleaved([self.default, best, best_random], rounds=rounds, steps=final_steps)
        ship, shipped_from = shipped(final, [self.default, best, best_random])
        return dict(
            default_launch=self.default, tuned_launch=ship, network_launch=best, best_random_launch=best_random,
            shipped_from=shipped_from, default_ms=final[0], tuned_ms=min(final), network_ms=final[1],
            best_random_ms=final[2], factor_vs_default=final[0] / min(final),
            factor_vs_best_random=final[2] / min(final), network_factor_vs_default=final[0] / final[1],
            network_factor_vs_best_random=final[2] / final[1],
            r2_test=model["r2_test"], r2_train=model["r2_train"], n_samples=len(samples),
            n_valid=len(good), n_train=model["n_train"], n_test=model["n_test"],
            epochs=len(model["losses"]), final_loss=float(model["losses"][-1]) if len(model["losses"]) else None,
            space_size=self.space.size, sweep_seconds=t_sweep, collect_seconds=t_collect,
            top_pred=[v * model["t_std"] + model["t_mean"] for v in top_val], top_measured_ms=[m for m, _ in cand_ms], steps_per_sample=self.steps,
            samples_requested=count, sampling_budget_s=budget_s, sampling_budget_hit=self.budget_hit,
        )

    def close(self):
        self.solver.close()


class FusedAutotuner(Autotuner):
    """The same loop on the fused path of one grid (the kernels the headline
    step runs): the launch surface is FusedSpace, each stage's segment height
    and wave count; the reference is the library's own table (automatic
    segment height, one wave per work item). Every table gives the same bits,
    which each sample's check confirms."""

    def make_space(self):
        from .tune_space import FusedSpace
        self.solver.set_path(fv.FV_PATH_FUSED, 0, 0)
        return FusedSpace(self.spec, fv.fv_fused_slots(self.solver.ctx))

    def default_launch(self):
        seg, waves = self.solver.get_fused_launch()
        return [seg[0], waves[0], seg[1], waves[1], seg[2], waves[2]] + [0] * 8

    def apply_launch(self, launch):
        from .tune_space import FusedSpace
        seg, waves = FusedSpace.table(launch)
        self.solver.set_fused_launch(seg, waves)


class BatchAutotuner:
    """The same method applied to the schedule of a batch of 2D grids: the
    segment height per grid-size bucket and the work-list order (BatchSpace),
    each sample timed as graph-replayed batch steps. The reference schedule is
    the library's own choice (one automatic segment height, given order)."""

    def __init__(self, grids, states, seed=0, steps=10, warmup=2, check_steps=1, log_path=None):
        import torch
        from .tune_space import BatchSpace
        self.torch = torch
        self.space = BatchSpace(grids)
        self.batch = fv.Batch(grids, seg=0, order=fv.FV_ORDER_GIVEN)
        self.batch.set_states(states)
        self.U_start = self.batch.U.clone()
        self.seed = seed
        self.steps = steps
        self.warmup = warmup
        self.check_steps = check_steps
        self.log_path = log_path
        segs, order, _ = self.batch.info()
        self.default = (list(segs), order)
        self.ref = self._run(self.default, check_steps)

    def _run(self, schedule, nsteps):
        B = self.batch
        B.set_schedule(*schedule)
        B.U.copy_(self.U_start)
        B.step(nsteps)
        return B.U.clone()

    def _time(self, schedule, steps):
        torch = self.torch
        B = self.batch
        B.set_schedule(*schedule)
        B.U.copy_(self.U_start)
        B.step(self.warmup)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.step(steps)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / steps

    def measure(self, schedule):
        """(ms per step, valid): valid when bitwise equal to the reference schedule."""
        got = self._run(schedule, self.check_steps)
        rc, flags = self.batch.status()
        valid = bool(self.torch.equal(got, self.ref)) and not flags
        return self._time(schedule, self.steps), valid

    def collect(self, count, budget_s=None):
        t0 = time.perf_counter()
        self.budget_hit = False
        samples = []
        for idx in self.space.sample(min(count, self.space.size), self.seed):
            if budget_s is not None and time.perf_counter() - t0 > budget_s:
                self.budget_hit = True
                break
            segs, order = self.space.schedule(idx)
            ms, valid = self.measure((segs, order))
            d = self.space.digits(idx)
            smp = Sample(idx, [self.space.choices[b][d[b]][0] for b in range(4)] + [order], ms, valid)
            samples.append(smp)
            if self.log_path:
                with open(self.log_path, "a") as f:
                    f.write(json.dumps(smp.__dict__) + "\n")
        return samples

    def interleaved(self, schedules, rounds=5):
        res = [[] for _ in schedules]
        for _ in range(rounds):
            for i, sc in enumerate(schedules):
                res[i].append(self._time(sc, self.steps))
        return [float(np.median(r)) for r in res]

    def run(self, count=300, k=8, rounds=5, budget_s=None):
        t0 = time.perf_counter()
        samples = self.collect(count, budget_s)
        t_collect = time.perf_counter() - t0
        model = fit_samples(self.space, samples, self.seed)
        top_idx, top_val, t_sweep = sweep_space(self.space, model, k)
        cands = [self.space.schedule(i) for i in top_idx]
        cand_ms = [self.measure(c) for c in cands]
        ok = [(ms, i) for i, (ms, v) in enumerate(cand_ms) if v]
        best = cands[min(ok)[1]] if ok else self.default
        good = model["good"]
        rnd = min(good, key=lambda s: s.ms)
        best_random = self.space.schedule(rnd.index)
        final = self.interleaved([self.default, best, best_random], rounds=rounds)
        ship, shipped_from = shipped(final, [self.default, best, best_random])
        per_bucket = lambda sc: {b: sc[0][self.space.bucket.index(b)] for b in sorted(set(self.space.bucket))}
        return dict(
            default_schedule={"seg_per_bucket": per_bucket(self.default), "order": self.default[1]},
            tuned_schedule={"seg_per_bucket": per_bucket(ship), "order": ship[1]},
            network_schedule={"seg_per_bucket": per_bucket(best), "order": best[1]},
            best_random_schedule={"seg_per_bucket": per_bucket(best_random), "order": best_random[1]},
            tuned=ship, shipped_from=shipped_from, default_ms=final[0], tuned_ms=min(final), network_ms=final[1],
            best_random_ms=final[2], factor_vs_default=final[0] / min(final),
            factor_vs_best_random=final[2] / min(final), network_factor_vs_default=final[0] / final[1],
            network_factor_vs_best_random=final[2] / final[1],
            r2_test=model["r2_test"], r2_train=model["r2_train"], n_samples=len(samples), n_valid=len(good),
            n_train=model["n_train"], n_test=model["n_test"], epochs=len(model["losses"]),
            space_size=self.space.size, sweep_seconds=t_sweep, collect_seconds=t_collect,
            top_measured_ms=[m for m, _ in cand_ms], samples_requested=count, sampling_budget_s=budget_s,
            sampling_budget_hit=self.budget_hit,
        )

    def close(self):
        self.batch.close()


class SizedAutotuner:
    """One network for several problem sizes, the extension proposed in the
    paper's Sec. "Broader Impact" (and the single-GPU analog of Sec. "Combined
    Training", where a hardware figure joins the launch features): the
    network has fv.FV_MLP_IN_SIZED inputs, the 14 launch features followed by
    the grid's problem features (tune_space.problem_features: log2 of the
    cell count, dimension). Samples of every grid not in `holdout` are pooled
    into one training set (75 / 25 split over the pool); the target is the
    log runtime relative to its grid (grid_relative_target). Every grid, held
    out or not, is then swept with its own problem features, its k best
    predictions are measured and the fastest valid one is kept."""

    def __init__(self, grids, states, seed=0, holdout=(), **tuner_kw):
        self.grids = list(grids)
        self.holdout = set(int(h) for h in holdout)
        self.seed = seed
        self.extra = [problem_features(g) for g in self.grids]
        self.tuners = [Autotuner(g, U, seed=seed + 1000 * i, **tuner_kw)
                       for i, (g, U) in enumerate(zip(self.grids, states))]

    def fit(self, samples):
        """samples[g]: the samples of grid g (None for a held-out grid)."""
        rows, extra, t, gid = [], [], [], []
        for g, smp in enumerate(samples):
            if smp is None:
                continue
            good = [s for s in smp if s.valid and np.isfinite(s.ms) and s.ms > 0.0]
            rows.append(self.tuners[g].space.features([s.index for s in good]))
            extra += [self.extra[g]] * len(good)
            t += [s.ms for s in good]
            gid += [g] * len(good)
        F = np.hstack([np.vstack(rows), np.asarray(extra, dtype=np.float64)])
        t = np.asarray(t, dtype=np.float64)
        gid = np.asarray(gid)
        tr, te = split_indices(len(t), self.seed)
        y, (z_mean, z_std), _ = grid_relative_target(t, gid, tr)
        mean = F[tr].mean(axis=0)
        std = F[tr].std(axis=0)
        std = np.where(std == 0.0, 1.0, std)
        X = (F - mean) / std
        net = Network(self.seed, n_in=fv.FV_MLP_IN_SIZED)
        losses = net.train(X[tr], y[tr])
        pred = net.predict(X)
        per_grid = {}
        for g in sorted(set(gid.tolist())):
            m = te[gid[te] == g]
            per_grid[g] = r2_score(y[m], pred[m]) if len(m) >= 3 else None
        return dict(net=net, mean=mean, std=std, z_mean=z_mean, z_std=z_std, losses=losses,
                    r2_test=r2_score(y[te], pred[te]), r2_train=r2_score(y[tr], pred[tr]),
                    r2_test_per_grid=per_grid, n_train=len(tr), n_test=len(te))

    def sweep(self, model, g, k=8):
        import torch
        at = self.tuners[g]
        sp = at.space.struct(model["mean"], model["std"], self.extra[g])
        t0 = time.perf_counter()
        idx, val = model["net"].sweep(sp, 0, at.space.size, k)
        torch.cuda.synchronize()
        return idx, val, time.perf_counter() - t0

    def run(self, count=300, k=8, rounds=5, budget_s=None):
        """budget_s: time budget of each grid's sampling (seconds), or None."""
        t0 = time.perf_counter()
        samples = [None if g in self.holdout else at.collect(count, budget_s) for g, at in enumerate(self.tuners)]
        t_collect = time.perf_counter() - t0
        model = self.fit(samples)
        out = []
        for g, at in enumerate(self.tuners):
            top_idx, top_val, t_sweep = self.sweep(model, g, k)
            cands = [at.space.decode(i) for i in top_idx]
            cand_ms = [at.measure(l) for l in cands]
            ok = [(ms, i) for i, (ms, v) in enumerate(cand_ms) if v]
            best = cands[min(ok)[1]] if ok else at.default
            final = at.interleaved([at.default, best], rounds=rounds)
            ship, shipped_from = shipped(final, [at.default, best], ("default", "network"))
            spec = self.grids[g]
            out.append(dict(
                n=[int(v) for v in spec.n[:spec.ndim]], ndim=spec.ndim, held_out=g in self.holdout,
                n_samples=0 if samples[g] is None else len(samples[g]),
                n_valid=0 if samples[g] is None else sum(1 for s in samples[g] if s.valid),
                default_launch=at.default, tuned_launch=ship, network_launch=best, shipped_from=shipped_from,
                default_ms=final[0], tuned_ms=min(final), network_ms=final[1],
                factor_vs_default=final[0] / min(final), network_factor_vs_default=final[0] / final[1],
                n_valid_candidates=len(ok),
                top_pred_relative=[float(math.exp(v * model["z_std"] + model["z_mean"])) for v in top_val],
                top_measured_ms=[m for m, _ in cand_ms], r2_test=model["r2_test_per_grid"].get(g),
                sweep_seconds=t_sweep, space_size=at.space.size, steps_per_sample=at.steps))
        return dict(grids=out, r2_test=model["r2_test"], r2_train=model["r2_train"], n_train=model["n_train"],
                    n_test=model["n_test"], epochs=len(model["losses"]), collect_seconds=t_collect,
                    sampling_budget_s=budget_s,
                    sampling_budget_hit=any(getattr(at, "budget_hit", False) for at in self.tuners))

    def close(self):
        for at in self.tuners:
            at.close()
