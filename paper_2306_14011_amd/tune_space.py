"""The 14-parameter launch space searched by the autotuner.

The paper tunes two OpenACC parameters (gang, vector) for each of seven
kernels (Sec. "Tuning Parameters", Table tuning-parameters: 10 gang values x
12 vector values per kernel). Here the seven sites of the split step each
take two CDNA launch parameters:
  * stencil sites (flux x/y/z): block width along x in {16, ..., 256} and
    threads per block in {64, ..., 1024}, width <= threads: 22 pairs;
  * one-dimensional sites (residual, update, bc, cfl): threads per block t in
    {64, ..., 1024} and elements per thread e in {1, 2, 4, 8, 16}: 25 pairs.
    e = 1 is the launch with one thread per element (gang 0); otherwise the
    gang is the power of two nearest to N / (t e) for the site's element
    count N (cells, or ghost cells for the fill), clamped to [1, 65536], and
    the kernel runs a grid-stride loop. The gang is thus relative to the
    problem size, as the paper's gang range was relative to its grid.
In 2D the z-flux site is pinned to one pair, so the space has
22^2 * 25^4 = 1.89e8 points; in 3D 22^3 * 25^4 = 4.16e9. The default launch
table (stencil (64, 256), one-dimensional (0, 256)) is a point of the space.
Indices are mixed radix with site 0 fastest.

Network features per site: log2 of (block width, threads) for stencil sites
and log2 of (elements per thread, threads) for one-dimensional sites. The
problem-size-conditioned network (the extension proposed in Sec.
"Broader Impact") appends two features of the grid, the same for every launch vector:
log2 of its interior cell count and its dimension (problem_features).
"""
from __future__ import annotations

import math

import numpy as np

THREADS = (64, 128, 256, 512, 1024)
STENCIL_WIDTHS = (16, 32, 64, 128, 256)
ELEMS_PER_THREAD = (1, 2, 4, 8, 16)
STENCIL_PAIRS = tuple((w, t) for w in STENCIL_WIDTHS for t in THREADS if w <= t)
PINNED_FLUX_Z = ((64, 256),)
NSITES = 7
ONE_D_SITES = (3, 4, 5, 6)   # residual, update, bc, cfl


def gang_for(n_elements: int, threads: int, e: int) -> int:
    """Blocks of a grid-stride launch giving about e elements per thread (0 for e = 1)."""
    if e == 1:
        return 0
    g = max(1.0, n_elements / float(threads * e))
    return int(min(65536, max(1, 2 ** int(round(math.log2(g))))))


def site_elements(spec):
    """Element counts of the one-dimensional sites: residual, update, bc, cfl."""
    nx, ny, nz = (int(v) for v in spec.n)
    ncell = nx * ny * nz
    ghosts = 4 * ny * nz + 4 * nx * nz + (4 * nx * ny if spec.ndim == 3 else 0)
    return {3: ncell, 4: ncell, 5: ghosts, 6: ncell}


def problem_features(spec):
    """Raw problem features of a grid for the size-conditioned network:
    (log2 of the interior cell count, dimension)."""
    cells = 1
    for v in spec.n[:spec.ndim]:
        cells *= int(v)
    return [math.log2(cells), float(spec.ndim)]


class MixedRadixSpace:
    """Choices per site (at most 7 sites, 2 parameters and 2 raw network
    features each); an index is the mixed-radix number of the per-site choice
    digits, site 0 fastest."""

    choices: list
    feats: list
    radix: list
    size: int

    def digits(self, idx: int):
        if not 0 <= idx < self.size:
            raise ValueError("index outside the space")
        out = []
        for s in range(NSITES):
            out.append(idx % self.radix[s])
            idx //= self.radix[s]
        return out

    def decode(self, idx: int):
        """14-vector of launch parameters of index idx."""
        out = []
        for s, c in enumerate(self.digits(idx)):
            out += list(self.choices[s][c])
        return out

    def encode(self, vec):
        """Index of a launch vector (the first choice matching each pair)."""
        idx = 0
        mul = 1
        for s in range(NSITES):
            c = self.choices[s].index((int(vec[2 * s]), int(vec[2 * s + 1])))
            idx += c * mul
            mul *= self.radix[s]
        return idx

    def sample(self, count: int, seed: int):
        """count distinct indices drawn uniformly from the space."""
        rng = np.random.default_rng(seed)
        seen = set()
        out = []
        while len(out) < count:
            i = int(rng.integers(0, self.size))
            if i not in seen:
                seen.add(i)
                out.append(i)
        return out

    def features(self, indices):
        """Raw (unscaled) network features of the given indices, one row each."""
        X = np.zeros((len(indices), 2 * NSITES))
        for r, idx in enumerate(indices):
            for s, c in enumerate(self.digits(int(idx))):
                X[r, 2 * s], X[r, 2 * s + 1] = self.feats[s][c]
        return X

    def tables(self, mean, std):
        """Standardised feature value of every choice: (f1, f2) per site, lists."""
        f1, f2 = [], []
        for s in range(NSITES):
            f1.append([(a - mean[2 * s]) / std[2 * s] for a, _ in self.feats[s]])
            f2.append([(b - mean[2 * s + 1]) / std[2 * s + 1] for _, b in self.feats[s]])
        return f1, f2

    def struct(self, mean, std, extra=None):
        """fv_tune_space describing this space with the given feature scaler.
        extra: raw problem features appended to every vector (the size-
        conditioned network), standardised with the scaler's trailing columns."""
        from .fv import FV_MLP_MAX_EXTRA, fv_tune_space
        sp = fv_tune_space()
        if extra is not None:
            extra = list(extra)
            if len(extra) != FV_MLP_MAX_EXTRA or len(mean) != 2 * NSITES + len(extra) or len(std) != len(mean):
                raise ValueError("extra features do not match the scaler")
            sp.n_extra = len(extra)
            for j, v in enumerate(extra):
                sp.extra[j] = (v - mean[2 * NSITES + j]) / std[2 * NSITES + j]
        f1, f2 = self.tables(mean, std)
        for s in range(NSITES):
            sp.radix[s] = self.radix[s]
            for c, (a, b) in enumerate(self.choices[s]):
                sp.p1[s][c] = a
                sp.p2[s][c] = b
                sp.f1[s][c] = f1[s][c]
                sp.f2[s][c] = f2[s][c]
        return sp


class LaunchSpace(MixedRadixSpace):
    def __init__(self, ndim: int, counts=None):
        """counts: element count per one-dimensional site (defaults to a 2048^2 grid)."""
        self.ndim = ndim
        if counts is None:
            counts = {3: 2048 * 2048, 4: 2048 * 2048, 5: 8 * 2048, 6: 2048 * 2048}
        self.counts = dict(counts)
        self.choices = []   # (p1, p2) launch parameters per choice
        self.feats = []     # (f1, f2) raw network features per choice
        for s in range(NSITES):
            if s in ONE_D_SITES:
                ch = [(gang_for(self.counts[s], t, e), t) for e in ELEMS_PER_THREAD for t in THREADS]
                ft = [(math.log2(e), math.log2(t)) for e in ELEMS_PER_THREAD for t in THREADS]
            else:
                pairs = STENCIL_PAIRS if (s < 2 or ndim == 3) else PINNED_FLUX_Z
                ch = list(pairs)
                ft = [(math.log2(a), math.log2(b)) for a, b in pairs]
            self.choices.append(ch)
            self.feats.append(ft)
        self.radix = [len(c) for c in self.choices]
        self.size = int(np.prod([int(r) for r in self.radix], dtype=object))

    @classmethod
    def for_grid(cls, spec):
        return cls(spec.ndim, site_elements(spec))



BATCH_SEGS = (4, 8, 12, 16, 20, 24, 32, 40, 48, 64)
BATCH_BUCKET_EDGES = (352, 576, 800)   # grid size buckets by sqrt(cells)


def batch_bucket(spec) -> int:
    side = math.sqrt(float(spec.n[0]) * float(spec.n[1]))
    return sum(side >= e for e in BATCH_BUCKET_EDGES)


class BatchSpace(MixedRadixSpace):
    """Schedule space of a batch of 2D grids: the segment height of each of
    four grid-size buckets (sites 0-3; a bucket with no grid is pinned) and
    the work-list order (site 4: given, largest first); sites 5 and 6 are
    pinned. Features: log2 of the segment height, the order flag."""

    def __init__(self, grids):
        self.bucket = [batch_bucket(g) for g in grids]
        used = set(self.bucket)
        self.choices, self.feats = [], []
        for b in range(4):
            segs = BATCH_SEGS if b in used else (16,)
            self.choices.append([(sg, 0) for sg in segs])
            self.feats.append([(math.log2(sg), 0.0) for sg in segs])
        self.choices.append([(0, 0), (1, 0)])
        self.feats.append([(0.0, 0.0), (1.0, 0.0)])
        for _ in range(2):
            self.choices.append([(0, 0)])
            self.feats.append([(0.0, 0.0)])
        self.radix = [len(c) for c in self.choices]
        self.size = int(np.prod([int(r) for r in self.radix], dtype=object))

    def schedule(self, idx: int):
        """(segment height per grid, order) of index idx."""
        d = self.digits(idx)
        segs = [self.choices[b][d[b]][0] for b in self.bucket]
        return segs, self.choices[4][d[4]][0]


FUSED_SEGS = (8, 12, 16, 20, 24, 32, 40, 48)
FUSED_WAVE_FACTORS = (0, 0.5, 1.0, 2.0)   # 0: one wave per work item, else x the resident wave slots


def fused_items(spec, seg: int) -> int:
    """Work items of one fused stage launch at segment height seg: 60-column
    strips x row segments in 2D, 32 x 7-cell tiles x plane segments in 3D
    (each 3D item is a workgroup of four waves)."""
    nx, ny, nz = (int(v) for v in spec.n)
    if spec.ndim == 2:
        return -(-nx // 60) * -(-ny // seg)
    return -(-nx // 32) * -(-ny // 7) * -(-nz // seg)


class FusedSpace(MixedRadixSpace):
    """Launch space of the fused path, the paper's method applied to the
    kernels the headline step runs: for each Runge-Kutta stage (sites 0-2)
    the segment height of its work items and the number of waves its launch
    holds (one per item, or a grid-stride loop over 1/2, 1 or 2 times the
    device's resident wave slots); sites 3-6 are pinned. 8 x 4 choices per
    stage: 32^3 = 32768 points. Features: log2 of the segment height and
    log2 of the waves actually launched (at most one per item)."""

    def __init__(self, spec, slots: int):
        self.spec = spec
        self.slots = int(slots)
        self.choices, self.feats = [], []
        for _ in range(3):
            ch, ft = [], []
            for sg in FUSED_SEGS:
                items = fused_items(spec, sg)
                per_item = items if spec.ndim == 2 else 4 * items
                for f in FUSED_WAVE_FACTORS:
                    w = 0 if f == 0 else max(4, int(round(f * self.slots)))
                    eff = per_item if w == 0 else min(w, per_item)
                    ch.append((sg, w))
                    ft.append((math.log2(sg), math.log2(eff)))
            self.choices.append(ch)
            self.feats.append(ft)
        for _ in range(4):
            self.choices.append([(0, 0)])
            self.feats.append([(0.0, 0.0)])
        self.radix = [len(c) for c in self.choices]
        self.size = int(np.prod([int(r) for r in self.radix], dtype=object))

    @staticmethod
    def table(vec):
        """(seg[3], waves[3]) of a decoded 14-vector."""
        return [int(vec[0]), int(vec[2]), int(vec[4])], [int(vec[1]), int(vec[3]), int(vec[5])]
