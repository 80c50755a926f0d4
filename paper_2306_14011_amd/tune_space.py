"""The 14-parameter launch space searched by the autotuner.

The paper tunes two OpenACC parameters (gang, vector) for each of seven
kernels (Sec. "Tuning Parameters", Table tuning-parameters: 10 gang values x
12 vector values per kernel). Here the seven sites of the split step each
take two CDNA launch parameters:
  * stencil sites (flux x/y/z): block width along x in {16, ..., 256} and
    threads per block in {64, ..., 1024}, width <= threads: 22 pairs;
  * one-dimensional sites (residual, update, bc, cfl): gang (blocks of a
    grid-stride loop) in {512, 2048, 8192, 32768} or 0 (one thread per
    element, as many blocks as that takes) and threads per block in
    {64, ..., 1024}: 25 pairs.
In 2D the z-flux site is pinned to one pair, so the space has
22^2 * 25^4 = 1.89e8 points; in 3D 22^3 * 25^4 = 4.16e9. The default launch
table (stencil (64, 256), one-dimensional (0, 256)) is a point of the space.
Indices are mixed radix with site 0 fastest.

Network features are log2 of the 14 parameters; a gang of 0 (one thread per
element: more blocks than any finite choice) is encoded as 2^17, one octave
above the largest finite gang.
"""
from __future__ import annotations

import math

import numpy as np

THREADS = (64, 128, 256, 512, 1024)
STENCIL_WIDTHS = (16, 32, 64, 128, 256)
GANGS = (512, 2048, 8192, 32768, 0)
GANG_AUTO_FEATURE = 2 ** 17
STENCIL_PAIRS = tuple((w, t) for w in STENCIL_WIDTHS for t in THREADS if w <= t)
GANG_PAIRS = tuple((g, t) for g in GANGS for t in THREADS)
PINNED_FLUX_Z = ((64, 256),)
NSITES = 7


class LaunchSpace:
    def __init__(self, ndim: int):
        self.ndim = ndim
        self.choices = [STENCIL_PAIRS, STENCIL_PAIRS, STENCIL_PAIRS if ndim == 3 else PINNED_FLUX_Z,
                        GANG_PAIRS, GANG_PAIRS, GANG_PAIRS, GANG_PAIRS]
        self.radix = [len(c) for c in self.choices]
        self.size = int(np.prod([int(r) for r in self.radix], dtype=object))

    def decode(self, idx: int):
        """14-vector of launch parameters of index idx."""
        if not 0 <= idx < self.size:
            raise ValueError("index outside the space")
        out = []
        for s in range(NSITES):
            c = idx % self.radix[s]
            idx //= self.radix[s]
            out += list(self.choices[s][c])
        return out

    def encode(self, vec):
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

    @staticmethod
    def encode_params(vecs):
        """Launch vectors with gang 0 replaced by its feature value 2^17."""
        P = np.asarray(vecs, dtype=np.float64).copy()
        P[P == 0] = GANG_AUTO_FEATURE
        return P

    @staticmethod
    def raw_features(vecs):
        """log2 of the 14 (encoded) launch parameters, one row per vector."""
        return np.log2(LaunchSpace.encode_params(vecs))

    def tables(self, mean, std):
        """Standardised feature value of every choice: (f1, f2) per site, lists."""
        f1, f2 = [], []
        for s in range(NSITES):
            f1.append([(math.log2(a if a else GANG_AUTO_FEATURE) - mean[2 * s]) / std[2 * s]
                       for a, _ in self.choices[s]])
            f2.append([(math.log2(b) - mean[2 * s + 1]) / std[2 * s + 1] for _, b in self.choices[s]])
        return f1, f2

    def struct(self, mean, std):
        """fv_tune_space describing this space with the given feature scaler."""
        from .fv import fv_tune_space
        sp = fv_tune_space()
        f1, f2 = self.tables(mean, std)
        for s in range(NSITES):
            sp.radix[s] = self.radix[s]
            for c, (a, b) in enumerate(self.choices[s]):
                sp.p1[s][c] = a
                sp.p2[s][c] = b
                sp.f1[s][c] = f1[s][c]
                sp.f2[s][c] = f2[s][c]
        return sp
