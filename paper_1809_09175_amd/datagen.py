"""Seeded synthetic COO tensors and factor matrices shaped like the paper's workloads.

This module draws random numbers only; it holds none of the MTTKRP / CP-ALS arithmetic, so both
the HIP path and the CPU oracle can be fed from it.  All generation is host-side numpy PCG64.

Workload recipes (the paper's real tensors come from the FROSTT collection, which is not
available; skewed index distributions stand in for real-data contention, Sec. 7.2):

  cpals_small   3-way 100 x 80 x 60, 10,000 distinct uniform coordinates, values U(0,1) FP64,
                factors U(0,1)                                        (seed 1)
  powerlaw3     3-way 500,000 x 500,000 x 20,000, 1e8 entries, each mode bounded Zipf(1.1)
                (P(rank r) ~ (r+1)^-1.1) followed by a random relabelling of the mode, duplicate
                coordinates kept (a COO tensor is the sum of its entries), values
                lognormal(0,1) FP32, factors U(0,1) FP32                 (seed 2)
  skewed4       4-way 1e6 x 1e5 x 1e4 x 365, 5e7 distinct entries, Zipf(1.2) + relabel on modes
                0-1 and uniform on modes 2-3, values lognormal(0,1) FP32  (seed 3)
  batch64       64 independent 3-way tensors, dims log-uniform in [1e3, 5e4], entries
                log-uniform in [1e4, 2e6], Zipf(1.1) + relabel, R from {8, 16, 32}  (seeds 4000+t)
  gcp_counts    3-way 2e5 x 1e5 x 5e3, 5e7 distinct uniform nonzeros with zero-truncated
                Poisson(2) counts, plus 5e7 distinct uniform cells outside the nonzero set
                with value 0, factors U(0, c), c = 2 (ln 2 / R)^(1/3)   (seed 5)

Every generator takes a ``scale`` (fraction of the entries) and optional dims so the same recipe
produces small parity-test cases.

  max_entries   3-way 2e6 x 1.5e6 x 1e6 with 2^31 - 1 entries (the int32 limit of the
                subscripts and permutations), uniform subscripts and U(0,1) FP32 values, drawn
                on the GPU with torch's seeded generator (too large to draw on the host)
                                                                        (seed 6)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_CHUNK = 1 << 23


@dataclass
class CooTensor:
    subs: np.ndarray          # P x d int32, row-major
    vals: np.ndarray          # P, float32 or float64
    dims: tuple               # d ints
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.subs.shape[0])

    @property
    def d(self) -> int:
        return len(self.dims)


class _Alias:
    """Walker/Vose alias table for a discrete distribution over 0..I-1."""

    def __init__(self, probs: np.ndarray):
        I = probs.size
        q = probs * (I / probs.sum())
        prob = np.ones(I)
        alias = np.arange(I, dtype=np.int64)
        small = list(np.flatnonzero(q < 1.0)[::-1])
        large = list(np.flatnonzero(q >= 1.0)[::-1])
        q = q.copy()
        while small and large:
            s = small.pop()
            l = large.pop()
            prob[s] = q[s]
            alias[s] = l
            q[l] = q[l] + q[s] - 1.0
            if q[l] < 1.0:
                small.append(l)
            else:
                large.append(l)
        self.I = I
        self.prob = prob
        self.alias = alias

    def sample_into(self, rng: np.random.Generator, out: np.ndarray) -> None:
        n = out.shape[0]
        for s in range(0, n, _CHUNK):
            e = min(n, s + _CHUNK)
            u = rng.random(e - s) * self.I
            k = u.astype(np.int64)
            np.minimum(k, self.I - 1, out=k)
            frac = u - k
            out[s:e] = np.where(frac < self.prob[k], k, self.alias[k])


def zipf_probs(I: int, s: float) -> np.ndarray:
    p = (np.arange(I, dtype=np.float64) + 1.0) ** (-s)
    return p / p.sum()


def zipf_mode(rng: np.random.Generator, I: int, s: float, n: int, out=None) -> np.ndarray:
    """n draws of a bounded Zipf(s) rank on [0, I), then a random relabelling of the ranks."""
    if out is None:
        out = np.empty(n, dtype=np.int32)
    if s == 0.0:
        for a in range(0, n, _CHUNK):
            b = min(n, a + _CHUNK)
            out[a:b] = rng.integers(0, I, size=b - a, dtype=np.int64)
        return out
    tab = _Alias(zipf_probs(I, s))
    tab.sample_into(rng, out)
    relabel = rng.permutation(I).astype(np.int32)
    for a in range(0, n, _CHUNK):
        b = min(n, a + _CHUNK)
        out[a:b] = relabel[out[a:b]]
    return out


def _lognormal_f32(rng, n):
    v = np.empty(n, dtype=np.float32)
    for a in range(0, n, _CHUNK):
        b = min(n, a + _CHUNK)
        v[a:b] = rng.lognormal(0.0, 1.0, size=b - a)
    return v


def _linear(subs: np.ndarray, dims) -> np.ndarray:
    lin = np.zeros(subs.shape[0], dtype=np.int64)
    for m, I in enumerate(dims):
        lin = lin * int(I) + subs[:, m].astype(np.int64)
    return lin


def _unlinear(lin: np.ndarray, dims) -> np.ndarray:
    subs = np.empty((lin.size, len(dims)), dtype=np.int32)
    rest = lin.copy()
    for m in range(len(dims) - 1, -1, -1):
        subs[:, m] = rest % int(dims[m])
        rest //= int(dims[m])
    return subs


def skewed_tensor(dims, nnz, skew, seed, distinct=False, values="lognormal", name=""):
    """Entries with independent per-mode indices: bounded Zipf(skew[m]) (0 = uniform) + relabel.

    distinct=True draws, removes repeated coordinates (keeping the first draw, in draw order)
    and tops up until exactly nnz distinct coordinates exist."""
    rng = np.random.default_rng(seed)
    d = len(dims)
    if not distinct:
        subs = np.empty((nnz, d), dtype=np.int32)
        col = np.empty(nnz, dtype=np.int32)
        for m in range(d):
            zipf_mode(rng, int(dims[m]), float(skew[m]), nnz, out=col)
            subs[:, m] = col
    else:
        cells = 1
        for I in dims:
            cells *= int(I)
        if nnz > cells:
            raise ValueError("more distinct entries than cells")
        # per-mode distributions are fixed up front so top-up draws come from the same law
        tabs = [None if skew[m] == 0.0 else _Alias(zipf_probs(int(dims[m]), float(skew[m])))
                for m in range(d)]
        relabels = [None if skew[m] == 0.0 else rng.permutation(int(dims[m])).astype(np.int32)
                    for m in range(d)]
        have = np.empty(0, dtype=np.int64)
        need = nnz
        while need > 0:
            draw = int(need * 1.05) + 16
            part = np.empty((draw, d), dtype=np.int32)
            col = np.empty(draw, dtype=np.int32)
            for m in range(d):
                if tabs[m] is None:
                    col[:] = rng.integers(0, int(dims[m]), size=draw, dtype=np.int64)
                else:
                    tabs[m].sample_into(rng, col)
                    col[:] = relabels[m][col]
                part[:, m] = col
            lin = np.concatenate([have, _linear(part, dims)])
            _, first = np.unique(lin, return_index=True)
            first.sort()
            have = lin[first[:nnz]]
            need = nnz - have.size
        subs = _unlinear(have, dims)
    if values == "lognormal":
        vals = _lognormal_f32(rng, nnz)
    elif values == "uniform64":
        vals = rng.random(nnz)
    else:
        raise ValueError(values)
    return CooTensor(subs, vals, tuple(int(x) for x in dims), name,
                     {"seed": seed, "skew": list(skew), "distinct": distinct})


def factors(dims, R, seed, dtype=np.float32, high=1.0):
    """Factor matrices U(0, high), one I_m x R row-major array per mode."""
    rng = np.random.default_rng(seed)
    return [(rng.random((int(I), R)) * high).astype(dtype) for I in dims]


# ---------------------------------------------------------------------------------------------
# the workload recipes
# ---------------------------------------------------------------------------------------------

def cpals_small(seed=1, dims=(100, 80, 60), nnz=10_000, R=16):
    rng = np.random.default_rng(seed)
    cells = int(np.prod(dims))
    lin = rng.choice(cells, size=nnz, replace=False).astype(np.int64)
    subs = _unlinear(lin, dims)
    vals = rng.random(nnz)
    X = CooTensor(subs, vals, tuple(dims), "cpals_small", {"seed": seed})
    A = [rng.random((I, R)) for I in dims]
    return X, A


def powerlaw3(scale=1.0, dims=(500_000, 500_000, 20_000), seed=2, s=1.1):
    nnz = max(1, int(round(1e8 * scale)))
    return skewed_tensor(dims, nnz, (s,) * 3, seed, distinct=False, name="powerlaw3")


def skewed4(scale=1.0, dims=(1_000_000, 100_000, 10_000, 365), seed=3):
    nnz = max(1, int(round(5e7 * scale)))
    return skewed_tensor(dims, nnz, (1.2, 1.2, 0.0, 0.0), seed, distinct=True, name="skewed4")


def batch64(count=64, seed0=4000, nnz_range=(1e4, 2e6), dim_range=(1e3, 5e4)):
    out = []
    for t in range(count):
        rng = np.random.default_rng(seed0 + t)
        dims = tuple(int(round(math.exp(rng.uniform(math.log(dim_range[0]),
                                                     math.log(dim_range[1]))))) for _ in range(3))
        nnz = int(round(math.exp(rng.uniform(math.log(nnz_range[0]), math.log(nnz_range[1])))))
        R = int(rng.choice([8, 16, 32]))
        X = skewed_tensor(dims, nnz, (1.1, 1.1, 1.1), int(rng.integers(1 << 31)), name=f"batch{t}")
        X.meta["R"] = R
        out.append(X)
    return out


def gcp_counts(scale=1.0, dims=(200_000, 100_000, 5_000), seed=5, R=32):
    """Nonzeros (zero-truncated Poisson(2) counts) followed by sampled zeros, weights 1.

    2 * nz distinct cells are drawn uniformly (draw, dedupe, top up), put in random order, and
    split: the first nz are the nonzeros, the rest the sampled zeros (so the two sets are
    disjoint)."""
    rng = np.random.default_rng(seed)
    nz = max(1, int(round(5e7 * scale)))
    nzero = nz
    cells = 1
    for I in dims:
        cells *= int(I)
    if nz + nzero > cells:
        raise ValueError("more entries than cells")
    u = np.unique(rng.integers(0, cells, size=int((nz + nzero) * 1.001) + 16, dtype=np.int64))
    while u.size < nz + nzero:
        u = np.unique(np.concatenate([u, rng.integers(0, cells, size=nz + nzero - u.size + 16,
                                                      dtype=np.int64)]))
    u = u[rng.permutation(u.size)[:nz + nzero]]
    lin, zeros = u[:nz], u[nz:]
    counts = rng.poisson(2.0, size=nz)
    while True:
        bad = np.flatnonzero(counts == 0)
        if bad.size == 0:
            break
        counts[bad] = rng.poisson(2.0, size=bad.size)
    subs = _unlinear(np.concatenate([lin, zeros]), dims)
    vals = np.concatenate([counts.astype(np.float32), np.zeros(nzero, dtype=np.float32)])
    X = CooTensor(subs, vals, tuple(dims), "gcp_counts", {"seed": seed, "nonzeros": nz})
    c = 2.0 * (math.log(2.0) / R) ** (1.0 / 3.0)
    A = factors(dims, R, seed + 1000, np.float32, high=c)
    return X, A



def max_entries(seed=6, dims=(2_000_000, 1_500_000, 1_000_000), nnz=(1 << 31) - 1, device="cuda"):
    """(subs, vals) as device tensors: nnz x 3 int32 subscripts, uniform per mode, and U(0,1)
    FP32 values, from torch's Philox-based generator on the device."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    subs = torch.empty((nnz, len(dims)), dtype=torch.int32, device=device)
    for m, I in enumerate(dims):
        subs[:, m] = torch.randint(0, I, (nnz,), dtype=torch.int32, device=device, generator=g)
    vals = torch.rand(nnz, dtype=torch.float32, device=device, generator=g)
    return subs, vals, tuple(dims)
