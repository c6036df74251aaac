"""Seeded synthetic inputs for nonnegative tensor completion.

This module only *draws inputs*: observed index sets, planted nonnegative CPD
factors, observed values, a train/test split and optional FP32 initial
factors.  It holds none of the solver's arithmetic (no sampling of
minibatches, no gradients, no step sizes), so the FP64 oracle and the HIP
library can both consume what it produces without sharing any method code.

Data model (Section II): the planted tensor is the CPD of nonnegative factors
``U^(m)`` with i.i.d. Uniform[0,1] entries (eq. Xo_densef); observations are
``X = X^o + E`` on an index set ``Omega`` (eq. M_def).  The experiments of
Section IV draw Gaussian noise ``N(0, sigma^2)``; the second argument is read
as a variance.

All randomness comes from NumPy's PCG64 seeded by the caller, so every array
is reproducible from ``(recipe, seed)``.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Problem:
    """One completion instance: dims, train/test COO and the planted truth."""

    dims: List[int]
    rank: int                     # rank used by the solver
    coords: np.ndarray            # int32 [nnz, N], 0-based, train
    values: np.ndarray            # float32 [nnz], train
    test_coords: np.ndarray       # int32 [n_test, N]
    test_values: np.ndarray       # float32 [n_test]
    planted: Optional[List[np.ndarray]] = None   # FP64 planted factors
    snr: Optional[float] = None   # ||M*X^o||^2 / ||M*E||^2 (Section IV-B)
    name: str = ""

    @property
    def nmodes(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.values.shape[0])


# ---------------------------------------------------------------- index sets
_CHUNK = 1 << 22          # draws per child generator (fixed: results do not depend on thread count)
_THREADS = max(1, min(16, os.cpu_count() or 1))


def _pmap(fn, items):
    items = list(items)
    if _THREADS == 1 or len(items) == 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(_THREADS) as ex:
        return list(ex.map(fn, items))


def _zipf_cdf(n: int, s: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    c /= c[-1]
    return c


def _draw_keys(seed_seq, dims, strides, count, zipf_s, cdfs, relabels) -> np.ndarray:
    """`count` linearised cell keys, i.i.d. per mode, in fixed-size chunks."""
    nchunks = (count + _CHUNK - 1) // _CHUNK
    children = seed_seq.spawn(nchunks)

    def chunk(ci):
        rng = np.random.default_rng(children[ci])
        cnt = min(_CHUNK, count - ci * _CHUNK)
        key = np.zeros(cnt, dtype=np.int64)
        for m, d in enumerate(dims):
            if zipf_s is None:
                ix = rng.integers(0, d, size=cnt, dtype=np.int64)
            else:
                rank = np.searchsorted(cdfs[m], rng.random(cnt), side="right")
                np.minimum(rank, d - 1, out=rank)
                ix = relabels[m][rank]
            key += ix * strides[m]
        return key

    return np.concatenate(_pmap(chunk, range(nchunks))) if nchunks else np.zeros(0, np.int64)


_NB = 64   # hash buckets of the de-duplication (duplicates always share a bucket)


def _buckets(keys: np.ndarray):
    h = ((keys.astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(58)).astype(np.uint8)
    order = np.argsort(h, kind="stable")          # radix sort on 8-bit ids
    ks = keys[order]
    bounds = np.concatenate([[0], np.cumsum(np.bincount(h, minlength=_NB))])
    return [ks[bounds[b]:bounds[b + 1]] for b in range(_NB)]


def _merge_unique(state, keys: np.ndarray):
    """state: _NB sorted arrays of distinct keys; returns state with `keys` added."""
    new = _buckets(keys)
    return _pmap(lambda b: np.union1d(state[b], new[b]), range(_NB))


def distinct_cells(rng, dims: Sequence[int], nnz: int, zipf_s: Optional[float] = None) -> np.ndarray:
    """``nnz`` distinct cells of the grid ``dims``, in random order.

    Uniform positions when ``zipf_s`` is None; otherwise each mode's index is
    Zipf(s) over a seeded random relabelling of its range, cells are
    de-duplicated on a linearised int64 key, and the set is topped up with
    fresh draws until ``nnz`` distinct cells exist.
    """
    dims = [int(d) for d in dims]
    total = 1
    for d in dims:
        total *= d
    if nnz > total:
        raise ValueError("more cells requested than the grid holds")
    if total >= 2 ** 62:
        raise ValueError("grid too large for an int64 key")
    strides = [1] * len(dims)
    for m in range(len(dims) - 2, -1, -1):
        strides[m] = strides[m + 1] * dims[m + 1]
    cdfs, relabels = [], []
    for d in dims:
        if zipf_s is None:
            cdfs.append(None)
            relabels.append(None)
        else:
            cdfs.append(_zipf_cdf(d, zipf_s))
            relabels.append(rng.permutation(d).astype(np.int64))
    if zipf_s is None and nnz * 4 > total:
        # dense fraction: a random subset of the grid directly
        keys = rng.choice(total, size=nnz, replace=False).astype(np.int64)
    else:
        seq = np.random.SeedSequence(int(rng.integers(0, 2 ** 63)))
        state = [np.zeros(0, np.int64)] * _NB
        have, yield_rate = 0, 1.0
        while have < nnz:
            deficit = nnz - have
            draw = int(deficit / max(yield_rate, 0.02) * 1.1) + 1024
            state = _merge_unique(state, _draw_keys(seq.spawn(1)[0], dims, strides, draw, zipf_s, cdfs,
                                                    relabels))
            now = sum(x.shape[0] for x in state)
            yield_rate = (now - have) / draw
            have = now
        keys = np.concatenate(state)        # deterministic order: bucket, then key
        keys = keys[rng.permutation(keys.shape[0])[:nnz]]
    coords = np.empty((nnz, len(dims)), dtype=np.int32)
    rem = keys
    for m in range(len(dims)):
        coords[:, m] = rem // strides[m]
        rem = rem % strides[m]
    return coords


# ------------------------------------------------------------------- values
def planted_factors(rng, dims: Sequence[int], rank: int) -> List[np.ndarray]:
    """i.i.d. Uniform[0,1] nonnegative factors (Section IV-B)."""
    return [rng.random((int(d), rank)) for d in dims]


def planted_values(factors: Sequence[np.ndarray], coords: np.ndarray, chunk: int = 1 << 20) -> np.ndarray:
    """FP64 entries of the planted CPD at ``coords`` (eq. Xo_densef)."""
    nnz = coords.shape[0]
    out = np.empty(nnz, dtype=np.float64)

    def part(s):
        e = min(nnz, s + chunk)
        acc = factors[0][coords[s:e, 0]]
        for m in range(1, len(factors)):
            acc = acc * factors[m][coords[s:e, m]]
        out[s:e] = acc.sum(axis=1)

    _pmap(part, range(0, nnz, chunk))
    return out


def _normal(seed_seq, n: int, sigma: float) -> np.ndarray:
    nchunks = (n + _CHUNK - 1) // _CHUNK
    children = seed_seq.spawn(max(nchunks, 1))
    out = np.empty(n, dtype=np.float64)

    def part(ci):
        s = ci * _CHUNK
        e = min(n, s + _CHUNK)
        out[s:e] = np.random.default_rng(children[ci]).normal(0.0, sigma, size=e - s)

    _pmap(part, range(nchunks))
    return out


def split_holdout(rng, coords: np.ndarray, values: np.ndarray, test_frac: float):
    n = coords.shape[0]
    n_test = int(round(n * test_frac))
    perm = rng.permutation(n)
    te, tr = perm[:n_test], perm[n_test:]
    return coords[tr], values[tr], coords[te], values[te]


def make_problem(dims: Sequence[int], nnz: int, planted_rank: int, *, rank: Optional[int] = None,
                 zipf_s: Optional[float] = None, noise_var: float = 0.0, value_model: str = "exact",
                 test_frac: float = 0.1, seed: int = 0, name: str = "",
                 grid_factors: Optional[int] = None) -> Problem:
    """Draw one instance.

    value_model:
      * ``exact``   -- X = X^o (+ noise if ``noise_var`` > 0)
      * ``clip0``   -- X = max(0, X^o + E)
      * ``ratings`` -- affine map of X^o onto [1,5] by its empirical min/max
        over the observed cells, plus noise, rounded to an integer, clipped to 1..5
    grid_factors: if set, planted factors are drawn from the dyadic grid
      {0, 1/g, ..., 1} so every CPD value is exact in FP32 and FP64.
    """
    rng = np.random.default_rng(seed)
    dims = [int(d) for d in dims]
    coords = distinct_cells(rng, dims, nnz, zipf_s)
    if grid_factors:
        fac = [rng.integers(0, grid_factors + 1, size=(d, planted_rank)) / float(grid_factors) for d in dims]
    else:
        fac = planted_factors(rng, dims, planted_rank)
    xo = planted_values(fac, coords)
    if value_model == "ratings":
        lo, hi = float(xo.min()), float(xo.max())
        xo = 1.0 + 4.0 * (xo - lo) / (hi - lo if hi > lo else 1.0)
    noise = (_normal(np.random.SeedSequence(int(rng.integers(0, 2 ** 63))), nnz, math.sqrt(noise_var))
             if noise_var > 0 else np.zeros(nnz))
    x = xo + noise
    if value_model == "ratings":
        x = np.clip(np.rint(x), 1.0, 5.0)
    elif value_model == "clip0":
        x = np.maximum(x, 0.0)
    en = float(np.sum((x - xo) ** 2))
    snr = float(np.sum(xo ** 2)) / en if en > 0 else math.inf
    vals = x.astype(np.float32)
    trc, trv, tec, tev = split_holdout(rng, coords, vals, test_frac)
    return Problem(dims=dims, rank=rank or planted_rank, coords=np.ascontiguousarray(trc),
                   values=np.ascontiguousarray(trv), test_coords=np.ascontiguousarray(tec),
                   test_values=np.ascontiguousarray(tev), planted=fac, snr=snr, name=name)


def uniform_init(dims: Sequence[int], rank: int, seed: int, scale: float = 1.0) -> List[np.ndarray]:
    """FP32 initial factors, Uniform[0,1) * scale (an explicit, caller-side U_0)."""
    rng = np.random.default_rng(seed + 0x5EED)
    return [(rng.random((int(d), rank), dtype=np.float32) * np.float32(scale)).astype(np.float32)
            for d in dims]


def init_scale(values: np.ndarray, rank: int, nmodes: int) -> float:
    """Scale s so that a CPD of Uniform[0,s) factors matches the data mean."""
    mean = float(np.mean(values.astype(np.float64)))
    return float(np.float32((max(mean, 1e-30) / (rank * 2.0 ** (-nmodes))) ** (1.0 / nmodes)))


# ------------------------------------------------------------------ recipes
def tiny(seed: int = 0, dims=(7, 6, 5), nnz: int = 120, rank: int = 3, **kw) -> Problem:
    """Small instance for brute-force checks."""
    kw.setdefault("test_frac", 0.1)
    return make_problem(dims, nnz, rank, seed=seed, name="tiny", **kw)


def c0(seed: int = 0) -> Problem:
    """3-way 100x80x60, 24,000 uniform cells, planted rank 8, exact CPD, 10% test."""
    return make_problem((100, 80, 60), 24000, 8, zipf_s=None, noise_var=0.0,
                        value_model="exact", test_frac=0.1, seed=seed, name="c0")


def c1(seed: int = 0, scale: float = 1.0) -> Problem:
    """3-way 480,000x18,000x2,000, 100M Zipf(1.1) cells, rank-16 ratings 1..5 with
    N(0,0.1) noise, 5% test.  ``scale`` < 1 shrinks nnz (dims kept) for smaller runs."""
    nnz = int(round(100_000_000 * scale))
    return make_problem((480_000, 18_000, 2_000), nnz, 16, zipf_s=1.1, noise_var=0.1,
                        value_model="ratings", test_frac=0.05, seed=seed, name="c1")


def c1_small(seed: int = 0) -> Problem:
    """Same recipe as c1 on a 1/100-scale grid and nnz (parity-sized, Zipf skew kept)."""
    return make_problem((4_800, 1_800, 200), 1_000_000, 16, zipf_s=1.1, noise_var=0.1,
                        value_model="ratings", test_frac=0.05, seed=seed, name="c1_small")


def c2(seed: int = 0, scale: float = 1.0) -> Problem:
    """4-way 1,000,000x500,000x1,000x100, 500M Zipf(1.05) cells, rank-32 CPD +
    N(0,0.05) clipped at 0, 5% test."""
    nnz = int(round(500_000_000 * scale))
    return make_problem((1_000_000, 500_000, 1_000, 100), nnz, 32, zipf_s=1.05, noise_var=0.05,
                        value_model="clip0", test_frac=0.05, seed=seed, name="c2")


def scaling_twin(seed: int = 0) -> Problem:
    """Synthetic twin of the timing workload of Section IV-C: a 4-way
    183x24x1140x1717 tensor with 3,309,490 uniformly placed observed cells of a
    noiseless rank-10 CPD with i.i.d. U[0,1] factors; no held-out set."""
    return make_problem((183, 24, 1140, 1717), 3_309_490, 10, zipf_s=None, noise_var=0.0,
                        value_model="exact", test_frac=0.0, seed=seed, name="scaling")


# E[x^2] of one entry of a rank-10 3-way CPD with i.i.d. U[0,1] factors:
# 10 (1/3)^3 + 90 (1/8)^2
_CPD10_3WAY_MEAN_SQ = 10.0 / 27.0 + 90.0 / 64.0


def convergence_twin(seed: int = 0, snr: float = 100.0, nnz: int = 10_000_054) -> Problem:
    """Synthetic twin of the convergence experiment of Section IV-B: a
    71567x65133x730 tensor (the MovieLens 10M shape) with nnz uniformly
    placed observed cells of a rank-10 CPD with i.i.d. U[0,1] factors plus
    N(0, sigma^2) noise, sigma^2 set for the given SNR (the paper's ratio of
    squared norms over the observed cells); 5% held out."""
    return make_problem((71_567, 65_133, 730), nnz, 10, zipf_s=None, noise_var=_CPD10_3WAY_MEAN_SQ / snr,
                        value_model="exact", test_frac=0.05, seed=seed, name=f"conv_snr{snr:g}")


def c3_shapes(n_instances: int = 256, base_seed: int = 1000):
    """Size mixture of the batching workload: per instance dims log-U[50,2000],
    nnz log-U[10k,2M] capped at half the grid, rank from {8,16,32}."""
    out = []
    for i in range(n_instances):
        rng = np.random.default_rng(base_seed + i)
        dims = [int(round(math.exp(rng.uniform(math.log(50), math.log(2000))))) for _ in range(3)]
        nnz = int(round(math.exp(rng.uniform(math.log(10_000), math.log(2_000_000)))))
        cap = (dims[0] * dims[1] * dims[2]) // 2
        nnz = min(nnz, cap)
        rank = int(rng.choice([8, 16, 32]))
        out.append((dims, nnz, rank, base_seed + i))
    return out


def c3_instance(dims, nnz, rank, seed) -> Problem:
    return make_problem(dims, nnz, rank, zipf_s=None, noise_var=0.01, value_model="exact",
                        test_frac=0.05, seed=seed, name="c3")
