"""Schedule autotuner.

The row schedule decides how the rows of each mode are cut into work for the
kernels: rows with at most ``tiny_max`` samples run one per lane, rows with at
most ``group_max`` one per 16-lane group (R <= 16), longer ones as chunks of
``item_samples`` samples.  It changes the order of floating-point sums only,
never which entries are sampled, so any candidate gives a valid run; the
tuner times a few sweeps of each candidate on the caller's problem and
returns the fastest.

    best, table = tune(dims, coords, values, rank, c=0.1)
    prob = Problem(dims, coords, values, rank, c=0.1, schedule=best)
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

from . import Problem

DEFAULT_CANDIDATES_16 = [
    {},  # the library's defaults
    {"item_samples": 4096},
    {"item_samples": 8192},
    {"group_max": 256},
    {"group_max": 384},
    {"tiny_max": 2},
    {"tiny_max": 0},
    {"overlap": 0},
    {"overlap": 2},
]
DEFAULT_CANDIDATES_WIDE = [
    {},
    {"item_samples": 512},
    {"item_samples": 2048},
    {"item_samples": 4096},
]


def candidates_for(rank: int) -> List[dict]:
    return [dict(c) for c in (DEFAULT_CANDIDATES_16 if rank <= 16 else DEFAULT_CANDIDATES_WIDE)]


def tune(dims: Sequence[int], coords: np.ndarray, values: np.ndarray, rank: int, *,
         candidates: Optional[Iterable[dict]] = None, sweeps: int = 5, warmup: int = 1,
         **problem_kw) -> Tuple[dict, List[Tuple[dict, float]]]:
    """Time `sweeps` sweeps per candidate schedule (device time, after
    `warmup` sweeps) and return (best schedule, [(schedule, ms per sweep)])."""
    table: List[Tuple[dict, float]] = []
    for cand in (candidates if candidates is not None else candidates_for(rank)):
        prob = Problem(dims, coords, values, rank, schedule=cand, stream=0, **problem_kw)
        try:
            if warmup:
                prob.time_sweeps(warmup)
            ms = prob.time_sweeps(sweeps) / sweeps
        finally:
            prob.close()
        table.append((dict(cand), ms))
    best = min(table, key=lambda t: t[1])[0]
    return best, table


def tune_classes(problems: Sequence[Tuple[Sequence[int], np.ndarray, np.ndarray, int]], *, sweeps: int = 5,
                 **problem_kw) -> Dict[int, dict]:
    """One schedule per padded-rank class (16, 32, 64) of a batch of problems,
    tuned on the class member with the most entries."""
    by_class: Dict[int, Tuple[int, int]] = {}
    for i, (_, co, _, R) in enumerate(problems):
        cls = 16 if R <= 16 else 32 if R <= 32 else 64
        if cls not in by_class or co.shape[0] > by_class[cls][1]:
            by_class[cls] = (i, co.shape[0])
    out = {}
    for cls, (i, _) in by_class.items():
        dims, co, va, R = problems[i]
        out[cls], _ = tune(dims, co, va, R, sweeps=sweeps, **problem_kw)
    return out
