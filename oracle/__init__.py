"""ctypes binding of the FP64 CPU oracle (``ntc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The product path never imports this
package, and this package never imports the product.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ntc_oracle.c")
_LIB = os.path.join(_HERE, "libntc_oracle.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math).  A forced
    build also compiles the sanitizer driver (syntax and types only; the
    sanitized executable is built by its test)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    if force:
        subprocess.check_call(["gcc", "-std=c99", "-fsyntax-only", "-Wall",
                               os.path.join(_HERE, "sanitize_driver.c")])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_create.argtypes = [ctypes.c_int, _i64p, ctypes.c_int64, _i32p, _f32p, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_uint64, ctypes.c_int64, _i32p, _f32p,
                                 ctypes.POINTER(_f32p)]
        L.ora_free.argtypes = [ctypes.c_void_p]
        L.ora_sweep.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_update_mode.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_update_rows.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p, ctypes.c_int64, _f64p]
        L.ora_loss.argtypes = [ctypes.c_void_p, _f64p]
        L.ora_get_factors.argtypes = [ctypes.c_void_p, ctypes.c_int, _f64p]
        L.ora_set_factors.argtypes = [ctypes.c_void_p, ctypes.c_int, _f64p]
        L.ora_get_sweep.restype = ctypes.c_int64
        L.ora_get_sweep.argtypes = [ctypes.c_void_p]
        L.ora_set_sweep.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.ora_get_csr.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p, _i64p]
        L.ora_set_threads.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_philox4x32.argtypes = [_u32p, _u32p, ctypes.c_int, _u32p]
        L.ora_sample_keys.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int64, _u32p]
        L.ora_feistel_width.restype = ctypes.c_int
        L.ora_feistel_width.argtypes = [ctypes.c_int64]
        L.ora_feistel_rounds.restype = ctypes.c_int
        L.ora_feistel_rounds.argtypes = [ctypes.c_int]
        L.ora_feistel_net.restype = ctypes.c_uint32
        L.ora_feistel_net.argtypes = [ctypes.c_uint32, ctypes.c_int64, _u32p]
        L.ora_feistel_domain.restype = ctypes.c_int64
        L.ora_feistel_domain.argtypes = [ctypes.c_int64]
        L.ora_feistel_pos.restype = ctypes.c_uint32
        L.ora_feistel_pos.argtypes = [ctypes.c_uint32, ctypes.c_int64, _u32p]
        L.ora_sample_size.restype = ctypes.c_int64
        L.ora_sample_size.argtypes = [ctypes.c_double, ctypes.c_int64]
        L.ora_sample_positions.restype = ctypes.c_int64
        L.ora_sample_positions.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _i32p]
        L.ora_power_lmax.restype = ctypes.c_double
        L.ora_power_lmax.argtypes = [_f64p, ctypes.c_int, ctypes.c_int]
        L.ora_lmax_cw.restype = ctypes.c_double
        L.ora_lmax_cw.argtypes = [_f64p, ctypes.c_int, ctypes.c_int]
        L.ora_set_lp_bound.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_set_gather_bf16.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_bf16.restype = ctypes.c_double
        L.ora_bf16.argtypes = [ctypes.c_double]
        L.ora_row_step.restype = ctypes.c_int64
        L.ora_row_step.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _f64p, _f64p,
                                   _f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


# ------------------------------------------------------------ free functions
def philox4x32(ctr, key, rounds: int = 10) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32(_p(c, _u32p), _p(k, _u32p), rounds, _p(out, _u32p))
    return out


def sample_keys(seed: int, k: int, mode: int, l: int, row: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_sample_keys(seed, k, mode, l, row, _p(out, _u32p))
    return out


def feistel_width(n: int) -> int:
    return lib().ora_feistel_width(n)


def feistel_rounds(w: int) -> int:
    return int(lib().ora_feistel_rounds(w))


def feistel_net(x: int, n: int, keys) -> int:
    """One pass of the network for a row of length n (x < feistel_domain(n))."""
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    return int(lib().ora_feistel_net(x, n, _p(k, _u32p)))


def feistel_domain(n: int) -> int:
    return int(lib().ora_feistel_domain(n))


def feistel_pos(j: int, n: int, keys) -> int:
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    return int(lib().ora_feistel_pos(j, n, _p(k, _u32p)))


def sample_size(c: float, n: int) -> int:
    return int(lib().ora_sample_size(c, n))


def sample_positions(seed: int, k: int, mode: int, l: int, row: int, n: int, c: float) -> np.ndarray:
    out = np.zeros(max(1, n), dtype=np.int32)
    b = lib().ora_sample_positions(seed, k, mode, l, row, n, c, _p(out, _i32p))
    return out[:b].copy()


def power_lmax(H: np.ndarray, iters: int = 20) -> float:
    H = np.ascontiguousarray(H, dtype=np.float64)
    return float(lib().ora_power_lmax(_p(H, _f64p), H.shape[0], iters))


def lmax_cw(H: np.ndarray, iters: int = 20) -> float:
    """Collatz-Wielandt upper bound max_i (H v)_i / v_i at the power method's
    `iters`-th normalised iterate (v_0 = ones / sqrt(R))."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    return float(lib().ora_lmax_cw(_p(H, _f64p), H.shape[0], iters))


def bf16(x: float) -> float:
    """The BF16 copy of a factor value (via its FP32 rounding), as the
    precision form gathers it."""
    return float(lib().ora_bf16(float(x)))


def set_threads(n: int) -> int:
    return int(lib().ora_set_threads(n))


# -------------------------------------------------------------------- solver
class Oracle:
    """FP64 reference solver for one completion instance."""

    def __init__(self, dims: Sequence[int], coords: np.ndarray, values: np.ndarray, rank: int, *,
                 c: float = 0.1, lam: float = 1e-3, max_inner: int = 1, power_iters: int = 20,
                 seed: int = 0, test_coords: Optional[np.ndarray] = None,
                 test_values: Optional[np.ndarray] = None, init: Optional[Sequence[np.ndarray]] = None,
                 lp_bound: int = 0, gather_bf16: bool = False):
        L = lib()
        self.dims = [int(d) for d in dims]
        self.N = len(self.dims)
        self.R = int(rank)
        d = np.asarray(self.dims, dtype=np.int64)
        co = np.ascontiguousarray(coords, dtype=np.int32)
        va = np.ascontiguousarray(values, dtype=np.float32)
        nnz = va.shape[0]
        if test_coords is None:
            tc = np.zeros((0, self.N), dtype=np.int32)
            tv = np.zeros(0, dtype=np.float32)
        else:
            tc = np.ascontiguousarray(test_coords, dtype=np.int32)
            tv = np.ascontiguousarray(test_values, dtype=np.float32)
        self._keep = [d, co, va, tc, tv]
        init_pp = None
        if init is not None:
            arrs = [np.ascontiguousarray(u, dtype=np.float32).reshape(-1) for u in init]
            self._keep.extend(arrs)
            init_pp = (_f32p * self.N)(*[_p(a, _f32p) for a in arrs])
        h = L.ora_create(self.N, _p(d, _i64p), nnz, _p(co, _i32p), _p(va, _f32p), self.R, c, lam,
                         max_inner, power_iters, seed, tv.shape[0], _p(tc, _i32p), _p(tv, _f32p), init_pp)
        if not h:
            raise ValueError("oracle rejected the problem")
        self._h = ctypes.c_void_p(h)
        L.ora_set_lp_bound(self._h, int(lp_bound))
        L.ora_set_gather_bf16(self._h, int(bool(gather_bf16)))
        self.c, self.lam, self.max_inner, self.power_iters, self.seed = c, lam, max_inner, power_iters, seed
        self.lp_bound = int(lp_bound)
        self.gather_bf16 = bool(gather_bf16)

    def close(self):
        if getattr(self, "_h", None):
            lib().ora_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n: int = 1):
        lib().ora_sweep(self._h, n)

    def update_mode(self, mode: int):
        lib().ora_update_mode(self._h, mode)

    def update_rows(self, mode: int, rows) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros((rows.shape[0], self.R), dtype=np.float64)
        lib().ora_update_rows(self._h, mode, _p(rows, _i64p), rows.shape[0], _p(out, _f64p))
        return out

    def loss(self) -> np.ndarray:
        out = np.zeros(4, dtype=np.float64)
        lib().ora_loss(self._h, _p(out, _f64p))
        return out

    def factors(self, mode: int) -> np.ndarray:
        out = np.zeros((self.dims[mode], self.R), dtype=np.float64)
        lib().ora_get_factors(self._h, mode, _p(out, _f64p))
        return out

    def set_factors(self, mode: int, U: np.ndarray):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (self.dims[mode], self.R)
        lib().ora_set_factors(self._h, mode, _p(U, _f64p))

    @property
    def sweep_count(self) -> int:
        return int(lib().ora_get_sweep(self._h))

    @sweep_count.setter
    def sweep_count(self, k: int):
        lib().ora_set_sweep(self._h, k)

    def csr(self, mode: int):
        rp = np.zeros(self.dims[mode] + 1, dtype=np.int64)
        perm = np.zeros(max(1, int(self._keep[2].shape[0])), dtype=np.int64)
        lib().ora_get_csr(self._h, mode, _p(rp, _i64p), _p(perm, _i64p))
        return rp, perm[: self._keep[2].shape[0]]

    def row_step(self, mode: int, l: int, row: int, y: np.ndarray, a: np.ndarray):
        """One inner step of one row: returns dict(a, y, g, H, L, beta, b)."""
        R = self.R
        y = np.ascontiguousarray(y, dtype=np.float64)
        a = np.ascontiguousarray(a, dtype=np.float64)
        an = np.zeros(R)
        yn = np.zeros(R)
        g = np.zeros(R)
        H = np.zeros((R, R))
        Lp = np.zeros(1)
        beta = np.zeros(1)
        b = lib().ora_row_step(self._h, mode, l, row, _p(y, _f64p), _p(a, _f64p), _p(an, _f64p),
                               _p(yn, _f64p), _p(g, _f64p), _p(H, _f64p), _p(Lp, _f64p), _p(beta, _f64p))
        return dict(a=an, y=yn, g=g, H=H, L=float(Lp[0]), beta=float(beta[0]), b=int(b))
