"""Python binding of libntc (AO accelerated stochastic nonnegative tensor
completion on an MI355X).

Argument marshalling only: every step of the method runs in the HIP library
behind the C ABI of ``include/ntc.h``.  PyTorch is used, optionally, for the
HIP stream the work is enqueued on and for device memory (its caching
allocator).  If ``libntc.so`` has not been built, importing works but every
call raises ``LibraryMissing`` -- there is no CPU fallback.

PyTorch wheels bundle their own HIP runtime under the same soname
(libamdhip64.so.7) as the system ROCm runtime libntc links.  Whichever is
loaded first serves the whole process: to share streams and memory with
torch, import torch before the first call into this module; torch interop
is refused when two HIP runtimes are mapped.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

__all__ = ["Problem", "NtcError", "LibraryMissing", "lib", "host_sample", "host_csr", "library_path",
           "hip_runtimes"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libntc.so")

NTC_OK, NTC_EINVAL, NTC_ENOMEM, NTC_EDEVICE, NTC_EUNSUPPORTED, NTC_ENONFINITE, NTC_ESTATE = 0, -1, -2, -3, -4, -5, -6
_STATUS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED", -5: "ENONFINITE", -6: "ESTATE"}

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class LibraryMissing(RuntimeError):
    pass


class NtcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ntc {_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [
        ("c", ctypes.c_double),
        ("lam", ctypes.c_double),
        ("max_inner", ctypes.c_int32),
        ("power_iters", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("gather_bf16", ctypes.c_int32),
        ("tiny_max", ctypes.c_int32),
        ("n_test", ctypes.c_int64),
        ("test_coords", _i32p),
        ("test_values", _f32p),
        ("init_factors", ctypes.POINTER(_f32p)),
        ("stream", ctypes.c_void_p),
        ("dev_alloc", _ALLOC_FN),
        ("dev_free", _FREE_FN),
        ("alloc_ctx", ctypes.c_void_p),
        ("item_samples", ctypes.c_int32),
        ("overlap", ctypes.c_int32),
        ("group_max", ctypes.c_int32),
        ("lp_bound", ctypes.c_int32),
    ]


class _PoolParams(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("window", ctypes.c_int32), ("max_sweeps", ctypes.c_int32), ("tol", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class LaunchRecord(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("mode", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("samples", ctypes.c_int64), ("rows", ctypes.c_int64),
                ("ms", ctypes.c_double)]


_lib = None

# (name, restype, argtypes) of every exported entry point of include/ntc.h
_SIGNATURES = [
    ("ntc_params_default", None, [ctypes.POINTER(_Params)]),
    ("ntc_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, _i64p, ctypes.c_int64, _i32p,
                                  _f32p, ctypes.c_int32, ctypes.POINTER(_Params)]),
    ("ntc_create_device_csr", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, _i64p,
                                             ctypes.c_int64, _i32p, _f32p, ctypes.c_int32,
                                             ctypes.POINTER(_Params)]),
    ("ntc_sweep", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("ntc_update_mode", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("ntc_loss", ctypes.c_int, [ctypes.c_void_p, _f64p]),
    ("ntc_loss_coo_noalloc", ctypes.c_int, [ctypes.c_int32, _i64p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.c_double, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    ("ntc_get_factors", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f32p]),
    ("ntc_set_factors", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f32p]),
    ("ntc_get_factors_device", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    ("ntc_get_sweep", ctypes.c_int, [ctypes.c_void_p, _i64p]),
    ("ntc_set_sweep", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    ("ntc_get_work", ctypes.c_int, [ctypes.c_void_p, _i64p, _i64p]),
    ("ntc_debug_sample", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int64, _i32p, _i32p]),
    ("ntc_debug_csr", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _i64p, ctypes.POINTER(ctypes.c_uint32)]),
    ("ntc_host_sample", ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _i32p, _i64p]),
    ("ntc_host_csr", ctypes.c_int, [ctypes.c_int32, _i64p, ctypes.c_int64, _i32p, ctypes.c_int32, _i64p, _i64p]),
    ("ntc_synchronize", ctypes.c_int, [ctypes.c_void_p]),
    ("ntc_time_sweeps", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p]),
    ("ntc_profile_sweep", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(LaunchRecord), ctypes.c_int32,
                                         _i32p]),
    ("ntc_profile_sweeps", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(LaunchRecord), ctypes.c_int32, _i32p]),
    ("ntc_release", ctypes.c_int, [ctypes.c_void_p]),
    ("ntc_estimate_bytes", ctypes.c_int, [ctypes.c_int32, _i64p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_size_t)]),
    ("ntc_prepare", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, _i64p, ctypes.c_int64, _i32p,
                                   _f32p, ctypes.c_int32, ctypes.POINTER(_Params)]),
    ("ntc_create_prepared", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                           ctypes.POINTER(_Params)]),
    ("ntc_prepared_bytes", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    ("ntc_prepared_release", ctypes.c_int, [ctypes.c_void_p]),
    ("ntc_prepared_schedule", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _i64p, _i64p, _i32p, _i32p, _i32p,
                                             _i32p]),
    ("ntc_pool_admit_prepared", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _i32p]),
    ("ntc_pool_params_default", None, [ctypes.POINTER(_PoolParams)]),
    ("ntc_pool_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(_PoolParams)]),
    ("ntc_pool_admit", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _i64p, ctypes.c_int64, _i32p, _f32p,
                                      ctypes.c_int32, ctypes.POINTER(_Params), _i32p]),
    ("ntc_pool_admit_device_csr", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _i64p, ctypes.c_int64, _i32p,
                                                 _f32p, ctypes.c_int32, ctypes.POINTER(_Params), _i32p]),
    ("ntc_pool_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("ntc_pool_query", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _i32p, _i64p, _f64p]),
    ("ntc_pool_loss", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p]),
    ("ntc_pool_get_factors", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _f32p]),
    ("ntc_pool_stopped", ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int32, _i32p]),
    ("ntc_pool_evict", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("ntc_pool_info", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t), _i32p, _i32p, _i64p]),
    ("ntc_pool_release", ctypes.c_int, [ctypes.c_void_p]),
    ("ntc_last_error", ctypes.c_char_p, []),
    ("ntc_version", ctypes.c_char_p, []),
]


def library_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libntc.so; raises LibraryMissing if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise LibraryMissing(f"{_LIB_PATH} is not built; run `python -m paper_2109_09534_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def hip_runtimes() -> List[str]:
    """Paths of the HIP runtime libraries mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return sorted(paths)


def _require_single_runtime():
    rt = hip_runtimes()
    if len(rt) > 1:
        raise NtcError(NTC_ESTATE, "two HIP runtimes are loaded (" + ", ".join(rt) + "); import torch before "
                       "paper_2109_09534_amd to share streams and memory with it")


def _check(status: int):
    if status != NTC_OK:
        raise NtcError(status, lib().ntc_last_error().decode(errors="replace"))


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def loss_coo_noalloc(dims: Sequence[int], rank: int, n_train: int, train_coords: int, train_values: int,
                     n_test: int, test_coords: int, test_values: int, factors: Sequence[int], lam: float, out: int,
                     stream: int = 0):
    """ntc_loss_coo_noalloc: every array argument is a DEVICE address (an
    int, e.g. a torch tensor's data_ptr()); out receives 4 doubles on
    `stream`.  Nothing is allocated, copied or synchronised."""
    d = np.ascontiguousarray(dims, dtype=np.int64)
    fp = (ctypes.c_void_p * len(factors))(*[ctypes.c_void_p(int(f)) for f in factors])
    _check(lib().ntc_loss_coo_noalloc(len(dims), _p(d, _i64p), rank, n_train, ctypes.c_void_p(train_coords),
                                      ctypes.c_void_p(train_values), n_test, ctypes.c_void_p(test_coords),
                                      ctypes.c_void_p(test_values), fp, lam, ctypes.c_void_p(out),
                                      ctypes.c_void_p(stream)))


def host_sample(seed: int, k: int, mode: int, l: int, row: int, n: int, c: float) -> np.ndarray:
    """The library's host copy of the minibatch sampler (no device)."""
    out = np.zeros(max(1, n), dtype=np.int32)
    cnt = ctypes.c_int64(0)
    _check(lib().ntc_host_sample(seed, k, mode, l, row, n, c, _p(out, _i32p), ctypes.byref(cnt)))
    return out[: cnt.value].copy()


def host_csr(dims: Sequence[int], coords: np.ndarray, mode: int):
    """The library's host CSR build of one mode: (rowptr, perm)."""
    d = np.asarray(dims, dtype=np.int64)
    co = np.ascontiguousarray(coords, dtype=np.int32)
    nnz = co.shape[0]
    rp = np.zeros(int(d[mode]) + 1, dtype=np.int64)
    perm = np.zeros(max(1, nnz), dtype=np.int64)
    _check(lib().ntc_host_csr(len(dims), _p(d, _i64p), nnz, _p(co, _i32p), mode, _p(rp, _i64p), _p(perm, _i64p)))
    return rp, perm[:nnz]


def _make_params(N, c, lam, max_inner, power_iters, seed, gather_bf16, test_coords, test_values, init, schedule,
                 lp_bound=0):
    """ntc_params for ntc_create / ntc_pool_admit, plus the arrays it points into."""
    prm = _Params()
    lib().ntc_params_default(ctypes.byref(prm))
    prm.c, prm.lam, prm.max_inner, prm.power_iters, prm.seed = c, lam, max_inner, power_iters, seed
    prm.gather_bf16 = 1 if gather_bf16 else 0
    prm.lp_bound = int(lp_bound)
    for key, val in (schedule or {}).items():
        if key not in ("tiny_max", "item_samples", "overlap", "group_max"):
            raise ValueError(f"unknown schedule field {key}")
        setattr(prm, key, int(val))
    keep = []
    if test_coords is not None:
        tc = np.ascontiguousarray(test_coords, dtype=np.int32)
        tv = np.ascontiguousarray(test_values, dtype=np.float32)
        keep += [tc, tv]
        prm.n_test = tv.shape[0]
        prm.test_coords = _p(tc, _i32p)
        prm.test_values = _p(tv, _f32p)
    if init is not None:
        arrs = [np.ascontiguousarray(u, dtype=np.float32).reshape(-1) for u in init]
        keep += arrs
        ptrs = (_f32p * N)(*[_p(a, _f32p) for a in arrs])
        keep.append(ptrs)
        prm.init_factors = ptrs
    return prm, keep


def estimate_bytes(dims: Sequence[int], nnz: int, rank: int, **kw) -> int:
    """Upper bound of the device bytes ntc_create allocates (ntc_estimate_bytes)."""
    d = np.asarray([int(x) for x in dims], dtype=np.int64)
    prm, _ = _make_params(len(d), kw.get("c", 0.1), kw.get("lam", 1e-3), kw.get("max_inner", 1),
                          kw.get("power_iters", 20), kw.get("seed", 0), kw.get("gather_bf16", False), None, None,
                          None, kw.get("schedule"))
    prm.n_test = int(kw.get("n_test", 0))
    out = ctypes.c_size_t()
    _check(lib().ntc_estimate_bytes(len(d), _p(d, _i64p), int(nnz), int(rank), ctypes.byref(prm),
                                    ctypes.byref(out)))
    return out.value


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self, device: int):
        import torch
        self._torch = torch
        self._device = device

        def _alloc(nbytes, stream, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self._device, stream))
            except Exception:
                return None

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc = _ALLOC_FN(_alloc)
        self.free = _FREE_FN(_free)


class Problem:
    """One completion instance resident on the GPU (ntc_create ... ntc_release).

    ``stream``: None or 0 for the null stream, a raw hipStream_t int, or a
    ``torch.cuda.Stream`` (torch must share libntc's HIP runtime).
    ``torch_allocator``: route device memory through torch's caching allocator.
    ``device_csr``: build the per-mode CSR on the GPU (ntc_create_device_csr);
    every result is bit-identical to the host build.
    """

    def __init__(self, dims: Sequence[int], coords: np.ndarray, values: np.ndarray, rank: int, *,
                 c: float = 0.1, lam: float = 1e-3, max_inner: int = 1, power_iters: int = 20, seed: int = 0,
                 gather_bf16: bool = False, test_coords: Optional[np.ndarray] = None,
                 test_values: Optional[np.ndarray] = None, init: Optional[Sequence[np.ndarray]] = None,
                 stream=None, torch_allocator: bool = False, schedule: Optional[dict] = None,
                 lp_bound: int = 0, device_csr: bool = False):
        L = lib()
        self.dims = [int(d) for d in dims]
        self.N = len(self.dims)
        self.R = int(rank)
        d = np.asarray(self.dims, dtype=np.int64)
        co = np.ascontiguousarray(coords, dtype=np.int32)
        va = np.ascontiguousarray(values, dtype=np.float32)
        if co.ndim != 2 or co.shape[1] != self.N or co.shape[0] != va.shape[0]:
            raise ValueError("coords must be [nnz, nmodes] and values [nnz]")
        prm, keep = _make_params(self.N, c, lam, max_inner, power_iters, seed, gather_bf16, test_coords,
                                 test_values, init, schedule, lp_bound)
        keep += [d, co, va]
        if torch_allocator or (stream is not None and not isinstance(stream, int)):
            _require_single_runtime()
        prm.stream = self._stream_handle(stream)
        self._allocator = None
        if torch_allocator:
            import torch
            self._allocator = _TorchAllocator(torch.cuda.current_device())
            prm.dev_alloc = self._allocator.alloc
            prm.dev_free = self._allocator.free
        h = ctypes.c_void_p()
        create = L.ntc_create_device_csr if device_csr else L.ntc_create
        _check(create(ctypes.byref(h), self.N, _p(d, _i64p), co.shape[0], _p(co, _i32p), _p(va, _f32p),
                      self.R, ctypes.byref(prm)))
        self._h = h
        self.c, self.lam, self.max_inner, self.power_iters, self.seed = c, lam, max_inner, power_iters, seed
        self.gather_bf16 = gather_bf16

    @classmethod
    def from_prepared(cls, prepared: "Prepared", *, c: float = 0.1, lam: float = 1e-3, max_inner: int = 1,
                      power_iters: int = 20, seed: int = 0, gather_bf16: bool = False, stream=None) -> "Problem":
        """The device half of ntc_create on a Prepared problem.  The method
        parameters are those the problem was prepared with; the ones given
        here only label the Python object."""
        self = cls.__new__(cls)
        prm = _Params()
        lib().ntc_params_default(ctypes.byref(prm))
        if stream is not None and not isinstance(stream, int):
            _require_single_runtime()
        prm.stream = cls._stream_handle(stream)
        h = ctypes.c_void_p()
        _check(lib().ntc_create_prepared(ctypes.byref(h), prepared._h, ctypes.byref(prm)))
        self._h = h
        self._allocator = None
        self.dims, self.N, self.R = list(prepared.dims), len(prepared.dims), prepared.rank
        self.c, self.lam, self.max_inner, self.power_iters, self.seed = c, lam, max_inner, power_iters, seed
        self.gather_bf16 = gather_bf16
        return self

    @staticmethod
    def _stream_handle(stream):
        if stream is None or stream == 0:
            return None
        if isinstance(stream, int):
            return stream
        return stream.cuda_stream

    # -------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ntc_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- method
    def sweep(self, n: int = 1):
        _check(lib().ntc_sweep(self._h, n))

    def synchronize(self):
        _check(lib().ntc_synchronize(self._h))

    def time_sweeps(self, n: int) -> float:
        """Device milliseconds of `n` sweeps between HIP events on the handle's stream."""
        ms = ctypes.c_double(0.0)
        _check(lib().ntc_time_sweeps(self._h, n, ctypes.byref(ms)))
        return ms.value

    def profile_sweep(self):
        """One sweep with HIP events around every launch, all on one stream: list of dicts."""
        return self.profile_sweeps(1, concurrent=False)

    def profile_sweeps(self, nsweeps: int, concurrent: bool = True):
        """`nsweeps` sweeps with HIP events around every launch on its own
        stream (concurrent: with the side-stream overlap of a plain sweep):
        list of dicts in launch order, sweep after sweep."""
        cap = 4096 * max(nsweeps, 1)
        buf = (LaunchRecord * cap)()
        cnt = ctypes.c_int32(0)
        _check(lib().ntc_profile_sweeps(self._h, nsweeps, int(bool(concurrent)), buf, cap, ctypes.byref(cnt)))
        return [dict(kernel=("row_items", "row_finalize", "row_tiny", "row_chunks", "row_reduce", "row_few")[r.kernel], mode=r.mode, inner=r.inner, blocks=r.blocks,
                     samples=r.samples, rows=r.rows, ms=r.ms) for r in buf[: min(cnt.value, cap)]]

    def update_mode(self, mode: int):
        _check(lib().ntc_update_mode(self._h, mode))

    def loss(self) -> np.ndarray:
        """[objective, train RMSE, test RMSE, test relative error]."""
        out = np.zeros(4, dtype=np.float64)
        _check(lib().ntc_loss(self._h, _p(out, _f64p)))
        return out

    def factors(self, mode: int) -> np.ndarray:
        out = np.zeros((self.dims[mode], self.R), dtype=np.float32)
        _check(lib().ntc_get_factors(self._h, mode, _p(out, _f32p)))
        return out

    def all_factors(self) -> List[np.ndarray]:
        return [self.factors(m) for m in range(self.N)]

    def set_factors(self, mode: int, U: np.ndarray):
        U = np.ascontiguousarray(U, dtype=np.float32)
        if U.shape != (self.dims[mode], self.R):
            raise ValueError("factor shape mismatch")
        _check(lib().ntc_set_factors(self._h, mode, _p(U, _f32p)))

    def factors_into(self, mode: int, tensor):
        """Copy mode's factor into a device torch tensor (float32, I x R)."""
        if tensor.dtype.itemsize != 4 or tensor.numel() != self.dims[mode] * self.R or not tensor.is_contiguous():
            raise ValueError("need a contiguous float32 tensor of I_m * R elements")
        _check(lib().ntc_get_factors_device(self._h, mode, ctypes.c_void_p(tensor.data_ptr())))

    @property
    def sweep_count(self) -> int:
        k = ctypes.c_int64(0)
        _check(lib().ntc_get_sweep(self._h, ctypes.byref(k)))
        return k.value

    @sweep_count.setter
    def sweep_count(self, k: int):
        _check(lib().ntc_set_sweep(self._h, k))

    def work(self):
        """(sampled-entry updates per sweep, row steps per sweep)."""
        u = ctypes.c_int64(0)
        r = ctypes.c_int64(0)
        _check(lib().ntc_get_work(self._h, ctypes.byref(u), ctypes.byref(r)))
        return u.value, r.value

    def debug_sample(self, k: int, mode: int, l: int, row: int, n_hint: int) -> np.ndarray:
        """Positions drawn by the device sampler for one row (n_hint >= row length)."""
        out = np.zeros(max(1, n_hint), dtype=np.int32)
        cnt = ctypes.c_int32(0)
        _check(lib().ntc_debug_sample(self._h, k, mode, l, row, _p(out, _i32p), ctypes.byref(cnt)))
        return out[: cnt.value].copy()

    def debug_csr(self, mode: int, nnz: int):
        """(rowptr [I+1] int64, records [nnz][W] uint32) of one mode as held on the device."""
        W = 4 if self.N <= 4 else 8
        rp = np.zeros(self.dims[mode] + 1, dtype=np.int64)
        rec = np.zeros((max(1, nnz), W), dtype=np.uint32)
        _check(lib().ntc_debug_csr(self._h, mode, _p(rp, _i64p), rec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
        return rp, rec[:nnz]


SLOT_FREE, SLOT_RUNNING, SLOT_STOPPED = 0, 1, 2


class Prepared:
    """The host half of ntc_create (ntc_prepare): CSR of every mode, row
    schedule and copies of the held-out set and init, with no device work.
    The C call releases the GIL, so problems can be prepared on worker
    threads while the GPU sweeps."""

    def __init__(self, dims: Sequence[int], coords: np.ndarray, values: np.ndarray, rank: int, *, c: float = 0.1,
                 lam: float = 1e-3, max_inner: int = 1, power_iters: int = 20, seed: int = 0,
                 gather_bf16: bool = False, test_coords=None, test_values=None, init=None,
                 schedule: Optional[dict] = None, lp_bound: int = 0):
        d = np.asarray([int(x) for x in dims], dtype=np.int64)
        co = np.ascontiguousarray(coords, dtype=np.int32)
        va = np.ascontiguousarray(values, dtype=np.float32)
        if co.ndim != 2 or co.shape[1] != d.size or co.shape[0] != va.shape[0]:
            raise ValueError("coords must be [nnz, nmodes] and values [nnz]")
        prm, keep = _make_params(d.size, c, lam, max_inner, power_iters, seed, gather_bf16, test_coords,
                                 test_values, init, schedule, lp_bound)
        h = ctypes.c_void_p()
        _check(lib().ntc_prepare(ctypes.byref(h), d.size, _p(d, _i64p), co.shape[0], _p(co, _i32p), _p(va, _f32p),
                                 int(rank), ctypes.byref(prm)))
        self._h = h
        self.dims, self.rank = [int(x) for x in d], int(rank)

    def row_schedule(self, mode: int) -> dict:
        """The host row schedule of one mode (ntc_prepared_schedule): rowptr and
        the tiny/items/split/groups tables as [n, 4] int32 arrays."""
        cnt = np.zeros(7, dtype=np.int64)
        _check(lib().ntc_prepared_schedule(self._h, mode, _p(cnt, _i64p), None, None, None, None, None))
        rp = np.zeros(self.dims[mode] + 1, dtype=np.int64)
        arr = {k: np.zeros((max(1, int(n)), 4), dtype=np.int32)
               for k, n in zip(("tiny", "items", "split", "groups"), (cnt[0], cnt[1], cnt[3], cnt[4]))}
        _check(lib().ntc_prepared_schedule(self._h, mode, _p(cnt, _i64p), _p(rp, _i64p), _p(arr["tiny"], _i32p),
                                           _p(arr["items"], _i32p), _p(arr["split"], _i32p), _p(arr["groups"], _i32p)))
        out = {k: arr[k][: int(n)] for k, n in zip(("tiny", "items", "split", "groups"), (cnt[0], cnt[1], cnt[3],
                                                                                          cnt[4]))}
        out.update(rowptr=rp, n_group=int(cnt[2]), n_slots=int(cnt[5]), samples=int(cnt[6]))
        return out

    @property
    def device_bytes(self) -> int:
        out = ctypes.c_size_t()
        _check(lib().ntc_prepared_bytes(self._h, ctypes.byref(out)))
        return out.value

    def close(self):
        if getattr(self, "_h", None):
            lib().ntc_prepared_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Many independent problems on one GPU (ntc_pool_*): one device memory
    arena, batched launches over all running problems, a HIP graph per sweep,
    and a held-out plateau stop rule."""

    def __init__(self, arena_bytes: int = 0, max_slots: int = 1024, use_graph: bool = True, window: int = 5,
                 max_sweeps: int = 500, tol: float = 1e-4):
        L = lib()
        prm = _PoolParams()
        L.ntc_pool_params_default(ctypes.byref(prm))
        prm.arena_bytes, prm.max_slots, prm.use_graph = int(arena_bytes), int(max_slots), 1 if use_graph else 0
        prm.window, prm.max_sweeps, prm.tol = int(window), int(max_sweeps), float(tol)
        h = ctypes.c_void_p()
        _check(L.ntc_pool_create(ctypes.byref(h), ctypes.byref(prm)))
        self._h = h
        self._dims = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().ntc_pool_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def admit(self, dims: Sequence[int], coords: np.ndarray, values: np.ndarray, rank: int, *, c: float = 0.1,
              lam: float = 1e-3, max_inner: int = 1, power_iters: int = 20, seed: int = 0,
              gather_bf16: bool = False, test_coords=None, test_values=None, init=None,
              schedule: Optional[dict] = None, lp_bound: int = 0, device_csr: bool = False) -> Optional[int]:
        """Slot index, or None when the pool cannot hold the problem now.
        device_csr: build the CSR on the device (ntc_pool_admit_device_csr)."""
        d = np.asarray([int(x) for x in dims], dtype=np.int64)
        co = np.ascontiguousarray(coords, dtype=np.int32)
        va = np.ascontiguousarray(values, dtype=np.float32)
        if co.ndim != 2 or co.shape[1] != d.size or co.shape[0] != va.shape[0]:
            raise ValueError("coords must be [nnz, nmodes] and values [nnz]")
        prm, keep = _make_params(d.size, c, lam, max_inner, power_iters, seed, gather_bf16, test_coords,
                                 test_values, init, schedule, lp_bound)
        slot = ctypes.c_int32(-1)
        fn = lib().ntc_pool_admit_device_csr if device_csr else lib().ntc_pool_admit
        st = fn(self._h, d.size, _p(d, _i64p), co.shape[0], _p(co, _i32p), _p(va, _f32p), int(rank),
                ctypes.byref(prm), ctypes.byref(slot))
        if st == -2:      # NTC_ENOMEM: not admitted now
            return None
        _check(st)
        self._dims[slot.value] = (list(int(x) for x in d), int(rank))
        return slot.value

    def admit_prepared(self, prepared: "Prepared") -> Optional[int]:
        """Slot index, or None when the pool cannot hold it now."""
        slot = ctypes.c_int32(-1)
        st = lib().ntc_pool_admit_prepared(self._h, prepared._h, ctypes.byref(slot))
        if st == -2:      # NTC_ENOMEM: not admitted now
            return None
        _check(st)
        self._dims[slot.value] = (list(prepared.dims), prepared.rank)
        return slot.value

    def step(self, n: int = 1):
        _check(lib().ntc_pool_step(self._h, int(n)))

    def query(self, slot: int):
        """(state, sweeps, last held-out RMSE)."""
        st, sw, rm = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().ntc_pool_query(self._h, int(slot), ctypes.byref(st), ctypes.byref(sw), ctypes.byref(rm)))
        return st.value, sw.value, rm.value

    def loss(self, slot: int) -> np.ndarray:
        out = np.zeros(4, dtype=np.float64)
        _check(lib().ntc_pool_loss(self._h, int(slot), _p(out, _f64p)))
        return out

    def factors(self, slot: int, mode: int) -> np.ndarray:
        dims, R = self._dims[slot]
        out = np.empty((dims[mode], R), dtype=np.float32)
        _check(lib().ntc_pool_get_factors(self._h, int(slot), int(mode), _p(out, _f32p)))
        return out

    def stopped(self) -> List[int]:
        n = ctypes.c_int32()
        _check(lib().ntc_pool_stopped(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(lib().ntc_pool_stopped(self._h, _p(out, _i32p), out.size, ctypes.byref(n)))
        return [int(x) for x in out[:n.value]]

    def evict(self, slot: int):
        _check(lib().ntc_pool_evict(self._h, int(slot)))
        self._dims.pop(slot, None)

    def info(self) -> dict:
        used, free = ctypes.c_size_t(), ctypes.c_size_t()
        run, stp, sw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().ntc_pool_info(self._h, ctypes.byref(used), ctypes.byref(free), ctypes.byref(run),
                                   ctypes.byref(stp), ctypes.byref(sw)))
        return {"used": used.value, "free": free.value, "running": run.value, "stopped": stp.value,
                "sweeps": sw.value}
