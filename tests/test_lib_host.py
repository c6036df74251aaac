"""CPU checks of libntc: it loads, exports every entry point of include/ntc.h,
and its host-side parts (sampler copy, CSR build, argument checks) agree
with the oracle bit for bit.  No compute call touches a device here."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle as O
import paper_2109_09534_amd as ntc
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(ntc_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_entry_point():
    L = ntc.lib()
    declared = _declared_symbols()
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", ntc.library_path()], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ntc_[a-z_0-9]+)$", out, flags=re.M))
    for name in declared:
        assert name in exported, name
        assert hasattr(L, name)
    # the binding wraps every declared entry point
    wrapped = {n for n, _, _ in ntc._SIGNATURES}
    assert set(declared) <= wrapped, set(declared) - wrapped
    assert b"gfx950" in L.ntc_version()


def test_host_sampler_is_bit_identical_to_the_oracle_sampler():
    rng = np.random.default_rng(0)
    for _ in range(400):
        n = int(rng.choice([1, 2, 3, 5, 9, 16, 17, 100, 1023, 1024, 1025, 70000, 2_000_001]))
        c = float(rng.choice([0.02, 0.1, 0.5, 0.57, 1.0]))
        args = dict(seed=int(rng.integers(0, 2**63)), k=int(rng.integers(0, 2**31)), mode=int(rng.integers(0, 8)),
                    l=int(rng.integers(0, 5)), row=int(rng.integers(0, 2**31 - 1)))
        if n * c > 300000:
            c = 0.02
        a = ntc.host_sample(n=n, c=c, **args)
        b = O.sample_positions(n=n, c=c, **args)
        assert np.array_equal(a, b), (n, c, args)


def test_host_csr_is_bit_identical_to_the_oracle_csr():
    for seed, dims, nnz in [(0, (30, 20, 10), 3000), (1, (7, 1, 9, 4), 200), (2, (1000, 50, 3), 120000)]:
        p = synth.make_problem(dims, nnz, 2, seed=seed, zipf_s=1.1 if nnz > 10000 else None)
        o = O.Oracle(p.dims, p.coords, p.values, 2)
        for m in range(len(dims)):
            rp, perm = ntc.host_csr(p.dims, p.coords, m)
            orp, operm = o.csr(m)
            assert np.array_equal(rp, orp)
            assert np.array_equal(perm, operm)


@pytest.mark.parametrize("kw,msg", [
    (dict(rank=0), "rank"), (dict(rank=65), "rank"), (dict(c=0.0), "c must"), (dict(c=1.5), "c must"),
    (dict(lam=-1.0), "lambda"), (dict(max_inner=0), "max_inner"), (dict(power_iters=-1), "power_iters"),
    (dict(lp_bound=2), "lp_bound"), (dict(schedule={"overlap": 3}), "overlap"),
    (dict(device_csr=True, c=0.0), "c must"), (dict(device_csr=True, rank=65), "rank"),
])
def test_create_rejects_invalid_parameters_before_touching_a_device(kw, msg):
    p = synth.tiny(seed=0)
    args = dict(rank=3)
    args.update(kw)
    rank = args.pop("rank")
    with pytest.raises(ntc.NtcError) as e:
        ntc.Problem(p.dims, p.coords, p.values, rank, stream=0, **args)
    assert e.value.status == ntc.NTC_EINVAL and msg in str(e.value)


def test_create_rejects_bad_data():
    p = synth.tiny(seed=0)
    bad = p.coords.copy()
    bad[3, 1] = p.dims[1]
    with pytest.raises(ntc.NtcError, match="coordinate out of range"):
        ntc.Problem(p.dims, bad, p.values, 3, stream=0)
    v = p.values.copy()
    v[0] = np.nan
    with pytest.raises(ntc.NtcError, match="non-finite"):
        ntc.Problem(p.dims, p.coords, v, 3, stream=0)
    init = synth.uniform_init(p.dims, 3, 0)
    init[1][0, 0] = -1.0
    with pytest.raises(ntc.NtcError, match="negative"):
        ntc.Problem(p.dims, p.coords, p.values, 3, init=init, stream=0)
    with pytest.raises(ntc.NtcError, match="nmodes"):
        ntc.Problem([5], np.zeros((0, 1), np.int32), np.zeros(0, np.float32), 3, stream=0)


def test_estimate_bytes_bounds_the_allocations():
    """The admission estimate is host-only arithmetic: it covers at least the
    records and factors and grows with every size."""
    import paper_2109_09534_amd as ntc
    dims = [480_000, 18_000, 2_000]
    b = ntc.estimate_bytes(dims, 95_000_000, 16, n_test=5_000_000)
    records = 3 * 95_000_000 * 16
    factors = sum((d + 1) * 16 * 4 for d in dims)
    assert b >= records + factors
    assert ntc.estimate_bytes(dims, 95_000_000, 16, n_test=5_000_000, gather_bf16=True) > b
    assert ntc.estimate_bytes(dims, 95_000_000, 32, n_test=5_000_000) > b
    assert ntc.estimate_bytes(dims, 96_000_000, 16, n_test=5_000_000) > b
    assert ntc.estimate_bytes(dims, 95_000_000, 16, n_test=5_000_000, max_inner=2) > b
    with pytest.raises(ntc.NtcError):
        ntc.estimate_bytes([10, 0, 3], 5, 4)


def test_autotune_candidates_cover_both_kernel_families():
    from paper_2109_09534_amd import autotune
    narrow, wide = autotune.candidates_for(16), autotune.candidates_for(32)
    assert {} in narrow and {} in wide
    allowed = {"tiny_max", "item_samples", "overlap", "group_max"}
    for c in narrow + wide:
        assert set(c) <= allowed
        for v in c.values():
            assert isinstance(v, int)


def test_prepare_runs_on_the_host_and_bounds_its_bytes():
    """ntc_prepare needs no device: the CSR, schedule and copies are host work.
    Its exact byte count stays under the admission upper bound."""
    import paper_2109_09534_amd as ntc
    for dims, nnz, R in [((100, 80, 60), 21600, 8), ((30, 20, 10, 8), 20000, 24), ((400, 300), 30000, 50)]:
        p = synth.make_problem(dims, nnz, min(R, 8), seed=1, test_frac=0.1)
        q = ntc.Prepared(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values)
        exact = q.device_bytes
        bound = ntc.estimate_bytes(p.dims, p.nnz, R, n_test=p.test_values.shape[0])
        assert 0 < exact <= bound, (dims, exact, bound)
        q.close()
    bad = synth.tiny()
    co = bad.coords.copy()
    co[0, 0] = bad.dims[0]
    with pytest.raises(ntc.NtcError):
        ntc.Prepared(bad.dims, co, bad.values, 3)


def test_scaling_twin_is_the_timing_workload_of_section_iv_c():
    """The twin of the paper's timing workload: 183x24x1140x1717, 3,309,490
    distinct cells, values the noiseless rank-10 CPD of U[0,1] factors."""
    p = synth.scaling_twin(seed=0)
    assert p.dims == [183, 24, 1140, 1717] and p.nnz == 3_309_490 and p.test_values.shape[0] == 0
    co = p.coords.astype(np.int64)
    assert np.all(co >= 0) and np.all(co < np.asarray(p.dims))
    key = ((co[:, 0] * 24 + co[:, 1]) * 1140 + co[:, 2]) * 1717 + co[:, 3]
    assert np.unique(key).shape[0] == p.nnz
    assert len(p.planted) == 4 and all(f.shape[1] == 10 and f.min() >= 0 and f.max() <= 1 for f in p.planted)
    idx = np.arange(0, p.nnz, 9973)
    ref = np.ones((idx.shape[0], 10))
    for m in range(4):
        ref *= p.planted[m][co[idx, m]]
    np.testing.assert_allclose(p.values[idx], ref.sum(axis=1).astype(np.float32), rtol=0, atol=0)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus above 1 exits with status 2 and a message, before any work."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""
