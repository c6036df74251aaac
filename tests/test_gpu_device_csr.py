"""ntc_create_device_csr: the per-mode CSR built on the GPU (stable radix
sort by coordinate) must give exactly what the host build gives, so every
later result is bit-identical; bad entries are reported as ntc_create
reports them."""
import sys

import numpy as np
import pytest

import paper_2109_09534_amd as ntc
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "3way_r8": lambda: (synth.c0(seed=1), 8, {}),
    "zipf_r16_split": lambda: (synth.c1_small(seed=2), 16, {}),
    "4way_r32_bf16": lambda: (synth.make_problem((60, 50, 40, 30), 80_000, 12, seed=3, zipf_s=1.1), 32,
                              dict(gather_bf16=True)),
    "matrix_r20": lambda: (synth.make_problem((500, 400), 60_000, 8, seed=4), 20, {}),
    "5way_r10": lambda: (synth.make_problem((20, 15, 12, 10, 8), 40_000, 5, seed=5), 10, dict(max_inner=2)),
    "4way_r50": lambda: (synth.make_problem((183, 24, 114, 171), 100_000, 10, seed=6), 50, dict(c=0.5)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_device_csr_is_bit_identical_to_the_host_build(case):
    p, R, kw = CASES[case]()
    kw = dict(kw)
    kw.setdefault("c", 0.1)
    _say(f"case {case}: dims {p.dims} nnz {p.nnz} R {R} {kw}")
    out = []
    for dev in (False, True):
        g = ntc.Problem(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                        seed=7, stream=0, device_csr=dev, **kw)
        work = g.work()
        l0 = g.loss()
        g.sweep(3)
        out.append(([g.factors(m) for m in range(len(p.dims))], [l0, g.loss()], work))
        g.close()
    (fh, lh, wh), (fd, ld, wd) = out
    assert wh == wd
    for m in range(len(p.dims)):
        assert np.array_equal(fh[m], fd[m]), (case, m)
    for a, b in zip(lh, ld):
        assert np.array_equal(a, b), (case, a, b)


def test_device_csr_reports_bad_entries_like_the_host():
    p = synth.c0(seed=3)
    co = p.coords.copy()
    co[1234, 1] = p.dims[1]
    msgs = []
    for dev in (False, True):
        with pytest.raises(Exception) as ex:
            ntc.Problem(p.dims, co, p.values, 8, stream=0, device_csr=dev)
        msgs.append(str(ex.value))
    assert "entry 1234" in msgs[0] and msgs[0] == msgs[1], msgs
    va = p.values.copy()
    va[77] = np.nan
    va[900] = np.inf
    msgs = []
    for dev in (False, True):
        with pytest.raises(Exception) as ex:
            ntc.Problem(p.dims, p.coords, va, 8, stream=0, device_csr=dev)
        msgs.append(str(ex.value))
    assert "entry 77" in msgs[0] and msgs[0] == msgs[1], msgs


def test_device_csr_with_no_entries():
    dims = [5, 4, 3]
    co = np.zeros((0, 3), dtype=np.int32)
    va = np.zeros(0, dtype=np.float32)
    init = synth.uniform_init(dims, 4, 1, 1.0)
    g = ntc.Problem(dims, co, va, 4, init=init, stream=0, device_csr=True)
    g.sweep(2)
    for m in range(3):
        assert np.array_equal(g.factors(m), init[m])
    g.close()


@pytest.mark.parametrize("case", ["3way_r8", "zipf_r16_split", "4way_r32_bf16", "matrix_r20", "5way_r10"])
def test_csr_on_the_device_equals_the_oracle_csr(case):
    """The row pointers and records the library holds on the device, from the
    device build and from the host build, against the oracle's CSR (a stable
    counting sort by coordinate, ties in COO order): rowptr equal, and record
    q of mode m is entry perm[q]'s other coordinates times R in increasing
    mode order, then its value bits, then zeros (mode 0 with N < W: word N
    holds the entry's own coordinate times R)."""
    import oracle as O
    O.build(force=False)
    p, R, kw = CASES[case]()
    N = len(p.dims)
    W = 4 if N <= 4 else 8
    o = O.Oracle(p.dims, p.coords, p.values, R, c=0.1)
    vbits = np.ascontiguousarray(p.values, dtype=np.float32).view(np.uint32)
    for dev in (False, True):
        g = ntc.Problem(p.dims, p.coords, p.values, R, c=0.1, stream=0, device_csr=dev)
        for m in range(N):
            rp_o, perm = o.csr(m)
            rp_g, rec = g.debug_csr(m, p.nnz)
            assert np.array_equal(rp_g, rp_o), (case, dev, m)
            want = np.zeros((p.nnz, W), dtype=np.uint32)
            others = [mm for mm in range(N) if mm != m]
            for w, mm in enumerate(others):
                want[:, w] = p.coords[perm, mm].astype(np.uint32) * np.uint32(R)
            want[:, N - 1] = vbits[perm]
            if m == 0 and N < W:
                want[:, N] = p.coords[perm, 0].astype(np.uint32) * np.uint32(R)
            assert np.array_equal(rec, want), (case, dev, m)
        g.close()
        _say(f"  {case} ({'device' if dev else 'host'} build): rowptr and records equal the oracle's CSR")
    o.close()
