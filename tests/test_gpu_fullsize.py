"""Full-size parity on the benchmark workload (480,000 x 18,000 x 2,000, 100M
Zipf(1.1) entries, R = 16, c = 0.1), in the launch configuration bench.py
times.  The oracle cannot afford whole sweeps here in a test, so each mode
update starts from the same FP32 factors on both sides and the oracle
recomputes sampled rows one by one: the heaviest rows (split over many work
items), random active rows and rows with a single sampled entry."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2109_09534_amd as ntc
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(900)
def test_full_size_mode_updates_match_oracle_on_sampled_rows():
    O.build(force=False)
    O.set_threads(16)
    _say("full-size: generating 480000x18000x2000 Zipf(1.1) 100M entries, seed 0")
    p = synth.c1(seed=0)
    R = 16
    init = synth.uniform_init(p.dims, R, 1, synth.init_scale(p.values, R, 3))
    _say("full-size: ntc_create (R=16, c=0.1)")
    g = ntc.Problem(p.dims, p.coords, p.values, R, c=0.1, init=init, stream=0)
    _say("full-size: oracle create")
    o = O.Oracle(p.dims, p.coords, p.values, R, c=0.1, init=init)
    rng = np.random.default_rng(0)
    for m in range(3):
        n = np.bincount(p.coords[:, m], minlength=p.dims[m])
        b = np.floor(0.1 * n)
        active = np.nonzero(b > 0)[0]
        heavy = active[np.argsort(-n[active], kind="stable")[:6]]
        ones = np.nonzero(b == 1)[0]
        rows = np.unique(np.concatenate([heavy, rng.choice(active, 250), rng.choice(ones, min(50, ones.size))]))
        _say(f"full-size: mode {m} update ({active.size} active rows), checking {rows.size} rows "
             f"(heaviest n = {n[heavy].tolist()})")
        g.update_mode(m)
        got = g.factors(m)[rows].astype(np.float64)
        ref = o.update_rows(m, rows)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        scale = np.sqrt(np.mean(ref ** 2))
        worst = np.max(np.abs(got - ref) / (np.abs(ref) + scale))
        _say(f"  mode {m}: rel Frobenius {err:.3e}, worst element {worst:.3e}")
        assert np.all(got >= 0)
        assert err <= 1e-5 and worst <= 1e-5
        # untouched rows (no sample) keep their initial values exactly
        idle = np.nonzero(b == 0)[0][:1000]
        assert np.array_equal(g.factors(m)[idle], init[m][idle])
        g.set_factors(m, init[m])      # the next mode starts from the shared factors again


@pytest.mark.timeout(600)
def test_records_past_the_cache_load_non_temporally_and_match_the_oracle():
    """17 <= R <= 32, 4-way, with more than 256 MB of records (4.7M training entries x 16 B x 4 modes): the row
    kernels take the non-temporal record loads; every mode update, from the same FP32 factors, matches
    the oracle's whole update element by element."""
    O.build(force=False)
    O.set_threads(16)
    p = synth.make_problem((20000, 10000, 200, 50), 5_200_000, 16, zipf_s=1.05, noise_var=0.05, seed=50)
    assert p.nnz * 16 * 4 > (256 << 20)
    R = 32
    init = synth.uniform_init(p.dims, R, 1, synth.init_scale(p.values, R, 4))
    _say(f"records past the cache: dims {p.dims} nnz {p.nnz} R {R}")
    g = ntc.Problem(p.dims, p.coords, p.values, R, c=0.1, init=init, stream=0)
    o = O.Oracle(p.dims, p.coords, p.values, R, c=0.1, init=init)
    for m in range(4):
        g.update_mode(m)
        o.update_mode(m)
        got = g.factors(m).astype(np.float64)
        ref = o.factors(m)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        scale = np.sqrt(np.mean(ref ** 2))
        worst = np.max(np.abs(got - ref) / (np.abs(ref) + scale))
        _say(f"  mode {m}: rel Frobenius {err:.3e}, worst element {worst:.3e}")
        assert np.all(got >= 0)
        assert err <= 1e-5 and worst <= 1e-5
        o.set_factors(m, g.factors(m).astype(np.float64))
    g.close()
    o.close()
