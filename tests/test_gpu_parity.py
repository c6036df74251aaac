"""GPU parity of libntc against the FP64 oracle, through the C ABI.

Inputs are seeded synthetic tensors shaped like the paper's workloads; both
sides start from the same FP32 factors.  Bars: sampled positions bit-exact;
one sweep from identical iterates within 1e-5 relative (Frobenius, per mode)
and element-wise within 1e-5 relative to the factor scale; final test RMSE
within 1e-3 of the oracle's.
"""
import functools
import os
import subprocess
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


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    O.set_threads(8)
    ntc.lib()


def _pair(p, R, *, init_seed=1, scale=None, ora_bf16=False, **kw):
    """(gpu problem, oracle) on identical FP32 init.  The oracle is the plain
    FP64 method unless ora_bf16 asks for its BF16-gather form."""
    if scale is None:
        scale = synth.init_scale(p.values, R, len(p.dims))
    init = synth.uniform_init(p.dims, R, init_seed, scale)
    g = ntc.Problem(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                    init=init, stream=0, **kw)
    okw = {k: v for k, v in kw.items() if k not in ("gather_bf16", "schedule")}
    o = O.Oracle(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                 init=init, gather_bf16=ora_bf16, **okw)
    return g, o, init


def _assert_factor_close(gpu, ora, tag, rel=1e-5):
    err = np.linalg.norm(gpu - ora) / max(np.linalg.norm(ora), 1e-300)
    scale = np.sqrt(np.mean(ora ** 2)) + 1e-300
    worst = np.max(np.abs(gpu - ora) / (np.abs(ora) + scale))
    _say(f"  {tag}: rel Frobenius {err:.3e}, worst element {worst:.3e}")
    assert err <= rel, (tag, err)
    assert worst <= rel, (tag, worst)


# ------------------------------------------------------------------ sampler
def test_device_sampler_is_bit_exact():
    p = synth.c1_small(seed=3)
    g = ntc.Problem(p.dims, p.coords, p.values, 16, c=0.1, seed=77, stream=0)
    o = O.Oracle(p.dims, p.coords, p.values, 16, c=0.1, seed=77)
    rng = np.random.default_rng(0)
    checked = 0
    for mode in range(3):
        rp, _ = o.csr(mode)
        n = np.diff(rp)
        rows = np.concatenate([np.argsort(-n)[:5], rng.integers(0, p.dims[mode], 30)])
        for row in rows:
            for k, l in [(0, 0), (5, 1), (2**31 + 3, 0)]:
                dev = g.debug_sample(k, mode, l, int(row), int(n.max()))
                ref = O.sample_positions(77, k, mode, l, int(row), int(n[row]), 0.1)
                assert np.array_equal(dev, ref), (mode, row, k, l)
                checked += dev.shape[0]
    _say(f"  {checked} sampled positions identical")
    assert checked > 100000


# ---------------------------------------------------------- one-sweep parity
@functools.lru_cache(maxsize=1)
def _twin():
    return synth.scaling_twin(seed=0)


@functools.lru_cache(maxsize=1)
def _conv():
    return synth.convergence_twin(seed=0, snr=2.0)


CASES = {
    "cpu_sized_r8": lambda: (synth.c0(seed=0), 8, dict(c=0.1)),
    "cpu_sized_r8_inner2": lambda: (synth.c0(seed=0), 8, dict(c=0.1, max_inner=2)),
    "zipf_r16_split_rows": lambda: (synth.c1_small(seed=0), 16, dict(c=0.1)),
    "zipf_r16_c05": lambda: (synth.c1_small(seed=1), 16, dict(c=0.5)),
    "r32": lambda: (synth.make_problem((300, 200, 100), 200_000, 32, noise_var=0.05, value_model="clip0",
                                       seed=4, zipf_s=1.05, test_frac=0.05), 32, dict(c=0.1)),
    "r50_4way": lambda: (synth.make_problem((183, 24, 114, 171), 150_000, 10, seed=5, test_frac=0.05), 50,
                         dict(c=0.5)),
    "r10_5way_generic": lambda: (synth.make_problem((20, 15, 12, 10, 8), 60_000, 5, seed=6), 10, dict(c=0.3)),
    "r12_matrix": lambda: (synth.make_problem((400, 300), 40_000, 6, seed=7), 12, dict(c=0.2)),
    "full_batch_inner3": lambda: (synth.make_problem((60, 50, 40), 30_000, 6, seed=8), 6,
                                  dict(c=1.0, max_inner=3, lam=0.01)),
    "lambda0_inner5": lambda: (synth.make_problem((80, 60, 50), 40_000, 4, seed=9, noise_var=0.01), 4,
                               dict(c=0.25, lam=0.0, max_inner=5)),
    # unconverged power method: every kernel must reproduce the oracle's T-th iterate, not lambda_max
    "zipf_power0": lambda: (synth.c1_small(seed=6), 16, dict(c=0.1, power_iters=0)),
    "zipf_power1": lambda: (synth.c1_small(seed=6), 16, dict(c=0.1, power_iters=1)),
    "zipf_power3_inner2": lambda: (synth.c1_small(seed=7), 16, dict(c=0.1, power_iters=3, max_inner=2)),
    "r8_power2_lam0": lambda: (synth.c0(seed=3), 8, dict(c=0.3, power_iters=2, lam=0.0)),
    # 17 <= R <= 32: two 32-lane groups per wave, split rows through the partial slots
    "r24_4way_split": lambda: (synth.make_problem((60, 50, 40, 30), 120_000, 12, seed=11, zipf_s=1.1), 24,
                               dict(c=0.2, schedule={"item_samples": 128})),
    "r32_inner2_power3": lambda: (synth.make_problem((200, 150, 80), 100_000, 16, seed=12), 32,
                                  dict(c=0.3, max_inner=2, power_iters=3)),
    "r20_matrix": lambda: (synth.make_problem((500, 400), 60_000, 8, seed=13), 20, dict(c=0.2)),
    # rows split into more than 64 items: partial slots summed in groups first
    "r24_slot_groups": lambda: (synth.make_problem((60, 50, 40), 70_000, 8, seed=14, zipf_s=1.1), 24,
                                dict(c=0.8, schedule={"item_samples": 16})),
    # 33 <= R <= 64, N <= 4: four columns per lane (one load of four, two pairs, or four singles),
    # whole rows finished in the kernel, heavy rows through partial slots
    "r40_3way_quads": lambda: (synth.make_problem((300, 200, 100), 150_000, 10, seed=15, zipf_s=1.1), 40,
                               dict(c=0.3)),
    "r64_4way_inner2": lambda: (synth.make_problem((80, 60, 50, 40), 100_000, 12, seed=16), 64,
                                dict(c=0.4, max_inner=2)),
    "r33_matrix_singles": lambda: (synth.make_problem((400, 300), 60_000, 8, seed=17), 33, dict(c=0.3)),
    "r46_slot_groups": lambda: (synth.make_problem((60, 50, 40), 70_000, 8, seed=18, zipf_s=1.1), 46,
                                dict(c=0.8, schedule={"item_samples": 16})),
    # L_p as the Collatz-Wielandt bound of the power iterate, in every finishing path: one lane per
    # row (Krylov form), 16-lane groups, chunks and split rows, R <= 32, R <= 64, and the generic kernel
    "cw_r8_tiny_and_groups": lambda: (synth.c0(seed=4), 8, dict(c=0.1, lp_bound=1)),
    "cw_zipf_r16_rowsum": lambda: (synth.c1_small(seed=8), 16, dict(c=0.1, lp_bound=1, power_iters=0)),
    "cw_r32_inner2": lambda: (synth.make_problem((200, 150, 80), 100_000, 16, seed=20), 32,
                              dict(c=0.3, max_inner=2, lp_bound=1)),
    "cw_r50_power3": lambda: (synth.make_problem((183, 24, 114, 171), 150_000, 10, seed=21), 50,
                              dict(c=0.5, lp_bound=1, power_iters=3)),
    "cw_r24_5way_generic": lambda: (synth.make_problem((20, 15, 12, 10, 8), 60_000, 5, seed=22), 24,
                                    dict(c=0.3, lp_bound=1)),
    # items that end exactly on a block boundary (64 samples for R > 16, 16 batches of 16 for the
    # chunks): the prefetch of the block after the last one has no sample and reads zero records
    "r32_items_of_64": lambda: (synth.make_problem((200, 150, 80), 100_000, 16, seed=23), 32,
                                dict(c=0.5, schedule={"item_samples": 64})),
    "r48_items_of_64": lambda: (synth.make_problem((120, 100, 60), 100_000, 12, seed=24), 48,
                                dict(c=0.5, schedule={"item_samples": 64})),
    "zipf_r16_chunks_of_256": lambda: (synth.c1_small(seed=9), 16,
                                       dict(c=0.2, schedule={"item_samples": 256, "group_max": 64})),
    # the twin of the paper's timing workload at full size (3.3M cells, c = 0.5), every rank it uses:
    # 24 to 1717 rows per mode, so every row of modes 0 and 1 is split over many items
    "scaling_twin_r10": lambda: (_twin(), 10, dict(c=0.5)),
    "scaling_twin_r30": lambda: (_twin(), 30, dict(c=0.5)),
    "scaling_twin_r50": lambda: (_twin(), 50, dict(c=0.5)),
    # the twin of the convergence experiment at full size (71567x65133x730, 10M cells, SNR 2), with the
    # extrapolated inner steps of the MAX_INNER study
    "convergence_twin_c005_inner2": lambda: (_conv(), 10, dict(c=0.05, max_inner=2)),
    "convergence_twin_c05_inner2": lambda: (_conv(), 10, dict(c=0.5, max_inner=2)),
    # long power iterations: the iterate is rescaled every 32 products, so T_pow = 200 stays finite in every
    # finishing path (16-lane groups and chunks, 32-lane halves, whole waves, the generic kernel)
    "zipf_r16_power200": lambda: (synth.c1_small(seed=10), 16, dict(c=0.1, power_iters=200)),
    "r32_power200_split": lambda: (synth.make_problem((200, 150, 80), 100_000, 16, seed=26, zipf_s=1.1), 32,
                                   dict(c=0.3, power_iters=200, schedule={"item_samples": 128})),
    "r64_power200": lambda: (synth.make_problem((80, 60, 50, 40), 100_000, 12, seed=27), 64,
                             dict(c=0.4, power_iters=200)),
    "r24_5way_power200": lambda: (synth.make_problem((20, 15, 12, 10, 8), 60_000, 5, seed=28), 24,
                                  dict(c=0.3, power_iters=200)),
    # 17 <= R <= 32, N <= 4: rows of at most 16 samples four to a wave, one sample per lane, the power
    # method on (alpha, u) with v = alpha v_0 + K^T u; every load width (four, two, one column), two to four
    # modes, unconverged and long power iterations, lambda = 0, MAX_INNER = 2, the Collatz-Wielandt bound
    "few_r25_odd_zipf": lambda: (synth.c1_small(seed=13), 25, dict(c=0.1)),
    "few_r30_4way_inner2": lambda: (synth.make_problem((2000, 1500, 40, 16), 200_000, 12, zipf_s=1.05, seed=44), 30,
                                    dict(c=0.1, max_inner=2)),
    "few_r32_power0": lambda: (synth.c1_small(seed=14), 32, dict(c=0.1, power_iters=0)),
    "few_r32_power1_lam0": lambda: (synth.c1_small(seed=15), 32, dict(c=0.1, power_iters=1, lam=0.0)),
    "few_r20_power3": lambda: (synth.c1_small(seed=16), 20, dict(c=0.15, power_iters=3)),
    "few_r28_power200": lambda: (synth.c1_small(seed=17), 28, dict(c=0.1, power_iters=200)),
    "few_r18_matrix": lambda: (synth.make_problem((3000, 2000), 60_000, 8, seed=46, zipf_s=1.1), 18, dict(c=0.2)),
    "cw_few_r24_zipf": lambda: (synth.c1_small(seed=18), 24, dict(c=0.1, lp_bound=1)),
    "cw_few_r31_4way_power3": lambda: (synth.make_problem((2000, 1500, 40, 16), 200_000, 12, zipf_s=1.05, seed=45),
                                       31, dict(c=0.1, lp_bound=1, power_iters=3)),
    # R <= 16, N <= 4: whole rows with 5 <= B_p <= 16 in the same four-rows-per-wave kernel (16 columns)
    "few16_r12_quads": lambda: (synth.c1_small(seed=21), 12, dict(c=0.1)),
    "few16_r10_pairs": lambda: (synth.c1_small(seed=22), 10, dict(c=0.1, max_inner=2)),
    "few16_r7_odd": lambda: (synth.c1_small(seed=23), 7, dict(c=0.1)),
    "few16_r14_4way": lambda: (synth.make_problem((2000, 1500, 40, 16), 200_000, 12, zipf_s=1.05, seed=48), 14,
                               dict(c=0.1)),
    "few16_r16_matrix_zipf": lambda: (synth.make_problem((3000, 2000), 60_000, 8, seed=49, zipf_s=1.1), 16,
                                      dict(c=0.2)),
    "few16_group_max_8": lambda: (synth.c1_small(seed=24), 16, dict(c=0.1, schedule={"group_max": 8})),
    "cw_few16_r16_power3": lambda: (synth.c1_small(seed=25), 16, dict(c=0.1, lp_bound=1, power_iters=3)),
    # R <= 16 chunks that are whole rows read their samples in position order when the records exceed the
    # last-level cache (281 MB here) and the row has at most 65536 entries and 6144 samples: rows on both
    # sides of 65536 entries in one launch; then, in cached problems, rows of 90000 entries and rows of 9000
    # samples (item_samples 16384), which keep the sampler's order
    "chunk_sorted_rows_near_65536": lambda: (synth.make_problem((3000, 400, 89), 6_500_000, 8, seed=60), 16,
                                             dict(c=0.09)),
    "chunk_unsorted_rows_of_90000": lambda: (synth.make_problem((1500, 300, 4), 400_000, 8, seed=61), 16,
                                             dict(c=0.05)),
    "chunk_unsorted_rows_of_9000_samples": lambda: (synth.make_problem((1500, 300, 8), 400_000, 8, seed=62), 12,
                                                    dict(c=0.2, schedule={"item_samples": 16384})),
}


@pytest.mark.parametrize("case", list(CASES))
def test_one_sweep_matches_oracle(case):
    p, R, kw = CASES[case]()
    _say(f"case {case}: dims {p.dims} nnz {p.nnz} R {R} {kw}")
    g, o, init = _pair(p, R, **kw)
    upd, rows = g.work()
    assert upd > 0
    g.sweep(1)
    o.sweep(1)
    for m in range(len(p.dims)):
        gm = g.factors(m).astype(np.float64)
        assert np.all(gm >= 0.0)
        _assert_factor_close(gm, o.factors(m), f"mode {m}")
    assert g.sweep_count == 1


def test_each_mode_update_matches_oracle_from_the_same_factors():
    """Mode by mode from shared FP32 factors (no Gauss-Seidel drift)."""
    p = synth.c1_small(seed=2)
    g, o, init = _pair(p, 16, c=0.1)
    for m in range(3):
        g.update_mode(m)
        o.update_mode(m)
        gm = g.factors(m)
        _assert_factor_close(gm.astype(np.float64), o.factors(m), f"mode {m}")
        o.set_factors(m, gm.astype(np.float64))   # continue both from the GPU's FP32 values


# ----------------------------------------------------------- multi-sweep
def test_final_test_rmse_within_1e3_of_oracle():
    p = synth.c0(seed=0)
    g, o, init = _pair(p, 8, c=0.1)
    g.sweep(20)
    o.sweep(20)
    lg, lo = g.loss(), o.loss()
    _say(f"  GPU loss {lg}, oracle {lo}")
    assert abs(lg[2] - lo[2]) <= 1e-3
    for m in range(3):
        assert np.all(g.factors(m) >= 0)


def test_bf16_gathers_final_rmse_within_1e3_of_oracle():
    p = synth.c0(seed=0)
    g, o, init = _pair(p, 8, c=0.1, gather_bf16=True)
    g.sweep(1)
    o.sweep(1)
    errs = [np.linalg.norm(g.factors(m) - o.factors(m)) / np.linalg.norm(o.factors(m)) for m in range(3)]
    _say(f"  BF16 one-sweep error vs FP64 oracle per mode: {errs}")
    assert max(errs) < 2e-2
    g.sweep(19)
    o.sweep(19)
    lg, lo = g.loss(), o.loss()
    _say(f"  BF16 GPU loss {lg}, oracle {lo}")
    assert abs(lg[2] - lo[2]) <= 1e-3


# The precision form against the oracle's BF16-gather form (other-mode factor values rounded to bfloat16 from
# their FP32 values, everything else FP64).  Mode by mode from shared FP32 factors both sides gather the same
# bfloat16 numbers, so the one-update bar of the plain path applies element by element.
BF16_CASES = {
    # the 4-way R = 32 kernel of the 500M-entry precision workload (column pairs), Zipf(1.05) heads split
    # over many items
    "c2_kernel_r32_4way_split": lambda: (synth.make_problem((300, 200, 60, 20), 300_000, 32, noise_var=0.05,
                                                            value_model="clip0", zipf_s=1.05, seed=40,
                                                            test_frac=0.05), 32,
                                         dict(c=0.1, schedule={"item_samples": 128})),
    "r27_4way_odd_columns": lambda: (synth.make_problem((200, 150, 40, 16), 200_000, 12, zipf_s=1.05, seed=41,
                                                        test_frac=0.05), 27, dict(c=0.2)),
    "r8_zipf_tiny_groups_chunks": lambda: (synth.c1_small(seed=11), 8, dict(c=0.1)),
    "r16_zipf_chunks_of_256": lambda: (synth.c1_small(seed=12), 16,
                                       dict(c=0.2, schedule={"item_samples": 256, "group_max": 64})),
    "r48_4way_quads": lambda: (synth.make_problem((120, 100, 60, 30), 150_000, 12, seed=42, zipf_s=1.1,
                                                  test_frac=0.05), 48, dict(c=0.3)),
    "r24_5way_generic": lambda: (synth.make_problem((20, 15, 12, 10, 8), 60_000, 5, seed=43, test_frac=0.05), 24,
                                 dict(c=0.3)),
    # the four-rows-per-wave kernel's BF16 loads: eight, two and one column at a time
    "few_r24_3way_bf16": lambda: (synth.c1_small(seed=19), 24, dict(c=0.1)),
    "few_r30_4way_bf16_pairs": lambda: (synth.make_problem((2000, 1500, 40, 16), 200_000, 12, zipf_s=1.05, seed=47),
                                        30, dict(c=0.1)),
    "few_r19_odd_bf16": lambda: (synth.c1_small(seed=20), 19, dict(c=0.1)),
    "few16_r12_bf16_pairs": lambda: (synth.c1_small(seed=26), 12, dict(c=0.1)),
    "few16_r9_odd_bf16": lambda: (synth.c1_small(seed=27), 9, dict(c=0.1)),
}


@pytest.mark.parametrize("case", list(BF16_CASES))
def test_bf16_mode_updates_match_the_oracle_bf16_form(case):
    p, R, kw = BF16_CASES[case]()
    _say(f"case {case}: dims {p.dims} nnz {p.nnz} R {R} {kw}")
    g, o, init = _pair(p, R, gather_bf16=True, ora_bf16=True, **kw)
    for m in range(len(p.dims)):
        g.update_mode(m)
        o.update_mode(m)
        gm = g.factors(m)
        assert np.all(gm >= 0.0)
        _assert_factor_close(gm.astype(np.float64), o.factors(m), f"mode {m}")
        o.set_factors(m, gm.astype(np.float64))


def test_bf16_c2_kernel_error_against_fp64_is_what_bf16_rounding_implies():
    """The 4-way R = 32 precision kernel against the plain FP64 oracle: its
    one-sweep error is the error that rounding the gathers to bfloat16
    causes in the oracle itself (same samples, FP64 elsewhere), not more,
    and after 20 sweeps its held-out RMSE is within 1e-3 of the FP64
    oracle's."""
    p, R, kw = BF16_CASES["c2_kernel_r32_4way_split"]()
    g, o, init = _pair(p, R, gather_bf16=True, **kw)
    ob = O.Oracle(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                  init=init, gather_bf16=True, c=kw["c"])
    g.sweep(1)
    o.sweep(1)
    ob.sweep(1)
    for m in range(len(p.dims)):
        ref = o.factors(m)
        e_gpu = np.linalg.norm(g.factors(m) - ref) / np.linalg.norm(ref)
        e_ora = np.linalg.norm(ob.factors(m) - ref) / np.linalg.norm(ref)
        _say(f"  mode {m}: BF16 GPU vs FP64 oracle {e_gpu:.3e}; oracle's own BF16 form vs FP64 {e_ora:.3e}")
        assert e_ora > 1e-5                     # the rounding is visible at this size
        assert abs(e_gpu - e_ora) <= 0.02 * e_ora + 1e-6, (m, e_gpu, e_ora)
    g.sweep(19)
    o.sweep(19)
    lg, lo = g.loss(), o.loss()
    _say(f"  after 20 sweeps: BF16 GPU test RMSE {lg[2]:.6f}, FP64 oracle {lo[2]:.6f}")
    assert abs(lg[2] - lo[2]) <= 1e-3


def test_bf16_gathers_at_r_above_32_stay_within_1e3_of_oracle():
    p = synth.make_problem((200, 150, 100), 120_000, 10, seed=19, test_frac=0.1)
    g, o, init = _pair(p, 48, c=0.2, gather_bf16=True)
    g.sweep(10)
    o.sweep(10)
    lg, lo = g.loss(), o.loss()
    _say(f"  R=48 BF16 GPU loss {lg}, oracle {lo}")
    assert abs(lg[2] - lo[2]) <= 1e-3


def test_loss_matches_oracle_on_identical_factors():
    p = synth.c1_small(seed=4)
    g, o, init = _pair(p, 16)
    lg, lo = g.loss(), o.loss()
    np.testing.assert_allclose(lg, lo, rtol=1e-11)


def test_fixed_point_is_bit_exact_on_gpu():
    p = synth.make_problem((40, 30, 20), 5000, 4, grid_factors=16, seed=2)
    U0 = [u.astype(np.float32) for u in p.planted]
    g = ntc.Problem(p.dims, p.coords, p.values, 4, c=0.5, lam=0.0, max_inner=2, init=U0, stream=0)
    g.sweep(2)
    for m in range(3):
        assert np.array_equal(g.factors(m), U0[m])


def test_runs_are_bit_identical_and_resumable():
    p = synth.c1_small(seed=5)
    init = synth.uniform_init(p.dims, 16, 3, synth.init_scale(p.values, 16, 3))
    a = ntc.Problem(p.dims, p.coords, p.values, 16, init=init, stream=0)
    b = ntc.Problem(p.dims, p.coords, p.values, 16, init=init, stream=0)
    a.sweep(4)
    b.sweep(2)
    mid = b.all_factors()
    c = ntc.Problem(p.dims, p.coords, p.values, 16, init=mid, stream=0)
    c.sweep_count = b.sweep_count
    c.sweep(2)
    b.sweep(2)
    for m in range(3):
        fa = a.factors(m)
        assert np.array_equal(fa, b.factors(m))
        assert np.array_equal(fa, c.factors(m))


def test_profiled_sweeps_are_ordinary_sweeps():
    """ntc_profile_sweeps runs the sweeps ntc_sweep runs (serial or with the
    side-stream overlap), so the factors match plain sweeps bit for bit; it
    returns one record per launch, sweep after sweep, with a duration."""
    p = synth.c1_small(seed=6)
    init = synth.uniform_init(p.dims, 16, 4, synth.init_scale(p.values, 16, 3))
    ref = ntc.Problem(p.dims, p.coords, p.values, 16, init=init, stream=0)
    ref.sweep(3)
    one = None
    for concurrent in (False, True):
        g = ntc.Problem(p.dims, p.coords, p.values, 16, init=init, stream=0)
        first = g.profile_sweep()
        rest = g.profile_sweeps(2, concurrent=concurrent)
        assert len(rest) == 2 * len(first) and len(first) > 0
        one = len(first)
        for a, b in zip(rest[:one], rest[one:]):
            assert (a["kernel"], a["mode"], a["blocks"], a["samples"]) == (b["kernel"], b["mode"], b["blocks"],
                                                                           b["samples"])
        assert all(r["ms"] > 0.0 for r in first + rest)
        assert g.sweep_count == 3
        for m in range(3):
            assert np.array_equal(g.factors(m), ref.factors(m)), (concurrent, m)
        g.close()
    _say(f"  {one} launches per sweep; profiled sweeps identical to plain ones")


def test_default_init_matches_oracle_bit_exactly():
    p = synth.c0(seed=1)
    g = ntc.Problem(p.dims, p.coords, p.values, 8, seed=99, stream=0)
    o = O.Oracle(p.dims, p.coords, p.values, 8, seed=99)
    for m in range(3):
        assert np.array_equal(g.factors(m).astype(np.float64), o.factors(m))


# ---------------------------------------------------------------- edges
def test_empty_and_degenerate_problems():
    # no observed entries: nothing moves, loss is the regulariser
    dims = [5, 4, 3]
    init = synth.uniform_init(dims, 3, 0)
    g = ntc.Problem(dims, np.zeros((0, 3), np.int32), np.zeros(0, np.float32), 3, init=init, stream=0)
    g.sweep(2)
    for m in range(3):
        assert np.array_equal(g.factors(m), init[m])
    lg = g.loss()
    assert lg[1] == 0.0 and lg[0] == pytest.approx(0.5e-3 * sum(float(np.sum(u.astype(np.float64) ** 2)) for u in init))
    # every row below 1/c entries: all rows skipped
    p = synth.tiny(seed=4, dims=(30, 30, 30), nnz=200, rank=2)
    init = synth.uniform_init(p.dims, 2, 0)
    g = ntc.Problem(p.dims, p.coords, p.values, 2, c=0.02, init=init, stream=0)
    assert g.work() == (0, 0)
    g.sweep(1)
    assert all(np.array_equal(g.factors(m), init[m]) for m in range(3))
    # a mode of size one, rank one
    p = synth.make_problem((1, 50, 40), 1500, 1, seed=3)
    g, o, _ = _pair(p, 1, c=0.5)
    g.sweep(1)
    o.sweep(1)
    for m in range(3):
        _assert_factor_close(g.factors(m).astype(np.float64), o.factors(m), f"mode {m}")


_INTEROP = """
import torch                       # first, so libntc binds to torch's HIP runtime
import numpy as np
import paper_2109_09534_amd as ntc
import synth
assert torch.cuda.is_available()
ntc.lib()
assert len(ntc.hip_runtimes()) == 1, ntc.hip_runtimes()
p = synth.c0(seed=2)
init = synth.uniform_init(p.dims, 8, 5, 1.0)
a = ntc.Problem(p.dims, p.coords, p.values, 8, init=init, stream=0)
s = torch.cuda.Stream()
with torch.cuda.stream(s):
    b = ntc.Problem(p.dims, p.coords, p.values, 8, init=init, stream=s, torch_allocator=True)
    b.sweep(3)
    dev = torch.empty(p.dims[0] * 8, dtype=torch.float32, device="cuda")
    b.factors_into(0, dev)
s.synchronize()
a.sweep(3)
assert np.array_equal(a.factors(0), b.factors(0))
assert np.array_equal(a.factors(0).reshape(-1), dev.cpu().numpy())
b.close()
print("interop ok", flush=True)
"""


@pytest.mark.timeout(400)
def test_torch_stream_and_allocator_interop_in_a_fresh_process():
    """torch's stream and caching allocator drive the same kernels and give
    bit-identical results (child process: torch must load the runtime first)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _INTEROP], cwd=root, capture_output=True, text=True, timeout=380,
                       env=dict(os.environ, PYTHONPATH=root))
    _say(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0 and "interop ok" in r.stdout
