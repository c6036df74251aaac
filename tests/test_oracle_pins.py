"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them compares the oracle with a
retyped copy of itself: the references are published test vectors, dense
matrix forms of the paper's equations (tests/brute.py), LAPACK/SciPy
routines, finite differences, closed forms and invariants.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy import optimize, stats

import brute
import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)
    O.set_threads(4)


# ------------------------------------------------------------------ sampler
def test_philox_known_answers():
    """Philox4x32-R against the published known-answer vectors."""
    n = 0
    with open(os.path.join(GOLDEN, "philox4x32_kat.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            tok = line.split()
            rounds = int(tok[0])
            ctr = [int(t, 16) for t in tok[1:5]]
            key = [int(t, 16) for t in tok[5:7]]
            want = [int(t, 16) for t in tok[7:11]]
            got = [int(v) for v in O.philox4x32(ctr, key, rounds)]
            assert got == want, (tok, [hex(g) for g in got])
            n += 1
    assert n >= 5


def test_feistel_is_a_permutation_for_every_small_domain():
    """With c = 1 the sample is pi(0..n-1): it must be a permutation of
    [0, n) for every n up to 4096 (exhaustive)."""
    for n in range(1, 4097):
        pos = O.sample_positions(seed=11, k=n, mode=n % 3, l=0, row=n * 7, n=n, c=1.0)
        assert pos.shape[0] == n
        assert np.array_equal(np.sort(pos), np.arange(n)), n


def test_feistel_network_is_a_permutation_of_its_word_domain():
    """One pass permutes [0, A*B) with A = 2^ceil(w/2), B = ceil(n/A), and
    A*B - n < A (so cycle walking is short)."""
    for n in [1, 2, 3, 4, 5, 7, 9, 16, 17, 100, 1000, 4097, 50000]:
        keys = O.sample_keys(3, n, 0, 0, 0)
        D = O.feistel_domain(n)
        w = O.feistel_width(n)
        A = 1 << ((w + 1) // 2)
        assert n <= D < n + A
        img = sorted(O.feistel_net(x, n, keys) for x in range(D))
        assert img == list(range(D)), n
    assert O.feistel_width(1) == 2 and O.feistel_width(4) == 2 and O.feistel_width(5) == 3
    assert O.feistel_width(1 << 20) == 20 and O.feistel_width((1 << 20) + 1) == 21


def test_sample_size_is_floor_of_one_binary64_product():
    """B_{l,p} = floor(c ||M(p,:)||_0) (Section II-B)."""
    assert O.sample_size(0.57, 100) == 56          # 0.57*100 = 56.99999999999999 in binary64
    assert O.sample_size(0.1, 9) == 0
    assert O.sample_size(0.1, 10) == 1
    assert O.sample_size(0.1, 30) == 3             # 3.0000000000000004 -> 3
    assert O.sample_size(1.0, 12345) == 12345
    for c in [0.02, 0.05, 0.1, 0.2, 0.5, 0.9]:
        for n in [0, 1, 7, 99, 1000, 123457]:
            assert O.sample_size(c, n) == math.floor(c * n)


@pytest.mark.parametrize("n,b_frac", [(10, 0.1), (13, 0.3), (37, 0.2), (100, 0.1), (1000, 0.05), (5000, 0.5)])
def test_sampler_inclusion_is_uniform(n, b_frac):
    """Each observed entry of a row is included with probability b/n
    (uniform sampling, Section II-B): chi-square over 20000 fresh keys."""
    T = 20000
    counts = np.zeros(n)
    b = O.sample_size(b_frac, n)
    for k in range(T):
        pos = O.sample_positions(seed=5, k=k, mode=1, l=0, row=3, n=n, c=b_frac)
        assert pos.shape[0] == b
        assert np.unique(pos).shape[0] == b             # without replacement
        counts[pos] += 1
    p = b / n
    chi = np.sum((counts - T * p) ** 2 / (T * p * (1 - p)))
    assert stats.chi2.sf(chi, n - 1) > 1e-4, chi


@pytest.mark.parametrize("n,b", [(2, 1), (3, 1), (4, 2), (5, 2), (6, 3), (7, 3), (8, 4)])
def test_sampler_subsets_are_uniform_on_tiny_rows(n, b):
    """All C(n, b) subsets about equally likely (enumeration, n <= 8)."""
    T = 30000
    c = b / n
    assert O.sample_size(c, n) == b
    seen = {}
    for k in range(T):
        s = tuple(sorted(O.sample_positions(seed=9, k=k, mode=0, l=0, row=1, n=n, c=c)))
        seen[s] = seen.get(s, 0) + 1
    subs = list(itertools.combinations(range(n), b))
    exp = T / len(subs)
    chi = sum((seen.get(s, 0) - exp) ** 2 / exp for s in subs)
    assert stats.chi2.sf(chi, len(subs) - 1) > 1e-4, (chi, len(subs))


def test_sample_depends_on_every_counter_field():
    base = O.sample_positions(seed=1, k=2, mode=1, l=0, row=5, n=1000, c=0.1)
    for kw in [dict(seed=2), dict(k=3), dict(mode=2), dict(l=1), dict(row=6)]:
        args = dict(seed=1, k=2, mode=1, l=0, row=5)
        args.update(kw)
        other = O.sample_positions(n=1000, c=0.1, **args)
        assert not np.array_equal(base, other), kw


# --------------------------------------------------------------------- CSR
def test_csr_is_a_stable_sort_by_mode_index():
    p = synth.tiny(seed=1, dims=(9, 7, 5), nnz=200, rank=3)
    o = O.Oracle(p.dims, p.coords, p.values, 3)
    for m in range(3):
        rp, perm = o.csr(m)
        ref = np.argsort(p.coords[:, m], kind="stable")
        assert np.array_equal(perm, ref)
        assert np.array_equal(rp, np.concatenate([[0], np.cumsum(np.bincount(p.coords[:, m], minlength=p.dims[m]))]))


# ---------------------------------------------------- gradient and Hessian
def _row_setup(seed=3, dims=(6, 5, 4), nnz=90, R=3, c=0.5, lam=0.05):
    p = synth.tiny(seed=seed, dims=dims, nnz=nnz, rank=R)
    init = synth.uniform_init(p.dims, R, seed=seed)
    o = O.Oracle(p.dims, p.coords, p.values, R, c=c, lam=lam, seed=seed, init=init)
    U = [o.factors(m) for m in range(len(dims))]
    return p, o, U


def _sampled_mask(p, o, mode, row, k=0, l=0):
    """Dense mode-`mode` mask of the entries the oracle's sampler picks in `row`."""
    rp, perm = o.csr(mode)
    n = rp[row + 1] - rp[row]
    pos = O.sample_positions(o.seed, k, mode, l, row, n, o.c)
    ents = perm[rp[row] + pos]
    Mhat = np.zeros(p.dims)
    idx = tuple(p.coords[ents, m] for m in range(len(p.dims)))
    Mhat[idx] = 1.0
    return Mhat, ents


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_row_hessian_is_the_row_block_of_the_dense_kronecker_hessian(mode):
    """The per-row H equals the row-p block of eq. hessian_F with the sampled
    mask, after the column-major -> row-major permutation of vec(A)."""
    p, o, U = _row_setup()
    X, _ = brute.dense_data(p.dims, p.coords, p.values)
    B = brute.kr_for_mode(U, mode)
    P = p.dims[mode]
    for row in range(P):
        Mhat, ents = _sampled_mask(p, o, mode, row)
        if ents.shape[0] == 0:
            continue
        Hfull = brute.nmc_hessian(brute.unfold(Mhat, mode), B, o.lam)
        blk = Hfull[np.ix_(np.arange(o.R) * P + row, np.arange(o.R) * P + row)]
        y = U[mode][row]
        st = o.row_step(mode, 0, row, y, y)
        assert st["b"] == ents.shape[0]
        np.testing.assert_allclose(st["H"], blk, rtol=1e-13, atol=1e-14)
        # block-diagonal over rows: other rows' blocks do not couple to row p
        other = (row + 1) % P
        cross = Hfull[np.ix_(np.arange(o.R) * P + row, np.arange(o.R) * P + other)]
        assert np.all(cross == 0)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_row_gradient_matches_dense_formula_and_finite_differences(mode):
    """g equals row p of eq. gradient_F (sampled mask), and central finite
    differences of f_hat(a) = 1/2 ||M_hat(p,:)*(X(p,:) - a B^T)||^2 + lam/2 ||a||^2."""
    p, o, U = _row_setup()
    X, _ = brute.dense_data(p.dims, p.coords, p.values)
    Xi = brute.unfold(X, mode)
    B = brute.kr_for_mode(U, mode)
    for row in range(p.dims[mode]):
        Mhat, ents = _sampled_mask(p, o, mode, row)
        if ents.shape[0] == 0:
            continue
        Mi = brute.unfold(Mhat, mode)
        y = U[mode][row] + 0.05            # any point; the gradient is affine in y
        A = U[mode].copy()
        A[row] = y
        G = brute.nmc_gradient(Xi, Mi, A, B, o.lam)
        st = o.row_step(mode, 0, row, y, y)
        np.testing.assert_allclose(st["g"], G[row], rtol=1e-12, atol=1e-13)

        def f(a):
            r = Mi[row] * (Xi[row] - B @ a)
            return 0.5 * r @ r + 0.5 * o.lam * a @ a
        h = 1e-6
        fd = np.array([(f(y + h * e) - f(y - h * e)) / (2 * h) for e in np.eye(o.R)])
        np.testing.assert_allclose(st["g"], fd, rtol=1e-7, atol=1e-8)


# ------------------------------------------------------------- L_p and beta
def test_power_method_matches_eigvalsh_and_closed_forms():
    rng = np.random.default_rng(0)
    for R in [1, 2, 3, 8, 16, 32]:
        for b in [1, 2, 5, 50]:
            K = rng.random((b, R)) * rng.random((b, R))      # Khatri-Rao rows of nonnegative factors
            lam = 1e-3
            H = K.T @ K + lam * np.eye(R)
            L = O.power_lmax(H, 20)
            ev = np.linalg.eigvalsh(H).max()
            assert abs(L - ev) <= 1e-10 * ev, (R, b, L, ev)
            # Rayleigh quotient <= lambda_max (sandwich lower side)
            assert L <= ev * (1 + 1e-14)
            if b == 1:
                assert abs(L - (K[0] @ K[0] + lam)) <= 1e-12 * L
    # lambda_max <= Collatz-Wielandt bound max_r (H v)_r / v_r for any v > 0
    H = np.array([[2.0, 1.0], [1.0, 3.0]])
    ev = np.linalg.eigvalsh(H).max()
    assert O.power_lmax(H, 60) == pytest.approx(ev, rel=1e-14)
    assert O.power_lmax(np.zeros((4, 4)), 20) == 0.0
    # T_pow = 0 returns the Rayleigh quotient of the start vector 1/sqrt(R)
    assert O.power_lmax(H, 0) == pytest.approx(np.ones(2) @ H @ np.ones(2) / 2)


def test_collatz_wielandt_bound_brackets_lambda_max():
    """For entrywise nonnegative H and any positive v, lambda_max <= max_r
    (H v)_r / v_r (Collatz-Wielandt); at v = ones it is the largest row sum,
    and along the power iterates it converges to lambda_max."""
    rng = np.random.default_rng(1)
    for R in [1, 2, 3, 8, 16, 33, 50, 64]:
        for b in [1, 3, 20, 200]:
            K = rng.random((b, R)) * rng.random((b, R))
            H = K.T @ K + 1e-3 * np.eye(R)
            ev = np.linalg.eigvalsh(H).max()
            assert O.lmax_cw(H, 0) == pytest.approx(H.sum(axis=1).max(), rel=1e-14)
            for T in [0, 1, 2, 5, 20]:
                assert O.lmax_cw(H, T) >= ev * (1 - 1e-13), (R, b, T)
            # with a spectral gap the bound meets lambda_max along the iterates
            if b >= 20 or R == 1:
                assert O.lmax_cw(H, 400) == pytest.approx(ev, rel=1e-9), (R, b)
    # a diagonal H: every iterate has ratio d_r in coordinate r, the bound is max d exactly
    d = np.array([0.5, 4.0, 2.0, 3.5])
    for T in [0, 3, 20]:
        assert O.lmax_cw(np.diag(d), T) == pytest.approx(4.0, rel=1e-15)
    assert O.lmax_cw(np.zeros((3, 3)), 5) == 0.0


def test_collatz_wielandt_steps_meet_the_rayleigh_steps_when_the_iterate_converges():
    """With many power iterations both estimators give lambda_max, so one sweep
    with either is the same up to rounding; with few iterations the bound is
    larger, so every step is a shorter (safe) projected step."""
    p = synth.c0(seed=2)
    init = synth.uniform_init(p.dims, 8, 3, synth.init_scale(p.values, 8, 3))
    runs = {}
    for bound, T in [(0, 400), (1, 400), (0, 2), (1, 2)]:
        o = O.Oracle(p.dims, p.coords, p.values, 8, c=0.5, power_iters=T, init=init, lp_bound=bound)
        o.sweep(1)
        runs[(bound, T)] = [o.factors(m) for m in range(3)]
        o.close()
    for m in range(3):
        a, b = runs[(0, 400)][m], runs[(1, 400)][m]
        assert np.max(np.abs(a - b)) <= 1e-9 * np.max(np.abs(a))
    assert any(np.max(np.abs(runs[(0, 2)][m] - runs[(1, 2)][m])) > 1e-6 for m in range(3))


def test_beta_and_step_closed_form_on_one_row():
    p, o, U = _row_setup(c=1.0)
    mode, row = 1, 2
    y = U[mode][row].copy()
    st = o.row_step(mode, 0, row, y, y)
    L = st["L"]
    beta = (math.sqrt(L) - math.sqrt(o.lam)) / (math.sqrt(L) + math.sqrt(o.lam))
    assert st["beta"] == pytest.approx(beta, rel=1e-15)
    a_ref = np.maximum(0.0, y - st["g"] / L)
    np.testing.assert_allclose(st["a"], a_ref, rtol=1e-15, atol=0)
    np.testing.assert_allclose(st["y"], a_ref + beta * (a_ref - y), rtol=1e-14, atol=1e-16)
    assert L == pytest.approx(brute.row_lmax(st["H"]), rel=1e-10)


def test_lambda_zero_gives_beta_one():
    p, o, U = _row_setup(c=1.0, lam=0.0)
    st = o.row_step(0, 0, 1, U[0][1], U[0][1])
    assert st["beta"] == 1.0


def test_row_with_no_sample_is_left_unchanged():
    """Rows with floor(c * n_p) = 0 are skipped (Section II-B): no ridge
    shrinkage, no change; rows with a sample do move."""
    p = synth.tiny(seed=4, dims=(6, 5, 4), nnz=60, rank=2)
    o = O.Oracle(p.dims, p.coords, p.values, 2, c=0.1, lam=1e-3)
    before = [o.factors(m) for m in range(3)]
    o.sweep(2)
    moved = 0
    for m in range(3):
        n = np.bincount(p.coords[:, m], minlength=p.dims[m])
        after = o.factors(m)
        for row in range(p.dims[m]):
            if n[row] < 10:
                assert np.array_equal(after[row], before[m][row]), (m, row)
            else:
                moved += int(not np.array_equal(after[row], before[m][row]))
    assert moved > 0


# --------------------------------------------------------- full-batch steps
@pytest.mark.parametrize("max_inner", [1, 2, 3])
def test_full_batch_mode_update_matches_dense_algorithm(max_inner):
    """c = 1: every row's minibatch is the whole row, so S_NMC is
    deterministic; compare with Alg. 1 written on dense matrices (eq.
    gradient_F, per-row L_p from eigvalsh, beta of the constant step scheme)."""
    p, o, U = _row_setup(c=1.0, lam=0.01)
    o2 = O.Oracle(p.dims, p.coords, p.values, o.R, c=1.0, lam=0.01, max_inner=max_inner, seed=o.seed,
                  init=[u.astype(np.float32) for u in U])
    X, M = brute.dense_data(p.dims, p.coords, p.values)
    Ud = [o2.factors(m) for m in range(3)]
    for mode in range(3):                       # Gauss-Seidel: later modes see updated earlier ones
        o2.update_mode(mode)
        Ud[mode] = brute.full_batch_mode_update(X, M, Ud, mode, 0.01, max_inner)
        np.testing.assert_allclose(o2.factors(mode), Ud[mode], rtol=1e-9, atol=1e-12)


def test_fixed_point_at_noiseless_truth_is_bit_exact():
    """lambda = 0, exact dyadic CPD data, start at the planted factors: the
    residual is exactly zero, so g = 0, beta = 1 and one sweep returns U^o."""
    p = synth.make_problem((12, 10, 8), 500, 4, grid_factors=16, seed=2)
    U0 = [u.astype(np.float32) for u in p.planted]
    for c in [0.1, 0.5, 1.0]:
        o = O.Oracle(p.dims, p.coords, p.values, 4, c=c, lam=0.0, max_inner=2, init=U0)
        o.sweep(2)
        for m in range(3):
            assert np.array_equal(o.factors(m), p.planted[m])


def test_objective_does_not_increase_in_full_batch_mode_updates():
    """c = 1, MAX_INNER = 1: each mode update is a projected gradient step
    with step 1/L_p on a row-separable convex quadratic (H_p <= L_p I)."""
    p = synth.tiny(seed=6, dims=(9, 8, 7), nnz=300, rank=4, noise_var=0.01)
    o = O.Oracle(p.dims, p.coords, p.values, 4, c=1.0, lam=1e-3, seed=1)
    prev = o.loss()[0]
    for sweep in range(6):
        for mode in range(3):
            o.update_mode(mode)
            cur = o.loss()[0]
            assert cur <= prev * (1 + 1e-13), (sweep, mode, prev, cur)
            prev = cur
        o.sweep_count = o.sweep_count + 1


def test_many_inner_steps_converge_to_nnls():
    """c = 1 and many inner steps: each row solves
    min_{a>=0} ||K_p a - x_p||^2 + lam ||a||^2, i.e. NNLS on [K_p; sqrt(lam) I]."""
    p = synth.tiny(seed=7, dims=(6, 7, 8), nnz=200, rank=3, noise_var=0.05)
    lam = 1.0
    o = O.Oracle(p.dims, p.coords, p.values, 3, c=1.0, lam=lam, max_inner=400, seed=3)
    U = [o.factors(m) for m in range(3)]
    o.update_mode(1)
    got = o.factors(1)
    X, M = brute.dense_data(p.dims, p.coords, p.values)
    Xi, Mi = brute.unfold(X, 1), brute.unfold(M, 1)
    B = brute.kr_for_mode(U, 1)
    for row in range(p.dims[1]):
        obs = Mi[row] > 0
        A = np.vstack([B[obs], math.sqrt(lam) * np.eye(3)])
        rhs = np.concatenate([Xi[row][obs], np.zeros(3)])
        ref, _ = optimize.nnls(A, rhs)
        np.testing.assert_allclose(got[row], ref, rtol=1e-7, atol=1e-9)


# -------------------------------------------------------- loss and sweeps
def test_loss_matches_dense_objective_and_errors():
    p = synth.tiny(seed=8, dims=(7, 6, 5), nnz=150, rank=3, noise_var=0.01)
    init = synth.uniform_init(p.dims, 3, seed=1)
    lam = 0.02
    o = O.Oracle(p.dims, p.coords, p.values, 3, lam=lam, test_coords=p.test_coords,
                 test_values=p.test_values, init=init)
    U = [o.factors(m) for m in range(3)]
    out = o.loss()
    assert out[0] == pytest.approx(brute.ntc_objective(p.dims, p.coords, p.values, U, lam), rel=1e-12)
    Xh = brute.cpd_full(U)
    tr = Xh[tuple(p.coords.T)] - p.values
    te = Xh[tuple(p.test_coords.T)] - p.test_values
    assert out[1] == pytest.approx(np.sqrt(np.mean(tr ** 2)), rel=1e-12)
    assert out[2] == pytest.approx(np.sqrt(np.mean(te ** 2)), rel=1e-12)
    assert out[3] == pytest.approx(np.linalg.norm(te) / np.linalg.norm(p.test_values.astype(np.float64)), rel=1e-12)


def test_iterates_stay_nonnegative():
    p = synth.tiny(seed=9, dims=(20, 15, 10), nnz=1500, rank=4, noise_var=0.5)
    o = O.Oracle(p.dims, p.coords, p.values, 4, c=0.3, lam=1e-3, max_inner=3, seed=2)
    for _ in range(5):
        o.sweep(1)
        for m in range(3):
            assert np.all(o.factors(m) >= 0.0)


def test_default_init_is_scaled_uniform():
    p = synth.tiny(seed=10, dims=(40, 30, 20), nnz=3000, rank=5)
    o = O.Oracle(p.dims, p.coords, p.values, 5, seed=123)
    s = synth.init_scale(p.values, 5, 3)
    allv = np.concatenate([o.factors(m).ravel() for m in range(3)])
    assert allv.min() >= 0.0 and allv.max() < s
    q = allv / s * 2.0 ** 24        # multiples of 2^-24 * s (24-bit uniform words)
    assert np.allclose(q, np.round(q), atol=1e-3)
    assert abs(allv.mean() / s - 0.5) < 0.02


def test_sweeps_are_deterministic_and_resumable():
    """The sampler is counter-based: state = factors + sweep counter."""
    p = synth.tiny(seed=11, dims=(30, 20, 10), nnz=2000, rank=4, noise_var=0.01)
    a = O.Oracle(p.dims, p.coords, p.values, 4, c=0.2, seed=5)
    a.sweep(4)
    b = O.Oracle(p.dims, p.coords, p.values, 4, c=0.2, seed=5)
    b.sweep(2)
    saved = [b.factors(m) for m in range(3)]
    c = O.Oracle(p.dims, p.coords, p.values, 4, c=0.2, seed=5,
                 init=[np.zeros((d, 4), np.float32) for d in p.dims])
    for m in range(3):
        c.set_factors(m, saved[m])
    c.sweep_count = b.sweep_count
    c.sweep(2)
    for m in range(3):
        assert np.array_equal(a.factors(m), c.factors(m))


def test_update_rows_matches_a_full_mode_update():
    p = synth.tiny(seed=12, dims=(25, 20, 15), nnz=2500, rank=4, noise_var=0.01)
    o = O.Oracle(p.dims, p.coords, p.values, 4, c=0.3, max_inner=2, seed=1)
    rows = np.array([0, 3, 7, 24])
    want = o.update_rows(0, rows)
    o.update_mode(0)
    np.testing.assert_array_equal(o.factors(0)[rows], want)


def test_planted_recovery_on_the_cpu_sized_workload():
    """100x80x60, 5% observed, planted rank 8, noiseless.  The paper prints
    no error level, so the 1e-2 threshold is ours (parity unpinned level)."""
    p = synth.c0(seed=0)
    o = O.Oracle(p.dims, p.coords, p.values, 8, c=0.5, lam=1e-3, seed=0,
                 test_coords=p.test_coords, test_values=p.test_values)
    before = o.loss()[3]
    o.sweep(1000)
    after = o.loss()[3]
    assert after < before
    assert after <= 1e-2, after


# ------------------------------------------------------ BF16 precision form
def test_bf16_copy_is_the_nearest_bfloat16_of_the_fp32_value():
    """ora_bf16 against torch's float32 -> bfloat16 conversion (round to
    nearest, ties to even), on random magnitudes and on exact ties."""
    import torch
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(0, 1, 4000), rng.uniform(0, 40, 2000),
                        np.exp(rng.uniform(-60, 60, 2000)), [0.0, 1.0, 2.0 ** -130]])
    # exact ties between two neighbouring bfloat16 numbers, both parities
    ties = [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 2 + 2.0 ** -7, 0.5 + 3 * 2.0 ** -9]
    x = np.concatenate([x, ties, -np.asarray(ties)])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([O.bf16(v) for v in x])
    assert np.array_equal(got, ref)
    assert O.bf16(1 + 2.0 ** -8) == 1.0 and O.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6
    assert O.bf16(2 + 2.0 ** -7) == 2.0 and O.bf16(0.5 + 3 * 2.0 ** -9) == 0.5 + 2.0 ** -7
    # the FP32 rounding comes first: a value just above a tie in binary64 but
    # equal to the tie in FP32 rounds to even
    assert O.bf16(1 + 2.0 ** -8 + 2.0 ** -40) == 1.0


def test_bf16_gathers_change_nothing_when_the_factors_are_bfloat16_numbers():
    """Factors with at most 8 significant bits are their own bfloat16 copies,
    so a mode update is bit-identical with and without BF16 gathers; with
    ordinary FP32 factors the option does change the result."""
    p = synth.make_problem((14, 12, 10), 900, 3, seed=31, test_frac=0.0)
    rng = np.random.default_rng(3)
    exact = [(rng.integers(0, 256, (d, 5)) * 2.0 ** -8).astype(np.float32) for d in p.dims]
    plain = [rng.uniform(0, 1, (d, 5)).astype(np.float32) for d in p.dims]
    for init, same in [(exact, True), (plain, False)]:
        a = O.Oracle(p.dims, p.coords, p.values, 5, c=0.5, init=init)
        b = O.Oracle(p.dims, p.coords, p.values, 5, c=0.5, init=init, gather_bf16=True)
        a.update_mode(0)
        b.update_mode(0)
        assert np.array_equal(a.factors(0), b.factors(0)) == same


@pytest.mark.parametrize("max_inner", [1, 2])
def test_bf16_full_batch_mode_update_matches_dense_algorithm_on_rounded_factors(max_inner):
    """c = 1 with BF16 gathers equals the dense Alg. 1 whose Khatri-Rao matrix
    is built from the bfloat16 copies (torch's conversion) of the other
    modes' FP32 factors, while the row's own iterate stays unrounded."""
    import torch
    p, o, U = _row_setup(c=1.0, lam=0.01)
    init = [u.astype(np.float32) for u in U]
    o2 = O.Oracle(p.dims, p.coords, p.values, o.R, c=1.0, lam=0.01, max_inner=max_inner, seed=o.seed,
                  init=init, gather_bf16=True)
    X, M = brute.dense_data(p.dims, p.coords, p.values)
    Ud = [o2.factors(m) for m in range(3)]
    for mode in range(3):
        rounded = [torch.tensor(u.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
                   if m != mode else u for m, u in enumerate(Ud)]
        o2.update_mode(mode)
        Ud[mode] = brute.full_batch_mode_update(X, M, rounded, mode, 0.01, max_inner)
        np.testing.assert_allclose(o2.factors(mode), Ud[mode], rtol=1e-9, atol=1e-12)
