"""Batching and serving form (ntc_pool_*), through the C ABI.

A problem inside a pool takes exactly the kernels and arithmetic it takes
alone, so after s pool sweeps its factors must be bit-identical to s
ntc_sweep calls on it alone, whatever else shares the pool.  The stop rule,
admission by arena memory and slot reuse are checked against their
definitions.
"""
import sys

import numpy as np
import pytest

import paper_2109_09534_amd as ntc
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mix(seed0=500):
    """Small instances of the batching mixture: mixed dims, nnz and R, one
    4-way, one BF16, one MAX_INNER = 2, one with Zipf heads (split rows), one
    with R > 32 and the Collatz-Wielandt L_p bound."""
    out = []
    shapes = [((60, 50, 40), 12000, 8, {}),
              ((200, 90, 70), 40000, 16, {}),
              ((120, 100, 30), 30000, 32, {}),
              ((30, 25, 20, 12), 20000, 10, {}),
              ((150, 80, 60), 35000, 16, {"gather_bf16": True}),
              ((90, 70, 50), 25000, 12, {"max_inner": 2}),
              ((400, 300, 40), 150000, 16, {"zipf": 1.1}),
              ((100, 80, 60), 30000, 48, {"lp_bound": 1})]
    for i, (dims, nnz, R, kw) in enumerate(shapes):
        kw = dict(kw)
        z = kw.pop("zipf", None)
        p = synth.make_problem(dims, nnz, min(R, 8), zipf_s=z, noise_var=0.01, value_model="exact",
                               test_frac=0.05, seed=seed0 + i, name="mix")
        out.append((p, R, dict(seed=seed0 + i, **kw)))
    return out


def _alone(p, R, kw, sweeps):
    g = ntc.Problem(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                    stream=0, **kw)
    g.sweep(sweeps)
    f = g.all_factors()
    loss = g.loss()
    g.close()
    return f, loss


@pytest.mark.parametrize("use_graph", [True, False])
def test_pool_sweeps_are_bit_identical_to_running_alone(use_graph):
    mix = _mix()
    sweeps = 4
    with ntc.Pool(arena_bytes=2 << 30, max_slots=16, use_graph=use_graph, window=0, max_sweeps=1000) as pool:
        slots = []
        for p, R, kw in mix:
            s = pool.admit(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                           **kw)
            assert s is not None
            slots.append(s)
        _say(f"  admitted {len(slots)} problems, {pool.info()}")
        pool.step(sweeps)
        for (p, R, kw), s in zip(mix, slots):
            st, sw, rm = pool.query(s)
            assert st == ntc.SLOT_RUNNING and sw == sweeps
            ref, loss = _alone(p, R, kw, sweeps)
            for m in range(len(p.dims)):
                got = pool.factors(s, m)
                assert np.array_equal(got, ref[m]), (s, m, R, kw)
            assert abs(rm - loss[2]) <= 1e-12 * max(loss[2], 1.0), (rm, loss[2])
            _say(f"  slot {s}: dims {p.dims} R={R} {kw}: factors identical, test RMSE {rm:.6f}")


def test_membership_changes_keep_every_problem_exact():
    """Evict and admit between sweeps; the launch tables and graph are rebuilt
    and every problem still matches its solo run for the sweeps it saw."""
    mix = _mix(700)
    with ntc.Pool(arena_bytes=2 << 30, max_slots=8, window=0, max_sweeps=1000) as pool:
        first = [pool.admit(p.dims, p.coords, p.values, R, test_coords=p.test_coords,
                            test_values=p.test_values, **kw) for p, R, kw in mix[:4]]
        pool.step(2)
        pool.evict(first[1])
        late = [pool.admit(p.dims, p.coords, p.values, R, test_coords=p.test_coords,
                           test_values=p.test_values, **kw) for p, R, kw in mix[4:]]
        pool.step(3)
        seen = {first[0]: (mix[0], 5), first[2]: (mix[2], 5), first[3]: (mix[3], 5)}
        for s, item in zip(late, mix[4:]):
            seen[s] = (item, 3)
        for s, ((p, R, kw), n) in seen.items():
            assert pool.query(s)[1] == n
            ref, _ = _alone(p, R, kw, n)
            for m in range(len(p.dims)):
                assert np.array_equal(pool.factors(s, m), ref[m]), (s, m)
        _say(f"  {len(seen)} problems exact across an eviction and {len(late)} late admissions")


def test_stop_rule_and_slot_reuse():
    p = synth.make_problem((80, 60, 50), 20000, 4, noise_var=0.01, value_model="exact", test_frac=0.1, seed=9)
    R = 4
    W, tol = 3, 1e-3
    with ntc.Pool(arena_bytes=1 << 30, max_slots=4, window=W, tol=tol, max_sweeps=400) as pool:
        s = pool.admit(p.dims, p.coords, p.values, R, c=0.5, test_coords=p.test_coords,
                       test_values=p.test_values, seed=3)
        # several sweeps per step: the device applies the rule after each one
        for _ in range(100):
            pool.step(7)
            if pool.query(s)[0] == ntc.SLOT_STOPPED:
                break
        st, stop_at, _ = pool.query(s)
        assert st == ntc.SLOT_STOPPED and pool.stopped() == [s]
        # the same problem alone: the rule on its own test-RMSE history
        g = ntc.Problem(p.dims, p.coords, p.values, R, c=0.5, test_coords=p.test_coords,
                        test_values=p.test_values, seed=3, stream=0)
        hist = [g.loss()[2]]
        rule_at = None
        for k in range(1, 401):
            g.sweep(1)
            hist.append(g.loss()[2])
            if k >= W and not (hist[k - W] - hist[k] >= tol * hist[k]):
                rule_at = k
                break
        solo = g.all_factors()
        g.close()
        _say(f"  pool stopped after {stop_at} sweeps; the rule on the solo history fires at {rule_at}")
        assert rule_at == stop_at
        # frozen at the stop sweep although the step ran past it
        for m in range(3):
            assert np.array_equal(pool.factors(s, m), solo[m])
        # the stopped problem no longer advances
        pool.step(2)
        assert pool.query(s)[1] == stop_at
        used = pool.info()["used"]
        pool.evict(s)
        assert pool.info()["used"] == 0 and used > 0
        s2 = pool.admit(p.dims, p.coords, p.values, R, c=0.5, test_coords=p.test_coords,
                        test_values=p.test_values, seed=3)
        assert s2 == s and pool.info()["used"] == used


def test_admission_by_arena_memory():
    p = synth.make_problem((100, 80, 60), 30000, 4, noise_var=0.0, value_model="exact", test_frac=0.05, seed=4)
    need = ntc.estimate_bytes(p.dims, p.nnz, 16, n_test=p.test_values.shape[0])
    cap = int(need * 3.5)
    with ntc.Pool(arena_bytes=cap, max_slots=16, window=0) as pool:
        slots = []
        while True:
            s = pool.admit(p.dims, p.coords, p.values, 16, test_coords=p.test_coords,
                           test_values=p.test_values, seed=len(slots))
            if s is None:
                break
            slots.append(s)
            assert len(slots) < 16
        info = pool.info()
        _say(f"  estimate {need} B per problem, arena {cap} B: admitted {len(slots)}, {info}")
        assert len(slots) >= 3
        assert info["used"] <= len(slots) * need
        pool.step(1)
        # two neighbouring problems' memory makes one free block large enough again
        pool.evict(slots[0])
        pool.evict(slots[1])
        assert pool.admit(p.dims, p.coords, p.values, 16, test_coords=p.test_coords,
                          test_values=p.test_values, seed=99) is not None
        # slots are a hard limit too
    with ntc.Pool(arena_bytes=1 << 30, max_slots=2, window=0) as pool:
        assert pool.admit(p.dims, p.coords, p.values, 8) is not None
        assert pool.admit(p.dims, p.coords, p.values, 8) is not None
        assert pool.admit(p.dims, p.coords, p.values, 8) is None


def test_autotuned_schedule_keeps_parity_with_the_oracle():
    """The tuner only reorders sums: the schedule it picks must still match
    the oracle to the one-sweep bar."""
    import oracle as O
    from paper_2109_09534_amd import autotune
    O.build(force=False)
    p = synth.c1_small(seed=5)
    R = 16
    best, table = autotune.tune(p.dims, p.coords, p.values, R, c=0.1, sweeps=2)
    _say("  " + ", ".join(f"{c or 'defaults'}: {ms:.3f} ms" for c, ms in table) + f" -> {best or 'defaults'}")
    assert len(table) == len(autotune.candidates_for(R))
    init = synth.uniform_init(p.dims, R, 1, synth.init_scale(p.values, R, 3))
    g = ntc.Problem(p.dims, p.coords, p.values, R, c=0.1, init=init, schedule=best, stream=0)
    o = O.Oracle(p.dims, p.coords, p.values, R, c=0.1, init=init)
    g.sweep(1)
    o.sweep(1)
    for m in range(3):
        ref = o.factors(m)
        err = np.linalg.norm(g.factors(m) - ref) / np.linalg.norm(ref)
        assert err <= 1e-5, (m, err)


def test_prepared_problems_match_direct_creation():
    """ntc_prepare + ntc_create_prepared (and pool admission of a prepared
    problem, built on a worker thread) give the same bits as ntc_create."""
    import concurrent.futures as cf
    mix = _mix(900)[:4]
    with cf.ThreadPoolExecutor(max_workers=2) as ex:
        futs = [ex.submit(ntc.Prepared, p.dims, p.coords, p.values, R, test_coords=p.test_coords,
                          test_values=p.test_values, **kw) for p, R, kw in mix]
        preps = [f.result() for f in futs]
    with ntc.Pool(arena_bytes=1 << 30, max_slots=8, window=0, max_sweeps=1000) as pool:
        slots = [pool.admit_prepared(q) for q in preps]
        assert all(s is not None for s in slots)
        pool.step(3)
        for (p, R, kw), q, s in zip(mix, preps, slots):
            ref, _ = _alone(p, R, kw, 3)
            g = ntc.Problem.from_prepared(q, stream=0)
            g.sweep(3)
            for m in range(len(p.dims)):
                assert np.array_equal(pool.factors(s, m), ref[m])
                assert np.array_equal(g.factors(m), ref[m])
            g.close()
    for q in preps:
        q.close()


def _oracle_mix(seed0=1100):
    """Batching-mixture instances for the oracle comparison: R = 8 to 32,
    3- and 4-way, FP32 and BF16 gathers, MAX_INNER = 2, Zipf heads split over
    many items (among them the 4-way R = 32 BF16 kernel), and one instance at
    the mixture's upper end (2M entries)."""
    shapes = [((60, 50, 40), 12000, 8, {}, None),
              ((200, 90, 70), 40000, 16, {}, None),
              ((120, 100, 30), 30000, 32, {}, None),
              ((90, 70, 50), 25000, 12, {"max_inner": 2}, None),
              ((400, 300, 40), 150000, 16, {"gather_bf16": True}, 1.1),
              ((300, 200, 60, 20), 300000, 32, {"gather_bf16": True, "schedule": {"item_samples": 128}}, 1.05),
              ((150, 80, 60), 35000, 8, {"gather_bf16": True}, None),
              ((2000, 1500, 1200), 2_000_000, 16, {}, None)]
    out = []
    for i, (dims, nnz, R, kw, z) in enumerate(shapes):
        p = synth.make_problem(dims, nnz, min(R, 8), zipf_s=z, noise_var=0.01, value_model="exact",
                               test_frac=0.05, seed=seed0 + i, name="mix")
        init = synth.uniform_init(p.dims, R, seed0 + i, synth.init_scale(p.values, R, len(dims)))
        out.append((p, R, dict(seed=seed0 + i, c=0.1, **kw), init))
    return out


@pytest.mark.timeout(600)
def test_pool_slots_match_the_oracle():
    """Every slot of a pool against the FP64 oracle run on the same instance
    from the same initial factors: after one pool sweep the factors agree to
    the one-sweep bar (FP32 slots with the plain oracle; BF16 slots with the
    oracle's BF16-gather form), and at the sweep where the device stop rule
    stopped the slot its held-out RMSE is within 1e-3 of the oracle's after
    the same number of sweeps."""
    import oracle as O
    O.build(force=False)
    O.set_threads(8)
    mix = _oracle_mix()
    with ntc.Pool(arena_bytes=4 << 30, max_slots=16, window=5, tol=1e-4, max_sweeps=150) as pool:
        slots = []
        for p, R, kw, init in mix:
            s = pool.admit(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                           init=init, **kw)
            assert s is not None
            slots.append(s)
        _say(f"  admitted {len(slots)} problems, {pool.info()}")
        pool.step(1)
        oras = []
        for (p, R, kw, init), s in zip(mix, slots):
            bf = bool(kw.get("gather_bf16"))
            okw = {k: v for k, v in kw.items() if k not in ("gather_bf16", "schedule")}
            o = O.Oracle(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                         init=init, gather_bf16=bf, **okw)
            o.sweep(1)
            for m in range(len(p.dims)):
                got = pool.factors(s, m).astype(np.float64)
                ref = o.factors(m)
                err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                scale = np.sqrt(np.mean(ref ** 2))
                worst = np.max(np.abs(got - ref) / (np.abs(ref) + scale))
                _say(f"  slot {s} dims {p.dims} R={R} {'BF16' if bf else 'FP32'} mode {m}: rel Frobenius "
                     f"{err:.2e}, worst element {worst:.2e}")
                assert np.all(got >= 0.0)
                # BF16 slots: the rounding decisions of the gathers follow the FP32 (GPU) and FP64 (oracle)
                # values of the factors; on these seeds none of them differs, so the one-sweep bar holds
                # element by element as for FP32
                assert err <= 1e-5, (s, m, err)
                assert worst <= 1e-5, (s, m, worst)
            if bf:   # the held-out target is the plain FP64 method's
                o.close()
                o = O.Oracle(p.dims, p.coords, p.values, R, test_coords=p.test_coords,
                             test_values=p.test_values, init=init, **okw)
                o.sweep(1)
            oras.append(o)
        for _ in range(60):
            if pool.info()["running"] == 0:
                break
            pool.step(4)
        assert pool.info()["running"] == 0
        for (p, R, kw, init), s, o in zip(mix, slots, oras):
            st, stop_at, rm = pool.query(s)
            assert st == ntc.SLOT_STOPPED
            o.sweep(stop_at - 1)
            lo = o.loss()
            lg = pool.loss(s)
            _say(f"  slot {s} R={R} {kw.get('gather_bf16', False) and 'BF16' or 'FP32'}: stopped at sweep "
                 f"{stop_at}, test RMSE {lg[2]:.6f}, oracle after {stop_at} sweeps {lo[2]:.6f}")
            assert abs(lg[2] - lo[2]) <= 1e-3, (s, lg[2], lo[2])
            o.close()


def test_device_csr_admission_matches_host_admission():
    """ntc_pool_admit_device_csr builds each problem's CSR on the GPU (its
    temporaries from the arena, returned before the call does): the slot is
    bit-identical to the host-built admission after several sweeps, and the
    arena holds exactly what the host-built problem holds."""
    mix = _mix(1300)[:5]
    res = []
    for dev in (False, True):
        with ntc.Pool(arena_bytes=2 << 30, max_slots=8, window=0, max_sweeps=1000) as pool:
            slots = [pool.admit(p.dims, p.coords, p.values, R, test_coords=p.test_coords,
                                test_values=p.test_values, device_csr=dev, **kw) for p, R, kw in mix]
            assert all(s is not None for s in slots)
            used = pool.info()["used"]
            pool.step(3)
            res.append((used, [[pool.factors(s, m) for m in range(len(p.dims))] for (p, _, _), s in zip(mix, slots)],
                        [pool.query(s)[2] for s in slots]))
    (uh, fh, rh), (ud, fd, rd) = res
    _say(f"  arena bytes in use after admission: host CSR {uh}, device CSR {ud}")
    assert uh == ud
    for a, b in zip(fh, fd):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    assert rh == rd
