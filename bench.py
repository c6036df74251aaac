#!/usr/bin/env python3
"""Benchmark: AO accelerated stochastic NTC on one MI355X.

Workload (default): 3-way 480,000 x 18,000 x 2,000 tensor, 100M distinct
observed cells with Zipf(1.1) index popularity per mode, values a rank-16
nonnegative CPD scaled to [1,5] + N(0, 0.1) noise rounded to 1..5, 5% held
out; R = 16, c = 0.1, lambda = 1e-3, MAX_INNER = 1, FP32 factors.

A step is one AO sweep (Alg. 2: every mode updated once by Alg. 1).  The
reported value is observed-entry updates per second: sampled entries
consumed per sweep (sum over modes of sum_p floor(c n_p)) times the timed
sweeps, over the wall time of the timed region (device synchronised on
both sides, inputs resident in HBM).

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 2] [--scale 1.0]
                       [--no-cpu-baseline] [--bf16]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
PROFILES = os.path.join(ROOT, "profiles")


CACHED_RECORD_BYTES = 256 << 20  # records (all modes) above this are loaded non-temporally


def kernel_name(kind: str, nmodes: int, R: int, bf16: bool, nnz: int) -> str:
    """The kernel rocprofv3 reports for one of profile_sweep's launch kinds (N <= 4)."""
    b = "true" if bf16 else "false"
    nt = "true" if nnz * 16 * nmodes > CACHED_RECORD_BYTES else "false"
    if R <= 16:
        v4 = "true" if R % 4 == 0 else "false"
        return {"row_items": f"k_rows16<{nmodes}, 4, {b}, {nt}>", "row_chunks": f"k_chunk16<{nmodes}, 4, {b}, {nt}>",
                "row_tiny": f"k_quad16<{nmodes}, {b}, {v4}, {nt}>", "row_finalize": f"k_finalize16<{b}>",
                "row_few": f"k_few16<{nmodes}, {b}, {v4}, {nt}>"}[kind]
    if R <= 32:
        pairs = "true" if R % 2 == 0 else "false"
        w = 3 if R == 32 else (2 if R % 8 == 0 else 1 if R % 2 == 0 else 0) if bf16 else \
            (2 if R % 4 == 0 else 1 if R % 2 == 0 else 0)
        return {"row_items": f"k_rows32<{nmodes}, {b}, {pairs}, {nt}>", "row_finalize": f"k_finalize32<{b}>",
                "row_reduce": "k_reduce_slots<32>", "row_tiny": f"k_few32<{nmodes}, {b}, {w}, {nt}>"}[kind]
    vec = 4 if R % 4 == 0 else 2 if R % 2 == 0 else 1
    return {"row_items": f"k_rows64<{nmodes}, {b}, {vec}, {nt}>", "row_finalize": f"k_row_finalize<64, {b}>",
            "row_reduce": "k_reduce_slots<64>"}[kind]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(nmodes: int, R: int, samples: int, rows: int, max_inner: int, bf16: bool):
    """Bytes the method must move for one mode update (per Alg. 1 inner step
    summed): per sampled entry the record (N-1 int32 coordinates + FP32 value)
    and the N-1 gathered factor rows (R x 4 B, or R x 2 B from the BF16
    shadow); per row step the two rowptr words, Y(p) read, A_l(p) read when
    l >= 1, A_{l+1}(p) write, Y_{l+1}(p) write when l+1 < MAX_INNER, and the
    BF16 shadow write in the precision form."""
    sf = 2 if bf16 else 4
    per_upd = 4 * nmodes + (nmodes - 1) * R * sf
    return per_upd, samples * per_upd, rows * 16 + rows * 4 * R * 2 + (rows * 2 * R if bf16 else 0)


def load_traffic(name: str):
    """Measured HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 --pmc summary, if it was taken on the current kernel source."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2109_09534_amd.profiling import source_hash
    if d.get("kernel_source_hash") != source_hash(bool(d.get("wide"))):
        return None
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the 100M entries (dims kept)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--bf16", action="store_true", help="BF16 shadow gathers (precision form)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-errors", action="store_true",
                    help="c2: skip the FP32/BF16 error statement against the FP64 oracle (1/10-nnz instance)")
    ap.add_argument("--oracle-sweeps", type=int, default=4,
                    help="c2: sweeps of the precision check against the oracle")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--workload", choices=["c1", "c2", "batch", "serve", "scaling", "convergence"], default="c1",
                    help="c1: one 100M-entry problem (default); c2: one 4-way 500M-entry R=32 problem; "
                         "batch: many small problems in one pool; "
                         "serve: Poisson arrivals into a pool; "
                         "scaling: the twin of the paper's timing workload, time per epoch per rank; "
                         "convergence: the twin of the paper's convergence experiment, RRE per epoch")
    ap.add_argument("--epochs", type=int, default=100, help="convergence: epochs per run")
    ap.add_argument("--oracle-epochs", type=int, default=4, help="convergence: epochs the oracle repeats")
    ap.add_argument("--estimators", default="rq20",
                    help="convergence: L_p estimators, comma separated: rqT = Rayleigh quotient after T power "
                         "iterations (the paper's), cwT = Collatz-Wielandt bound of the same iterate")
    ap.add_argument("--inner", default="1,2", help="convergence: MAX_INNER values")
    ap.add_argument("--lp-bound", type=int, default=0,
                    help="c1/c2: 1 = L_p as the Collatz-Wielandt bound of the power iterate")
    ap.add_argument("--power-iters", type=int, default=20, help="c1/c2: power iterations T_pow")
    ap.add_argument("--device-csr", action="store_true",
                    help="c1/c2: build the per-mode CSR on the GPU (ntc_create_device_csr)")
    ap.add_argument("--ranks", default="10,30,50", help="scaling: ranks R")
    ap.add_argument("--instances", type=int, default=256, help="batch/serve: number of problems")
    ap.add_argument("--no-plain", action="store_true", help="batch/serve: skip the one-at-a-time FP32 baseline")
    ap.add_argument("--oracle-instances", type=int, default=32,
                    help="batch/serve: problems (evenly spread over the stream) whose final held-out RMSE is "
                         "checked against the FP64 oracle run to the same plateau rule (0 = none)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch: library default schedule instead of one tuned per kernel family")
    ap.add_argument("--rates", default="0.25,0.5,1,2", help="serve: arrival rates as fractions of saturation")
    ap.add_argument("--admit-device-csr", type=int, default=0,
                    help="serve: requests with at least this many entries are admitted with the CSR built on the "
                         "GPU (ntc_pool_admit_device_csr) instead of prepared on a host thread (0 = never)")
    ap.add_argument("--prepare-threads", type=int, default=2,
                    help="serve: host threads building arriving requests' CSR while the pool sweeps")
    ap.add_argument("--sweeps-per-step", type=int, default=4,
                    help="batch/serve: pool sweeps between host checks (the stop rule runs on the device)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} (WORLD_SIZE={world}) is not supported; "
              "sharding the rows over several GPUs is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "scaling":
        return run_scaling(args)
    if args.workload == "convergence":
        return run_convergence(args)

    import numpy as np

    import paper_2109_09534_amd as ntc
    import synth

    ntc.lib()       # fails loudly without the HIP library
    c, lam, max_inner = 0.1, 1e-3, 1
    t0 = time.perf_counter()
    if args.workload == "c2":
        R = 32
        log(f"generating the 1000000x500000x1000x100 Zipf(1.05) workload, scale {args.scale} ...")
        p = synth.c2(seed=args.seed, scale=args.scale)
        wl = ("4-way 1000000x500000x1000x100, 500M Zipf(1.05) entries, rank-32 CPD + N(0,0.05) clipped at 0, "
              "5% test; R=32, c=0.1, lambda=1e-3, MAX_INNER=1")
        args.no_cpu_baseline = True     # the oracle is timed on the 1/10-nnz instance of the precision check
    else:
        R = 16
        log(f"generating the 480000x18000x2000 Zipf(1.1) workload, scale {args.scale} ...")
        p = synth.c1(seed=args.seed, scale=args.scale)
        wl = ("3-way 480000x18000x2000, 100M Zipf(1.1) entries, rank-16 ratings 1..5, 5% test; R=16, c=0.1, "
              "lambda=1e-3, MAX_INNER=1")
    gen_s = time.perf_counter() - t0
    log(f"generated {p.nnz} train / {p.test_values.shape[0]} test entries in {gen_s:.1f} s (SNR {p.snr:.2f})")

    t0 = time.perf_counter()
    prob = ntc.Problem(p.dims, p.coords, p.values, R, c=c, lam=lam, max_inner=max_inner, seed=args.seed,
                       gather_bf16=args.bf16, test_coords=p.test_coords, test_values=p.test_values, stream=0,
                       power_iters=args.power_iters, lp_bound=args.lp_bound, device_csr=args.device_csr)
    create_s = time.perf_counter() - t0
    upd_sweep, rows_sweep = prob.work()
    log(f"ntc_create {create_s:.1f} s; {upd_sweep} sampled entries and {rows_sweep} row steps per sweep")

    loss0 = prob.loss()
    if args.warmup > 0:
        prob.time_sweeps(args.warmup)
    prob.synchronize()
    log(f"warmup {args.warmup} sweeps done; timing {args.steps} sweeps")
    t0 = time.perf_counter()
    dev_ms = prob.time_sweeps(args.steps)        # ends with a stream synchronisation
    prob.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = upd_sweep * args.steps / wall
    log(f"timed: {wall * 1e3:.2f} ms wall, {dev_ms:.2f} ms device for {args.steps} sweeps")

    # Per-launch HIP events over a second run of the same K sweeps in the same
    # launch configuration (side-stream overlap on), each pair of events on the
    # stream its launch runs on: the roofline of the dominant kernel, the one
    # with the largest share of the launch time.
    launches = prob.profile_sweeps(args.steps, concurrent=True)
    per_sweep = len(launches) // max(args.steps, 1)
    per_kernel = {}
    sweep_bytes = 0
    per_mode = []
    for i, rec in enumerate(launches):
        _, b_upd, b_rows = algorithmic_bytes(p.nmodes, R, rec["samples"], rec["rows"], max_inner, args.bf16)
        k = per_kernel.setdefault(rec["kernel"], {"bytes": 0, "ms": 0.0, "launches": 0})
        k["bytes"] += b_upd + b_rows
        k["ms"] += rec["ms"]
        k["launches"] += 1
        if i < per_sweep:
            sweep_bytes += b_upd + b_rows
            per_mode.append(dict(rec))
        else:
            per_mode[i % per_sweep]["ms"] += rec["ms"]
    for rec in per_mode:  # mean over the K sweeps
        rec["ms"] = round(rec["ms"] / max(args.steps, 1), 4)
    dom = max(per_kernel, key=lambda n: per_kernel[n]["ms"])
    kd = per_kernel[dom]
    avg_ms = kd["ms"] / kd["launches"]
    bytes_per_launch = kd["bytes"] / kd["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kfile = kernel_name(dom, p.nmodes, R, args.bf16, p.nnz).split("<")[0]
    traffic_rec = load_traffic(f"{kfile}_{args.workload}{'_bf16' if args.bf16 else ''}_traffic.json")
    traffic = traffic_rec["hbm_bytes_per_launch"] if traffic_rec else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_name(dom, p.nmodes, R, args.bf16, p.nnz), "avg_launch_ms": round(avg_ms, 4),
                "launches_per_sweep": kd["launches"] // max(args.steps, 1),
                "algorithmic_bytes_per_launch": round(bytes_per_launch),
                "sweep_share": round(kd["ms"] / sum(v["ms"] for v in per_kernel.values()), 3)}
    hbm_frac = sweep_bytes * args.steps / wall / (HBM_PEAK_GBS * 1e9)

    t0 = time.perf_counter()
    loss = prob.loss()
    loss_ms = (time.perf_counter() - t0) * 1e3
    log(f"loss before {loss0}, after {loss} ({loss_ms:.1f} ms)")

    other = None
    if args.workload == "c2":
        # the other precision on the same data, same seed and sweep count: rate and held-out quality
        prob.close()
        alt = not args.bf16
        q = ntc.Problem(p.dims, p.coords, p.values, R, c=c, lam=lam, max_inner=max_inner, seed=args.seed,
                        gather_bf16=alt, test_coords=p.test_coords, test_values=p.test_values, stream=0,
                        power_iters=args.power_iters, lp_bound=args.lp_bound)
        if args.warmup > 0:
            q.time_sweeps(args.warmup)
        q.synchronize()
        t1 = time.perf_counter()
        q.time_sweeps(args.steps)
        q.synchronize()
        wall_q = time.perf_counter() - t1
        q.time_sweeps(args.steps)  # the main problem's profiled sweeps: the same count before its loss
        loss_q = q.loss()
        q.close()
        other = {"gather": "bf16" if alt else "f32", "value": round(upd_sweep * args.steps / wall_q, 1),
                 "ms_per_step": round(wall_q * 1e3 / args.steps, 4), "test_rmse": round(float(loss_q[2]), 6)}
        log(f"{other['gather']} gathers: {other['ms_per_step']} ms per sweep, test RMSE {other['test_rmse']}")

    cpu = None
    precision = None
    if args.workload == "c2" and not args.no_oracle_errors:
        precision, cpu = c2_precision_vs_oracle(args, c, lam, max_inner)
    if not args.no_cpu_baseline:
        import oracle as O
        threads = args.cpu_threads or len(os.sched_getaffinity(0))
        used = O.set_threads(threads)
        log(f"cpu baseline: FP64 oracle, {used} threads: building its CSR ...")
        t0 = time.perf_counter()
        o = O.Oracle(p.dims, p.coords, p.values, R, c=c, lam=lam, max_inner=max_inner, seed=args.seed)
        log(f"oracle create {time.perf_counter() - t0:.1f} s; timing one full sweep")
        t0 = time.perf_counter()
        o.sweep(1)
        cpu_s = time.perf_counter() - t0
        o.close()
        cpu = {"value": round(upd_sweep / cpu_s, 1), "unit": "updates/s", "cores": used, "kind": "oracle",
               "sample": f"one full AO sweep ({upd_sweep} sampled entries, all 3 modes) of the same workload "
                         f"from the same initial factors, FP64, {cpu_s:.2f} s"}
        log(f"oracle sweep {cpu_s:.2f} s -> {upd_sweep / cpu_s:.3e} updates/s")

    out = {
        "metric": "observed-entry updates/s",
        "value": round(value, 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if not args.bf16 else "bf16-gather/f32",
        "data": "synthetic",
        "config": {"workload": wl + (" (BF16 gathers)" if args.bf16 else "")
                   + ("" if (args.lp_bound, args.power_iters) == (0, 20) else
                      f" (L_p: {'Collatz-Wielandt bound' if args.lp_bound else 'Rayleigh quotient'}, "
                      f"T_pow={args.power_iters})"),
                   "nnz_train": p.nnz, "scale": args.scale, "seed": args.seed,
                   "updates_per_sweep": upd_sweep, "row_steps_per_sweep": rows_sweep},
        "pct_hbm_peak": round(100 * hbm_frac, 2),
        "algorithmic_bytes_per_sweep": sweep_bytes,
        "device_ms_per_step": round(dev_ms / args.steps, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "create_s": round(create_s, 2),
        "create": "device CSR build" if args.device_csr else "host CSR build",
        "generate_s": round(gen_s, 2),
        "loss_ms": round(loss_ms, 2),
        "test_rmse": round(float(loss[2]), 6),
        "train_rmse": round(float(loss[1]), 6),
        "launches": per_mode,
    }
    if other is not None:
        out["other_precision"] = other
    if precision is not None:
        out["precision_vs_oracle"] = precision
    print(json.dumps(out), flush=True)


def c2_precision_vs_oracle(args, c, lam, max_inner):
    """The precision form's error against the FP64 oracle, on a 1/10-nnz
    instance of the 4-way workload (same dims and distributions, 50M
    entries, so the oracle finishes in seconds): from the same default
    initial factors, the relative Frobenius error of every factor after one
    sweep for FP32 and for BF16 gathers, and the held-out RMSE of both after
    `oracle_sweeps` sweeps beside the oracle's.  The oracle's first sweep is
    also the CPU baseline of this workload."""
    import numpy as np

    import oracle as O
    import paper_2109_09534_amd as ntc
    import synth

    R, K = 32, args.oracle_sweeps
    t0 = time.perf_counter()
    p = synth.c2(seed=args.seed, scale=0.1)
    log(f"precision check: 1/10-nnz instance, {p.nnz} train entries, generated in {time.perf_counter() - t0:.1f} s")
    res = {}
    for bf in (False, True):
        g = ntc.Problem(p.dims, p.coords, p.values, R, c=c, lam=lam, max_inner=max_inner, seed=args.seed,
                        gather_bf16=bf, test_coords=p.test_coords, test_values=p.test_values, stream=0)
        g.sweep(1)
        res[bf] = {"f1": g.all_factors()}
        g.sweep(K - 1)
        res[bf]["loss"] = g.loss()
        g.close()
    threads = args.cpu_threads or len(os.sched_getaffinity(0))
    used = O.set_threads(threads)
    o = O.Oracle(p.dims, p.coords, p.values, R, c=c, lam=lam, max_inner=max_inner, seed=args.seed,
                 test_coords=p.test_coords, test_values=p.test_values)
    upd = _updates_per_sweep(p, c)
    t0 = time.perf_counter()
    o.sweep(1)
    cpu_s = time.perf_counter() - t0
    f1 = [o.factors(m) for m in range(p.nmodes)]
    log(f"oracle: first sweep {cpu_s:.2f} s on {used} threads; {K - 1} more sweeps")
    o.sweep(K - 1)
    lo = o.loss()
    o.close()
    out = {"instance": f"4-way 1000000x500000x1000x100, {p.nnz} Zipf(1.05) train entries (1/10 of the "
                       f"workload's, same dims and distributions), {p.test_values.shape[0]} held out",
           "sweeps": K, "oracle_test_rmse": round(float(lo[2]), 6)}
    for bf in (False, True):
        errs = [float(np.linalg.norm(res[bf]["f1"][m] - f1[m]) / np.linalg.norm(f1[m])) for m in range(p.nmodes)]
        tr = float(res[bf]["loss"][2])
        out["bf16" if bf else "f32"] = {"one_sweep_rel_err_per_mode": [float(f"{e:.3e}") for e in errs],
                                        "test_rmse": round(tr, 6), "test_rmse_minus_oracle": float(f"{tr - lo[2]:.3e}")}
        log(f"{'BF16' if bf else 'FP32'} gathers: one-sweep error vs FP64 per mode {errs}; test RMSE after {K} "
            f"sweeps {tr:.6f} (oracle {lo[2]:.6f})")
    cpu = {"value": round(upd / cpu_s, 1), "unit": "updates/s", "cores": used, "kind": "oracle",
           "sample": f"one full AO sweep ({upd} sampled entries, all 4 modes) of the 1/10-nnz instance, FP64, "
                     f"{cpu_s:.2f} s"}
    return out, cpu


# ------------------------------------------------------------ scaling twin
def run_scaling(args):
    """Twin of the paper's timing workload (Section IV-C): 4-way
    183x24x1140x1717, 3,309,490 uniform cells of a noiseless rank-10 CPD,
    c = 0.5, MAX_INNER = 1; one epoch is ceil(1/c) = 2 sweeps.  Per rank R:
    the GPU's time per epoch (mean of 5 epochs after a warm-up epoch), the FP64
    oracle's time per epoch against its thread count, and the largest
    difference of the factors after the first epoch from identical initial
    factors (relative to each mode's largest entry)."""
    import math

    import numpy as np

    import oracle as O
    import paper_2109_09534_amd as ntc
    import synth

    ntc.lib()
    O.build(force=False)
    c, lam = 0.5, 1e-3
    epoch = int(math.ceil(1.0 / c))
    ranks = [int(r) for r in args.ranks.split(",") if r]
    tmax = args.cpu_threads or len(os.sched_getaffinity(0))
    thread_sweep = sorted({t for t in (1, 2, 4, 8, 16) if t < tmax} | {tmax})
    t0 = time.perf_counter()
    p = synth.scaling_twin(seed=args.seed)
    gen_s = time.perf_counter() - t0
    upd_sweep = _updates_per_sweep(p, c)
    log(f"generated the 183x24x1140x1717 twin, {p.nnz} cells, in {gen_s:.1f} s; {upd_sweep} updates per sweep")
    per_rank = []
    for R in ranks:
        init = synth.uniform_init(p.dims, R, 1, synth.init_scale(p.values, R, len(p.dims)))
        g = ntc.Problem(p.dims, p.coords, p.values, R, c=c, lam=lam, seed=args.seed, init=init, stream=0)
        g.sweep(epoch)  # the first epoch, from init: compared with the oracle's below
        gf = g.all_factors()
        g.time_sweeps(epoch)  # warm-up epoch
        trials = []
        for _ in range(5):
            t1 = time.perf_counter()
            g.time_sweeps(epoch)  # ends with a synchronisation
            trials.append(time.perf_counter() - t1)
        g.close()
        gpu_s = sum(trials) / len(trials)
        o = O.Oracle(p.dims, p.coords, p.values, R, c=c, lam=lam, seed=args.seed, init=init)
        O.set_threads(tmax)
        o.sweep(epoch)
        diff = max(float(np.max(np.abs(gf[m] - o.factors(m))) / max(float(np.max(np.abs(o.factors(m)))), 1e-30))
                   for m in range(len(p.dims)))
        cpu = {}
        for t in (thread_sweep if R == ranks[0] else [tmax]):
            used = O.set_threads(t)
            t1 = time.perf_counter()
            o.sweep(epoch)
            cpu[str(used)] = round(time.perf_counter() - t1, 4)
        o.close()
        row = {"R": R, "gpu_s_per_epoch": round(gpu_s, 6), "gpu_updates_per_s": round(epoch * upd_sweep / gpu_s, 1),
               "oracle_s_per_epoch_by_threads": cpu, "first_epoch_max_rel_diff": diff}
        log(f"R={R}: GPU {gpu_s * 1e3:.2f} ms per epoch; oracle {cpu} s per epoch; "
            f"first-epoch factors differ by {diff:.2e}")
        per_rank.append(row)
    head = per_rank[0]
    out = {
        "metric": "time per epoch", "value": head["gpu_s_per_epoch"], "unit": "s/epoch", "n_gpus": 1,
        "steps": 5, "warmup": 1, "ms_per_step": round(head["gpu_s_per_epoch"] * 1e3, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "twin of the Section IV-C timing workload: 4-way 183x24x1140x1717, 3,309,490 "
                               "uniform cells, noiseless rank-10 CPD with U[0,1] factors; c=0.5, MAX_INNER=1, "
                               f"1 epoch = {epoch} sweeps; value is R={head['R']}",
                   "nnz_train": p.nnz, "seed": args.seed, "updates_per_sweep": upd_sweep},
        "ranks": per_rank,
        "cpu_baseline": {"value": head["oracle_s_per_epoch_by_threads"][str(tmax)], "unit": "s/epoch",
                         "cores": tmax, "kind": "oracle",
                         "sample": f"one epoch of the same workload at R={head['R']}, FP64"},
        "generate_s": round(gen_s, 2),
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------------------ convergence twin
def run_convergence(args):
    """Twin of the paper's convergence experiment (Section IV-B): a
    71567x65133x730 tensor with 10,000,054 uniform cells (5% held out) of a
    rank-10 CPD with U[0,1] factors plus Gaussian noise at two SNRs, R = 10,
    lambda = 1e-3, c in {0.05, 0.2, 0.5}, MAX_INNER in {1, 2}; the held-out
    relative reconstruction error after every epoch (ceil(1/c) sweeps) for
    `--epochs` epochs.  The FP64 oracle repeats the first `--oracle-epochs`
    epochs of two runs from the same default initialisation."""
    import math

    import oracle as O
    import paper_2109_09534_amd as ntc
    import synth

    ntc.lib()
    O.build(force=False)
    tmax = args.cpu_threads or len(os.sched_getaffinity(0))
    O.set_threads(tmax)
    R, lam = 10, 1e-3
    snrs = {"S1": 100.0, "S2": 2.0}
    cs = (0.05, 0.2, 0.5)
    inners = tuple(int(x) for x in args.inner.split(",") if x)
    ests = []
    for e in args.estimators.split(","):
        e = e.strip()
        if e[:2] not in ("rq", "cw"):
            raise SystemExit(f"unknown estimator {e}")
        ests.append((e, 1 if e[:2] == "cw" else 0, int(e[2:])))
    checks = {("S1", 0.5, 1, ests[0][0]), ("S2", 0.05, 2, ests[0][0])} | {("S1", 0.2, inners[0], e[0])
                                                                             for e in ests[1:]}
    runs, oracle_checks = [], []
    gen_s = 0.0
    for name, snr in snrs.items():
        t0 = time.perf_counter()
        p = synth.convergence_twin(seed=args.seed, snr=snr)
        gen_s += time.perf_counter() - t0
        log(f"{name}: generated {p.nnz} train / {p.test_values.shape[0]} test entries, SNR {p.snr:.2f}")
        for (est, lpb, T), c, mi in [(e, c, mi) for e in ests for c in cs for mi in inners]:
            spe = int(math.ceil(1.0 / c))
            g = ntc.Problem(p.dims, p.coords, p.values, R, c=c, lam=lam, max_inner=mi, seed=args.seed,
                            test_coords=p.test_coords, test_values=p.test_values, stream=0,
                            power_iters=T, lp_bound=lpb)
            rre = [float(g.loss()[3])]
            t1 = time.perf_counter()
            sweep_s = 0.0
            for _ in range(args.epochs):
                t2 = time.perf_counter()
                g.sweep(spe)
                g.synchronize()
                sweep_s += time.perf_counter() - t2
                rre.append(float(g.loss()[3]))
            wall = time.perf_counter() - t1
            g.close()
            run = {"data": name, "snr": round(p.snr, 3), "estimator": est, "c": c, "max_inner": mi,
                   "sweeps_per_epoch": spe,
                   "gpu_s_per_epoch": round(sweep_s / args.epochs, 6), "wall_s": round(wall, 3),
                   "rre": [round(x, 6) for x in rre]}
            runs.append(run)
            log(f"{name} {est} c={c} MAX_INNER={mi}: RRE {rre[0]:.4f} -> {rre[min(10, args.epochs)]:.4f} "
                f"(10 epochs) -> {rre[-1]:.4f} ({args.epochs} epochs); "
                f"{run['gpu_s_per_epoch'] * 1e3:.2f} ms per epoch")
            if (name, c, mi, est) in checks and args.oracle_epochs > 0:
                o = O.Oracle(p.dims, p.coords, p.values, R, c=c, lam=lam, max_inner=mi, seed=args.seed,
                             test_coords=p.test_coords, test_values=p.test_values, power_iters=T,
                             lp_bound=lpb)
                orre = [float(o.loss()[3])]
                t2 = time.perf_counter()
                for _ in range(args.oracle_epochs):
                    o.sweep(spe)
                    orre.append(float(o.loss()[3]))
                o_s = time.perf_counter() - t2
                o.close()
                diff = max(abs(a - b) for a, b in zip(orre, rre))
                oracle_checks.append({"data": name, "estimator": est, "c": c, "max_inner": mi,
                                      "epochs": args.oracle_epochs,
                                      "oracle_rre": [round(x, 6) for x in orre], "max_abs_rre_diff": diff,
                                      "oracle_s_per_epoch": round(o_s / args.oracle_epochs, 3),
                                      "threads": tmax})
                log(f"  oracle, {args.oracle_epochs} epochs: max |RRE difference| {diff:.2e}, "
                    f"{o_s / args.oracle_epochs:.2f} s per epoch on {tmax} threads")

    def final(name, c, mi, e):
        for r in runs:
            if r["data"] == name and r["c"] == c and r["max_inner"] == mi and r["estimator"] == ests[0][0]:
                return r["rre"][min(e, len(r["rre"]) - 1)]
        return None
    # the paper's reading of its figure: small c pays at high SNR, not at low SNR
    ordering = {name: {f"epoch{e}": {str(c): final(name, c, 1, e) for c in cs} for e in (10, args.epochs)}
                for name in snrs}
    head = final("S1", 0.5, 1, args.epochs)
    out = {
        "metric": "held-out RRE after the last epoch (S1, c=0.5, MAX_INNER=1)", "value": head, "unit": "RRE",
        "n_gpus": 1, "steps": args.epochs, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "twin of the Section IV-B convergence experiment: 71567x65133x730, 10,000,054 "
                               "uniform cells (5% held out), rank-10 CPD with U[0,1] factors + N(0, sigma^2) at "
                               "SNR 100 (S1) and 2 (S2); R=10, lambda=1e-3, c in {0.05, 0.2, 0.5}, "
                               "MAX_INNER in {1, 2}", "epochs": args.epochs, "seed": args.seed},
        "runs": runs, "oracle_checks": oracle_checks, "rre_by_c": ordering, "generate_s": round(gen_s, 2),
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------ batching form
def _updates_per_sweep(p, c=0.1):
    import numpy as np
    u = 0
    for m in range(len(p.dims)):
        n = np.bincount(p.coords[:, m], minlength=p.dims[m]).astype(np.float64)
        u += int(np.floor(c * n).sum())
    return u


def _stop_at(hist, W=5, tol=1e-4, cap=500):
    """Sweep at which the held-out plateau rule stops (hist[k] after k sweeps)."""
    for k in range(1, len(hist)):
        if k >= cap or (k >= W and not (hist[k - W] - hist[k] >= tol * hist[k])):
            return k
    return None


def _batch_problems(n, seed):
    import synth
    shapes = synth.c3_shapes(n, base_seed=1000 + 7919 * seed)
    return shapes, [synth.c3_instance(*sh) for sh in shapes]


def run_batch(args):
    """Many independent 3-way problems (dims log-U[50,2000], nnz log-U[10k,2M],
    R in {8,16,32}) solved to the held-out plateau in one pool, against the
    same problems run one at a time through ntc_create/ntc_sweep/ntc_loss."""
    import numpy as np

    import paper_2109_09534_amd as ntc
    ntc.lib()
    n = args.instances
    t0 = time.perf_counter()
    shapes, probs = _batch_problems(n, args.seed)
    gen_s = time.perf_counter() - t0
    nnz = sum(p.nnz for p in probs)
    log(f"generated {n} problems, {nnz} train entries in {gen_s:.1f} s")
    kw = dict(c=0.1, lam=1e-3, gather_bf16=args.bf16)
    kw_plain = dict(c=0.1, lam=1e-3, gather_bf16=False)   # the plain method: FP32 gathers

    # one schedule per kernel family (R <= 16, R <= 32), tuned on its largest problem
    sched = {}
    tune_s = 0.0
    if not args.no_autotune:
        from paper_2109_09534_amd import autotune
        t0 = time.perf_counter()
        sched = autotune.tune_classes([(p.dims, p.coords, p.values, sh[2]) for sh, p in zip(shapes, probs)],
                                      sweeps=3, **kw)
        tune_s = time.perf_counter() - t0
        log(f"autotuned schedules {sched} in {tune_s:.1f} s")

    def schedule_of(R):
        return sched.get(16 if R <= 16 else 32 if R <= 32 else 64, {})

    pool = ntc.Pool(max_slots=n, window=5, tol=1e-4, max_sweeps=500)
    t0 = time.perf_counter()
    slots = []
    # host preparation (CSR build, schedule) on worker threads, admission in
    # submission order on this thread
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=max(1, args.prepare_threads)) as ex:
        futs = [ex.submit(ntc.Prepared, p.dims, p.coords, p.values, R, seed=sd, test_coords=p.test_coords,
                          test_values=p.test_values, schedule=schedule_of(R), **kw)
                for (dims, _, R, sd), p in zip(shapes, probs)]
        for f in futs:
            q = f.result()
            s = pool.admit_prepared(q)
            q.close()
            if s is None:
                raise RuntimeError("the pool could not hold every problem")
            slots.append(s)
    admit_s = time.perf_counter() - t0
    log(f"admitted {n} problems in {admit_s:.2f} s; {pool.info()}")
    t0 = time.perf_counter()
    sweeps = 0
    while pool.info()["running"] > 0:
        pool.step(args.sweeps_per_step)
        sweeps += args.sweeps_per_step
    run_s = time.perf_counter() - t0
    per = [pool.query(s) for s in slots]
    upd = sum(_updates_per_sweep(p) * q[1] for p, q in zip(probs, per))
    log(f"all stopped after {sweeps} pool sweeps, {run_s:.3f} s; {upd} updates")
    pool.close()

    plain = None
    plain_rmse = None
    if not args.no_plain:
        t0 = time.perf_counter()
        diffs = []
        plain_rmse = []
        for (dims, _, R, sd), p, q in zip(shapes, probs, per):
            g = ntc.Problem(p.dims, p.coords, p.values, R, seed=sd, test_coords=p.test_coords,
                            test_values=p.test_values, stream=0, schedule=schedule_of(R), **kw_plain)
            hist = [g.loss()[2]]
            while _stop_at(hist) is None:
                g.sweep(1)
                hist.append(g.loss()[2])
            g.close()
            plain_rmse.append(hist[-1])
            diffs.append((len(hist) - 1 - q[1], abs(hist[-1] - q[2])))
        plain_s = time.perf_counter() - t0
        plain = {"value": round(n / plain_s, 3), "unit": "instances/s", "seconds": round(plain_s, 3),
                 "dtype": "f32",
                 "kind": "the same problems one at a time through ntc_create/ntc_sweep/ntc_loss with FP32 "
                         "gathers, create included",
                 "max_stop_sweep_diff_vs_pool": int(max(abs(d[0]) for d in diffs)),
                 "max_final_rmse_diff_vs_pool": float(max(d[1] for d in diffs))}
        log(f"plain one-at-a-time (FP32): {plain_s:.2f} s")

    check = None
    if args.oracle_instances > 0:
        idx = sorted(set(np.linspace(0, n - 1, min(n, args.oracle_instances)).astype(int).tolist()))
        t0 = time.perf_counter()
        targets, threads = _oracle_plateau([(probs[i], shapes[i][2], shapes[i][3]) for i in idx], args.cpu_threads)
        ora_s = time.perf_counter() - t0
        check = _rmse_check(idx, targets, [per[i][2] for i in idx],
                            None if plain_rmse is None else [plain_rmse[i] for i in idx])
        check.update({"oracle": f"FP64 oracle from the same default initial factors and seeds, same plateau "
                                f"rule, {threads} threads, {ora_s:.1f} s"})
        log(f"oracle check on {len(idx)} problems: {check}")
    out = {
        "metric": "instances/s", "value": round(n / (admit_s + run_s), 3), "unit": "instances/s",
        "n_gpus": 1, "steps": sweeps, "warmup": 0, "ms_per_step": round(run_s * 1e3 / max(sweeps, 1), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-gather/f32" if args.bf16 else "f32", "data": "synthetic",
        "config": {"workload": f"{n} 3-way problems, dims log-U[50,2000], nnz log-U[10k,2M], R in {{8,16,32}}, "
                               "planted CPD + N(0,0.01), 5% test; c=0.1, lambda=1e-3, plateau stop (W=5, 1e-4, "
                               "cap 500)", "instances": n, "nnz_train": nnz, "seed": args.seed},
        "instances_per_s_solve_only": round(n / run_s, 3),
        "admit_s": round(admit_s, 3), "solve_s": round(run_s, 3), "generate_s": round(gen_s, 2),
        "autotune_s": round(tune_s, 2), "schedules": {str(k): v for k, v in sched.items()},
        "updates_per_s_solve": round(upd / run_s, 1),
        "sweeps_per_instance": {"min": int(min(q[1] for q in per)), "median": float(np.median([q[1] for q in per])),
                                "max": int(max(q[1] for q in per))},
        "plain": plain,
        "speedup_vs_plain": None if plain is None else round((n / (admit_s + run_s)) / plain["value"], 2),
        "oracle_check": check,
    }
    print(json.dumps(out), flush=True)


def _oracle_plateau(items, cpu_threads=0, W=5, tol=1e-4, cap=500):
    """Run the FP64 oracle on each (problem, R, seed) from the default initial
    factors to the held-out plateau (the pool's stop rule): returns the final
    held-out RMSE and stop sweep of each, and the threads used."""
    import oracle as O
    threads = O.set_threads(cpu_threads or len(os.sched_getaffinity(0)))
    out = []
    for p, R, sd in items:
        o = O.Oracle(p.dims, p.coords, p.values, R, c=0.1, lam=1e-3, seed=sd, test_coords=p.test_coords,
                     test_values=p.test_values)
        hist = [o.loss()[2]]
        t_log = time.time()
        while _stop_at(hist, W, tol, cap) is None:
            o.sweep(1)
            hist.append(o.loss()[2])
            if time.time() - t_log > 30.0:  # a long oracle run reports its progress
                t_log = time.time()
                log(f"oracle {len(out) + 1}/{len(items)}: {p.nnz} entries, sweep {len(hist) - 1}, "
                    f"test RMSE {hist[-1]:.6f}")
        o.close()
        out.append((float(hist[-1]), len(hist) - 1))
        log(f"oracle {len(out)}/{len(items)}: {p.nnz} entries, R={R}: plateau at sweep {len(hist) - 1}, "
            f"test RMSE {hist[-1]:.6f}")
    return out, threads


def _rmse_check(idx, targets, got, plain=None, tol=1e-3):
    """Final held-out RMSE of the sampled problems against the oracle's:
    within tol (|diff| <= tol) and at or below the target oracle + tol."""
    import numpy as np
    d = np.asarray(got) - np.asarray([t[0] for t in targets])
    out = {"instances": len(idx), "indices": idx, "tolerance": tol,
           "within_tol": int(np.sum(np.abs(d) <= tol)), "at_or_below_target": int(np.sum(d <= tol)),
           "max_abs_diff": float(f"{np.max(np.abs(d)):.3e}"),
           "oracle_stop_sweeps": {"min": int(min(t[1] for t in targets)), "max": int(max(t[1] for t in targets))}}
    out["outside_tol"] = [{"index": int(i), "rmse": round(float(g), 6), "oracle": round(float(t[0]), 6),
                           "oracle_stop_sweep": int(t[1])}
                          for i, g, t, x in zip(idx, got, targets, d) if abs(x) > tol]
    if plain is not None:
        dp = np.asarray(plain) - np.asarray([t[0] for t in targets])
        out["plain_within_tol"] = int(np.sum(np.abs(dp) <= tol))
        out["plain_max_abs_diff"] = float(f"{np.max(np.abs(dp)):.3e}")
    return out


def run_serve(args):
    """Poisson arrivals into a pool (95% batching mixture, 5% 200000x50000x500
    problems with 20M Zipf(1.1) entries, R = 16), BF16 gathers; latency is
    arrival -> plateau stop, admission (host CSR build) included.  Beside it:
    the plain method (FP32 gathers, one request at a time through
    ntc_create/ntc_sweep/ntc_loss) on the same arrival times, and for a sample
    of requests the FP64 oracle's final held-out RMSE as the target."""
    import collections

    import numpy as np

    import paper_2109_09534_amd as ntc
    import synth
    ntc.lib()
    rng = np.random.default_rng(args.seed)
    n = args.instances
    t0 = time.perf_counter()
    shapes, small = _batch_problems(n, args.seed)
    large = [synth.make_problem((200_000, 50_000, 500), 20_000_000, 16, zipf_s=1.1, noise_var=0.01,
                                value_model="exact", test_frac=0.05, seed=90_000 + i, name="large")
             for i in range(2)]
    log(f"generated {n} small and {len(large)} large problems in {time.perf_counter() - t0:.1f} s")
    reqs = []
    for i in range(n):
        if rng.random() < 0.05:
            reqs.append((large[i % len(large)], 16, 50_000 + i))
        else:
            dims, _, R, sd = shapes[i]
            reqs.append((small[i], R, sd))
    kw = dict(c=0.1, lam=1e-3, gather_bf16=True)
    dev_min = args.admit_device_csr
    rates = [float(x) for x in args.rates.split(",") if x]
    unit_gaps = rng.exponential(1.0, (len(rates), n))   # arrival gaps at rate 1, scaled per rate

    def serve(arrive):
        """Open loop with the given arrival times (all zero: everything at
        once).  A request's host work (CSR, schedule) starts on a worker thread
        when it arrives; the pool admits it once that is done, without
        waiting.  Returns the wall time, each request's latency and the
        held-out RMSE at which it stopped."""
        import concurrent.futures as cf
        pool = ntc.Pool(max_slots=min(n, 1024), window=5, tol=1e-4, max_sweeps=500)
        ex = cf.ThreadPoolExecutor(max_workers=args.prepare_threads)
        queue = collections.deque()
        slot_req = {}
        lat = np.zeros(n)
        rmse = np.zeros(n)
        nxt = done = 0
        start = time.perf_counter()
        while done < n:
            now = time.perf_counter() - start
            while nxt < n and arrive[nxt] <= now:
                p, R, sd = reqs[nxt]
                if dev_min and p.nnz >= dev_min:   # CSR built on the GPU at admission
                    queue.append((nxt, None))
                else:
                    queue.append((nxt, ex.submit(ntc.Prepared, p.dims, p.coords, p.values, R, seed=sd,
                                                 test_coords=p.test_coords, test_values=p.test_values, **kw)))
                nxt += 1
            while queue and (queue[0][1] is None or queue[0][1].done()):
                i, fut = queue[0]
                if fut is None:
                    p, R, sd = reqs[i]
                    s = pool.admit(p.dims, p.coords, p.values, R, seed=sd, test_coords=p.test_coords,
                                   test_values=p.test_values, device_csr=True, **kw)
                    if s is None:
                        break
                else:
                    q = fut.result()
                    s = pool.admit_prepared(q)
                    if s is None:
                        break
                    q.close()
                queue.popleft()
                slot_req[s] = i
            if pool.info()["running"] > 0:
                pool.step(args.sweeps_per_step)
            else:
                # nothing to sweep: wait for the next arrival or the head of the queue
                if queue and queue[0][1] is not None:
                    cf.wait([queue[0][1]], timeout=0.05)
                elif nxt < n:
                    time.sleep(max(0.0, min(arrive[nxt] - (time.perf_counter() - start), 0.05)))
            for s in pool.stopped():
                i = slot_req.pop(s)
                lat[i] = time.perf_counter() - start - arrive[i]
                rmse[i] = pool.query(s)[2]
                pool.evict(s)
                done += 1
        wall = time.perf_counter() - start
        ex.shutdown()
        pool.close()
        return wall, lat, rmse

    def fifo(arrive, service):
        """Latencies of one server taking requests one at a time in arrival order."""
        fin = np.zeros(n)
        t = 0.0
        for i in range(n):
            t = max(t, arrive[i]) + service[i]
            fin[i] = t
        return fin[-1] - arrive[0], fin - arrive

    def pct(x, q):
        return round(float(np.percentile(x, q)), 4)

    wall, lat, rm = serve(np.zeros(n))
    sat = n / wall
    log(f"saturation (all {n} at once): {wall:.2f} s -> {sat:.2f} requests/s")
    runs = [(0.0, np.zeros(n), wall, lat, rm)]
    for j, f in enumerate(rates):
        arrive = np.cumsum(unit_gaps[j] / (f * sat))
        arrive -= arrive[0]
        w, l, r = serve(arrive)
        runs.append((f, arrive, w, l, r))
        log(f"rate {f} x saturation: p50 {pct(l, 50)} s, p99 {pct(l, 99)} s")

    service = plain_rmse = None
    if not args.no_plain:
        service = np.zeros(n)
        plain_rmse = np.zeros(n)
        for i, (p, R, sd) in enumerate(reqs):
            t0 = time.perf_counter()
            g = ntc.Problem(p.dims, p.coords, p.values, R, seed=sd, test_coords=p.test_coords,
                            test_values=p.test_values, stream=0, c=0.1, lam=1e-3, gather_bf16=False)
            hist = [g.loss()[2]]
            while _stop_at(hist) is None:
                g.sweep(1)
                hist.append(g.loss()[2])
            g.close()
            service[i] = time.perf_counter() - t0
            plain_rmse[i] = hist[-1]
        log(f"plain one-at-a-time (FP32): {service.sum():.2f} s of service for {n} requests")

    idx = []
    targets = []
    ora_note = None
    if args.oracle_instances > 0:
        # evenly spread requests plus the first request on each large tensor
        idx = set(np.linspace(0, n - 1, min(n, args.oracle_instances)).astype(int).tolist())
        for big in large:
            first = [i for i, r in enumerate(reqs) if r[0] is big]
            idx |= set(first[:1])
        idx = sorted(idx)
        t0 = time.perf_counter()
        targets, threads = _oracle_plateau([reqs[i] for i in idx], args.cpu_threads)
        ora_note = (f"FP64 oracle from the same default initial factors and seeds, same plateau rule, "
                    f"{threads} threads, {time.perf_counter() - t0:.1f} s, on requests {idx} "
                    f"({sum(reqs[i][0].nnz > 10_000_000 for i in idx)} of them large)")
        log(ora_note)

    rows = []
    for f, arrive, w, l, r in runs:
        row = {"rate_fraction": f, "rate": None if f == 0 else round(f * sat, 3),
               "completions_per_s": round(n / w, 3), "p50_s": pct(l, 50), "p99_s": pct(l, 99)}
        if idx:
            row["oracle_check"] = _rmse_check(idx, targets, [r[i] for i in idx],
                                              None if plain_rmse is None else [plain_rmse[i] for i in idx])
        if service is not None:
            pw, pl = fifo(arrive, service)
            row["plain"] = {"completions_per_s": round(n / pw, 3), "p50_s": pct(pl, 50), "p99_s": pct(pl, 99)}
        rows.append(row)
    out = {"metric": "completions/s at saturation", "value": round(sat, 3), "unit": "requests/s", "n_gpus": 1,
           "steps": n, "warmup": 0, "ms_per_step": round(1e3 / sat, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16-gather/f32", "data": "synthetic",
           "config": {"workload": f"{n} requests: 95% batching mixture, 5% 200000x50000x500 20M Zipf(1.1) R=16; "
                                  "BF16 gathers, plateau stop; Poisson arrivals; host CSR on "
                                  f"{args.prepare_threads} worker threads"
                                  + (f", CSR on the GPU for requests of >= {dev_min} entries" if dev_min else ""),
                       "requests": n, "seed": args.seed, "admit_device_csr_min_nnz": dev_min},
           "latency": rows,
           "plain": None if service is None else {
               "kind": "FP32 gathers, one request at a time through ntc_create/ntc_sweep/ntc_loss (create "
                       "included); latencies are those of one server taking the requests in arrival order at "
                       "the same arrival times, from each request's measured service time",
               "saturation_per_s": round(n / float(service.sum()), 3),
               "max_final_rmse_diff_vs_pool": float(f"{np.max(np.abs(plain_rmse - runs[0][4])):.3e}")},
           "oracle": ora_note}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
