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
# profile_sweep's launch kinds -> the kernels rocprofv3 reports for them (R = 16, N = 3)
KERNEL_NAMES = {"row_items": "k_rows16<3, 4, false, 1>", "row_chunks": "k_chunk16<3, 4, false>",
                "row_tiny": "k_tiny16<3, 4, false>", "row_finalize": "k_finalize16<false>"}


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
    if d.get("kernel_source_hash") != source_hash():
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
    ap.add_argument("--cpu-threads", type=int, default=0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} (WORLD_SIZE={world}) is not supported; "
              "the multi-GPU row sharding is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import paper_2109_09534_amd as ntc
    import synth

    ntc.lib()       # fails loudly without the HIP library
    R, c, lam, max_inner = 16, 0.1, 1e-3, 1
    t0 = time.perf_counter()
    log(f"generating the 480000x18000x2000 Zipf(1.1) workload, scale {args.scale} ...")
    p = synth.c1(seed=args.seed, scale=args.scale)
    gen_s = time.perf_counter() - t0
    log(f"generated {p.nnz} train / {p.test_values.shape[0]} test entries in {gen_s:.1f} s (SNR {p.snr:.2f})")

    t0 = time.perf_counter()
    prob = ntc.Problem(p.dims, p.coords, p.values, R, c=c, lam=lam, max_inner=max_inner, seed=args.seed,
                       gather_bf16=args.bf16, test_coords=p.test_coords, test_values=p.test_values, stream=0)
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

    # per-launch event timing of one more sweep (all launches on one stream):
    # roofline of the dominant kernel, the one with the largest share of the sweep
    launches = prob.profile_sweep()
    per_kernel = {}
    sweep_bytes = 0
    per_mode = []
    for rec in launches:
        _, b_upd, b_rows = algorithmic_bytes(p.nmodes, R, rec["samples"], rec["rows"], max_inner, args.bf16)
        k = per_kernel.setdefault(rec["kernel"], {"bytes": 0, "ms": 0.0, "launches": 0})
        k["bytes"] += b_upd + b_rows
        k["ms"] += rec["ms"]
        k["launches"] += 1
        sweep_bytes += b_upd + b_rows
        per_mode.append({kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in rec.items()})
    dom = max(per_kernel, key=lambda n: per_kernel[n]["ms"])
    kd = per_kernel[dom]
    avg_ms = kd["ms"] / kd["launches"]
    bytes_per_launch = kd["bytes"] / kd["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kfile = KERNEL_NAMES[dom].split("<")[0]
    traffic_rec = load_traffic(f"{kfile}_c1{'_bf16' if args.bf16 else ''}_traffic.json")
    traffic = traffic_rec["hbm_bytes_per_launch"] if traffic_rec else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES[dom], "avg_launch_ms": round(avg_ms, 4),
                "launches_per_sweep": kd["launches"],
                "algorithmic_bytes_per_launch": round(bytes_per_launch),
                "sweep_share": round(kd["ms"] / sum(v["ms"] for v in per_kernel.values()), 3)}
    hbm_frac = sweep_bytes * args.steps / wall / (HBM_PEAK_GBS * 1e9)

    t0 = time.perf_counter()
    loss = prob.loss()
    loss_ms = (time.perf_counter() - t0) * 1e3
    log(f"loss before {loss0}, after {loss} ({loss_ms:.1f} ms)")

    cpu = None
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
        "config": {"workload": "3-way 480000x18000x2000, 100M Zipf(1.1) entries, rank-16 ratings 1..5, "
                               "5% test; R=16, c=0.1, lambda=1e-3, MAX_INNER=1" +
                               (" (BF16 gathers)" if args.bf16 else ""),
                   "nnz_train": p.nnz, "scale": args.scale, "seed": args.seed,
                   "updates_per_sweep": upd_sweep, "row_steps_per_sweep": rows_sweep},
        "pct_hbm_peak": round(100 * hbm_frac, 2),
        "algorithmic_bytes_per_sweep": sweep_bytes,
        "device_ms_per_step": round(dev_ms / args.steps, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "create_s": round(create_s, 2),
        "generate_s": round(gen_s, 2),
        "loss_ms": round(loss_ms, 2),
        "test_rmse": round(float(loss[2]), 6),
        "train_rmse": round(float(loss[1]), 6),
        "launches": per_mode,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
