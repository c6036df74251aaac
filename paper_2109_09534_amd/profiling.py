"""Summaries of rocprofv3 output for the row kernels.

rocprofv3 writes a SQLite database per run.  This module turns one into
the short text summaries kept beside the code:

* ``trace``   -- per-kernel statistics (``--kernel-trace --stats``) and the
  dispatch table of the last sweep's row kernels, as Markdown;
* ``ranges``  -- the library's ROCTX ranges (``--marker-trace``) with the
  kernels each one launched (``--kernel-trace --hip-runtime-trace``);
* ``traffic`` -- HBM bytes per launch of one kernel from two ``--pmc`` runs
  (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
  same counter reads for a plain device copy of known size, as JSON tagged
  with a hash of the row-kernel sources it was taken on.

Usage:
  python -m paper_2109_09534_amd.profiling trace DIR --title T --command C [--last 9] [--before NAME]
  python -m paper_2109_09534_amd.profiling ranges DIR --title T --command C
  python -m paper_2109_09534_amd.profiling counters DIR [DIR ...] --title T --command C
  python -m paper_2109_09534_amd.profiling traffic --kernel K --fetch DIR --write DIR
         --copy-fetch DIR --copy-write DIR --copy-bytes B --command C [--out FILE]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_HEADERS = ["ntc_dev.h", "ntc_few.h", "ntc_rng.h", "ntc_bf16.h", "ntc_internal.h"]
ROW_KERNELS = ("k_rows16", "k_chunk16", "k_tiny16", "k_finalize16", "k_row_items", "k_row_finalize",
               "k_rows16_nm", "k_rows32", "k_finalize32", "k_reduce_slots", "k_few16", "k_few32", "k_quad16")


def source_hash(wide: bool = False) -> str:
    """Hash of the sources a row kernel is compiled from: its translation
    unit (ntc_kernels.hip for R <= 16; wide: ntc_kernels_wide.hip for
    R > 16) and the headers both include."""
    h = hashlib.sha256()
    for fn in ["ntc_kernels_wide.hip" if wide else "ntc_kernels.hip"] + KERNEL_HEADERS:
        with open(os.path.join(PKG, "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _db(path: str) -> sqlite3.Connection:
    dbs = glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
    if not dbs:
        raise FileNotFoundError(f"no rocprofv3 database under {path}")
    return sqlite3.connect(dbs[0])


def short_name(name: str) -> str:
    name = name.replace("ntc::(anonymous namespace)::", "").replace("ntc::", "")
    return re.sub(r"^void ", "", name).split("(")[0]


def trace(path: str, title: str, command: str, last: int = 9, before: str = "") -> str:
    """``before``: take the sweep that ends where the first dispatch whose
    name contains it starts (a run that times two precisions in turn)."""
    con = _db(path)
    out = [f"# {title}", "", "Command (from the repository root; REPO is its absolute path):", "",
           "```", command, "```", "",
           "## Kernel statistics (rocprofv3 --stats; durations in microseconds)", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, calls, total, avg, pct in con.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        out.append(f"| `{short_name(name)}` | {calls} | {total:.1f} | {avg:.1f} | {pct:.2f} |")
    like = " or ".join(f"name like '%{k}%'" for k in ROW_KERNELS)
    rows = list(con.execute(f"select name, grid_x, workgroup_x, duration, vgpr_count, accum_vgpr_count, "
                            f"lds_size, scratch_size from kernels where {like} order by start"))
    if before:
        cut = next((i for i, r in enumerate(rows) if before in short_name(r[0])), len(rows))
        rows = rows[:cut]
    out += ["", f"## Row-kernel dispatches of the last sweep ({min(last, len(rows))} launches, in order)", "",
            "| kernel | grid (threads) | block | duration us | VGPR | AGPR | LDS B | scratch B |",
            "|---|---|---|---|---|---|---|---|"]
    for name, grid, wg, dur, vgpr, agpr, lds, scratch in rows[-last:]:
        out.append(f"| `{short_name(name)}` | {grid} | {wg} | {dur / 1e3:.1f} | {vgpr} | {agpr} | {lds} | {scratch} |")
    return "\n".join(out) + "\n"


def ranges(path: str, title: str, command: str) -> str:
    """The library's ROCTX ranges (``--marker-trace``) with the kernels
    rocprofv3 attributes to each (``--kernel-trace``: the innermost range
    open on the launching thread when the kernel was enqueued)."""
    con = _db(path)
    marks = []
    for name, extdata, start, end in con.execute("select name, extdata, start, end from regions where "
                                                 "category like '%MARKER%' and end > start order by start"):
        try:  # the range's message; the region's own name is the ROCTX call
            name = json.loads(extdata).get("message", name)
        except (TypeError, ValueError):
            pass
        marks.append((name, start, end))
    kern = {}
    for region, name, dur in con.execute("select region, name, duration from kernels order by start"):
        kern.setdefault(region or "", []).append((short_name(name), dur))
    out = [f"# {title}", "", "Command (from the repository root; REPO is its absolute path):", "",
           "```", command, "```", "",
           "Host time is the range's own interval on the calling thread (enqueue, not execution). Kernels are "
           "those rocprofv3 attributes to the range: the innermost range open when each was enqueued. Kernel us is "
           "the sum of their GPU durations; launches on the two streams of a mode overlap, so it can exceed the "
           "mode's span.", "",
           "| range | calls | host us per call | kernels per call | kernel us per call | kernels |",
           "|---|---|---|---|---|---|"]
    names = []
    for m in marks:
        if m[0] not in names:
            names.append(m[0])
    for n in names:
        calls = [m for m in marks if m[0] == n]
        host = sum(m[2] - m[1] for m in calls) / 1e3 / len(calls)
        ks = kern.get(n, [])
        gpu = sum(d for _, d in ks) / 1e3 / len(calls)
        counts = {}
        for k, _ in ks:
            counts[k] = counts.get(k, 0) + 1
        which = ", ".join(f"`{k}` x{v // len(calls) if v % len(calls) == 0 else v / len(calls):g}"
                          for k, v in counts.items()) or "-"
        out.append(f"| `{n}` | {len(calls)} | {host:.1f} | {len(ks) / len(calls):g} | {gpu:.1f} | {which} |")
    if kern.get(""):
        out += ["", f"{len(kern[''])} kernels ran outside every range."]
    return "\n".join(out) + "\n"


def counters(paths, title: str, command: str, kernels=ROW_KERNELS, clock_ghz: float = 2.4) -> str:
    """Per-dispatch counter values of the row kernels from one or more
    rocprofv3 --pmc runs of the same program (dispatch ids line up), with
    the derived memory figures: L2-to-memory read requests per microsecond
    and their mean number in flight (TCC_EA0_RDREQ_LEVEL over the cycles of
    the dispatch), whose ratio is the mean request latency (Little's law)."""
    per = {}
    dur = {}
    for path in paths:
        con = _db(path)
        for did, name, cn, v in con.execute(
                "select dispatch_id, kernel_name, counter_name, sum(value) from counters_collection "
                "group by dispatch_id, counter_name order by dispatch_id"):
            per.setdefault((did, short_name(name)), {})[cn] = v
        try:
            for did, start, end in con.execute("select dispatch_id, start, end from kernels"):
                dur.setdefault(did, (end - start) / 1e3)
        except sqlite3.Error:
            pass
    names = sorted({c for v in per.values() for c in v})
    derived = "TCC_EA0_RDREQ_sum" in names and "TCC_EA0_RDREQ_LEVEL_sum" in names
    head = ["dispatch", "kernel", "us"] + (["G req/s", "in flight", "latency ns"] if derived else []) + names
    out = [f"# {title}", "", "Command (from the repository root; REPO is its absolute path):", "", "```", command,
           "```", ""]
    if derived:
        out += ["Derived: G req/s = TCC_EA0_RDREQ_sum / duration; in flight = TCC_EA0_RDREQ_LEVEL_sum / "
                f"(duration x {clock_ghz} GHz); latency = in flight / rate.", ""]
    out += ["| " + " | ".join(head) + " |", "|" + "---|" * len(head)]
    for (did, name), c in sorted(per.items()):
        if not any(k in name for k in kernels):
            continue
        us = dur.get(did, 0.0)
        row = [str(did), f"`{name}`", f"{us:.1f}"]
        if derived:
            rate = c.get("TCC_EA0_RDREQ_sum", 0.0) / us / 1e3 if us > 0 else 0.0
            inflight = c.get("TCC_EA0_RDREQ_LEVEL_sum", 0.0) / (us * 1e3 * clock_ghz) if us > 0 else 0.0
            row += [f"{rate:.1f}", f"{inflight:.0f}", f"{inflight / rate:.0f}" if rate > 0 else ""]
        row += [f"{c[n]:.4g}" if n in c else "" for n in names]
        out.append("| " + " | ".join(row) + " |")
    return "\n".join(out) + "\n"


def _per_dispatch(path: str, counter: str):
    con = _db(path)
    q = ("select dispatch_id, kernel_name, sum(value) from counters_collection where counter_name = ? "
         "group by dispatch_id order by dispatch_id")
    return [(d, short_name(n), v) for d, n, v in con.execute(q, (counter,))]


def traffic(kernel: str, fetch: str, write: str, copy_fetch: str, copy_write: str, copy_bytes: int,
            command: str, wide: bool = False) -> dict:
    """HBM bytes per launch of `kernel` (name prefix, e.g. 'k_chunk16<3, 4, false, true>')."""
    kib = 1024.0
    scale = {}
    for counter, path, expect in (("FETCH_SIZE", copy_fetch, copy_bytes), ("WRITE_SIZE", copy_write, copy_bytes)):
        copies = [v for _, n, v in _per_dispatch(path, counter) if "copyBuffer" in n]
        if not copies:
            raise RuntimeError(f"no copy dispatch in {path}")
        counted = sum(copies) / len(copies) * kib
        scale[counter] = expect / counted
    per = {}
    for counter, path in (("FETCH_SIZE", fetch), ("WRITE_SIZE", write)):
        vals = [v for _, n, v in _per_dispatch(path, counter) if n.startswith(kernel)]
        if not vals:
            raise RuntimeError(f"no dispatch of {kernel} in {path}")
        per[counter] = vals
    n = min(len(per["FETCH_SIZE"]), len(per["WRITE_SIZE"]))
    fetch_b = sum(per["FETCH_SIZE"][:n]) / n * kib * scale["FETCH_SIZE"]
    write_b = sum(per["WRITE_SIZE"][:n]) / n * kib * scale["WRITE_SIZE"]
    return {"kernel": kernel, "launches": n, "hbm_bytes_per_launch": round(fetch_b + write_b),
            "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
            "fetch_kib_per_dispatch": per["FETCH_SIZE"][:n], "write_kib_per_dispatch": per["WRITE_SIZE"][:n],
            "copy_bytes": copy_bytes, "scale": {k: round(v, 4) for k, v in scale.items()},
            "kernel_source_hash": source_hash(wide), "wide": wide, "command": command}


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2109_09534_amd.profiling")
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--last", type=int, default=9)
    t.add_argument("--before", default="", help="end the dispatch table before the first kernel of this name")
    t.add_argument("--out")
    g = sub.add_parser("ranges")
    g.add_argument("dir")
    g.add_argument("--title", required=True)
    g.add_argument("--command", required=True)
    g.add_argument("--out")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--out")
    f = sub.add_parser("traffic")
    for k in ("kernel", "fetch", "write", "copy-fetch", "copy-write", "command"):
        f.add_argument("--" + k, required=True)
    f.add_argument("--copy-bytes", type=int, required=True)
    f.add_argument("--wide", action="store_true", help="the kernel is one of the R > 16 kernels")
    f.add_argument("--out")
    a = ap.parse_args(argv)
    if a.what == "trace":
        text = trace(a.dir, a.title, a.command, a.last, a.before)
    elif a.what == "ranges":
        text = ranges(a.dir, a.title, a.command)
    elif a.what == "counters":
        text = counters(a.dirs, a.title, a.command)
    else:
        text = json.dumps(traffic(a.kernel, a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.command,
                                  a.wide), indent=1) + "\n"
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    else:
        sys.stdout.write(text)


if __name__ == "__main__":
    main()
