"""The rocprofv3 summaries of profiling.py on a small database of the same
shape (the views ``regions`` and ``kernels`` that rocprofv3 writes)."""
import json
import os
import sqlite3

from paper_2109_09534_amd import profiling


def _db(tmp_path):
    d = tmp_path / "run"
    os.makedirs(d)
    con = sqlite3.connect(str(d / "x_results.db"))
    con.execute("create table regions (category text, name text, extdata text, tid int, start int, end int)")
    con.execute("create table kernels (region text, name text, start int, end int, duration int)")
    marks = [("ntc_sweep", 0, 100_000), ("ntc mode 0", 1_000, 40_000), ("ntc mode 1", 41_000, 90_000),
             ("ntc_sweep", 200_000, 300_000), ("ntc mode 0", 201_000, 240_000), ("ntc mode 1", 241_000, 290_000)]
    for msg, s, e in marks:
        con.execute("insert into regions values ('MARKER_CORE_RANGE_API', 'roctxThreadRangeA', ?, 1, ?, ?)",
                    (json.dumps({"message": msg}), s, e))
    con.execute("insert into regions values ('HIP_RUNTIME_API_EXT', 'hipLaunchKernel', '{}', 1, 5, 6)")
    t = 1_000_000
    for sweep in range(2):
        for region, name, dur in [("ntc mode 0", "void ntc::(anonymous namespace)::k_chunk16<3, 4, false, true>(a)",
                                   30_000),
                                  ("ntc mode 0", "void ntc::(anonymous namespace)::k_quad16<3, false, true, true>(a)",
                                   10_000),
                                  ("ntc mode 1", "void ntc::(anonymous namespace)::k_chunk16<3, 4, false, true>(a)",
                                   50_000),
                                  ("ntc_sweep", "void ntc::(anonymous namespace)::k_advance(long*, int)", 4_000),
                                  ("", "void ntc::(anonymous namespace)::k_advance(long*, int)", 4_000)]:
            con.execute("insert into kernels values (?, ?, ?, ?, ?)", (region, name, t, t + dur, dur))
            t += dur
    con.commit()
    con.close()
    return str(d)


def test_ranges_summary_attributes_kernels_to_the_innermost_range(tmp_path):
    text = profiling.ranges(_db(tmp_path), "title", "cmd")
    rows = {line.split("|")[1].strip(): [c.strip() for c in line.split("|")[2:-1]]
            for line in text.splitlines() if line.startswith("| `")}
    assert list(rows) == ["`ntc_sweep`", "`ntc mode 0`", "`ntc mode 1`"]
    # calls, host us per call, kernels per call, kernel us per call, names
    assert rows["`ntc_sweep`"][:4] == ["2", "100.0", "1", "4.0"]
    assert rows["`ntc mode 0`"][:4] == ["2", "39.0", "2", "40.0"]
    assert "`k_chunk16<3, 4, false, true>` x1" in rows["`ntc mode 0`"][4]
    assert "`k_quad16<3, false, true, true>` x1" in rows["`ntc mode 0`"][4]
    assert rows["`ntc mode 1`"][:4] == ["2", "49.0", "1", "50.0"]
    assert "2 kernels ran outside every range." in text
