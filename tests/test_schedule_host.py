"""Host-side bounds checks of the row schedule (no device).

ntc_prepare turns each mode's CSR into work for the row kernels: rows of at
most tiny_max samples (one per lane for R <= 16, four per wave for
17 <= R <= 32 with N <= 4), whole rows, chunks of long rows that
write partial slots, split rows combined from those slots, and (R > 16)
groups of slots summed first.  The kernels index rows, records and slots
from these tables without checks of their own, so the checker below states
what must hold, from the sampling rule (B_p = floor(c n_p), Section II-B)
and the CSR: every row with B_p > 0 is scheduled exactly once, its samples
[0, B_p) covered exactly once in order, every span and slot in range.  It
is run on schedules of several shapes, and shown to catch planted errors.
"""
import copy

import numpy as np
import pytest

import paper_2109_09534_amd as ntc
import synth


def _base(w2, w3):
    return (int(w2) & 0xFFFFFFFF) | (int(w3) << 32)


def check_schedule(s, *, c, R, N, nnz, tiny_max=4, group_max=512):
    rp = s["rowptr"]
    I = rp.shape[0] - 1
    assert rp[0] == 0 and rp[-1] == nnz and np.all(np.diff(rp) >= 0), "row pointers"
    n = np.diff(rp)
    b = np.floor(c * n.astype(np.float64)).astype(np.int64)
    covered = np.zeros(I, dtype=np.int64)
    seen = np.zeros(I, dtype=bool)

    def claim(row, cnt):
        assert 0 <= row < I, f"row {row} out of range"
        assert not seen[row], f"row {row} scheduled twice"
        seen[row] = True
        covered[row] = cnt

    for row, nn, lo, hi in s["tiny"]:
        assert 0 <= row < I and nn == n[row] and _base(lo, hi) == rp[row], f"tiny row {row} span"
        assert 1 <= b[row] <= tiny_max, f"tiny row {row} has {b[row]} samples"
        claim(row, b[row])
    row_items = R <= 16 and N <= 4
    n_slots = s["n_slots"]
    slot_item = {}
    for i, (w0, w1, w2, w3) in enumerate(s["items"]):
        if row_items and i < s["n_group"]:
            row = w0
            assert 0 <= row < I and w1 == n[row] and _base(w2, w3) == rp[row], f"group row {row} span"
            assert tiny_max < b[row] <= group_max, f"group row {row} has {b[row]} samples"
            claim(row, b[row])
            continue
        row, j0, j1, slot = int(w0), int(w1), int(w2), int(w3)
        assert 0 <= row < I, f"item row {row} out of range"
        assert 0 <= j0 < j1 <= b[row], f"item [{j0}, {j1}) of row {row} with {b[row]} samples"
        if slot < 0:
            assert j0 == 0 and j1 == b[row], f"whole item of row {row} covers [{j0}, {j1})"
            claim(row, b[row])
        else:
            assert slot < n_slots and slot not in slot_item, f"slot {slot} out of range or reused"
            slot_item[slot] = (row, j0, j1)
    group_of = {}
    for src, cnt, dst, _ in s["groups"]:
        assert cnt >= 1 and all(q in slot_item for q in range(src, src + cnt)), f"group sources {src}+{cnt}"
        assert len({slot_item[q][0] for q in range(src, src + cnt)}) == 1, "group spans two rows"
        assert dst not in slot_item and 0 <= dst < n_slots and dst not in group_of, f"group destination {dst}"
        group_of[dst] = list(range(src, src + cnt))
    used = set()
    for row, slot0, ns, _ in s["split"]:
        slots = list(range(slot0, slot0 + ns))
        if slots and slots[0] in group_of:
            slots = [q for d in slots for q in group_of[d]]
        assert slots and all(q in slot_item and slot_item[q][0] == row for q in slots), f"split row {row} slots"
        j = 0
        for q in slots:
            assert slot_item[q][1] == j, f"split row {row}: gap or overlap at sample {j}"
            j = slot_item[q][2]
            assert q not in used, f"slot {q} in two split rows"
            used.add(q)
        assert j == b[row], f"split row {row} covers {j} of {b[row]} samples"
        claim(row, b[row])
    assert used == set(slot_item), "partial slots that no split row reads"
    assert np.array_equal(covered, np.where(b > 0, b, 0)), "rows with samples left out"
    assert s["samples"] == int(b.sum()), "sample count"


CASES = {
    "zipf_r16_tiny_groups_chunks": lambda: (synth.c1_small(seed=0), 16, dict(c=0.1)),
    "zipf_r16_small_chunks": lambda: (synth.c1_small(seed=1), 16,
                                      dict(c=0.3, schedule={"item_samples": 64, "group_max": 32, "tiny_max": 2})),
    "r8_no_tiny": lambda: (synth.c0(seed=0), 8, dict(c=0.2, schedule={"tiny_max": 0})),
    "r32_slot_groups": lambda: (synth.make_problem((60, 50, 40), 70_000, 8, seed=14, zipf_s=1.1), 24,
                                dict(c=0.8, schedule={"item_samples": 16})),
    "r50_4way": lambda: (synth.make_problem((183, 24, 114, 171), 150_000, 10, seed=5), 50, dict(c=0.5)),
    "r16_5way": lambda: (synth.make_problem((20, 15, 12, 10, 8), 60_000, 5, seed=6), 16, dict(c=0.3)),
    "matrix_r64": lambda: (synth.make_problem((400, 300), 60_000, 8, seed=17), 64, dict(c=1.0)),
    # 17 <= R <= 32, N <= 4: rows of at most 16 samples four to a wave, the rest whole or split
    "zipf_r32_4way_few_rows": lambda: (synth.make_problem((3000, 2000, 60, 20), 300_000, 12, zipf_s=1.05,
                                                          seed=40), 32, dict(c=0.1, schedule={"item_samples": 128})),
    "zipf_r27_few_max_5": lambda: (synth.c1_small(seed=3), 27, dict(c=0.1, schedule={"tiny_max": 5})),
    "r24_5way_no_few_rows": lambda: (synth.make_problem((20, 15, 12, 10, 8), 60_000, 5, seed=6), 24, dict(c=0.05)),
}


def _tiny_max(R, N, sch):
    if R <= 16:
        return sch.get("tiny_max", 4)
    if R <= 32 and N <= 4:
        return sch.get("tiny_max", 16)
    return 0


@pytest.mark.parametrize("case", list(CASES))
def test_row_schedule_invariants(case):
    p, R, kw = CASES[case]()
    q = ntc.Prepared(p.dims, p.coords, p.values, R, **kw)
    sch = kw.get("schedule", {})
    for m in range(len(p.dims)):
        s = q.row_schedule(m)
        check_schedule(s, c=kw["c"], R=R, N=len(p.dims), nnz=p.nnz, tiny_max=_tiny_max(R, len(p.dims), sch),
                       group_max=sch.get("group_max", 512))
    q.close()


def test_few_sample_rows_of_the_r32_kernels_are_scheduled_apart():
    """17 <= R <= 32 with N <= 4: every row with 1 <= B_p <= 16 is in the few-row list, none with more."""
    p = synth.make_problem((3000, 2000, 60, 20), 300_000, 12, zipf_s=1.05, seed=40)
    q = ntc.Prepared(p.dims, p.coords, p.values, 32, c=0.1)
    s = q.row_schedule(0)
    q.close()
    b = np.floor(0.1 * np.diff(s["rowptr"]).astype(np.float64)).astype(np.int64)
    few = set(int(r) for r in s["tiny"][:, 0])
    assert few == set(int(r) for r in np.nonzero((b >= 1) & (b <= 16))[0])
    assert len(few) > 1000


def test_the_checker_catches_planted_schedule_errors():
    p = synth.c1_small(seed=2)
    q = ntc.Prepared(p.dims, p.coords, p.values, 16, c=0.1, schedule={"item_samples": 256})
    s0 = q.row_schedule(0)
    q.close()
    assert s0["tiny"].shape[0] > 1 and s0["n_group"] > 1 and s0["split"].shape[0] > 0
    kw = dict(c=0.1, R=16, N=3, nnz=p.nnz)
    check_schedule(s0, **kw)
    ng = s0["n_group"]
    chunk = next(i for i in range(ng, s0["items"].shape[0]) if s0["items"][i, 3] >= 0)
    mutations = {
        "tiny base off by one": lambda s: s["tiny"].__setitem__((0, 2), s["tiny"][0, 2] + 1),
        "tiny row dropped": lambda s: s.__setitem__("tiny", s["tiny"][1:]),
        "group row twice": lambda s: s["items"].__setitem__(1, s["items"][0]),
        "chunk end past the minibatch": lambda s: s["items"].__setitem__((chunk, 2), s["items"][chunk, 2] + 1),
        "slot out of range": lambda s: s["items"].__setitem__((chunk, 3), s["n_slots"]),
        "split row slot count": lambda s: s["split"].__setitem__((0, 2), s["split"][0, 2] - 1),
        "row pointer decreases": lambda s: s["rowptr"].__setitem__(5, s["rowptr"][6] + 1),
        "sample count": lambda s: s.__setitem__("samples", s["samples"] + 1),
    }
    for name, mutate in mutations.items():
        s = copy.deepcopy(s0)
        mutate(s)
        with pytest.raises(AssertionError):
            check_schedule(s, **kw)
