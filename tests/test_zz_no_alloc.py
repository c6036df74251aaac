"""The allocation-free entry point (ntc_loss_coo_noalloc) against ntc_loss.

Both evaluate the FP64 loss of eq. (Problem_TC) on the same factors; the
allocation-free form reads caller-held device COO arrays and keeps its
partial sums in a fixed device array.  Two calls in a row (the second on a
smaller problem, so it uses fewer partial blocks than the first left in the
array) must each agree with ntc_loss on their own problem.  The body runs in
a fresh process that imports torch first (device arrays come from torch).
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

_BODY = """
import torch                       # first: libntc then binds to torch's HIP runtime
import numpy as np
import paper_2109_09534_amd as ntc
import synth
assert torch.cuda.is_available()
ntc.lib()
cases = [(synth.c1_small(seed=13), 16, dict(c=0.1)), (synth.c0(seed=2), 8, dict(c=0.1)),
         (synth.make_problem((20, 15, 12, 10, 8), 6000, 5, seed=6, test_frac=0.1), 12, dict(c=0.3))]
stream = torch.cuda.current_stream()
for p, R, kw in cases:
    g = ntc.Problem(p.dims, p.coords, p.values, R, test_coords=p.test_coords, test_values=p.test_values,
                    stream=stream, torch_allocator=True, **kw)
    g.sweep(2)
    ref = g.loss()
    facs = [torch.empty(d * R, dtype=torch.float32, device="cuda") for d in p.dims]
    for m, t in enumerate(facs):
        g.factors_into(m, t)
    tc = torch.from_numpy(np.ascontiguousarray(p.coords, dtype=np.int32)).cuda()
    tv = torch.from_numpy(np.ascontiguousarray(p.values, dtype=np.float32)).cuda()
    ec = torch.from_numpy(np.ascontiguousarray(p.test_coords, dtype=np.int32)).cuda()
    ev = torch.from_numpy(np.ascontiguousarray(p.test_values, dtype=np.float32)).cuda()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    ntc.loss_coo_noalloc(p.dims, R, p.nnz, tc.data_ptr(), tv.data_ptr(), ev.shape[0], ec.data_ptr(), ev.data_ptr(),
                         [t.data_ptr() for t in facs], 1e-3, out.data_ptr(), stream.cuda_stream)
    got = out.cpu().numpy()
    print(f"dims {p.dims} nnz {p.nnz} R {R}: ntc_loss {ref.tolist()} allocation-free {got.tolist()}", flush=True)
    # the same FP64 sums in another order: agreement to a few ulps of the totals
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=0)
    g.close()
# argument checks
try:
    ntc.loss_coo_noalloc([5, 4], 65, 0, 0, 0, 0, 0, 0, [1, 1], 1e-3, 1, 0)
    raise SystemExit("rank 65 accepted")
except ntc.NtcError as e:
    assert e.status == ntc.NTC_EINVAL, e
try:
    ntc.loss_coo_noalloc([1 << 30, 4], 8, 0, 0, 0, 0, 0, 0, [1, 1], 1e-3, 1, 0)
    raise SystemExit("dims * rank >= 2^32 accepted")
except ntc.NtcError as e:
    assert e.status == ntc.NTC_EUNSUPPORTED, e
print("no-alloc ok", flush=True)
"""


@pytest.mark.timeout(400)
def test_allocation_free_loss_matches_ntc_loss_on_two_calls():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _BODY], cwd=root, capture_output=True, text=True, timeout=380,
                       env=dict(os.environ, PYTHONPATH=root))
    print(r.stdout[-3000:], r.stderr[-3000:], flush=True)
    assert r.returncode == 0 and "no-alloc ok" in r.stdout
