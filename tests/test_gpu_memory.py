"""Device memory one sort call holds, measured (the analogue of the paper's
memory table, section 3.2, Table 2).

A sort call allocates nothing itself: the caller gives the input, the output
and a workspace of intsort_workspace_size bytes.  Through the Python binding
the output and the workspace come from torch's allocator, so the device bytes
a call adds are what torch's allocator counts, and the driver's free memory
drops by what torch reserves.  The measured peak (input + what the call
allocated) must equal the figure every bench.py line reports
(workspace + input + output), up to torch's rounding: a block is 512-byte
aligned, and a large one keeps the rest of its 2 MiB-rounded segment when
that rest is under 1 MiB (so up to 1 MiB more per allocation)."""
import pytest
import torch

import bench
from paper_1206_3511_amd import intsort as I

pytestmark = pytest.mark.gpu

CASES = [("radix", 4, False, 10_000_000, {}),
         ("radix", 4, False, 10_000_000, {"digit_bits": 11}),
         ("radix", 8, True, 5_000_000, {}),
         ("bucket", 4, False, 10_000_000, {"num_buckets": 1024}),
         ("bucket", 8, True, 5_000_000, {"num_buckets": 65536}),
         ("bucket", 4, True, 3_000_000, {"num_buckets": 3_000_000, "key_bound": 10**6})]


def _call(algo, width, pairs, n, opt, keys, vals):
    if pairs:
        return I.sort_pairs(keys, vals, algo=algo, **opt)
    return I.sort(keys, algo=algo, **opt)


@pytest.mark.parametrize("algo,width,pairs,n,opt", CASES)
def test_call_holds_the_reported_bytes(algo, width, pairs, n, opt):
    dt = torch.int32 if width == 4 else torch.int64
    keys = torch.randint(0, 10**6, (n,), dtype=dt, device="cuda:0").view(torch.uint32 if width == 4 else torch.uint64)
    vals = torch.arange(n, dtype=torch.int32, device="cuda:0").view(torch.uint32) if pairs else None
    ctx = I.context(0)
    # once first: kernels load and the runtime sets up what it needs
    _call(algo, width, pairs, n, opt, keys, vals)
    torch.cuda.synchronize()
    ctx._ws.clear()
    torch.cuda.empty_cache()
    in_bytes = n * (width + (4 if pairs else 0))
    free0, _ = torch.cuda.mem_get_info()
    res0 = torch.cuda.memory_reserved()
    alloc0 = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    out = _call(algo, width, pairs, n, opt, keys, vals)
    torch.cuda.synchronize()
    assert I.device_error(0) == 0
    measured = torch.cuda.max_memory_allocated() - alloc0 + in_bytes
    m = bench._memory(width, pairs, n, algo=algo, **opt)
    allocations = 3 if pairs else 2   # output keys (and values), workspace
    assert 0 <= measured - m["peak_device_bytes"] <= allocations * ((1 << 20) + 512), (measured, m)
    # nothing besides torch's allocator took device memory during the call
    free1, _ = torch.cuda.mem_get_info()
    res1 = torch.cuda.memory_reserved()
    assert abs((free0 - free1) - (res1 - res0)) <= 8 << 20
    del out
