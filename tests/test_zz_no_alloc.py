"""intsort_sort_keys_noalloc, the key sort for callers that cannot allocate,
against intsort_sort_keys (the same sort with a caller workspace), called
through the C ABI: two calls in a row, the second with a smaller input (the
library's array then holds what the first call left), each equal to the
workspace entry point's output byte for byte; and a call that needs more
than the array refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1206_3511_amd import intsort as I

pytestmark = pytest.mark.gpu


def _noalloc(keys, out, **opt):
    ctx = I.context(0)
    o = I.make_options(**opt)
    return I.lib().intsort_sort_keys_noalloc(ctx.handle, I._key_type(keys), keys.data_ptr(), out.data_ptr(),
                                             keys.numel(), ctypes.byref(o), None)


def _keys(n, dtype, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    bits = torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, dtype=torch.int64)
    if dtype == torch.uint32:
        return bits.to(torch.int32).view(torch.uint32).to("cuda:0")
    hi = torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, dtype=torch.int64)
    return ((hi << 32) ^ (bits & 0xFFFFFFFF)).view(torch.uint64).to("cuda:0")


@pytest.mark.parametrize("algo,dtype,opt", [("radix", torch.uint32, {}), ("radix", torch.uint64, {}),
                                            ("bucket", torch.uint32, {"num_buckets": 1024}),
                                            ("radix", torch.uint32, {"digit_bits": 11})])
def test_noalloc_equals_workspace_entry_point(algo, dtype, opt):
    for i, n in enumerate((3_000_001, 100_003)):
        print(f"noalloc {algo} {dtype} n={n}", flush=True)
        keys = _keys(n, dtype, 17 + i)
        out = torch.empty_like(keys)
        assert _noalloc(keys, out, algo=algo, **opt) == I.OK
        ref = I.sort(keys, algo=algo, **opt)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32 if dtype == torch.uint32 else torch.int64),
                           ref.view(torch.int32 if dtype == torch.uint32 else torch.int64))
        assert I.device_error(0) == 0


def test_noalloc_refuses_more_than_its_array():
    n = 40_000_000   # a radix sort of 40M 32-bit keys needs about 160 MiB of workspace
    keys = torch.empty(16, dtype=torch.uint32, device="cuda:0")
    o = I.make_options()
    rc = I.lib().intsort_sort_keys_noalloc(I.context(0).handle, I.U32, keys.data_ptr(), keys.data_ptr(), n,
                                           ctypes.byref(o), None)
    assert rc == I.ERR_WORKSPACE_TOO_SMALL
