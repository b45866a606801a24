"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/intsort.h declares, validates arguments before it
touches a device, and sizes workspaces consistently."""
import ctypes
import os
import re

import pytest

from paper_1206_3511_amd import intsort as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "intsort.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(intsort_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_what_the_binding_uses():
    decl = declared_functions()
    assert set(I.EXPORTED) <= set(decl)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(I.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_status_strings():
    for s in range(0, 9):
        assert I.status_string(s) and I.status_string(s) != "unknown status"
    assert I.status_string(99) == "unknown status"


@pytest.fixture(scope="module")
def plan_ctx():
    return I.Context(-1)


def _call_sort(ctx, kt=I.U32, kin=0x1000, kout=0x100000, n=100, opts=None, ws=0x1000000, wsb=1 << 30):
    o = opts if opts is not None else I.make_options()
    return I.lib().intsort_sort_keys(ctx.handle, kt, kin, kout, n, ctypes.byref(o), ws, wsb, None)


def test_validation_order_on_planning_context(plan_ctx):
    # arguments that pass every check reach the device step, which a
    # planning context refuses
    assert _call_sort(plan_ctx) == I.ERR_UNSUPPORTED
    assert _call_sort(plan_ctx, n=0) == I.OK
    assert _call_sort(plan_ctx, kt=7) == I.ERR_INVALID_ARGUMENT
    assert _call_sort(plan_ctx, kin=None) == I.ERR_INVALID_ARGUMENT
    assert _call_sort(plan_ctx, kout=0x100004) == I.ERR_MISALIGNED
    # partial overlap of input and output
    assert _call_sort(plan_ctx, kin=0x1000, kout=0x1010, n=100) == I.ERR_INVALID_ARGUMENT
    # in place is allowed
    assert _call_sort(plan_ctx, kin=0x1000, kout=0x1000) == I.ERR_UNSUPPORTED
    assert _call_sort(plan_ctx, ws=None) == I.ERR_INVALID_ARGUMENT
    assert _call_sort(plan_ctx, ws=0x1000010) == I.ERR_MISALIGNED
    assert _call_sort(plan_ctx, wsb=16) == I.ERR_WORKSPACE_TOO_SMALL
    bad = I.make_options(digit_bits=5)
    assert _call_sort(plan_ctx, opts=bad) == I.ERR_UNSUPPORTED
    bad = I.make_options()
    bad.struct_size = 4
    assert _call_sort(plan_ctx, opts=bad) == I.ERR_INVALID_ARGUMENT
    bad = I.make_options()
    bad.flags = 0x80
    assert _call_sort(plan_ctx, opts=bad) == I.ERR_INVALID_ARGUMENT
    # more keys than a 30-bit status word can count
    assert _call_sort(plan_ctx, kout=1 << 40, n=1 << 31, wsb=1 << 62) == I.ERR_UNSUPPORTED
    # bucket counts up to 2^30; a declared range must fit the key width
    assert _call_sort(plan_ctx, wsb=1 << 62, opts=I.make_options("bucket", num_buckets=1 << 30)) == I.ERR_UNSUPPORTED
    assert _call_sort(plan_ctx, opts=I.make_options("bucket", num_buckets=(1 << 30) + 1)) == I.ERR_UNSUPPORTED
    assert _call_sort(plan_ctx, opts=I.make_options("bucket", key_bound=1 << 32)) == I.ERR_INVALID_ARGUMENT
    assert _call_sort(plan_ctx, opts=I.make_options("bucket", key_bound=(1 << 32) - 1)) == I.ERR_UNSUPPORTED
    assert _call_sort(plan_ctx, kt=I.U64, opts=I.make_options("bucket", key_bound=1 << 40)) == I.ERR_UNSUPPORTED


def test_pairs_validation(plan_ctx):
    o = I.make_options()
    L = I.lib()
    n = 64
    ok = L.intsort_sort_pairs(plan_ctx.handle, I.U32, 0x1000, 0x2000, 0x3000, 0x4000, n, ctypes.byref(o),
                              0x100000, 1 << 30, None)
    assert ok == I.ERR_UNSUPPORTED
    # values overlapping keys
    assert L.intsort_sort_pairs(plan_ctx.handle, I.U32, 0x1000, 0x2000, 0x1040, 0x4000, n, ctypes.byref(o),
                                0x100000, 1 << 30, None) == I.ERR_INVALID_ARGUMENT
    assert L.intsort_sort_pairs(plan_ctx.handle, I.U32, 0x1000, 0x2000, None, 0x4000, n, ctypes.byref(o),
                                0x100000, 1 << 30, None) == I.ERR_INVALID_ARGUMENT


def test_create_rejects_bad_device():
    h = ctypes.c_void_p()
    assert I.lib().intsort_create(ctypes.byref(h), -2) == I.ERR_INVALID_ARGUMENT
    assert I.lib().intsort_create(None, 0) == I.ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("kt", [I.U32, I.U64])
@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("bits", [4, 8, 11])
def test_workspace_monotone(plan_ctx, kt, pairs, bits):
    o = I.make_options(digit_bits=bits)
    prev = 0
    for n in [0, 1, 100, 4095, 4096, 4097, 10**5, 10**6, 10**8]:
        b = plan_ctx.workspace_size(kt, pairs, n, 0, o)
        assert b >= prev and b % 256 == 0
        prev = b
    # at least the scratch copy of keys (and values)
    w = 8 if kt == I.U64 else 4
    assert prev >= 10**8 * (w + (4 if pairs else 0))


@pytest.mark.parametrize("kt,kb", [(I.I32, 4), (I.I64, 8), (I.F32, 4), (I.F64, 8)])
def test_signed_and_float_keys_take_radix_with_8bit_digits(plan_ctx, kt, kb):
    L = I.lib()
    n = 1 << 20

    def ws(opts, segs=0):
        b = ctypes.c_size_t(0)
        st = L.intsort_workspace_size(plan_ctx.handle, kt, 1, n, segs, ctypes.byref(opts), ctypes.byref(b))
        return st, b.value

    same_width = I.U32 if kb == 4 else I.U64
    ref = ctypes.c_size_t(0)
    assert L.intsort_workspace_size(plan_ctx.handle, same_width, 1, n, 0, ctypes.byref(I.make_options()),
                                    ctypes.byref(ref)) == I.OK
    assert ws(I.make_options()) == (I.OK, ref.value)
    assert ws(I.make_options(digit_bits=11))[0] == I.ERR_UNSUPPORTED
    assert ws(I.make_options(digit_bits=4))[0] == I.ERR_UNSUPPORTED
    assert ws(I.make_options("bucket"))[0] == I.ERR_UNSUPPORTED
    assert ws(I.make_options(), segs=4)[0] == I.ERR_UNSUPPORTED
    assert _call_sort(plan_ctx, kt=kt, opts=I.make_options("bucket")) == I.ERR_UNSUPPORTED
    off = 0x200000
    assert L.intsort_segmented_sort_keys(plan_ctx.handle, kt, 0x1000, 0x100000, 100, 1, off,
                                         ctypes.byref(I.make_options()), 0x1000000, 1 << 30,
                                         None) == I.ERR_UNSUPPORTED
    mm = (ctypes.c_uint64 * 2)()
    assert L.intsort_minmax(plan_ctx.handle, kt, 0x1000, 100, mm, None) == I.ERR_UNSUPPORTED
    assert L.intsort_digit_histogram(plan_ctx.handle, kt, 0x1000, 100, 8, 0x2000, 0x1000000, 1 << 20,
                                     None) == I.ERR_UNSUPPORTED
    assert _call_sort(plan_ctx, kt=6) == I.ERR_INVALID_ARGUMENT


def test_msd_is_bucket_sort_over_the_full_range(plan_ctx):
    L = I.lib()
    n = 1 << 22
    for kt, top in ((I.U32, (1 << 32) - 1), (I.U64, (1 << 64) - 1)):
        for r in (4, 8, 11):
            a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
            assert L.intsort_workspace_size(plan_ctx.handle, kt, 1, n, 0,
                                            ctypes.byref(I.make_options("msd", digit_bits=r, num_buckets=77)),
                                            ctypes.byref(a)) == I.OK
            assert L.intsort_workspace_size(plan_ctx.handle, kt, 1, n, 0,
                                            ctypes.byref(I.make_options("bucket", num_buckets=1 << r,
                                                                        key_bound=top)),
                                            ctypes.byref(b)) == I.OK
            assert a.value == b.value
    assert _call_sort(plan_ctx, opts=I.make_options("msd", key_bound=5)) == I.ERR_INVALID_ARGUMENT
    assert _call_sort(plan_ctx, kt=I.I32, opts=I.make_options("msd")) == I.ERR_UNSUPPORTED
    bad = I.make_options()
    bad.algo = 3
    assert _call_sort(plan_ctx, opts=bad) == I.ERR_INVALID_ARGUMENT


def test_graph_capture_argument_checks(plan_ctx):
    L = I.lib()
    g = ctypes.c_void_p()
    assert L.intsort_capture_begin(plan_ctx.handle, None) == I.ERR_INVALID_ARGUMENT
    assert L.intsort_capture_begin(None, 0x1000) == I.ERR_INVALID_ARGUMENT
    # a planning context has no device to record on
    assert L.intsort_capture_begin(plan_ctx.handle, 0x1000) == I.ERR_UNSUPPORTED
    assert L.intsort_capture_end(plan_ctx.handle, None, ctypes.byref(g)) == I.ERR_INVALID_ARGUMENT
    assert L.intsort_capture_end(plan_ctx.handle, 0x1000, None) == I.ERR_INVALID_ARGUMENT
    assert L.intsort_graph_launch(None, None) == I.ERR_INVALID_ARGUMENT
    assert L.intsort_graph_destroy(None) == I.OK


def test_check_segments_flag_accepted(plan_ctx):
    b = ctypes.c_size_t(0)
    o = I.make_options(check_segments=True)
    assert o.flags == I.FLAG_CHECK_SEGMENTS
    assert I.lib().intsort_workspace_size(plan_ctx.handle, I.U32, 0, 1000, 10, ctypes.byref(o),
                                          ctypes.byref(b)) == I.OK
    bad = I.make_options()
    bad.flags = 0x4
    assert I.lib().intsort_workspace_size(plan_ctx.handle, I.U32, 0, 1000, 10, ctypes.byref(bad),
                                          ctypes.byref(b)) == I.ERR_INVALID_ARGUMENT


def test_host_tensors_are_refused():
    """Every step runs in the HIP kernels: host tensors are refused with an
    error, never sorted on the CPU."""
    import torch
    k = torch.arange(100, dtype=torch.int64).flip(0).to(torch.uint32)
    v = torch.arange(100, dtype=torch.int32).view(torch.uint32)
    offs = torch.tensor([0, 50, 100], dtype=torch.int64)
    with pytest.raises(ValueError, match="device tensor"):
        I.sort(k)
    with pytest.raises(ValueError, match="device tensor"):
        I.sort(k, algo="bucket")
    with pytest.raises(ValueError, match="device tensor"):
        I.sort_pairs(k, v)
    with pytest.raises(ValueError, match="device tensor"):
        I.segmented_sort(k, offs)
    with pytest.raises(ValueError, match="device tensor"):
        I.batched_sort([k, k[:10]])
    with pytest.raises(ValueError, match="device tensor"):
        I.sort(torch.zeros(4, dtype=torch.int16))


def test_bucket_histogram_requires_aligned_keys(plan_ctx):
    """The bucket histogram reads keys as 16-byte vectors: an unaligned base is
    refused before anything is enqueued."""
    L = I.lib()
    mm, counts = 0x200000, 0x300000
    assert L.intsort_bucket_histogram(plan_ctx.handle, I.U32, 0x1004, 100, mm, 1024, counts,
                                      None) == I.ERR_MISALIGNED
    assert L.intsort_bucket_histogram(plan_ctx.handle, I.U64, 0x1008, 100, mm, 1024, counts,
                                      None) == I.ERR_MISALIGNED
    # aligned keys pass every check and reach the device step
    assert L.intsort_bucket_histogram(plan_ctx.handle, I.U32, 0x1000, 100, mm, 1024, counts,
                                      None) == I.ERR_UNSUPPORTED


def test_segmented_pairs_refuse_keys_overlapping_values(plan_ctx):
    L = I.lib()
    o = I.make_options()
    n, off = 64, 0x900000

    def call(kin, kout, vin, vout):
        return L.intsort_segmented_sort_pairs(plan_ctx.handle, I.U32, kin, kout, vin, vout, n, 1, off,
                                              ctypes.byref(o), 0x1000000, 1 << 30, None)

    assert call(0x1000, 0x2000, 0x3000, 0x4000) == I.ERR_UNSUPPORTED
    assert call(0x1000, 0x2000, 0x1040, 0x4000) == I.ERR_INVALID_ARGUMENT   # values inside the input keys
    assert call(0x1000, 0x2000, 0x3000, 0x2000) == I.ERR_INVALID_ARGUMENT   # output values on output keys
    assert call(0x1000, 0x2000, 0x3000, 0x3010) == I.ERR_INVALID_ARGUMENT   # values partly overlap
    assert call(0x1000, 0x1000, 0x3000, 0x3000) == I.ERR_UNSUPPORTED        # both in place
