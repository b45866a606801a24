"""Python binding of libintsort.so (include/intsort.h).

Argument marshalling only: every step of every sort runs in the HIP kernels of
the library.  torch supplies device memory (inputs, outputs, workspaces) and
streams.  If the library is not built the calls raise; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libintsort.so")

# status codes (intsort_status)
OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_MISALIGNED = 2
ERR_WORKSPACE_TOO_SMALL = 3
ERR_UNSUPPORTED = 4
ERR_OVER_BUDGET = 5
ERR_HIP = 6
ERR_INTERNAL = 7
ERR_NOT_READY = 8

U32, U64, I32, I64, F32, F64 = 0, 1, 2, 3, 4, 5
RADIX, BUCKET, MSD = 0, 1, 2
FLAG_NO_PASS_SKIP = 0x1
FLAG_CHECK_SEGMENTS = 0x2
DEVERR_BAD_SEGMENTS = 0x8

EXPORTED = (
    "intsort_status_string", "intsort_default_options", "intsort_create", "intsort_destroy",
    "intsort_workspace_size", "intsort_sort_keys", "intsort_sort_keys_noalloc", "intsort_sort_pairs",
    "intsort_segmented_sort_keys", "intsort_segmented_sort_pairs", "intsort_digit_histogram",
    "intsort_minmax", "intsort_bucket_histogram", "intsort_read_device_error",
    "intsort_timing_enable", "intsort_timing_read", "intsort_batched_sort_keys",
    "intsort_server_create", "intsort_server_submit", "intsort_server_poll", "intsort_server_completed",
    "intsort_server_drain", "intsort_server_destroy", "intsort_server_fail_next_launches",
    "intsort_capture_begin", "intsort_capture_end", "intsort_graph_launch", "intsort_graph_destroy",
    "intsort_load_tuning", "intsort_device_key",
)

KERNEL_KINDS = ("init", "digit_histogram", "pass", "copy", "minmax", "bucket_histogram",
                "bucket_scatter", "segment_sort", "plan")


class IntsortError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class KernelTime(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("index", ctypes.c_uint32), ("ms", ctypes.c_float)]


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("algo", ctypes.c_uint32),
                ("digit_bits", ctypes.c_uint32), ("num_buckets", ctypes.c_uint32),
                ("lds_cutoff", ctypes.c_uint32), ("max_passes", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("key_bound", ctypes.c_uint64)]


_lib = None
_lock = threading.Lock()
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_i = ctypes.c_int
_st = ctypes.c_int


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        L.intsort_status_string.argtypes = [_st]
        L.intsort_status_string.restype = ctypes.c_char_p
        L.intsort_default_options.argtypes = [ctypes.POINTER(Options)]
        L.intsort_default_options.restype = None
        L.intsort_create.argtypes = [ctypes.POINTER(_vp), _i]
        L.intsort_destroy.argtypes = [_vp]
        L.intsort_workspace_size.argtypes = [_vp, _i, _i, _u64, _u64, ctypes.POINTER(Options),
                                             ctypes.POINTER(ctypes.c_size_t)]
        L.intsort_sort_keys.argtypes = [_vp, _i, _vp, _vp, _u64, ctypes.POINTER(Options), _vp,
                                        ctypes.c_size_t, _vp]
        L.intsort_sort_keys_noalloc.argtypes = [_vp, _i, _vp, _vp, _u64, ctypes.POINTER(Options), _vp]
        L.intsort_sort_pairs.argtypes = [_vp, _i, _vp, _vp, _vp, _vp, _u64, ctypes.POINTER(Options),
                                         _vp, ctypes.c_size_t, _vp]
        L.intsort_segmented_sort_keys.argtypes = [_vp, _i, _vp, _vp, _u64, _u64, _vp,
                                                  ctypes.POINTER(Options), _vp, ctypes.c_size_t, _vp]
        L.intsort_segmented_sort_pairs.argtypes = [_vp, _i, _vp, _vp, _vp, _vp, _u64, _u64, _vp,
                                                   ctypes.POINTER(Options), _vp, ctypes.c_size_t, _vp]
        L.intsort_digit_histogram.argtypes = [_vp, _i, _vp, _u64, ctypes.c_uint32, _vp, _vp,
                                              ctypes.c_size_t, _vp]
        L.intsort_minmax.argtypes = [_vp, _i, _vp, _u64, _vp, _vp]
        L.intsort_bucket_histogram.argtypes = [_vp, _i, _vp, _u64, _vp, ctypes.c_uint32, _vp, _vp]
        L.intsort_read_device_error.argtypes = [_vp, _vp, ctypes.c_size_t,
                                                ctypes.POINTER(ctypes.c_uint32), _vp]
        L.intsort_batched_sort_keys.argtypes = [_vp, _i, _vp, _u64, _u64, ctypes.POINTER(Options), _vp,
                                                ctypes.c_size_t, _vp]
        L.intsort_capture_begin.argtypes = [_vp, _vp]
        L.intsort_capture_end.argtypes = [_vp, _vp, ctypes.POINTER(_vp)]
        L.intsort_graph_launch.argtypes = [_vp, _vp]
        L.intsort_graph_destroy.argtypes = [_vp]
        L.intsort_server_create.argtypes = [_vp, _u64, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_vp)]
        L.intsort_server_submit.argtypes = [_vp, _i, _vp, _vp, _u64, ctypes.POINTER(_u64)]
        L.intsort_server_poll.argtypes = [_vp, _u64, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_double)]
        L.intsort_server_completed.argtypes = [_vp, ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_double),
                                               ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        L.intsort_server_drain.argtypes = [_vp]
        L.intsort_server_destroy.argtypes = [_vp]
        L.intsort_server_fail_next_launches.argtypes = [_vp, ctypes.c_uint32]
        L.intsort_load_tuning.argtypes = [_vp, ctypes.c_char_p]
        L.intsort_device_key.argtypes = [_vp, ctypes.c_char_p, ctypes.c_size_t]
        L.intsort_timing_enable.argtypes = [_vp, _i]
        L.intsort_timing_read.argtypes = [_vp, ctypes.POINTER(KernelTime), ctypes.c_uint32,
                                          ctypes.POINTER(ctypes.c_uint32)]
        for name in EXPORTED:
            if name not in ("intsort_status_string", "intsort_default_options"):
                getattr(L, name).restype = _st
        _lib = L
        return L


def status_string(s: int) -> str:
    return lib().intsort_status_string(s).decode()


def _check(rc: int, where: str):
    if rc != OK:
        raise IntsortError(rc, where)


def make_options(algo: str | int = "radix", digit_bits: int = 0, num_buckets: int = 0,
                 lds_cutoff: int = 0, max_passes: int = 0, skip_passes: bool = True,
                 key_bound: int = 0, check_segments: bool = False) -> Options:
    """intsort_options for a call.  Zero fields take the library defaults;
    skip_passes=False runs every digit pass (INTSORT_FLAG_NO_PASS_SKIP);
    check_segments=True makes the segmented and batched calls check their
    segment layout on the device first (INTSORT_FLAG_CHECK_SEGMENTS: a bad
    layout sets DEVERR_BAD_SEGMENTS in device_error() and sorts nothing)."""
    o = Options()
    lib().intsort_default_options(ctypes.byref(o))
    o.algo = algo if isinstance(algo, int) else {"radix": RADIX, "bucket": BUCKET, "msd": MSD}[algo]
    o.digit_bits = digit_bits
    o.num_buckets = num_buckets
    o.lds_cutoff = lds_cutoff
    o.max_passes = max_passes
    o.flags = (0 if skip_passes else FLAG_NO_PASS_SKIP) | (FLAG_CHECK_SEGMENTS if check_segments else 0)
    o.key_bound = key_bound
    return o


class Context:
    """One intsort context per device (device -1: planning only) and a cached
    workspace tensor per stream.

    A workspace must not be used by two calls that run at the same time, so
    each stream gets its own.  It is allocated while that stream is current:
    torch's caching allocator then hands its memory to a later allocation
    only in that stream's order, so dropping it to grow it cannot give it to
    work on another stream while kernels on its own stream still use it."""

    def __init__(self, device: int):
        self.device = device
        self.handle = _vp()
        _check(lib().intsort_create(ctypes.byref(self.handle), device), "intsort_create")
        self._ws: dict[int, torch.Tensor] = {}

    def __del__(self):
        try:
            if self.handle:
                lib().intsort_destroy(self.handle)
        except Exception:
            pass

    def workspace_size(self, kt: int, has_values: bool, n: int, num_segments: int, opts: Options) -> int:
        out = ctypes.c_size_t(0)
        _check(lib().intsort_workspace_size(self.handle, kt, int(has_values), n, num_segments,
                                            ctypes.byref(opts), ctypes.byref(out)), "intsort_workspace_size")
        return out.value

    def load_tuning(self, path: str | None):
        """Replaces the context's tuning table with the file at `path` (None
        empties it): zero digit_bits / num_buckets / lds_cutoff take its
        choices."""
        _check(lib().intsort_load_tuning(self.handle, None if path is None else path.encode()),
               "intsort_load_tuning")

    def device_key(self) -> str:
        buf = ctypes.create_string_buffer(512)
        _check(lib().intsort_device_key(self.handle, buf, 512), "intsort_device_key")
        return buf.value.decode()

    def timing(self, enable: bool = True):
        _check(lib().intsort_timing_enable(self.handle, int(enable)), "intsort_timing_enable")

    def kernel_times(self) -> list[tuple[str, int, float]]:
        """(kind, index, ms) of every kernel launched since the last read."""
        buf = (KernelTime * 1024)()
        cnt = ctypes.c_uint32(0)
        _check(lib().intsort_timing_read(self.handle, buf, 1024, ctypes.byref(cnt)), "intsort_timing_read")
        return [(KERNEL_KINDS[buf[i].kind], buf[i].index, buf[i].ms) for i in range(cnt.value)]

    def workspace(self, nbytes: int, stream=None) -> torch.Tensor:
        """A workspace of at least nbytes for calls on `stream` (None: the
        current stream)."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        key = s.cuda_stream
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            self._ws.pop(key, None)
            with torch.cuda.stream(s):
                ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
            self._ws[key] = ws
        return ws


_contexts: dict[int, Context] = {}


def context(device: int) -> Context:
    c = _contexts.get(device)
    if c is None:
        c = _contexts[device] = Context(device)
    return c


_KEY_TYPES = {torch.uint32: U32, torch.uint64: U64, torch.int32: I32, torch.int64: I64,
              torch.float32: F32, torch.float64: F64}


def _key_type(t: torch.Tensor) -> int:
    kt = _KEY_TYPES.get(t.dtype)
    if kt is None:
        raise TypeError(f"keys must be a 32- or 64-bit integer or float tensor, got {t.dtype}")
    return kt


def _dev_tensor(t: torch.Tensor, what: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t


def _stream_ptr(stream) -> int | None:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def _ptr(t):
    return None if t is None else t.data_ptr()


def sort(keys: torch.Tensor, algo: str = "radix", out: torch.Tensor | None = None, stream=None,
         **opt) -> torch.Tensor:
    """Nondecreasing permutation of `keys`.  Unsigned keys (uint32, uint64)
    take every algorithm; signed (int32, int64) and floating-point keys
    (float32, float64, in IEEE 754 totalOrder: -NaN < -inf < ... < -0 < +0
    < ... < +inf < +NaN) take radix sort with 8-bit digits."""
    _dev_tensor(keys, "keys")
    kt = _key_type(keys)
    out = torch.empty_like(keys) if out is None else _dev_tensor(out, "out")
    ctx = context(keys.device.index)
    o = make_options(algo, **opt)
    n = keys.numel()
    nb = ctx.workspace_size(kt, False, n, 0, o)
    ws = ctx.workspace(nb, stream)
    _check(lib().intsort_sort_keys(ctx.handle, kt, _ptr(keys), _ptr(out), n, ctypes.byref(o), ws.data_ptr(),
                                   ws.numel(), _stream_ptr(stream)), "intsort_sort_keys")
    return out


def sort_noalloc(keys: torch.Tensor, algo: str = "radix", out: torch.Tensor | None = None, stream=None,
                 **opt) -> torch.Tensor:
    """sort() through intsort_sort_keys_noalloc: the library's own device
    array is the workspace (nothing is allocated for it; `out` is allocated
    here when not given).  Calls that overlap on one device race."""
    _dev_tensor(keys, "keys")
    kt = _key_type(keys)
    out = torch.empty_like(keys) if out is None else _dev_tensor(out, "out")
    ctx = context(keys.device.index)
    o = make_options(algo, **opt)
    _check(lib().intsort_sort_keys_noalloc(ctx.handle, kt, _ptr(keys), _ptr(out), keys.numel(), ctypes.byref(o),
                                           _stream_ptr(stream)), "intsort_sort_keys_noalloc")
    return out


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, algo: str = "radix", out_keys=None, out_vals=None,
               stream=None, **opt):
    """Stable key-value sort: equal keys keep their input order."""
    _dev_tensor(keys, "keys")
    _dev_tensor(vals, "vals")
    if vals.dtype not in (torch.uint32, torch.int32) or vals.numel() != keys.numel():
        raise ValueError("vals must hold one 32-bit value per key")
    kt = _key_type(keys)
    ok = torch.empty_like(keys) if out_keys is None else out_keys
    ov = torch.empty_like(vals) if out_vals is None else out_vals
    ctx = context(keys.device.index)
    o = make_options(algo, **opt)
    n = keys.numel()
    ws = ctx.workspace(ctx.workspace_size(kt, True, n, 0, o), stream)
    _check(lib().intsort_sort_pairs(ctx.handle, kt, _ptr(keys), _ptr(ok), _ptr(vals), _ptr(ov), n,
                                    ctypes.byref(o), ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
           "intsort_sort_pairs")
    return ok, ov


def segmented_sort(keys: torch.Tensor, offsets: torch.Tensor, vals: torch.Tensor | None = None,
                   algo: str = "radix", out_keys=None, out_vals=None, stream=None, **opt):
    """Sort every segment [offsets[s], offsets[s+1]) of `keys` on its own.
    `offsets` is a device uint64/int64 tensor of num_segments + 1 entries,
    nondecreasing from 0 to keys.numel(); the host does not read it (pass
    check_segments=True to have the device check it)."""
    _dev_tensor(keys, "keys")
    _dev_tensor(offsets, "offsets")
    if offsets.dtype not in (torch.uint64, torch.int64):
        raise TypeError("offsets must be 64-bit")
    kt = _key_type(keys)
    S = offsets.numel() - 1
    ok = torch.empty_like(keys) if out_keys is None else out_keys
    ctx = context(keys.device.index)
    o = make_options(algo, **opt)
    n = keys.numel()
    ws = ctx.workspace(ctx.workspace_size(kt, vals is not None, n, max(S, 1), o), stream)
    if vals is None:
        _check(lib().intsort_segmented_sort_keys(ctx.handle, kt, _ptr(keys), _ptr(ok), n, S, _ptr(offsets),
                                                 ctypes.byref(o), ws.data_ptr(), ws.numel(),
                                                 _stream_ptr(stream)), "intsort_segmented_sort_keys")
        return ok
    ov = torch.empty_like(vals) if out_vals is None else out_vals
    _check(lib().intsort_segmented_sort_pairs(ctx.handle, kt, _ptr(keys), _ptr(ok), _ptr(vals), _ptr(ov), n, S,
                                              _ptr(offsets), ctypes.byref(o), ws.data_ptr(), ws.numel(),
                                              _stream_ptr(stream)), "intsort_segmented_sort_pairs")
    return ok, ov


def batched_sort(inputs: list, outputs: list | None = None, stream=None, **opt) -> list:
    """Sort several separate device arrays (all 32-bit or all 64-bit) in one
    set of launches; returns the output tensors.  `opt` are options
    (digit_bits, lds_cutoff, flags)."""
    if not inputs:
        return []
    kt = _key_type(inputs[0])
    outputs = [torch.empty_like(t) for t in inputs] if outputs is None else outputs
    desc = torch.empty((len(inputs), 3), dtype=torch.int64)
    for i, (a, b) in enumerate(zip(inputs, outputs)):
        _dev_tensor(a, "input")
        _dev_tensor(b, "output")
        if _key_type(a) != kt or a.numel() != b.numel():
            raise ValueError("all arrays must share the key type; outputs must match inputs")
        desc[i, 0] = a.data_ptr()
        desc[i, 1] = b.data_ptr()
        desc[i, 2] = a.numel()
    dev = inputs[0].device
    d_desc = desc.to(dev)
    total = int(sum(t.numel() for t in inputs))
    ctx = context(dev.index)
    o = make_options("radix", **opt)
    ws = ctx.workspace(ctx.workspace_size(kt, False, total, len(inputs), o), stream)
    _check(lib().intsort_batched_sort_keys(ctx.handle, kt, d_desc.data_ptr(), len(inputs), total, ctypes.byref(o),
                                           ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
           "intsort_batched_sort_keys")
    return outputs


def digit_histogram(keys: torch.Tensor, digit_bits: int = 8, stream=None) -> torch.Tensor:
    """counts[p, v]: keys whose digit p equals v, for every pass p."""
    _dev_tensor(keys, "keys")
    kt = _key_type(keys)
    passes = -(-8 * keys.element_size() // digit_bits)
    counts = torch.empty(passes * (1 << digit_bits), dtype=torch.uint32, device=keys.device)
    ctx = context(keys.device.index)
    o = make_options("radix", digit_bits=digit_bits)
    ws = ctx.workspace(ctx.workspace_size(kt, False, 0, 0, o), stream)
    _check(lib().intsort_digit_histogram(ctx.handle, kt, _ptr(keys), keys.numel(), digit_bits, _ptr(counts),
                                         ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
           "intsort_digit_histogram")
    return counts.view(passes, 1 << digit_bits)


def minmax(keys: torch.Tensor, stream=None) -> torch.Tensor:
    _dev_tensor(keys, "keys")
    mm = torch.empty(2, dtype=torch.uint64, device=keys.device)
    ctx = context(keys.device.index)
    _check(lib().intsort_minmax(ctx.handle, _key_type(keys), _ptr(keys), keys.numel(), _ptr(mm),
                                _stream_ptr(stream)), "intsort_minmax")
    return mm


def bucket_histogram(keys: torch.Tensor, mm: torch.Tensor, num_buckets: int, stream=None) -> torch.Tensor:
    _dev_tensor(keys, "keys")
    counts = torch.empty(num_buckets, dtype=torch.uint32, device=keys.device)
    ctx = context(keys.device.index)
    _check(lib().intsort_bucket_histogram(ctx.handle, _key_type(keys), _ptr(keys), keys.numel(), _ptr(mm),
                                          num_buckets, _ptr(counts), _stream_ptr(stream)),
           "intsort_bucket_histogram")
    return counts


def device_error(device: int = 0, stream=None) -> int:
    """Error word left by the last sort that used the workspace this device's
    context keeps for `stream` (None: the current stream)."""
    ctx = context(device)
    s = stream if stream is not None else torch.cuda.current_stream(device)
    ws = ctx._ws.get(s.cuda_stream)
    if ws is None:
        return 0
    w = ctypes.c_uint32(0)
    _check(lib().intsort_read_device_error(ctx.handle, ws.data_ptr(), ws.numel(), ctypes.byref(w),
                                           _stream_ptr(s)), "intsort_read_device_error")
    return w.value


class Graph:
    """A recorded sequence of sort calls; launch() replays it on a stream."""

    def __init__(self, handle, device: int, keep=()):
        self.handle = handle
        self.device = device
        # the workspace the recorded calls use stays allocated while the
        # graph exists, even if the context later takes a larger one
        self._keep = list(keep)

    def launch(self, stream=None):
        _check(lib().intsort_graph_launch(self.handle, _stream_ptr(stream)), "intsort_graph_launch")

    def close(self):
        if self.handle:
            lib().intsort_graph_destroy(self.handle)
            self.handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture(fn, stream, device: int = 0) -> Graph:
    """Records the sort calls `fn()` makes on `stream` (a non-default
    torch.cuda.Stream) into one HIP graph.  fn runs once eagerly first, so
    that every workspace it needs exists before the recording (nothing may be
    allocated while recording); it must pass its output tensors and device
    offsets in, and use only this module's sort calls on `stream`."""
    if stream is None or not stream.cuda_stream:
        raise ValueError("capture needs a non-default stream")
    with torch.cuda.stream(stream):
        fn()
    stream.synchronize()
    ctx = context(device)
    _check(lib().intsort_capture_begin(ctx.handle, stream.cuda_stream), "intsort_capture_begin")
    g = _vp()
    try:
        with torch.cuda.stream(stream):
            fn()
    except BaseException:
        if lib().intsort_capture_end(ctx.handle, stream.cuda_stream, ctypes.byref(g)) == OK:
            lib().intsort_graph_destroy(g)
        raise
    _check(lib().intsort_capture_end(ctx.handle, stream.cuda_stream, ctypes.byref(g)), "intsort_capture_end")
    return Graph(g, device, keep=[ctx._ws.get(stream.cuda_stream)])


class ServerRequestsFailed(IntsortError):
    """Some requests listed by Server.completed failed (their batch's launch
    or completion reported a HIP error).  `tickets` are the failed ones,
    `results` everything that call listed, failed ones included."""

    def __init__(self, tickets, results):
        self.tickets = tickets
        self.results = results
        super().__init__(ERR_HIP, f"intsort_server_completed (failed tickets {tickets})")


class Server:
    """Continuous-batching sort server (intsort_server_*).  Keeps every
    submitted request's tensors alive until it completes.  `failed` holds the
    tickets that completed() has seen fail."""

    def __init__(self, device: int = 0, budget_bytes: int = 64 << 30, max_batch: int = 64, slots: int = 2):
        torch.cuda.set_device(device)
        self.handle = _vp()
        _check(lib().intsort_server_create(context(device).handle, budget_bytes, max_batch, slots,
                                           ctypes.byref(self.handle)), "intsort_server_create")
        self._live: dict[int, tuple] = {}
        self.failed: set[int] = set()

    def submit(self, keys: torch.Tensor, out: torch.Tensor) -> int:
        _dev_tensor(keys, "keys")
        _dev_tensor(out, "out")
        t = _u64(0)
        _check(lib().intsort_server_submit(self.handle, _key_type(keys), _ptr(keys), _ptr(out), keys.numel(),
                                           ctypes.byref(t)), "intsort_server_submit")
        self._live[t.value] = (keys, out)
        return t.value

    def completed(self, raise_on_failure: bool = True) -> list[tuple[int, float]]:
        """(ticket, latency seconds) of requests finished since the last call,
        failed ones included.  Failed tickets go into `failed`; with
        raise_on_failure the call then raises ServerRequestsFailed."""
        res, bad = [], []
        # buffers of this call (the C calls may run in several threads at once)
        buf_t, buf_l = (_u64 * 4096)(), (ctypes.c_double * 4096)()
        while True:
            cnt = ctypes.c_uint32(0)
            rc = lib().intsort_server_completed(self.handle, buf_t, buf_l, 4096, ctypes.byref(cnt))
            if rc not in (OK, ERR_HIP):
                raise IntsortError(rc, "intsort_server_completed")
            for i in range(cnt.value):
                t = int(buf_t[i])
                res.append((t, float(buf_l[i])))
                self._live.pop(t, None)
                if rc == ERR_HIP:
                    done = ctypes.c_int(0)
                    if lib().intsort_server_poll(self.handle, t, ctypes.byref(done), None) == ERR_HIP:
                        bad.append(t)
            if cnt.value < 4096:
                break
        self.failed.update(bad)
        if bad and raise_on_failure:
            raise ServerRequestsFailed(bad, res)
        return res

    def fail_next_launches(self, count: int):
        """Makes the next `count` batch launches fail before anything is
        enqueued (a test hook for the failure path)."""
        _check(lib().intsort_server_fail_next_launches(self.handle, count), "intsort_server_fail_next_launches")

    def poll(self, ticket: int):
        done = ctypes.c_int(0)
        lat = ctypes.c_double(0.0)
        rc = lib().intsort_server_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(lat))
        if rc not in (OK, ERR_NOT_READY):
            raise IntsortError(rc, "intsort_server_poll")
        return bool(done.value), lat.value

    def drain(self):
        _check(lib().intsort_server_drain(self.handle), "intsort_server_drain")

    def close(self):
        if self.handle:
            _check(lib().intsort_server_destroy(self.handle), "intsort_server_destroy")
            self.handle = _vp()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
