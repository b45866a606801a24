// abi.cpp -- the extern "C" entry points declared in include/intsort.h:
// argument validation on the host, workspace sizing, and dispatch to the
// kernel launchers.  No C++ exception leaves this file.

#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

#include "intsort.h"
#include "internal.hpp"
#include "sort_plans.hpp"
#include "tuning.hpp"

struct intsort_ctx {
    int device;
    int cus;
    intsort::Timer *timer = nullptr;   // set while per-kernel timing is on
    std::string dev_key;               // key of the device in the tuning table
    std::vector<intsort::TuneEntry> tune;   // tuned defaults of zero option fields
};

int intsort::ctx_device(const intsort_ctx *ctx) { return ctx ? ctx->device : -1; }

static_assert(INTSORT_DEVERR_LOOKBACK_TIMEOUT == intsort::DEVERR_LOOKBACK_TIMEOUT &&
                  INTSORT_DEVERR_BAD_TILE == intsort::DEVERR_BAD_TILE &&
                  INTSORT_DEVERR_SCATTER_RANGE == intsort::DEVERR_SCATTER_RANGE,
              "public error bits match the kernels'");

struct intsort_graph {
    int device;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

using namespace intsort;

int key_bytes_of(intsort_key_type kt)
{
    return kt == INTSORT_U64 || kt == INTSORT_I64 || kt == INTSORT_F64 ? 8 : 4;
}

bool valid_kt(intsort_key_type kt) { return kt >= INTSORT_U32 && kt <= INTSORT_F64; }

bool unsigned_kt(intsort_key_type kt) { return kt == INTSORT_U32 || kt == INTSORT_U64; }

// how a key's bits map to its rank: 0 as unsigned, 1 two's complement,
// 2 IEEE 754 totalOrder
int key_order(intsort_key_type kt)
{
    if (kt == INTSORT_I32 || kt == INTSORT_I64) return 1;
    if (kt == INTSORT_F32 || kt == INTSORT_F64) return 2;
    return 0;
}

// The options of a call on n keys (n_total for segmented and batched calls).
// A zero digit_bits (plain radix sort of unsigned keys), num_buckets (bucket
// sort) or lds_cutoff (segmented and batched calls) takes the value the
// context's table holds for its device, the key width and the size class of
// n, when there is one and a call can take it; otherwise the library default.
intsort_status read_opts(const intsort_ctx *ctx, const intsort_options *in, intsort_key_type kt, uint64_t n,
                         bool segmented, intsort_options *out)
{
    *out = intsort_options{};
    out->struct_size = sizeof(intsort_options);
    out->algo = INTSORT_RADIX_LSD;
    if (in) {
        if (in->struct_size != sizeof(intsort_options)) return INTSORT_ERR_INVALID_ARGUMENT;
        *out = *in;
    }
    if (out->algo != INTSORT_RADIX_LSD && out->algo != INTSORT_BUCKET && out->algo != INTSORT_RADIX_MSD)
        return INTSORT_ERR_INVALID_ARGUMENT;
    if (ctx && !ctx->tune.empty() && valid_kt(kt)) {
        const int w = key_bytes_of(kt);
        uint32_t v = 0;
        if (out->digit_bits == 0 && !segmented && out->algo == INTSORT_RADIX_LSD && unsigned_kt(kt) &&
            tune_lookup(ctx->tune, ctx->dev_key, TUNE_RADIX_BITS, w, n, &v) && (v == 4 || v == 8 || v == 11))
            out->digit_bits = v;
        if (out->num_buckets == 0 && out->algo == INTSORT_BUCKET &&
            tune_lookup(ctx->tune, ctx->dev_key, TUNE_BUCKETS, w, n, &v) && v >= 1 && v <= MAX_BUCKETS)
            out->num_buckets = v;
        if (out->lds_cutoff == 0 && segmented && tune_lookup(ctx->tune, ctx->dev_key, TUNE_LDS_CUTOFF, w, n, &v))
            out->lds_cutoff = v;
        if (out->digit_bits == 0 && segmented &&
            tune_lookup(ctx->tune, ctx->dev_key, TUNE_SEG_BITS, w, n, &v) && (v == 4 || v == 8))
            out->digit_bits = v;
    }
    if (out->digit_bits == 0) out->digit_bits = 8;
    if (out->digit_bits != 4 && out->digit_bits != 8 && out->digit_bits != 11) return INTSORT_ERR_UNSUPPORTED;
    if (out->algo == INTSORT_RADIX_MSD) {
        // the top r bits of the key are the bucket index floor(k * 2^r / 2^W)
        // of bucket sort over the declared range [0, 2^W - 1]
        if (out->key_bound != 0 || !unsigned_kt(kt)) return out->key_bound ? INTSORT_ERR_INVALID_ARGUMENT
                                                                           : INTSORT_ERR_UNSUPPORTED;
        out->algo = INTSORT_BUCKET;
        out->num_buckets = 1u << out->digit_bits;
        out->key_bound = kt == INTSORT_U64 ? ~0ull : 0xffffffffull;
    }
    // signed and floating-point keys: radix sort with 8-bit digits only
    if (!unsigned_kt(kt) && (out->algo != INTSORT_RADIX_LSD || out->digit_bits != 8)) return INTSORT_ERR_UNSUPPORTED;
    if (out->num_buckets == 0) out->num_buckets = kt == INTSORT_U64 ? 65536u : 1024u;
    if (out->num_buckets > MAX_BUCKETS) return INTSORT_ERR_UNSUPPORTED;
    if (out->flags & ~(INTSORT_FLAG_NO_PASS_SKIP | INTSORT_FLAG_CHECK_SEGMENTS)) return INTSORT_ERR_INVALID_ARGUMENT;
    // a declared bound beyond the key width says nothing a measured range
    // would not, and 32-bit keys compute their bucket with 32-bit ranges
    if (kt == INTSORT_U32 && out->key_bound > 0xffffffffull) return INTSORT_ERR_INVALID_ARGUMENT;
    return INTSORT_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// true when [a, a+bytes) and [b, b+bytes) intersect without being identical
bool partial_overlap(const void *a, const void *b, size_t bytes)
{
    if (a == b || bytes == 0) return false;
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

// key-value buffers: values in and out either identical or disjoint, and no
// key buffer sharing memory with a value buffer
bool pair_buffers_ok(const void *keys_in, const void *keys_out, const void *vals_in, const void *vals_out,
                     uint64_t n, int kb)
{
    if (partial_overlap(vals_in, vals_out, n * 4)) return false;
    const void *kbufs[2] = {keys_in, keys_out};
    const void *vbufs[2] = {vals_in, vals_out};
    for (auto kp : kbufs)
        for (auto vp : vbufs) {
            const uintptr_t k0 = reinterpret_cast<uintptr_t>(kp), v0 = reinterpret_cast<uintptr_t>(vp);
            if (k0 < v0 + n * 4 && v0 < k0 + n * (size_t)kb) return false;
        }
    return true;
}

intsort_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return INTSORT_OK;
    if (e == hipErrorNotSupported) return INTSORT_ERR_UNSUPPORTED;
    return INTSORT_ERR_HIP;
}

// a planning context (device -1) validates and sizes but never launches
intsort_status set_device(const intsort_ctx *ctx)
{
    if (ctx->device < 0) return INTSORT_ERR_UNSUPPORTED;
    return hipSetDevice(ctx->device) == hipSuccess ? INTSORT_OK : INTSORT_ERR_HIP;
}

// workspace bytes of a plain (unsegmented) sort
size_t plain_workspace(int kb, bool pairs, uint64_t n, const intsort_options &o)
{
    if (n == 0) return 0;
    if (o.algo == INTSORT_RADIX_LSD) return radix_layout(kb, pairs, n, (int)o.digit_bits).total;
    return bucket_layout(kb, pairs, n, o).total;
}

intsort_status check_ws(const void *ws, size_t ws_bytes, size_t need)
{
    if (need == 0) return INTSORT_OK;
    if (!ws) return INTSORT_ERR_INVALID_ARGUMENT;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return INTSORT_ERR_MISALIGNED;
    if (ws_bytes < need) return INTSORT_ERR_WORKSPACE_TOO_SMALL;
    return INTSORT_OK;
}

intsort_status sort_common(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in, void *keys_out,
                           const uint32_t *vals_in, uint32_t *vals_out, bool pairs, uint64_t n,
                           const intsort_options *opts_in, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx || !valid_kt(kt)) return INTSORT_ERR_INVALID_ARGUMENT;
    intsort_options o;
    intsort_status st = read_opts(ctx, opts_in, kt, n, false, &o);
    if (st != INTSORT_OK) return st;
    if (n == 0) return INTSORT_OK;
    if (!keys_in || !keys_out) return INTSORT_ERR_INVALID_ARGUMENT;
    if (pairs && (!vals_in || !vals_out)) return INTSORT_ERR_INVALID_ARGUMENT;
    if (!aligned16(keys_in) || !aligned16(keys_out)) return INTSORT_ERR_MISALIGNED;
    if (pairs && (!aligned16(vals_in) || !aligned16(vals_out))) return INTSORT_ERR_MISALIGNED;
    const int kb = key_bytes_of(kt);
    if (partial_overlap(keys_in, keys_out, n * (size_t)kb)) return INTSORT_ERR_INVALID_ARGUMENT;
    if (pairs && !pair_buffers_ok(keys_in, keys_out, vals_in, vals_out, n, kb)) return INTSORT_ERR_INVALID_ARGUMENT;
    if (n > MAX_KEYS) return INTSORT_ERR_UNSUPPORTED;
    const size_t need = plain_workspace(kb, pairs, n, o);
    if ((st = check_ws(ws, ws_bytes, need)) != INTSORT_OK) return st;
    if ((st = set_device(ctx)) != INTSORT_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);

    if (o.algo == INTSORT_RADIX_LSD) {
        RadixCall c{};
        c.keys_in = keys_in;
        c.keys_out = keys_out;
        c.vals_in = pairs ? vals_in : nullptr;
        c.vals_out = pairs ? vals_out : nullptr;
        c.n = n;
        c.key_bytes = kb;
        c.pairs = pairs;
        c.bits = (int)o.digit_bits;
        c.order = key_order(kt);
        c.L = radix_layout(kb, pairs, n, c.bits);
        c.max_passes = c.L.g.passes;
        c.skip_constant_digits = !(o.flags & INTSORT_FLAG_NO_PASS_SKIP);
        if (o.max_passes != 0) {
            if ((int)o.max_passes < c.max_passes) c.max_passes = (int)o.max_passes;
            c.skip_constant_digits = false;
        }
        c.ws = static_cast<char *>(ws);
        c.timer = ctx->timer;
        return from_hip(radix_sort_run(c, s));
    }
    BucketCall b{};
    b.keys_in = keys_in;
    b.keys_out = keys_out;
    b.vals_in = pairs ? vals_in : nullptr;
    b.vals_out = pairs ? vals_out : nullptr;
    b.n = n;
    b.key_bytes = kb;
    b.pairs = pairs;
    b.opts = o;
    b.L = bucket_layout(kb, pairs, n, o);
    b.ws = static_cast<char *>(ws);
    b.timer = ctx->timer;
    return from_hip(bucket_sort_run(b, s));
}

}  // namespace

extern "C" {

const char *intsort_status_string(intsort_status s)
{
    switch (s) {
    case INTSORT_OK: return "ok";
    case INTSORT_ERR_INVALID_ARGUMENT: return "invalid argument";
    case INTSORT_ERR_MISALIGNED: return "misaligned pointer";
    case INTSORT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case INTSORT_ERR_UNSUPPORTED: return "unsupported option or size";
    case INTSORT_ERR_OVER_BUDGET: return "request exceeds the memory budget";
    case INTSORT_ERR_HIP: return "HIP runtime error";
    case INTSORT_ERR_INTERNAL: return "internal error";
    case INTSORT_ERR_NOT_READY: return "not ready";
    }
    return "unknown status";
}

void intsort_default_options(intsort_options *o)
{
    if (!o) return;
    *o = intsort_options{};
    o->struct_size = sizeof(intsort_options);
    o->algo = INTSORT_RADIX_LSD;
    o->digit_bits = 8;
}

intsort_status intsort_create(intsort_ctx **ctx, int hip_device)
{
    try {
        if (!ctx) return INTSORT_ERR_INVALID_ARGUMENT;
        *ctx = nullptr;
        if (hip_device < -1) return INTSORT_ERR_INVALID_ARGUMENT;
        if (hip_device >= 0) {
            int count = 0;
            if (hipGetDeviceCount(&count) != hipSuccess) return INTSORT_ERR_HIP;
            if (hip_device >= count) return INTSORT_ERR_INVALID_ARGUMENT;
        }
        intsort_ctx *c = new (std::nothrow) intsort_ctx;
        if (!c) return INTSORT_ERR_INTERNAL;
        c->device = hip_device;
        c->cus = hip_device >= 0 ? device_cu_count(hip_device) : 0;
        c->dev_key = tune_device_key(hip_device);
        // the tuned defaults, when the default table file exists
        const std::string path = tune_default_path();
        if (!path.empty()) tune_load(path.c_str(), &c->tune);
        if (hip_device >= 0) {
            // once per device: the pass kernel's stable rank needs LDS atomics
            // that serve the lanes of one instruction in lane order; and the
            // device address of the no-allocation entry point's workspace
            int prev = 0;
            bool lane_order = false;
            const bool ran = hipGetDevice(&prev) == hipSuccess && hipSetDevice(hip_device) == hipSuccess &&
                             rank_check(hip_device, &lane_order) == hipSuccess &&
                             noalloc_setup(hip_device) == hipSuccess;
            hipSetDevice(prev);
            if (!ran || !lane_order) {
                delete c;
                return ran ? INTSORT_ERR_UNSUPPORTED : INTSORT_ERR_HIP;
            }
        }
        *ctx = c;
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_timing_enable(intsort_ctx *ctx, int enable)
{
    try {
        if (!ctx) return INTSORT_ERR_INVALID_ARGUMENT;
        if (enable && !ctx->timer) {
            if (ctx->device < 0) return INTSORT_ERR_UNSUPPORTED;
            intsort_status st = set_device(ctx);
            if (st != INTSORT_OK) return st;
            Timer *t = new (std::nothrow) Timer;
            if (!t) return INTSORT_ERR_INTERNAL;
            for (int i = 0; i < Timer::CAP; i++) {
                if (hipEventCreate(&t->ev[i]) != hipSuccess) {
                    for (int j = 0; j < i; j++) (void)hipEventDestroy(t->ev[j]);
                    delete t;
                    return INTSORT_ERR_HIP;
                }
            }
            ctx->timer = t;
        } else if (!enable && ctx->timer) {
            for (int i = 0; i < Timer::CAP; i++) (void)hipEventDestroy(ctx->timer->ev[i]);
            delete ctx->timer;
            ctx->timer = nullptr;
        }
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_timing_read(intsort_ctx *ctx, intsort_kernel_time *out, uint32_t capacity, uint32_t *count)
{
    try {
        if (!ctx || !count || (capacity > 0 && !out)) return INTSORT_ERR_INVALID_ARGUMENT;
        Timer *t = ctx->timer;
        *count = 0;
        if (!t || t->used == 0) return INTSORT_OK;
        if (hipEventSynchronize(t->ev[t->used - 1]) != hipSuccess) return INTSORT_ERR_HIP;
        uint32_t m = 0;
        for (int i = 1; i < t->used && m < capacity; i++) {
            if (t->kind[i] == Timer::CALL_START) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, t->ev[i - 1], t->ev[i]) != hipSuccess) return INTSORT_ERR_HIP;
            out[m].kind = t->kind[i];
            out[m].index = t->index[i];
            out[m].ms = ms;
            m++;
        }
        *count = m;
        t->used = 0;
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_destroy(intsort_ctx *ctx)
{
    if (ctx && ctx->timer) intsort_timing_enable(ctx, 0);
    delete ctx;
    return INTSORT_OK;
}

intsort_status intsort_load_tuning(intsort_ctx *ctx, const char *path)
{
    try {
        if (!ctx) return INTSORT_ERR_INVALID_ARGUMENT;
        if (!path) {
            ctx->tune.clear();
            return INTSORT_OK;
        }
        std::vector<TuneEntry> t;
        if (!tune_load(path, &t)) return INTSORT_ERR_INVALID_ARGUMENT;
        ctx->tune = std::move(t);
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_device_key(const intsort_ctx *ctx, char *buf, size_t len)
{
    if (!ctx || !buf || len == 0) return INTSORT_ERR_INVALID_ARGUMENT;
    if (ctx->dev_key.size() + 1 > len) return INTSORT_ERR_INVALID_ARGUMENT;
    for (size_t i = 0; i < ctx->dev_key.size(); i++) buf[i] = ctx->dev_key[i];
    buf[ctx->dev_key.size()] = '\0';
    return INTSORT_OK;
}

intsort_status intsort_workspace_size(const intsort_ctx *ctx, intsort_key_type kt, int has_values, uint64_t n,
                                      uint64_t num_segments, const intsort_options *opts, size_t *bytes)
{
    try {
        if (!ctx || !bytes || !valid_kt(kt)) return INTSORT_ERR_INVALID_ARGUMENT;
        intsort_options o;
        intsort_status st = read_opts(ctx, opts, kt, n, num_segments != 0, &o);
        if (st != INTSORT_OK) return st;
        if (n > MAX_KEYS) return INTSORT_ERR_UNSUPPORTED;
        const int kb = key_bytes_of(kt);
        size_t plain = plain_workspace(kb, has_values != 0, n, o);
        // the step entry points share the plain layout's counters
        if (plain == 0) plain = radix_layout(kb, false, 1, (int)o.digit_bits).total;
        if (num_segments == 0) {
            *bytes = plain;
        } else {
            if (num_segments > MAX_SEGMENTS || !unsigned_kt(kt)) return INTSORT_ERR_UNSUPPORTED;
            *bytes = segmented_layout(kb, has_values != 0, n, num_segments, o).total;
        }
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_sort_keys(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in, void *keys_out,
                                 uint64_t n, const intsort_options *opts, void *workspace,
                                 size_t workspace_bytes, void *stream)
{
    try {
        return sort_common(ctx, kt, keys_in, keys_out, nullptr, nullptr, false, n, opts, workspace,
                           workspace_bytes, stream);
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_sort_pairs(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in, void *keys_out,
                                  const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                                  const intsort_options *opts, void *workspace, size_t workspace_bytes,
                                  void *stream)
{
    try {
        return sort_common(ctx, kt, keys_in, keys_out, vals_in, vals_out, true, n, opts, workspace,
                           workspace_bytes, stream);
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

static intsort_status segmented_common(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in,
                                       void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                                       bool pairs, uint64_t n_total, uint64_t num_segments,
                                       const uint64_t *d_offsets, const intsort_options *opts_in, void *ws,
                                       size_t ws_bytes, void *stream)
{
    if (!ctx || !valid_kt(kt)) return INTSORT_ERR_INVALID_ARGUMENT;
    if (!unsigned_kt(kt)) return INTSORT_ERR_UNSUPPORTED;
    intsort_options o;
    intsort_status st = read_opts(ctx, opts_in, kt, n_total, true, &o);
    if (st != INTSORT_OK) return st;
    if (num_segments == 0 && n_total != 0) return INTSORT_ERR_INVALID_ARGUMENT;
    if (n_total == 0 || num_segments == 0) return INTSORT_OK;
    if (o.digit_bits != 4 && o.digit_bits != 8) return INTSORT_ERR_UNSUPPORTED;
    if (!d_offsets || !keys_in || !keys_out) return INTSORT_ERR_INVALID_ARGUMENT;
    if (pairs && (!vals_in || !vals_out)) return INTSORT_ERR_INVALID_ARGUMENT;
    if (!aligned16(keys_in) || !aligned16(keys_out)) return INTSORT_ERR_MISALIGNED;
    if (pairs && (!aligned16(vals_in) || !aligned16(vals_out))) return INTSORT_ERR_MISALIGNED;
    const int kb = key_bytes_of(kt);
    if (partial_overlap(keys_in, keys_out, n_total * (size_t)kb)) return INTSORT_ERR_INVALID_ARGUMENT;
    if (pairs && !pair_buffers_ok(keys_in, keys_out, vals_in, vals_out, n_total, kb))
        return INTSORT_ERR_INVALID_ARGUMENT;
    if (n_total > MAX_KEYS || num_segments > MAX_SEGMENTS) return INTSORT_ERR_UNSUPPORTED;
    const SegLayout L = segmented_layout(kb, pairs, n_total, num_segments, o);
    if ((st = check_ws(ws, ws_bytes, L.total)) != INTSORT_OK) return st;
    if ((st = set_device(ctx)) != INTSORT_OK) return st;
    SegCall c{};
    c.keys_in = keys_in;
    c.keys_out = keys_out;
    c.vals_in = pairs ? vals_in : nullptr;
    c.vals_out = pairs ? vals_out : nullptr;
    c.n = n_total;
    c.num_segments = num_segments;
    c.offsets = d_offsets;
    c.descs = nullptr;
    c.key_bytes = kb;
    c.pairs = pairs;
    c.opts = o;
    c.L = L;
    c.ws = static_cast<char *>(ws);
    c.timer = ctx->timer;
    return from_hip(segmented_sort_run(c, static_cast<hipStream_t>(stream)));
}

intsort_status intsort_segmented_sort_keys(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in,
                                           void *keys_out, uint64_t n_total, uint64_t num_segments,
                                           const uint64_t *d_offsets, const intsort_options *opts,
                                           void *workspace, size_t workspace_bytes, void *stream)
{
    try {
        return segmented_common(ctx, kt, keys_in, keys_out, nullptr, nullptr, false, n_total, num_segments,
                                d_offsets, opts, workspace, workspace_bytes, stream);
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_segmented_sort_pairs(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in,
                                            void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                                            uint64_t n_total, uint64_t num_segments, const uint64_t *d_offsets,
                                            const intsort_options *opts, void *workspace,
                                            size_t workspace_bytes, void *stream)
{
    try {
        return segmented_common(ctx, kt, keys_in, keys_out, vals_in, vals_out, true, n_total, num_segments,
                                d_offsets, opts, workspace, workspace_bytes, stream);
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_batched_sort_keys(intsort_ctx *ctx, intsort_key_type kt, const intsort_segment_desc *d_descs,
                                         uint64_t count, uint64_t total_keys, const intsort_options *opts,
                                         void *workspace, size_t workspace_bytes, void *stream)
{
    try {
        if (!ctx || !valid_kt(kt)) return INTSORT_ERR_INVALID_ARGUMENT;
        if (!unsigned_kt(kt)) return INTSORT_ERR_UNSUPPORTED;
        intsort_options o;
        intsort_status st = read_opts(ctx, opts, kt, total_keys, true, &o);
        if (st != INTSORT_OK) return st;
        if (count == 0 || total_keys == 0) return INTSORT_OK;
        if (!d_descs) return INTSORT_ERR_INVALID_ARGUMENT;
        if (o.digit_bits != 4 && o.digit_bits != 8) return INTSORT_ERR_UNSUPPORTED;
        if (total_keys > MAX_KEYS || count > MAX_SEGMENTS) return INTSORT_ERR_UNSUPPORTED;
        const int kb = key_bytes_of(kt);
        const SegLayout L = segmented_layout(kb, false, total_keys, count, o);
        if ((st = check_ws(workspace, workspace_bytes, L.total)) != INTSORT_OK) return st;
        if ((st = set_device(ctx)) != INTSORT_OK) return st;
        SegCall c{};
        c.n = total_keys;
        c.num_segments = count;
        c.descs = d_descs;
        c.key_bytes = kb;
        c.pairs = false;
        c.opts = o;
        c.L = L;
        c.ws = static_cast<char *>(workspace);
        c.timer = ctx->timer;
        return from_hip(segmented_sort_run(c, static_cast<hipStream_t>(stream)));
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_digit_histogram(intsort_ctx *ctx, intsort_key_type kt, const void *keys, uint64_t n,
                                       uint32_t digit_bits, uint32_t *counts, void *workspace,
                                       size_t workspace_bytes, void *stream)
{
    try {
        if (!ctx || !valid_kt(kt) || !counts) return INTSORT_ERR_INVALID_ARGUMENT;
        if (!unsigned_kt(kt)) return INTSORT_ERR_UNSUPPORTED;
        if (digit_bits != 4 && digit_bits != 8 && digit_bits != 11) return INTSORT_ERR_UNSUPPORTED;
        if (n > 0 && !keys) return INTSORT_ERR_INVALID_ARGUMENT;
        if (n > 0 && !aligned16(keys)) return INTSORT_ERR_MISALIGNED;
        if (n >= (1ull << 32)) return INTSORT_ERR_UNSUPPORTED;
        const int kb = key_bytes_of(kt);
        RadixCall c{};
        c.keys_in = keys;
        c.n = n;
        c.key_bytes = kb;
        c.bits = (int)digit_bits;
        c.L = radix_layout(kb, false, n > 0 ? n : 1, c.bits);
        c.max_passes = c.L.g.passes;
        intsort_status st = check_ws(workspace, workspace_bytes, (size_t)CTR_WORDS * 4);
        if (st != INTSORT_OK) return st;
        if ((st = set_device(ctx)) != INTSORT_OK) return st;
        c.ws = static_cast<char *>(workspace);
        return from_hip(digit_histogram_run(c, counts, static_cast<hipStream_t>(stream)));
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_minmax(intsort_ctx *ctx, intsort_key_type kt, const void *keys, uint64_t n,
                              uint64_t *minmax, void *stream)
{
    try {
        if (!ctx || !valid_kt(kt) || !minmax || n == 0 || !keys) return INTSORT_ERR_INVALID_ARGUMENT;
        if (!unsigned_kt(kt)) return INTSORT_ERR_UNSUPPORTED;
        if (!aligned16(keys)) return INTSORT_ERR_MISALIGNED;
        intsort_status st = set_device(ctx);
        if (st != INTSORT_OK) return st;
        return from_hip(minmax_run(key_bytes_of(kt), keys, n, minmax, static_cast<hipStream_t>(stream)));
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_bucket_histogram(intsort_ctx *ctx, intsort_key_type kt, const void *keys, uint64_t n,
                                        const uint64_t *minmax, uint32_t num_buckets, uint32_t *counts,
                                        void *stream)
{
    try {
        if (!ctx || !valid_kt(kt) || !minmax || !counts || num_buckets == 0) return INTSORT_ERR_INVALID_ARGUMENT;
        if (!unsigned_kt(kt)) return INTSORT_ERR_UNSUPPORTED;
        if (n > 0 && !keys) return INTSORT_ERR_INVALID_ARGUMENT;
        // the kernel reads the keys as 16-byte vectors
        if (n > 0 && !aligned16(keys)) return INTSORT_ERR_MISALIGNED;
        if (num_buckets > MAX_BUCKETS || n >= (1ull << 32)) return INTSORT_ERR_UNSUPPORTED;
        intsort_status st = set_device(ctx);
        if (st != INTSORT_OK) return st;
        return from_hip(bucket_histogram_run(key_bytes_of(kt), keys, n, minmax, num_buckets, counts,
                                             static_cast<hipStream_t>(stream)));
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_read_device_error(intsort_ctx *ctx, const void *workspace, size_t workspace_bytes,
                                         uint32_t *error_word, void *stream)
{
    try {
        if (!ctx || !workspace || !error_word) return INTSORT_ERR_INVALID_ARGUMENT;
        // every workspace layout starts with the counters block
        const size_t at = (size_t)CTR_ERROR * 4;
        if (workspace_bytes < (size_t)CTR_WORDS * 4) return INTSORT_ERR_INVALID_ARGUMENT;
        intsort_status st = set_device(ctx);
        if (st != INTSORT_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (hipMemcpyAsync(error_word, static_cast<const char *>(workspace) + at, 4, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
            return INTSORT_ERR_HIP;
        return from_hip(hipStreamSynchronize(s));
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_capture_begin(intsort_ctx *ctx, void *stream)
{
    try {
        if (!ctx || !stream) return INTSORT_ERR_INVALID_ARGUMENT;
        if (ctx->timer) return INTSORT_ERR_UNSUPPORTED;   // event records would be captured
        intsort_status st = set_device(ctx);
        if (st != INTSORT_OK) return st;
        return from_hip(hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal));
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_capture_end(intsort_ctx *ctx, void *stream, intsort_graph **graph)
{
    try {
        if (!ctx || !stream || !graph) return INTSORT_ERR_INVALID_ARGUMENT;
        *graph = nullptr;
        intsort_status st = set_device(ctx);
        if (st != INTSORT_OK) return st;
        hipGraph_t g = nullptr;
        // ending the capture also ends it after a failed call in between
        if (hipStreamEndCapture(static_cast<hipStream_t>(stream), &g) != hipSuccess || !g) return INTSORT_ERR_HIP;
        intsort_graph *h = new (std::nothrow) intsort_graph;
        if (!h) {
            (void)hipGraphDestroy(g);
            return INTSORT_ERR_INTERNAL;
        }
        h->device = ctx->device;
        h->graph = g;
        if (hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            delete h;
            return INTSORT_ERR_HIP;
        }
        *graph = h;
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_graph_launch(intsort_graph *graph, void *stream)
{
    try {
        if (!graph || !graph->exec) return INTSORT_ERR_INVALID_ARGUMENT;
        if (hipSetDevice(graph->device) != hipSuccess) return INTSORT_ERR_HIP;
        return from_hip(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_graph_destroy(intsort_graph *graph)
{
    if (!graph) return INTSORT_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return INTSORT_OK;
}

}  // extern "C"
