/*
 * intsort.h -- C ABI of an MI355X (gfx950) integer sorting library for the two
 * methods compared in "Comparison of Bucket Sort and RADIX Sort"
 * (P. Horsmalahti, arXiv 1206.3511): LSD radix sort (section 2.5,
 * Algorithm 4, with the counting sort of section 2.4, Algorithm 3, as its
 * stable digit sort) and bucket sort (section 2.3, Algorithm 2).
 *
 * Problem statement (section 2): a call takes a sequence of unsigned
 * integers and produces the permutation of it that is in nondecreasing
 * order.  The key-value calls produce the stable permutation: keys that
 * compare equal keep their input order (section 2, stability), so for every
 * input exactly one output is correct, and radix and bucket sort return the
 * same bytes.
 *
 * Conventions shared by every call
 *   - Memory.  Every key, value, offset and workspace pointer is a DEVICE
 *     pointer on the context's device, owned by the caller.  The library
 *     owns only the context (host memory).  Sort calls never allocate, never
 *     synchronise the host with the device and never read device memory back
 *     to the host: they enqueue kernels on `stream` and return.
 *   - stream.  A hipStream_t passed as void*; NULL means the null stream.
 *   - Layout.  Keys are contiguous little-endian uint32 or uint64; values
 *     are contiguous uint32, one per key.  Input and output base pointers
 *     must be 16-byte aligned.  keys_in == keys_out (in place) is allowed;
 *     any other overlap between an input and an output is an error.  The
 *     same holds for values.
 *   - Workspace.  A device buffer of at least the size returned by
 *     intsort_workspace_size() for the same arguments, 256-byte aligned.  Its
 *     contents on entry do not matter; it must not be used by another call
 *     that runs at the same time.
 *   - Errors.  Argument errors are detected on the host and returned before
 *     anything is enqueued.  A failed kernel launch returns
 *     INTSORT_ERR_HIP.  Faults during execution surface at the caller's next
 *     synchronisation of `stream`.  No C++ exception crosses this ABI.
 *   - Threads.  Calls are reentrant when they use different workspaces.
 */
#ifndef INTSORT_H
#define INTSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * The enumerations below are passed as 32-bit unsigned integers: that is the
 * type a C compiler gives them (no enumerator is negative), and C++ callers
 * and the library see them with that fixed underlying type, so an
 * out-of-range value from a C caller is an ordinary value there too, and is
 * rejected with INTSORT_ERR_INVALID_ARGUMENT.
 */
#ifdef __cplusplus
#define INTSORT_ENUM(name) enum name : uint32_t
#else
#define INTSORT_ENUM(name) enum name
#endif

typedef INTSORT_ENUM(intsort_status) {
    INTSORT_OK = 0,
    INTSORT_ERR_INVALID_ARGUMENT = 1, /* null pointer with n > 0, bad enum, overlap */
    INTSORT_ERR_MISALIGNED = 2,       /* a base pointer is not 16-byte aligned */
    INTSORT_ERR_WORKSPACE_TOO_SMALL = 3,
    INTSORT_ERR_UNSUPPORTED = 4,      /* option value or size the library does not handle */
    INTSORT_ERR_OVER_BUDGET = 5,      /* serving: a request larger than the whole budget */
    INTSORT_ERR_HIP = 6,              /* a HIP runtime call or kernel launch failed */
    INTSORT_ERR_INTERNAL = 7,
    INTSORT_ERR_NOT_READY = 8         /* serving: the ticket has not completed yet */
} intsort_status;

/*
 * Key types.  The paper sorts non-negative integers (section 2); unsigned
 * keys are that case.  Signed and floating-point keys are sorted by radix
 * sort with 8-bit digits only (any other algorithm, digit width or entry
 * point returns INTSORT_ERR_UNSUPPORTED): each digit is taken from an
 * order-preserving image of the key's bits, and the original bits are what
 * move, so the output holds the input's bit patterns.
 *   I32/I64  two's complement, ascending by value.
 *   F32/F64  IEEE 754 binary32/binary64 in the totalOrder of IEEE 754-2019
 *            section 5.10: -NaN < -inf < finite negatives < -0 < +0 <
 *            finite positives < +inf < +NaN, NaNs ordered by their payload
 *            bits; keys with identical bits keep their input order.
 */
typedef INTSORT_ENUM(intsort_key_type) {
    INTSORT_U32 = 0,
    INTSORT_U64 = 1,
    INTSORT_I32 = 2,
    INTSORT_I64 = 3,
    INTSORT_F32 = 4,
    INTSORT_F64 = 5
} intsort_key_type;

typedef INTSORT_ENUM(intsort_algo) {
    INTSORT_RADIX_LSD = 0, /* Algorithm 4 over a stable per-digit counting sort */
    INTSORT_BUCKET = 1,    /* Algorithm 2: range, bucket scatter, per-bucket sort;
                              keys found already in nondecreasing order by the
                              first full read (min/max, or with key_bound the
                              bucket histogram) skip the later steps and are
                              copied to the output */
    INTSORT_RADIX_MSD = 2  /* most significant digit first (section 2.5's other
                              variant): one stable counting-sort pass on the
                              top r = digit_bits bits of the key, then every one
                              of the 2^r buckets sorted on its remaining bits,
                              least significant digit first.  This is bucket
                              sort over the declared range [0, 2^key_bits - 1]
                              with 2^r buckets, and takes its options
                              (max_passes 1 stops after the top-digit pass);
                              num_buckets is ignored, key_bound must be 0.
                              Unsigned keys only. */
} intsort_algo;

/* option flags */
#define INTSORT_FLAG_NO_PASS_SKIP 0x1u /* radix: run every digit pass even when
                                          a digit is the same for all keys */
#define INTSORT_FLAG_CHECK_SEGMENTS 0x2u /* segmented and batched: first check
                                            on the device the layout the caller
                                            gave (offsets nondecreasing from 0 to
                                            n_total; every array at most
                                            total_keys long, with non-null,
                                            16-byte aligned buffers when not
                                            empty, and all of them together
                                            at most total_keys long); if a
                                            check fails, set
                                            INTSORT_DEVERR_BAD_SEGMENTS in the
                                            device error word and sort nothing
                                            (outputs unspecified); the other
                                            calls ignore the flag */

/*
 * Options.  A zero digit_bits, num_buckets or lds_cutoff means "tuned": the
 * value the context's tuning table (intsort_load_tuning) holds for the
 * context's device, the key width and the size class floor(log2 n) (n_total
 * for segmented and batched calls), when the table has one and the call can
 * take it; otherwise the library default given below.  Other zero fields
 * mean the library default.  A NULL options pointer means all zero.
 *   digit_bits   radix digit width r: 0 (tuned for plain radix sorts of
 *                unsigned keys and for segmented and batched calls, else
 *                8) | 4 | 8 | 11.  The number of passes is
 *                ceil(key_bits / r) (Algorithm 4's d for a key of key_bits
 *                bits).  Segmented and batched calls take 4 or 8 (the
 *                digit passes of segments longer than lds_cutoff; shorter
 *                ones are sorted on chip, with the same result) and return
 *                INTSORT_ERR_UNSUPPORTED for 11.
 *   num_buckets  bucket sort: number of buckets B, 1..2^30 (default 1024
 *                for u32, 65536 for u64).  The bucket of key k is
 *                floor((k - min) * B / (max - min + 1)), exact.
 *   key_bound    bucket sort: 0 = measure min and max of the keys on the
 *                device.  Otherwise the caller declares that every key lies
 *                in [0, key_bound], the bound M of section 2.3, and the
 *                bucket of k is floor(k * B / (key_bound + 1)); with
 *                B = n this is Algorithm 2's map.  A key above the bound
 *                goes to the last bucket, so the output is still sorted.
 *   lds_cutoff   bucket/segmented/batched: segments of at most this many
 *                keys are sorted by one workgroup entirely in LDS, longer
 *                ones by all workgroups together (0 or more than one
 *                workgroup holds = the largest size one workgroup holds:
 *                16384 32-bit or 8192 64-bit keys).
 *   max_passes   radix: stop after this many digit passes (0 = all).  With a
 *                value p the output is the input stably sorted on its low
 *                p*r bits; this exposes the intermediate arrays of
 *                Algorithm 4.  Implies INTSORT_FLAG_NO_PASS_SKIP.
 *                bucket: 1 stops after the scatter: the output holds every
 *                bucket's keys in input order, buckets concatenated
 *                (Algorithm 2 before its per-bucket sorts).
 *   flags        INTSORT_FLAG_*.
 */
typedef struct intsort_options {
    uint32_t struct_size; /* sizeof(intsort_options) */
    uint32_t algo;        /* intsort_algo */
    uint32_t digit_bits;
    uint32_t num_buckets;
    uint32_t lds_cutoff;
    uint32_t max_passes;
    uint32_t flags;
    uint32_t reserved;
    uint64_t key_bound;
} intsort_options;

typedef struct intsort_ctx intsort_ctx;

/* Human-readable name of a status code; never NULL. */
const char *intsort_status_string(intsort_status s);

/*
 * Tuning table of a context (the autotuner's choices, which zero option
 * fields take; any choice gives the same bytes, only the speed differs).
 * A text file, one entry per line, tab-separated:
 *   device key, kind, key bytes (4 | 8), size class, value
 * with kind "radix" (value: digit_bits), "bucket" (num_buckets),
 * "segmented" (lds_cutoff) or "segmented_bits" (digit_bits of segmented and
 * batched calls).  The device key is the one intsort_device_key
 * gives; "*" matches every device (and a planning context, whose key is
 * empty).  '#' starts a comment line; lines that do not parse, and values a
 * call cannot take, are ignored.  intsort_create loads the file named by
 * $INTSORT_TUNE_FILE, else ~/.cache/intsort/tune.tsv, when it exists.
 * intsort_load_tuning replaces the context's table with the file at `path`
 * (INTSORT_ERR_INVALID_ARGUMENT if it cannot be read; the table is then
 * unchanged); path == NULL empties it.  Not thread-safe against calls on the
 * same context.
 */
intsort_status intsort_load_tuning(intsort_ctx *ctx, const char *path);

/* The device key of a context (its device's name, architecture and HIP
 * runtime version; empty for a planning context) into buf, NUL-terminated;
 * INTSORT_ERR_INVALID_ARGUMENT when it does not fit in len bytes. */
intsort_status intsort_device_key(const intsort_ctx *ctx, char *buf, size_t len);

/* Fills *opts with the defaults (radix, 8-bit digits). */
void intsort_default_options(intsort_options *opts);

/*
 * Creates a context bound to HIP device `hip_device` (reads its properties).
 * The first context of a device also runs, once per process, a short
 * self-test kernel: the digit passes rank keys stably with LDS atomic adds,
 * which needs the lanes of one add instruction that hit the same word to be
 * served in lane order.  The test allocates and frees 4 bytes of device
 * memory and waits for its kernel; a device that fails it is refused with
 * INTSORT_ERR_UNSUPPORTED.  The calling thread's current device is left as
 * it was.  *ctx receives the handle; destroy it with
 * intsort_destroy (destroying NULL does nothing and returns INTSORT_OK).
 * hip_device = -1 makes a planning context that touches no
 * device: workspace sizes and argument checks work on it, and a sort call
 * whose arguments pass the checks returns INTSORT_ERR_UNSUPPORTED.
 */
intsort_status intsort_create(intsort_ctx **ctx, int hip_device);
intsort_status intsort_destroy(intsort_ctx *ctx);

/*
 * Bytes of workspace that a sort of n keys of type kt (with values when
 * has_values != 0; in num_segments segments for the segmented calls, 0 for
 * the plain calls) needs under `opts` (NULL = defaults).  The size is
 * monotone in n and num_segments.
 */
intsort_status intsort_workspace_size(const intsort_ctx *ctx, intsort_key_type kt,
                                      int has_values, uint64_t n, uint64_t num_segments,
                                      const intsort_options *opts, size_t *bytes);

/*
 * Sorts n keys (section 2): keys_out receives the nondecreasing permutation
 * of keys_in (in the order of intsort_key_type for signed and floating-point
 * keys).  opts->algo picks LSD radix (section 2.5), bucket (section 2.3) or
 * MSD-first radix sort; all give identical bytes.  n == 0 is a no-op.
 */
intsort_status intsort_sort_keys(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in,
                                 void *keys_out, uint64_t n, const intsort_options *opts,
                                 void *workspace, size_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * intsort_sort_keys with no workspace argument.  Its workspace is the
 * library's own device array of INTSORT_NOALLOC_SCRATCH_MB MiB, one per
 * device, whose address intsort_create takes once per device; the array is
 * held until the process ends.  The call allocates nothing and the caller
 * still passes keys_in and keys_out (device memory, as for
 * intsort_sort_keys, with the same argument rules and results).
 * Errors: those of intsort_sort_keys, and INTSORT_ERR_WORKSPACE_TOO_SMALL
 * when intsort_workspace_size for the call exceeds the array (radix sort of
 * 32-bit keys with 8-bit digits fits about 15 million keys, bucket sort
 * about 7 million).  Every call on one device shares that device's array:
 * calls that overlap on one device (other streams, other threads) race and
 * give undefined results; calls in one stream's order are safe.
 */
#define INTSORT_NOALLOC_SCRATCH_MB 64
intsort_status intsort_sort_keys_noalloc(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in,
                                         void *keys_out, uint64_t n, const intsort_options *opts,
                                         void *stream);

/*
 * Stable key-value sort (section 2, stability): keys as intsort_sort_keys,
 * and vals_out[i] is the value that travelled with keys_out[i]; among equal
 * keys, values keep their input order.
 */
intsort_status intsort_sort_pairs(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in,
                                  void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                                  uint64_t n, const intsort_options *opts, void *workspace,
                                  size_t workspace_bytes, void *stream);

/*
 * Segmented sort: the packed array of n_total keys is split by the device
 * array d_offsets[num_segments + 1] (uint64, nondecreasing, d_offsets[0] = 0,
 * d_offsets[num_segments] = n_total; empty segments allowed) and every
 * segment [d_offsets[s], d_offsets[s+1]) is sorted on its own; nothing moves
 * between segments.  The offsets live on the device and are not validated
 * on the host.  Segment starts need no alignment.  num_segments = 0 with
 * n_total > 0 is INTSORT_ERR_INVALID_ARGUMENT (no segment holds the keys).
 */
intsort_status intsort_segmented_sort_keys(intsort_ctx *ctx, intsort_key_type kt,
                                           const void *keys_in, void *keys_out, uint64_t n_total,
                                           uint64_t num_segments, const uint64_t *d_offsets,
                                           const intsort_options *opts, void *workspace,
                                           size_t workspace_bytes, void *stream);

intsort_status intsort_segmented_sort_pairs(intsort_ctx *ctx, intsort_key_type kt,
                                            const void *keys_in, void *keys_out,
                                            const uint32_t *vals_in, uint32_t *vals_out,
                                            uint64_t n_total, uint64_t num_segments,
                                            const uint64_t *d_offsets,
                                            const intsort_options *opts, void *workspace,
                                            size_t workspace_bytes, void *stream);

/*
 * One array of a batch: device input and output buffers (keys_in ==
 * keys_out sorts in place) and the number of keys.  16-byte aligned bases.
 */
typedef struct intsort_segment_desc {
    const void *keys_in;
    void *keys_out;
    uint64_t n;
} intsort_segment_desc;

/*
 * Batched sort, the serving form of the segmented sort: `count` separate
 * arrays of key type kt, described by the DEVICE array d_descs[count], are
 * sorted in one set of launches; array i's keys_out receives the
 * nondecreasing permutation of its keys_in.  total_keys must be at least the
 * sum of all n (it sizes the work; the descriptors are not read on the host).
 * The workspace is intsort_workspace_size(ctx, kt, 0, total_keys, count,
 * opts, &bytes).  Keys only; 8-bit digits.
 */
intsort_status intsort_batched_sort_keys(intsort_ctx *ctx, intsort_key_type kt,
                                         const intsort_segment_desc *d_descs, uint64_t count,
                                         uint64_t total_keys, const intsort_options *opts,
                                         void *workspace, size_t workspace_bytes, void *stream);

/*
 * Serving loop with continuous batching.  A server owns a worker thread and
 * `slots` streams (1..4), each with a workspace for batches of up to 2^27
 * keys, allocated once in intsort_server_create on the context's device.  Requests are (key type, device input, device output,
 * n); the caller owns those arrays and must keep them alive until the
 * request completes.  A request's footprint is 3*w*n + 4*n + 4096 bytes for
 * w-byte keys (its two arrays plus its share of a batch workspace); one
 * larger than hbm_budget_bytes, or with more than 2^27 keys, is refused with
 * INTSORT_ERR_OVER_BUDGET.  Whenever a slot is free the worker admits waiting
 * requests in arrival order while their footprints fit the budget next to
 * the requests still running, launches them as one batched sort per key type
 * (at most max_batch arrays each) and, when the batch's completion event has
 * fired, marks them done with latency = completion seen by the worker -
 * submission.  max_batch = 1 with slots = 1 is the plain one-request-per-
 * launch path.
 *
 * A batch whose launch fails (a HIP call returns an error) or whose
 * completion event reports an error fails as a whole: each of its requests
 * finishes as failed, after whatever part of the batch was enqueued has
 * finished, and the worker goes on with the next batch.
 *
 * intsort_server_poll: *done = 1 and INTSORT_OK when finished,
 *   INTSORT_ERR_NOT_READY while waiting or running, *done = 1 and
 *   INTSORT_ERR_HIP when the request failed.
 * intsort_server_completed: tickets (and latencies) finished since the last
 *   call, failed ones included, oldest first, at most `capacity`; returns
 *   INTSORT_ERR_HIP when at least one listed ticket failed (poll tells which).
 *   Finished tickets are forgotten, failed ones once poll has reported them.
 * intsort_server_drain: blocks until every submitted request has finished;
 *   INTSORT_ERR_HIP when a request failed since the previous drain.
 * intsort_server_destroy: drains, stops the worker, frees the workspaces.
 * submit, poll, completed, drain and fail_next_launches may be called from
 * several threads at once (the server serialises them); destroy must not
 * overlap any other call on the same server.  A finished ticket that
 * completed has listed is forgotten whichever thread submitted it: poll on
 * it then returns INTSORT_ERR_INVALID_ARGUMENT.
 */
typedef struct intsort_server intsort_server;

intsort_status intsort_server_create(intsort_ctx *ctx, uint64_t hbm_budget_bytes, uint32_t max_batch,
                                     uint32_t slots, intsort_server **server);
intsort_status intsort_server_submit(intsort_server *server, intsort_key_type kt, const void *d_in,
                                     void *d_out, uint64_t n, uint64_t *ticket);
intsort_status intsort_server_poll(intsort_server *server, uint64_t ticket, int *done, double *latency_s);
intsort_status intsort_server_completed(intsort_server *server, uint64_t *tickets, double *latency_s,
                                        uint32_t capacity, uint32_t *count);
intsort_status intsort_server_drain(intsort_server *server);
intsort_status intsort_server_destroy(intsort_server *server);

/*
 * For tests of the failure path (a fault-injection hook): the next `count`
 * batch launches of the server's worker fail before anything is enqueued,
 * as when the launch's first HIP call returns an error, so their requests
 * finish as failed as described above.  count = 0 cancels what is left.
 */
intsort_status intsort_server_fail_next_launches(intsort_server *server, uint32_t count);

/*
 * Step-level entry points.  Each runs one step of the sorts above on its own
 * so that the step can be checked against its definition.  Outputs are
 * device arrays owned by the caller.
 *
 * intsort_digit_histogram: counts[p * 2^r + v] = number of keys whose digit p
 *   ((k >> p*r) & (2^r - 1)) equals v, for every pass p < ceil(key_bits/r),
 *   from one read of the keys (the count loop of Algorithm 3, for all digits
 *   at once).  counts is uint32 [passes * 2^r]; n < 2^32.
 * intsort_minmax: minmax[0] = smallest key, minmax[1] = largest key (as
 *   uint64, also for 32-bit keys); n >= 1.
 * intsort_bucket_histogram: counts[b] = number of keys with
 *   floor((k - min) * B / (max - min + 1)) == b, with min/max read from the
 *   device array minmax[2] (uint64); counts is uint32 [B].
 * Each needs a workspace of intsort_workspace_size() for a plain sort of n.
 */
intsort_status intsort_digit_histogram(intsort_ctx *ctx, intsort_key_type kt, const void *keys,
                                       uint64_t n, uint32_t digit_bits, uint32_t *counts,
                                       void *workspace, size_t workspace_bytes, void *stream);
intsort_status intsort_minmax(intsort_ctx *ctx, intsort_key_type kt, const void *keys,
                              uint64_t n, uint64_t *minmax, void *stream);
intsort_status intsort_bucket_histogram(intsort_ctx *ctx, intsort_key_type kt, const void *keys,
                                        uint64_t n, const uint64_t *minmax, uint32_t num_buckets,
                                        uint32_t *counts, void *stream);

/*
 * Graph capture: one HIP graph launch replays a whole sequence of sort calls.
 *
 * intsort_capture_begin starts recording `stream` (not the null stream) in
 * thread-local capture mode; every sort call the caller then makes on that
 * stream is recorded, not run: every one of them only enqueues kernels (no
 * allocation, no synchronisation, no memset nodes), so each can be captured.
 * intsort_capture_end stops recording and instantiates the graph in *graph.
 * intsort_graph_launch enqueues one replay on `stream`: the same kernels on
 * the same buffers, sizes and options, reading whatever the input buffers
 * hold by then.  Each replay starts from the state its own first kernels
 * set up (counters, look-back words), so replays may follow each other and
 * other work freely.  The caller keeps every buffer the recorded calls name
 * (inputs, outputs, workspaces, device offsets) alive and unchanged in size
 * until intsort_graph_destroy.  Replays of one graph, or of graphs that
 * share a workspace, must not overlap (same rule as the calls themselves).
 * Timing must be off while recording (INTSORT_ERR_UNSUPPORTED otherwise).
 */
typedef struct intsort_graph intsort_graph;

intsort_status intsort_capture_begin(intsort_ctx *ctx, void *stream);
intsort_status intsort_capture_end(intsort_ctx *ctx, void *stream, intsort_graph **graph);
intsort_status intsort_graph_launch(intsort_graph *graph, void *stream);
intsort_status intsort_graph_destroy(intsort_graph *graph);

/*
 * Per-kernel timing, for profiling.  intsort_timing_enable(ctx, 1) creates the
 * HIP events the context needs (host-side objects, no device memory); while
 * it is on, every sort call on the context records an event on its stream
 * before its first kernel and after each kernel (up to 1024 events between
 * reads; later ones are dropped).  intsort_timing_read waits for the last
 * recorded event and fills out[0..*count) with one entry per kernel launched
 * since the previous read, in launch order: its kind, its index (the digit
 * pass for INTSORT_KERNEL_PASS), and the milliseconds between the event
 * before it and the event after it.  Then it forgets them.  Timing a context
 * from two threads at once is not supported.
 */
typedef INTSORT_ENUM(intsort_kernel_kind) {
    INTSORT_KERNEL_INIT = 0,
    INTSORT_KERNEL_DIGIT_HISTOGRAM = 1,
    INTSORT_KERNEL_PASS = 2,
    INTSORT_KERNEL_COPY = 3,
    INTSORT_KERNEL_MINMAX = 4,
    INTSORT_KERNEL_BUCKET_HISTOGRAM = 5,
    INTSORT_KERNEL_BUCKET_SCATTER = 6,
    INTSORT_KERNEL_SEGMENT_SORT = 7,
    INTSORT_KERNEL_PLAN = 8
} intsort_kernel_kind;

typedef struct intsort_kernel_time {
    uint32_t kind;  /* intsort_kernel_kind */
    uint32_t index;
    float ms;
} intsort_kernel_time;

intsort_status intsort_timing_enable(intsort_ctx *ctx, int enable);
intsort_status intsort_timing_read(intsort_ctx *ctx, intsort_kernel_time *out, uint32_t capacity,
                                   uint32_t *count);

/*
 * Device-side error word of the last sort that used `workspace`: 0 when no
 * kernel reported a problem; otherwise an OR of the bits below, and the
 * result is not valid.  Reads device memory, so it synchronises `stream`.
 */
#define INTSORT_DEVERR_LOOKBACK_TIMEOUT 0x1u /* a bounded wait inside a kernel gave up */
#define INTSORT_DEVERR_BAD_TILE 0x2u         /* a tile id or look-back walk left its range */
#define INTSORT_DEVERR_SCATTER_RANGE 0x4u    /* a computed destination fell outside [0, n) */
#define INTSORT_DEVERR_BAD_SEGMENTS 0x8u     /* INTSORT_FLAG_CHECK_SEGMENTS found a bad segment */
intsort_status intsort_read_device_error(intsort_ctx *ctx, const void *workspace,
                                         size_t workspace_bytes, uint32_t *error_word,
                                         void *stream);

#ifdef __cplusplus
}
#endif

#endif /* INTSORT_H */
