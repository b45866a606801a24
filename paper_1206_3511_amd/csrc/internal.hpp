// internal.hpp -- host-side declarations shared by the C ABI and the kernel
// translation units of the sort library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace intsort {

// buffer codes used by the device-side pass plan
enum BufCode : uint32_t { BUF_IN = 0, BUF_OUT = 1, BUF_TMP = 2 };

// status word of the decoupled look-back: 2 flag bits over a 30-bit count
constexpr uint32_t FLAG_SHIFT = 30;
constexpr uint32_t FLAG_AGG = 1u << FLAG_SHIFT;
constexpr uint32_t FLAG_INC = 2u << FLAG_SHIFT;
constexpr uint32_t COUNT_MASK = FLAG_AGG - 1u;
// largest key count one status word can describe
constexpr uint64_t MAX_KEYS = (1ull << 30) - 1;

// error bits written by kernels into the workspace error word
constexpr uint32_t DEVERR_LOOKBACK_TIMEOUT = 1u;   // a bounded wait gave up
constexpr uint32_t DEVERR_BAD_TILE = 2u;           // tile id or look-back walk out of range
constexpr uint32_t DEVERR_SCATTER_RANGE = 4u;      // a computed destination fell outside [0, n)

// plan words per pass: active, src, dst, ordinal
constexpr int PLAN_WORDS = 4;
// final-copy word of a plan (after the passes' words): what moves from the
// buffer the last pass left it in to the output
constexpr uint32_t COPY_KEYS = 1u;
constexpr uint32_t COPY_VALS = 2u;
constexpr int MAX_PASSES = 16;
// counters block: tile counters [MAX_PASSES], done counter, error word
constexpr int CTR_TILE = 0;
constexpr int CTR_DONE = MAX_PASSES;
constexpr int CTR_ERROR = MAX_PASSES + 1;
constexpr int CTR_SEG_CLASS = 32;   // [4] segments per on-chip size class
constexpr int CTR_SEG_SLOTS = 36;   // large segments
constexpr int CTR_SEG_TILES = 37;   // tiles of the large segments
constexpr int CTR_SEG_TMP = 38;     // scratch keys handed out to large separate arrays
constexpr int CTR_SEG_SUM = 40;     // [2] 64-bit sum of the segment lengths (the layout check)
constexpr int CTR_WORDS = 64;

// HIP events around kernels (profiling only).  Events accumulate over calls
// until they are read: every call records a start event, then one event after
// each kernel; a kernel's time is the gap from the event before it.
struct Timer {
    static constexpr int CAP = 1024;
    hipEvent_t ev[CAP];
    uint32_t kind[CAP];    // kernel kind, or CALL_START
    uint32_t index[CAP];
    int used = 0;
    static constexpr uint32_t CALL_START = 0xffffffffu;
    void start(hipStream_t s)
    {
        if (used + 2 > CAP) return;
        kind[used] = CALL_START;
        index[used] = 0;
        if (hipEventRecord(ev[used], s) == hipSuccess) used++;
    }
    void mark(uint32_t k, uint32_t i, hipStream_t s)
    {
        if (used == 0 || used >= CAP) return;
        kind[used] = k;
        index[used] = i;
        if (hipEventRecord(ev[used], s) == hipSuccess) used++;
    }
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// tile geometry of one radix configuration
struct RadixGeom {
    int bits;        // digit width r
    int radix;       // 2^r
    int passes;      // ceil(key_bits / r)
    int threads;     // workgroup size of the pass kernel
    int tile;        // keys per tile
    bool chunked;    // reduce-then-scan passes over chunks of tiles
};

// where every region of a radix sort's workspace sits (byte offsets)
struct RadixLayout {
    RadixGeom g;
    uint64_t n;
    uint64_t num_tiles;
    uint64_t status_words;   // words of each of the two status arrays
    size_t tmp_keys, tmp_vals, hist, excl, plan, counters, status0, status1, tile_offs, chunk_offs, total;
};

RadixGeom radix_geometry(int key_bytes, int bits);
RadixLayout radix_layout(int key_bytes, bool pairs, uint64_t n, int bits);

struct RadixCall {
    const void *keys_in;
    void *keys_out;
    const uint32_t *vals_in;
    uint32_t *vals_out;
    uint64_t n;
    int key_bytes;
    bool pairs;
    int bits;
    int order;        // 0 unsigned, 1 signed, 2 IEEE 754 totalOrder
    bool skip_constant_digits;
    int max_passes;   // passes to run at most (<= geometry passes)
    char *ws;         // workspace base
    RadixLayout L;
    Timer *timer;     // nullable
};

hipError_t radix_sort_run(const RadixCall &c, hipStream_t stream);
// one-read histogram of all digits into a caller array (uint32 [passes*radix])
hipError_t digit_histogram_run(const RadixCall &c, uint32_t *counts, hipStream_t stream);

// sorted (optional): set to 1 when the keys are in nondecreasing order, else 0
hipError_t minmax_run(int key_bytes, const void *keys, uint64_t n, uint64_t *minmax, hipStream_t s,
                      uint64_t *sorted = nullptr);
// skip (optional): a device word; when it is nonzero the kernel counts nothing.
// order (optional): a device word the caller set to 1; cleared unless the
// keys are in nondecreasing order
hipError_t bucket_histogram_run(int key_bytes, const void *keys, uint64_t n, const uint64_t *minmax,
                                uint32_t num_buckets, uint32_t *counts, hipStream_t s,
                                const uint64_t *skip = nullptr, uint64_t *order = nullptr);

int device_cu_count(int device);

// Runs the lane-order self-test of LDS atomics on a device once (the HIP
// device must be current) and says whether the device passed: the pass
// kernel's stable rank needs it.
hipError_t rank_check(int device, bool *ok);

// Takes, once per device (the device must be current), the device address of
// the array intsort_sort_keys_noalloc uses as its workspace.
hipError_t noalloc_setup(int device);

}  // namespace intsort

struct intsort_ctx;
namespace intsort {

// HIP device of a context (-1 for a planning context)
int ctx_device(const intsort_ctx *ctx);

}  // namespace intsort
