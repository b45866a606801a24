// tuning.hpp -- the table of tuned defaults (tuning.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace intsort {

enum TuneKind { TUNE_RADIX_BITS = 0, TUNE_BUCKETS = 1, TUNE_LDS_CUTOFF = 2, TUNE_SEG_BITS = 3 };

struct TuneEntry {
    std::string device;   // device key, or "*" for every device
    int kind;             // TuneKind
    int width;            // key bytes
    int size_class;       // floor(log2 n)
    uint32_t value;
};

// reads a table file; false if it cannot be opened (then *out is unchanged)
bool tune_load(const char *path, std::vector<TuneEntry> *out);
// $INTSORT_TUNE_FILE, else ~/.cache/intsort/tune.tsv
std::string tune_default_path();
// "<name>|<arch>|hip <runtime version>" of a HIP device; empty for -1
std::string tune_device_key(int device);
int size_class(uint64_t n);
// the tuned value of a kind for the device (or '*'), key width and size class of n
bool tune_lookup(const std::vector<TuneEntry> &table, const std::string &device, int kind, int width, uint64_t n,
                 uint32_t *value);

}  // namespace intsort
