// tuning.cpp -- the table of tuned defaults that zero option fields take:
// the autotuner's choice of digit width, bucket count and segmented LDS
// cutoff per device, key width and size class floor(log2 n).
//
// The table is a text file, one entry per line, tab-separated:
//   device key, kind (radix | bucket | segmented | segmented_bits), key bytes (4 | 8),
//   size class, value
// '#' starts a comment line; '*' as the device key matches every device.
// Lines that do not parse are skipped, and so are values a call could not
// take (the caller of tune_lookup checks them).

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "tuning.hpp"

namespace intsort {

namespace {

bool parse_kind(const std::string &s, int *kind)
{
    if (s == "radix") *kind = TUNE_RADIX_BITS;
    else if (s == "bucket") *kind = TUNE_BUCKETS;
    else if (s == "segmented") *kind = TUNE_LDS_CUTOFF;
    else if (s == "segmented_bits") *kind = TUNE_SEG_BITS;
    else return false;
    return true;
}

bool parse_uint(const std::string &s, uint64_t *v)
{
    if (s.empty() || s.size() > 19) return false;
    uint64_t x = 0;
    for (char c : s) {
        if (c < '0' || c > '9') return false;
        x = x * 10 + (uint64_t)(c - '0');
    }
    *v = x;
    return true;
}

}  // namespace

bool tune_load(const char *path, std::vector<TuneEntry> *out)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    std::vector<TuneEntry> e;
    std::string line;
    int ch;
    auto flush = [&]() {
        if (!line.empty() && line[0] != '#') {
            std::vector<std::string> fld;
            size_t at = 0;
            while (true) {
                const size_t tab = line.find('\t', at);
                fld.push_back(line.substr(at, tab == std::string::npos ? std::string::npos : tab - at));
                if (tab == std::string::npos) break;
                at = tab + 1;
            }
            TuneEntry t;
            uint64_t w = 0, cls = 0, val = 0;
            if (fld.size() == 5 && !fld[0].empty() && parse_kind(fld[1], &t.kind) && parse_uint(fld[2], &w) &&
                (w == 4 || w == 8) && parse_uint(fld[3], &cls) && cls < 64 && parse_uint(fld[4], &val) &&
                val <= 0xffffffffull) {
                t.device = fld[0];
                t.width = (int)w;
                t.size_class = (int)cls;
                t.value = (uint32_t)val;
                e.push_back(t);
            }
        }
        line.clear();
    };
    while ((ch = std::fgetc(f)) != EOF) {
        if (ch == '\n') flush();
        else if (ch != '\r') line.push_back((char)ch);
    }
    flush();
    std::fclose(f);
    *out = std::move(e);
    return true;
}

std::string tune_default_path()
{
    if (const char *p = std::getenv("INTSORT_TUNE_FILE")) return p;
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/intsort/tune.tsv";
    return std::string();
}

std::string tune_device_key(int device)
{
    if (device < 0) return std::string();
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return std::string();
    int rt = 0;
    if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
    return std::string(p.name) + "|" + p.gcnArchName + "|hip " + std::to_string(rt);
}

int size_class(uint64_t n)
{
    int c = 0;
    while (n > 1) {
        n >>= 1;
        c++;
    }
    return c;
}

bool tune_lookup(const std::vector<TuneEntry> &table, const std::string &device, int kind, int width, uint64_t n,
                 uint32_t *value)
{
    const int cls = size_class(n);
    // the device's own entry first, then one for every device
    for (int pass = 0; pass < 2; pass++) {
        for (const TuneEntry &t : table) {
            if (t.kind != kind || t.width != width || t.size_class != cls) continue;
            if (pass == 0 ? (device.empty() || t.device != device) : t.device != "*") continue;
            *value = t.value;
            return true;
        }
    }
    return false;
}

}  // namespace intsort
