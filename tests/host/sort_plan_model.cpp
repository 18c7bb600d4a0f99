// Host model of the radix sort's pass schedule: stable LSD passes of 8-bit
// digits over key - kmin, skipping digits that are the same for every key,
// moving the keys at the widths sort_pass_modes gives (64-bit, then 32-bit
// keys shifted past the sorted digits, none after the last pass; or 32-bit
// key - kmin from the start for the kept 32-bit form).  The order must be the
// stable order of the keys, and kept keys must leave sorted.
#include <stdint.h>

#include <vector>

#include "sort_plan.h"

extern "C" int plan_sort(const uint64_t *keys, int64_t n, int key_form, uint32_t *order, int *modes_out,
                         int *base_out, int64_t *bytes_out) {
    uint64_t kmin = ~0ull;
    for (int64_t i = 0; i < n; ++i) kmin = keys[i] < kmin ? keys[i] : kmin;
    int skip[8];
    for (int d = 0; d < 8; ++d) {
        skip[d] = 1;
        if (n <= 1) continue;
        const uint64_t first = ((keys[0] - kmin) >> (8 * d)) & 255u;
        for (int64_t i = 1; i < n; ++i)
            if ((((keys[i] - kmin) >> (8 * d)) & 255u) != first) {
                skip[d] = 0;
                break;
            }
    }
    const int base = jabba::sort_pass_modes(skip, key_form, modes_out);
    *base_out = base;
    std::vector<uint64_t> k64(keys, keys + n), t64(n);
    std::vector<uint32_t> k32(n), t32(n), v(n), tv(n);
    for (int64_t i = 0; i < n; ++i) v[i] = (uint32_t)i;
    bool have64 = true, have32 = false;
    if (key_form == jabba::kSortKeep32) {  // the caller writes key - kmin as 32-bit words
        for (int64_t i = 0; i < n; ++i) {
            if (keys[i] - kmin > 0xFFFFFFFFull) return -2;
            k32[i] = (uint32_t)(keys[i] - kmin);
        }
        have64 = false;
        have32 = true;
    }
    int64_t bytes = 0;
    for (int d = 0; d < 8; ++d) {
        if (skip[d]) continue;
        const int mode = modes_out[d];
        const bool in32 = (mode & jabba::kSortModeIn32) != 0;
        if ((in32 && !have32) || (!in32 && !have64)) return -1;  // a pass reads keys no pass wrote
        bytes += jabba::sort_pass_bytes(mode);
        auto digit = [&](int64_t i) -> uint32_t {
            return in32 ? (k32[i] >> (8 * d - base)) & 255u : (uint32_t)(((k64[i] - kmin) >> (8 * d)) & 255u);
        };
        int64_t cnt[257] = {0};
        for (int64_t i = 0; i < n; ++i) ++cnt[digit(i) + 1];
        for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
        for (int64_t i = 0; i < n; ++i) {
            const int64_t p = cnt[digit(i)]++;
            tv[p] = v[i];
            if (mode & jabba::kSortModeOut32)
                t32[p] = in32 ? k32[i] : (uint32_t)((k64[i] - kmin) >> base);
            else if (!(mode & jabba::kSortModeNoKeys))
                t64[p] = k64[i];
        }
        v.swap(tv);
        if (mode & jabba::kSortModeOut32) {
            k32.swap(t32);
            have32 = true;
            have64 = false;
        } else if (mode & jabba::kSortModeNoKeys) {
            have32 = have64 = false;
        } else {
            k64.swap(t64);
        }
    }
    for (int64_t i = 0; i < n; ++i) order[i] = v[i];
    *bytes_out = bytes;
    if (key_form == jabba::kSortKeep32) {  // the kept keys must leave in sorted order
        if (!have32) return -3;
        for (int64_t i = 0; i < n; ++i)
            if ((uint64_t)k32[i] + kmin != keys[v[i]]) return -4;
    }
    return 0;
}
