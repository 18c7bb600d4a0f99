// Key widths of the passes of the radix sort, shared by the sort's planning
// kernel and its host-side model test.  Plain C++ so the host compiler can
// build it too.
//
// The sort orders key - kmin, which is 0 on the smallest key, so a digit that
// is the same for every key (a skipped pass) is 0 in every key, and digits
// above the highest active one can be dropped.  A sort whose caller needs
// only the order carries 64-bit keys until the digits left to sort fit in 32
// bits, then 32-bit keys (key - kmin shifted past the digits already sorted);
// its last active pass writes the values alone.  A sort whose keys minus kmin
// are below 2^32 can carry them at 32 bits throughout and keep them.
#pragma once

#ifndef JB_HD
#if defined(__HIPCC__)
#define JB_HD __host__ __device__
#else
#define JB_HD
#endif
#endif

namespace jabba {

constexpr int kSortModeIn32 = 1;    // the pass reads 32-bit keys
constexpr int kSortModeOut32 = 2;   // the pass writes 32-bit keys
constexpr int kSortModeNoKeys = 4;  // the pass writes no keys (order only)

// what the sort's caller gets besides the order
constexpr int kSortOrderOnly = 0;  // nothing: keys narrow, the last pass writes values only
constexpr int kSortKeep64 = 1;     // the sorted 64-bit keys
constexpr int kSortKeep32 = 2;     // the sorted keys, stored as 32-bit key - kmin (< 2^32) from the start

// skip[d] (d = 0..7): digit d of key - kmin is the same for every key.
// Writes modes[d] (kSortMode* bits, 0 for skipped passes and 64-bit kept
// keys) and returns the bit offset of the 32-bit keys inside key - kmin
// (0 when no pass narrows).
JB_HD inline int sort_pass_modes(const int *skip, int key_form, int *modes) {
    if (key_form == kSortKeep32) {
        for (int d = 0; d < 8; ++d) modes[d] = skip[d] ? 0 : (kSortModeIn32 | kSortModeOut32);
        return 0;
    }
    const bool keep_keys = key_form != kSortOrderOnly;
    int top = -1;
    for (int d = 0; d < 8; ++d)
        if (!skip[d]) top = d;
    bool narrow = false;
    int base = 0;
    for (int d = 0; d < 8; ++d) {
        int mode = 0;
        if (!skip[d] && !keep_keys) {
            mode = narrow ? kSortModeIn32 : 0;
            if (d == top) {
                mode |= kSortModeNoKeys;
            } else if (narrow) {
                mode |= kSortModeOut32;
            } else if (top - d <= 4) {  // digits d+1..top fit in 32 bits
                mode |= kSortModeOut32;
                narrow = true;
                base = 8 * (d + 1);
            }
        }
        modes[d] = mode;
    }
    return base;
}

// bytes per pair that pass `mode` reads and writes (key and value)
JB_HD inline int sort_pass_bytes(int mode) {
    return ((mode & kSortModeIn32) ? 4 : 8) + 4 + ((mode & kSortModeNoKeys) ? 0 : (mode & kSortModeOut32) ? 4 : 8) + 4;
}

}  // namespace jabba
