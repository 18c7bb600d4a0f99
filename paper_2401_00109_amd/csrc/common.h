// Internal helpers shared by the HIP sources of libjabba (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "jabba.h"
#include "lane_ops.h"
#include "sort_plan.h"

namespace jabba {

constexpr int kWave = 64;
// The chip's accelerator dies (XCDs), each with its own L2.  The dispatcher
// hands workgroups to them round robin, so blockIdx.x % kXcds names the
// workgroup's XCD (a performance assumption only: no result depends on it).
constexpr int kXcds = 8;

// Device status bits (OR-ed into the first word of a workspace).
enum : int32_t {
    kStNonFinite = 1,
    kStCapacity = 2,
    kStOverflow = 4,
    kStInvalid = 8,
    kStInternal = 16,  // a bounded device-side wait ran out
};

// ---------------------------------------------------------------- host side
#define JB_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return JABBA_EHIP;       \
    } while (0)

#define JB_LAUNCH_CHECK()                               \
    do {                                                \
        hipError_t e_ = hipGetLastError();              \
        if (e_ != hipSuccess) return JABBA_EHIP;        \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carves typed sub-buffers out of one caller-provided workspace.  The same
// sequence of take() calls is used for the size query and for the call, so
// offsets always agree.
struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b = nullptr) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t n) {
        off = align_up(off, 256);
        T *p = reinterpret_cast<T *>(base + off);
        off += (n ? n : 1) * sizeof(T);
        return base ? p : nullptr;
    }
    size_t bytes() const { return align_up(off, 256); }
};

// Number of compute units of the current device (cached per device).
int device_cu_count();

// JABBA_OK when the current device is a gfx950 (cached per device), else
// JABBA_ENODEV (also when no device is visible).
int device_check();
#define JB_DEVICE_CHECK()                           \
    do {                                            \
        const int dc_ = ::jabba::device_check();    \
        if (dc_ != JABBA_OK) return dc_;            \
    } while (0)

// Opt-in per-kernel event timing (jabba_timing_*): a scope that records an
// event on `st` when created and another when destroyed, if timing is on.
// Times the launches enqueued during its lifetime on one stream as `launches`
// launches of `name` (one event pair around them all).
struct KernelTimer {
    KernelTimer(const char *name, hipStream_t st, int launches = 1);
    ~KernelTimer();
    const char *name_;
    hipStream_t st_;
    void *a_;
    int launches_;
};
// Launch with the optional event timing around it (the kernel expression's
// text is the timing name).
#define JB_LAUNCH(kernel, grid, block, lds, st, ...)                   \
    do {                                                               \
        ::jabba::KernelTimer jb_timer_(#kernel, st);                   \
        hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__); \
    } while (0)
// Same, with an explicit timing name (kernels launched for several purposes).
#define JB_LAUNCH_NAMED(name, kernel, grid, block, lds, st, ...)       \
    do {                                                               \
        ::jabba::KernelTimer jb_timer_(name, st);                      \
        hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__); \
    } while (0)

// ---------------------------------------------------------------- device side
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int ffs64(uint64_t m) { return m ? __builtin_ctzll(m) : -1; }

// One step of a wavefront scan: the value of a lane selected by a DPP
// control (row shifts within rows of 16 lanes, row broadcasts across rows);
// lanes without a source read 0.  Register-to-register, no LDS.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, true);
}

// value of lane l (l uniform across the wavefront): two scalar reads, no LDS
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src); }
__device__ __forceinline__ int64_t shfl_i64(int64_t v, int src) { return __shfl(v, src); }
__device__ __forceinline__ int shfl_i(int v, int src) { return __shfl(v, src); }

// Sum of a wavefront's values as a balanced pairwise tree over lanes
// (lane pairs (0,1), (2,3), ..., then pairs of pairs).  Floating-point
// addition is commutative, so every lane ends with the same bits.
__device__ __forceinline__ double wave_tree_sum(double v) {
    // step m: every lane adds the value of lane ^ m (lane moves in the VALU)
    v = v + xor_lane_f64<1>(v);
    v = v + xor_lane_f64<2>(v);
    v = v + xor_lane_f64<4>(v);
    v = v + xor_lane_f64<8>(v);
    v = v + xor_lane_f64<16>(v);
    v = v + xor_lane_f64<32>(v);
    return v;
}

// Pairwise tree over 1024 leaves (a 256-thread workgroup, every thread calls): 4 adjacent leaves per thread, then the
// wavefront butterfly, then the four wavefront sums pairwise.
__device__ __forceinline__ double block_tree_1024(double a0, double a1, double a2, double a3) {
    __shared__ double ws[4];
    double v = (a0 + a1) + (a2 + a3);
    v = wave_tree_sum(v);
    if (lane_id() == 0) ws[threadIdx.x / kWave] = v;
    __syncthreads();
    double r = (ws[0] + ws[1]) + (ws[2] + ws[3]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    uint64_t u = (uint64_t)v;
    u += xor_lane_u64<1>(u);
    u += xor_lane_u64<2>(u);
    u += xor_lane_u64<4>(u);
    u += xor_lane_u64<8>(u);
    u += xor_lane_u64<16>(u);
    u += xor_lane_u64<32>(u);
    return (int64_t)u;
}

__device__ __forceinline__ void set_status(int32_t *st, int32_t bit) {
    if (st) atomicOr(st, bit);
}

// Scaled coordinates of a piece (Eq. tupseq2); every kernel that needs x, y
// or the key evaluates them with this one function so the bits agree.
struct Scaled {
    double x, y;
};
__device__ __forceinline__ Scaled scale_piece(int32_t len, double inc, double scl, double sl, double si) {
    Scaled s;
    double q = (double)len / sl;
    s.x = scl * q;
    s.y = inc / si;
    return s;
}
__device__ __forceinline__ double piece_key(Scaled s) {
    double xx = s.x * s.x;
    double yy = s.y * s.y;
    return __dsqrt_rn(xx + yy);
}

// ---------------------------------------------------------------- launchers
// scan.hip: exclusive scans (out[0..n] with out[n] = total), n read on device
// when n_dev != nullptr (clamped to n_max), otherwise n = n_max.
size_t scan_workspace(int64_t n_max);
int scan_i32_to_i64(const int32_t *in, int64_t *out, const int64_t *n_dev, int64_t n_max, void *ws, hipStream_t st);
int scan_i64_to_i64(const int64_t *in, int64_t *out, const int64_t *n_dev, int64_t n_max, void *ws, hipStream_t st);
int scan_u32_to_u32(const uint32_t *in, uint32_t *out, const int64_t *n_dev, int64_t n_max, void *ws,
                    hipStream_t st);

// fill kernels (graph-safe replacements for memset)
int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
int fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st);

// sort.hip: stable LSD radix sort of (u64 key, u32 value) pairs.
struct SortBuffers {
    uint64_t *keys[2];
    uint32_t *vals[2];
    uint64_t *status;    // look-back words, 256 per tile
    int64_t n_status;
    uint32_t *ghist;     // 8 * 256 global digit histograms
    uint32_t *gbase;     // 8 * 256 bucket bases
    int32_t *tile_ctr;   // tile tickets, one counter per pass
    unsigned long long *kmin;  // smallest key; digits are taken from key - kmin
    int32_t *ctl;        // [0] = buffer with the sorted order, [1..8] = skip flags,
                         // [9..16] = buffer each pass reads, [32] = look-back error
};
size_t sort_workspace(int64_t n_max, Carve &c, SortBuffers *b);
// Resets the control words and the global digit histograms.
int radix_sort_init(const SortBuffers &b, hipStream_t st);
// ctl[kSortCtlMode + d]: the key widths (kSortMode* bits of sort_plan.h)
// pass d of the last sort moved.
constexpr int kSortCtlMode = 40;

// Global histograms of the eight digits of keys[0] (after the keys are written).
int radix_global_hist(const SortBuffers &b, const int64_t *n_dev, int64_t n_max, hipStream_t st);
// Sorts n (device count) pairs held in keys[0]/vals[0]; the result is in
// keys[ctl[0]], vals[ctl[0]] (read on device by consumers).  key_form
// (sort_plan.h): kSortKeep64 keeps the 64-bit keys; kSortKeep32 takes and
// keeps keys - kmin as 32-bit words (the key buffers read as uint32_t, every
// key - kmin below 2^32); with kSortOrderOnly only vals[ctl[0]] holds the
// result (the sorted order) and the key buffers hold intermediate, narrowed
// keys.  sparse: the live count is
// expected far below n_max (the passes then run persistent workgroups
// instead of one per possible tile).
// `tag` suffixes the timing names of the pass kernels ("" for the main sort).
// prefix_digits > 0: only the highest prefix_digits digits below the top
// non-constant one are sorted; the pairs leave grouped by
// (key - kmin) >> ctl[kSortCtlPrefixShift], in input order within a group
// (with kSortOrderOnly, the values alone).
int radix_sort_pairs(const SortBuffers &b, const int64_t *n_dev, int64_t n_max, hipStream_t st,
                     const char *tag = "", int key_form = kSortKeep64, bool sparse = false, int prefix_digits = 0);
// ctl words a consumer of the sort reads: [0] the buffer holding the result,
// [kSortCtlSkip + d] pass d skipped, [kSortCtlError] a look-back wait ran out,
// [kSortCtlPrefixShift] the prefix shift of a prefix sort.
constexpr int kSortCtlSkip = 1;
constexpr int kSortCtlError = 32;
constexpr int kSortCtlPrefixShift = 56;
constexpr int kSortCtlFirst = 57;  // first pass that moves data, 8 when none does

}  // namespace jabba
