// Device-wide exclusive scans and fill kernels.
//
// Three launches: per-tile totals, one workgroup scanning the tile totals,
// per-tile scan plus tile offset.  Element counts may live in device memory
// (n_dev), so the launches are sized from the host upper bound n_max and
// every tile beyond the live count contributes zero; this keeps the scans
// capturable in a HIP graph.  out has n + 1 entries: out[n] is the total.
#include "common.h"

namespace jabba {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kTile = kScanThreads * kScanItems;

template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *lds_wave, T *total) {
    // lane inclusive scan (wave64) then across the 4 waves
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds_wave[wave] = x;
    __syncthreads();
    T wave_off = 0, tot = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        T s = lds_wave[w];
        if (w < wave) wave_off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wave_off + x - v;
}

__device__ __forceinline__ int64_t live_n(const int64_t *n_dev, int64_t n_max) {
    if (!n_dev) return n_max;
    int64_t n = *n_dev;
    return n < 0 ? 0 : (n > n_max ? n_max : n);
}

template <class Tin, class Tout>
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const Tin *__restrict__ in, Tout *__restrict__ sums,
                                                             const int64_t *n_dev, int64_t n_max) {
    __shared__ Tout lds[kScanThreads / kWave];
    const int64_t n = live_n(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    Tout acc = 0;
    bool vec = false;
    if constexpr (sizeof(Tin) == 4 && kScanItems == 8)
        vec = base + kTile <= n && ((uintptr_t)in & 15) == 0;
    if (vec) {  // a full tile of 4-byte values: two 16-byte loads per thread (an exact sum, any order)
        const uint4 *p = reinterpret_cast<const uint4 *>(in + base + (int64_t)threadIdx.x * kScanItems);
        const uint4 a = p[0], b = p[1];
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            Tin t;
            __builtin_memcpy(&t, &w[i], sizeof(t));
            acc += (Tout)t;
        }
    } else if (base < n) {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;
            if (idx < n) acc += (Tout)in[idx];
        }
    }
    Tout tot;
    block_exclusive_scan<Tout>(acc, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile totals in place; total -> *grand.
template <class Tout>
__global__ __launch_bounds__(1024) void k_scan_sums(Tout *__restrict__ sums, int64_t n_tiles, Tout *grand) {
    __shared__ Tout lds[1024 / kWave];
    __shared__ Tout carry_s;
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    Tout carry = 0;
    for (int64_t b0 = 0; b0 < n_tiles; b0 += 1024) {
        int64_t i = b0 + threadIdx.x;
        Tout v = i < n_tiles ? sums[i] : 0;
        Tout x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            Tout y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) lds[wave] = x;
        __syncthreads();
        Tout off = carry;
        Tout tot = 0;
        for (int w = 0; w < 1024 / kWave; ++w) {
            Tout s = lds[w];
            if (w < wave) off += s;
            tot += s;
        }
        if (i < n_tiles) sums[i] = off + x - v;
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) {
        carry_s = carry;
        *grand = carry;
    }
}

template <class Tin, class Tout>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const Tin *__restrict__ in, Tout *__restrict__ out,
                                                             const Tout *__restrict__ sums, const int64_t *n_dev,
                                                             int64_t n_max, const Tout *grand) {
    __shared__ Tout lds[kScanThreads / kWave];
    const int64_t n = live_n(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *grand;
    if (base >= n) return;
    // each thread owns kScanItems consecutive elements of the tile; a full
    // tile of 4-byte types on 16-byte boundaries moves them as two 16-byte
    // loads and stores per thread
    const int64_t my0 = base + (int64_t)threadIdx.x * kScanItems;
    bool vec = false;
    if constexpr (sizeof(Tin) == 4 && sizeof(Tout) == 4 && kScanItems == 8)
        vec = base + kTile <= n && ((uintptr_t)in & 15) == 0 && ((uintptr_t)out & 15) == 0;
    Tout v[kScanItems];
    Tout acc = 0;
    if (vec) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in + my0);
        const uint4 a = p[0], b = p[1];
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            Tin t;
            __builtin_memcpy(&t, &w[i], sizeof(t));
            v[i] = (Tout)t;
            acc += v[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            int64_t idx = my0 + i;
            v[i] = idx < n ? (Tout)in[idx] : (Tout)0;
            acc += v[i];
        }
    }
    Tout tot;
    Tout run = block_exclusive_scan<Tout>(acc, lds, &tot) + sums[blockIdx.x];
    if (vec) {
        uint32_t w[8];
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            __builtin_memcpy(&w[i], &run, sizeof(uint32_t));
            run += v[i];
        }
        uint4 *q = reinterpret_cast<uint4 *>(out + my0);
        q[0] = make_uint4(w[0], w[1], w[2], w[3]);
        q[1] = make_uint4(w[4], w[5], w[6], w[7]);
        return;
    }
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = my0 + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
}

template <class Tin, class Tout>
int scan_impl(const Tin *in, Tout *out, const int64_t *n_dev, int64_t n_max, void *ws, hipStream_t st) {
    if (n_max < 0) return JABBA_EINVAL;
    int64_t tiles = (n_max + kTile - 1) / kTile;
    if (tiles < 1) tiles = 1;
    Carve c(ws);
    Tout *sums = c.take<Tout>(tiles);
    Tout *grand = c.take<Tout>(1);
    JB_LAUNCH((k_tile_sums<Tin, Tout>), dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, sums, n_dev,
                       n_max);
    JB_LAUNCH_CHECK();
    JB_LAUNCH((k_scan_sums<Tout>), dim3(1), dim3(1024), 0, st, sums, tiles, grand);
    JB_LAUNCH_CHECK();
    JB_LAUNCH((k_tile_scan<Tin, Tout>), dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, out, sums,
                       n_dev, n_max, grand);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
int fill_impl(T *p, T v, int64_t n, hipStream_t st) {
    if (n <= 0) return JABBA_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    JB_LAUNCH((k_fill<T>), dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

}  // namespace

size_t scan_workspace(int64_t n_max) {
    int64_t tiles = (n_max + kTile - 1) / kTile;
    if (tiles < 1) tiles = 1;
    Carve c;
    c.take<int64_t>(tiles);
    c.take<int64_t>(1);
    return c.bytes();
}

int scan_i32_to_i64(const int32_t *in, int64_t *out, const int64_t *n_dev, int64_t n_max, void *ws, hipStream_t st) {
    return scan_impl<int32_t, int64_t>(in, out, n_dev, n_max, ws, st);
}
int scan_i64_to_i64(const int64_t *in, int64_t *out, const int64_t *n_dev, int64_t n_max, void *ws, hipStream_t st) {
    return scan_impl<int64_t, int64_t>(in, out, n_dev, n_max, ws, st);
}
int scan_u32_to_u32(const uint32_t *in, uint32_t *out, const int64_t *n_dev, int64_t n_max, void *ws,
                    hipStream_t st) {
    return scan_impl<uint32_t, uint32_t>(in, out, n_dev, n_max, ws, st);
}
int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) { return fill_impl<int32_t>(p, v, n, st); }
int fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st) { return fill_impl<int64_t>(p, v, n, st); }

}  // namespace jabba
