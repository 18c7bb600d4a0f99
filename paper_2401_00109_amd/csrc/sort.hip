// Stable LSD radix sort of (u64 key, u32 value) pairs, 8-bit digits.
//
// Used for the global sorting index of Sec. 5: keys are the bit patterns of
// non-negative binary64 sort keys (their unsigned order is the numeric
// order) and values are canonical piece indices, so equal keys keep the
// canonical order.
//
// Per pass: tile histograms (digit-major, 256 x tiles) -> exclusive scan ->
// stable scatter.  Inside a tile the elements are ranked in index order:
// wavefront peers with the same digit are found with eight ballots, waves
// are ordered through LDS counters, and rounds of 256 elements follow each
// other; the ranked tile is staged in LDS and leaves in digit order.  A digit that is the same for every key is skipped; the decision is
// taken on the device from the global digit histograms, and the buffer that
// holds the current order is tracked in device memory (ctl[0]), so no host
// read-back is needed and the sort can be captured in a HIP graph.
#include "common.h"

namespace jabba {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int kTileN = kThreads * kRounds;

__device__ __forceinline__ int64_t live(const int64_t *n_dev, int64_t n_max) {
    int64_t n = *n_dev;
    return n < 0 ? 0 : (n > n_max ? n_max : n);
}

__global__ void k_sort_init(int32_t *ctl, uint32_t *ghist) {
    if (threadIdx.x == 0) ctl[0] = 0;
    for (int i = threadIdx.x; i < 8 * 256; i += blockDim.x) ghist[i] = 0;
}

// Global histograms of all eight digits.
__global__ __launch_bounds__(kThreads) void k_global_hist(const uint64_t *__restrict__ keys, const int64_t *n_dev,
                                                          int64_t n_max, uint32_t *__restrict__ ghist) {
    __shared__ uint32_t h[8][256];
    for (int i = threadIdx.x; i < 8 * 256; i += kThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t n = live(n_dev, n_max);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        uint64_t k = keys[i];
#pragma unroll
        for (int d = 0; d < 8; ++d) atomicAdd(&h[d][(k >> (8 * d)) & 255], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * 256; i += kThreads) {
        uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&ghist[i], v);
    }
}

// skip[d] = every key has the same digit d
__global__ void k_plan(const uint32_t *__restrict__ ghist, const int64_t *n_dev, int64_t n_max, int32_t *ctl) {
    const int d = threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (d >= 8) return;
    const int64_t n = live(n_dev, n_max);
    bool full = false;
    for (int b = lane; b < 256; b += 64) full |= (int64_t)ghist[d * 256 + b] == n;
    uint64_t m = __ballot(full);
    if (lane == 0) ctl[1 + d] = (m != 0ull || n <= 1) ? 1 : 0;
}

template <int Tag>
__global__ __launch_bounds__(kThreads) void k_tile_hist(const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                                                        const int64_t *n_dev, int64_t n_max, int64_t tiles_max,
                                                        int shift, const int32_t *ctl, int pass,
                                                        uint32_t *__restrict__ hist) {
    if (ctl[1 + pass]) return;
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t *keys = ctl[0] ? k1 : k0;
    const int64_t n = live(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kTileN;
    for (int r = 0; r < kRounds; ++r) {
        int64_t i = base + r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles_max + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of one value per thread over the 256 threads of the block.
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *s_wave) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_wave[w] = x;
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < w; ++q) add += s_wave[q];
    return x - v + add;
}

// Stable scatter of one tile.  The tile is first ranked into LDS in digit
// order (the rank of an element is its position among the tile's elements
// with the same digit, in index order), then written out in that order, so
// each digit's run of the tile lands in one contiguous stretch of the
// destination and the stores of consecutive threads are coalesced.
template <int Tag>
__global__ __launch_bounds__(kThreads) void k_scatter(uint64_t *__restrict__ k0, uint64_t *__restrict__ k1,
                                                      uint32_t *__restrict__ v0, uint32_t *__restrict__ v1,
                                                      const int64_t *n_dev, int64_t n_max, int64_t tiles_max, int shift,
                                                      const int32_t *ctl, int pass,
                                                      const uint32_t *__restrict__ offs) {
    if (ctl[1 + pass]) return;
    __shared__ uint64_t s_key[kTileN];
    __shared__ uint32_t s_val[kTileN];
    __shared__ uint32_t s_run[256];  // next free local slot per digit
    __shared__ uint32_t s_lo[256];   // local start per digit
    __shared__ uint32_t s_go[256];   // destination start per digit
    __shared__ uint32_t s_cnt[kThreads / kWave][256];
    __shared__ uint32_t s_pre[kThreads / kWave][256];
    __shared__ uint32_t s_wave[kThreads / kWave];
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    const bool src1 = ctl[0] != 0;
    const uint64_t *ks = src1 ? k1 : k0;
    const uint32_t *vs = src1 ? v1 : v0;
    uint64_t *kd = src1 ? k0 : k1;
    uint32_t *vd = src1 ? v0 : v1;
    const int64_t n = live(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kTileN;
    if (base >= n) return;
    const int m = (int)(n - base < kTileN ? n - base : kTileN);

    // all of this thread's elements in flight at once
    uint64_t kr[kRounds];
    uint32_t vr[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int li = r * kThreads + tid;
        kr[r] = li < m ? ks[base + li] : 0ull;
        vr[r] = li < m ? vs[base + li] : 0u;
    }
    // this tile's count of digit `tid`: difference of consecutive scanned
    // offsets (digit-major layout; the entry after the last is the total)
    const uint32_t g0 = offs[(int64_t)tid * tiles_max + blockIdx.x];
    const uint32_t g1 = offs[(int64_t)tid * tiles_max + blockIdx.x + 1];
    const uint32_t lo = block_excl_scan_256(g1 - g0, s_wave);
    s_lo[tid] = lo;
    s_run[tid] = lo;
    s_go[tid] = g0;
    for (int i = 0; i < kThreads / kWave; ++i) s_cnt[i][tid] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const bool ok = r * kThreads + tid < m;
        const uint64_t key = kr[r];
        const uint32_t dg = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (ok && rank == 0) s_cnt[w][dg] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t run = s_run[tid];
#pragma unroll
            for (int q = 0; q < kThreads / kWave; ++q) {
                s_pre[q][tid] = run;
                run += s_cnt[q][tid];
                s_cnt[q][tid] = 0;
            }
            s_run[tid] = run;
        }
        __syncthreads();
        if (ok) {
            const uint32_t lp = s_pre[w][dg] + rank;
            s_key[lp] = key;
            s_val[lp] = vr[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int j = r * kThreads + tid;
        if (j < m) {
            const uint64_t key = s_key[j];
            const uint32_t dg = (uint32_t)(key >> shift) & 255u;
            const uint32_t pos = s_go[dg] + ((uint32_t)j - s_lo[dg]);
            kd[pos] = key;
            vd[pos] = s_val[j];
        }
    }
}

__global__ void k_flip(int32_t *ctl, int pass) {
    if (threadIdx.x == 0 && !ctl[1 + pass]) ctl[0] ^= 1;
}

}  // namespace

size_t sort_workspace(int64_t n_max, Carve &c, SortBuffers *b) {
    const int64_t tiles = (n_max + kTileN - 1) / kTileN > 0 ? (n_max + kTileN - 1) / kTileN : 1;
    SortBuffers x;
    x.keys[0] = c.take<uint64_t>(n_max);
    x.keys[1] = c.take<uint64_t>(n_max);
    x.vals[0] = c.take<uint32_t>(n_max);
    x.vals[1] = c.take<uint32_t>(n_max);
    x.hist = c.take<uint32_t>(256 * tiles + 1);
    x.ghist = c.take<uint32_t>(8 * 256);
    x.ctl = c.take<int32_t>(64);
    x.scan_ws = c.take<char>(scan_workspace(256 * tiles));
    if (b) *b = x;
    return c.bytes();
}

int radix_sort_init(const SortBuffers &b, hipStream_t st) {
    JB_LAUNCH(k_sort_init, dim3(1), dim3(256), 0, st, b.ctl, b.ghist);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

int radix_global_hist(const SortBuffers &b, const int64_t *n_dev, int64_t n_max, hipStream_t st) {
    int64_t blocks = (n_max + kThreads * 8 - 1) / (kThreads * 8);
    int cap = device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    JB_LAUNCH(k_global_hist, dim3((unsigned)blocks), dim3(kThreads), 0, st, b.keys[0], n_dev, n_max,
                       b.ghist);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

int radix_sort_pairs(const SortBuffers &b, const int64_t *n_dev, int64_t n_max, hipStream_t st, const char *tag) {
    const bool main_sort = !tag || !tag[0];
    const int64_t tiles = (n_max + kTileN - 1) / kTileN > 0 ? (n_max + kTileN - 1) / kTileN : 1;
    JB_LAUNCH(k_plan, dim3(1), dim3(512), 0, st, b.ghist, n_dev, n_max, b.ctl);
    JB_LAUNCH_CHECK();
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        JB_LAUNCH_NAMED(main_sort ? "k_tile_hist" : "k_tile_hist_groups",
                        main_sort ? k_tile_hist<0> : k_tile_hist<1>, dim3((unsigned)tiles),
                        dim3(kThreads), 0, st, b.keys[0], b.keys[1], n_dev,
                           n_max, tiles, shift, b.ctl, pass, b.hist);
        JB_LAUNCH_CHECK();
        int rc = scan_u32_to_u32(b.hist, b.hist, nullptr, 256 * tiles, b.scan_ws, st);
        if (rc) return rc;
        JB_LAUNCH_NAMED(main_sort ? "k_scatter" : "k_scatter_groups",
                        main_sort ? k_scatter<0> : k_scatter<1>, dim3((unsigned)tiles),
                        dim3(kThreads), 0, st, b.keys[0], b.keys[1], b.vals[0],
                           b.vals[1], n_dev, n_max, tiles, shift, b.ctl, pass, b.hist);
        JB_LAUNCH_CHECK();
        JB_LAUNCH(k_flip, dim3(1), dim3(64), 0, st, b.ctl, pass);
        JB_LAUNCH_CHECK();
    }
    return JABBA_OK;
}

}  // namespace jabba
