// Stable LSD radix sort of (u64 key, u32 value) pairs, 8-bit digits.
//
// Used for the global sorting index of Sec. 5: keys are unsigned integers in
// the order of the binary64 sort keys and values are canonical piece
// indices, so equal keys keep the canonical order.
//
// One kernel per digit ("one sweep"): the global histograms of all eight
// digits are taken once, up front; a pass takes tiles in ticket order, counts
// the tile's digits, and finds the tile's offset inside each digit bucket by
// decoupled look-back over the earlier tiles' published counts (each status
// word carries the pass tag, an aggregate/prefix flag and the count).  Inside
// a tile each wavefront ranks its own contiguous slice in index order (peers
// with the same digit by eight ballots, a running count per digit in the
// wave's LDS row), and the slices are ordered by per-digit offsets; the
// ranked tile is staged in LDS and leaves in digit order, so each digit's run
// of the tile is one contiguous, coalesced stretch of the destination.  A
// digit that is the same for every key is skipped; the decision and the
// buffer parity of every pass are taken on the device from the global
// histograms, so no host read-back is needed and the sort can be captured in
// a HIP graph.
//
// A sort whose caller needs only the order (not the sorted keys) carries
// less: once the digits not yet sorted fit in 32 bits, the passes read and
// write 32-bit keys (key - kmin shifted past the sorted digits), and the last
// pass writes the values alone.
#include "common.h"
#include "sort_plan.h"

namespace jabba {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int kTileN = kThreads * kRounds;

// control words
constexpr int kCtlFinal = 0;   // buffer holding the sorted order after all passes
constexpr int kCtlSkip = 1;    // [1..8]: digit d is the same for every key
constexpr int kCtlSrc = 9;     // [9..16]: buffer pass d reads
constexpr int kCtlError = 32;  // a look-back wait ran out (never expected)
constexpr int kCtlMode = kSortCtlMode;  // [40..47]: key widths of pass d
constexpr int kCtlBase = 48;            // bit offset of the 32-bit keys inside key - kmin
constexpr int kCtlPrefixShift = kSortCtlPrefixShift;  // lowest bit a prefix sort ordered
constexpr int kCtlFirst = kSortCtlFirst;  // first pass that moves data
constexpr int kModeIn32 = kSortModeIn32;
constexpr int kModeOut32 = kSortModeOut32;
constexpr int kModeNoKeys = kSortModeNoKeys;

// status word: [63:56] pass tag, [55:54] flag, [31:0] count
constexpr uint64_t kFlagAgg = 1ull << 54;
constexpr uint64_t kFlagPre = 2ull << 54;
constexpr uint64_t kCountMask = 0xffffffffull;
constexpr int kSpinLimit = 1 << 22;

__device__ __forceinline__ int64_t live(const int64_t *n_dev, int64_t n_max) {
    int64_t n = *n_dev;
    return n < 0 ? 0 : (n > n_max ? n_max : n);
}

__device__ __forceinline__ int64_t n_tiles(int64_t n) { return (n + kTileN - 1) / kTileN; }

__global__ void k_sort_init(int32_t *ctl, uint32_t *ghist, int32_t *tile_ctr, unsigned long long *kmin) {
    if (threadIdx.x == 0) *kmin = ~0ull;
    for (int i = threadIdx.x; i < 64; i += blockDim.x) ctl[i] = 0;
    for (int i = threadIdx.x; i < 8; i += blockDim.x) tile_ctr[i] = 0;
    for (int i = threadIdx.x; i < 8 * 256; i += blockDim.x) ghist[i] = 0;
}

__global__ void k_status_clear(uint64_t *__restrict__ status, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        status[i] = 0;
}

// Smallest key.  The passes sort key - kmin, which has the same order and,
// for keys spanning less than 2^56, a constant top digit (one pass fewer).
__global__ __launch_bounds__(1024) void k_key_min(const uint64_t *__restrict__ keys, const int64_t *n_dev,
                                                  int64_t n_max, unsigned long long *__restrict__ kmin) {
    __shared__ unsigned long long s_min[1024 / kWave];
    const int64_t n = live(n_dev, n_max);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long m = ~0ull;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {  // four loads in flight
        const unsigned long long a = keys[i], b = keys[i + stride], c = keys[i + 2 * stride],
                                 d = keys[i + 3 * stride];
        const unsigned long long ab = a < b ? a : b, cd = c < d ? c : d;
        const unsigned long long x = ab < cd ? ab : cd;
        m = x < m ? x : m;
    }
    for (; i < n; i += stride) {
        const unsigned long long k = keys[i];
        m = k < m ? k : m;
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const unsigned long long y = __shfl_xor(m, o);
        m = y < m ? y : m;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) s_min[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / kWave); ++w) m = s_min[w] < m ? s_min[w] : m;
        if (m != ~0ull) atomicMin(kmin, m);  // one atomic per workgroup
    }
}

// Global histograms of all eight digits of key - kmin.
__global__ __launch_bounds__(kThreads) void k_global_hist(const uint64_t *__restrict__ keys, const int64_t *n_dev,
                                                          int64_t n_max, const unsigned long long *__restrict__ kmin,
                                                          uint32_t *__restrict__ ghist) {
    __shared__ uint32_t h[8][256];
    for (int i = threadIdx.x; i < 8 * 256; i += kThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t n = live(n_dev, n_max);
    const uint64_t k0 = *kmin;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        uint64_t k = keys[i] - k0;
        const uint64_t active = __ballot(true);
        const int leader = __ffsll((unsigned long long)active) - 1;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const uint32_t dg = (uint32_t)(k >> (8 * d)) & 255u;
            // a digit the whole wavefront shares (the high digits mostly):
            // one add of the lane count instead of colliding lane atomics
            const uint32_t first = __builtin_amdgcn_readfirstlane(dg);
            if (__ballot(dg == first) == active) {
                if (lane_id() == leader) atomicAdd(&h[d][first], (uint32_t)__popcll(active));
            } else {
                atomicAdd(&h[d][dg], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * 256; i += kThreads) {
        uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&ghist[i], v);
    }
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
    __syncthreads();
    return x - v + add;
}

// Per digit: skip flag, bucket bases (exclusive scan of the global
// histogram), the buffer each pass reads and the key widths it moves.  One
// workgroup of 256.  With prefix_digits > 0 only the highest prefix_digits
// digits below the top non-constant one are sorted (the lower digits are
// skipped), and ctl[kCtlPrefixShift] receives the lowest sorted bit: the
// keys then leave grouped by (key - kmin) >> that shift, in input order
// within a group (64 when no digit varies).
__global__ __launch_bounds__(kThreads) void k_plan(const uint32_t *__restrict__ ghist, const int64_t *n_dev,
                                                   int64_t n_max, int key_form, int prefix_digits, int32_t *ctl,
                                                   uint32_t *__restrict__ gbase) {
    __shared__ uint32_t s_wave[kThreads / kWave];
    __shared__ int s_full;
    __shared__ int s_const[8];
    const int64_t n = live(n_dev, n_max);
    for (int d = 0; d < 8; ++d) {
        if (threadIdx.x == 0) s_full = 0;
        __syncthreads();
        const uint32_t c = ghist[d * 256 + threadIdx.x];
        if ((int64_t)c == n) s_full = 1;
        gbase[d * 256 + threadIdx.x] = block_excl_scan_256(c, s_wave);
        if (threadIdx.x == 0) s_const[d] = (s_full != 0 || n <= 1) ? 1 : 0;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int top = -1;
        for (int d = 0; d < 8; ++d)
            if (!s_const[d]) top = d;
        const int low = prefix_digits > 0 ? top - prefix_digits + 1 : 0;
        int active = 0;
        int skip[8], modes[8];
        for (int d = 0; d < 8; ++d) {
            skip[d] = (s_const[d] || d < low) ? 1 : 0;
            ctl[kCtlSkip + d] = skip[d];
            ctl[kCtlSrc + d] = active & 1;
            active += skip[d] ? 0 : 1;
        }
        ctl[kCtlFinal] = active & 1;
        ctl[kCtlPrefixShift] = top < 0 ? 64 : 8 * (low > 0 ? low : 0);
        int first = 8;
        for (int d = 7; d >= 0; --d)
            if (!skip[d]) first = d;
        ctl[kCtlFirst] = first;
        ctl[kCtlBase] = sort_pass_modes(skip, key_form, modes);
        for (int d = 0; d < 8; ++d) ctl[kCtlMode + d] = modes[d];
    }
}

// Exclusive scan over the NT threads of a block (one value per thread).
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_wave) {
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
    __syncthreads();
    return x - v + add;
}

// A pass over one tile of kTileN pairs with kSweepThreads threads: threads
// below 256 own one digit each (histogram, look-back, bucket bases).  The
// per-wave digit counts and the tile histogram share LDS with the staged
// keys (they are dead before the tile is staged), and the values are loaded
// only for the staging, after the look-back: 50 KB of LDS and at most 80
// registers let three workgroups share a compute unit, so one tile's
// look-back and loads overlap the others' work.  Each element finds its slot
// with one LDS read (per-wave offsets that start at the digit's local start)
// and its destination with one more (a per-digit distance).
constexpr int kSweepThreads = 512;
constexpr int kSweepRounds = kTileN / kSweepThreads;
constexpr int kSweepWavesPerSimd = 6;

template <int Tag, bool Persistent>
__global__ __launch_bounds__(kSweepThreads, kSweepWavesPerSimd) void k_onesweep(
    uint64_t *__restrict__ k0, uint64_t *__restrict__ k1, uint32_t *__restrict__ v0, uint32_t *__restrict__ v1,
    const int64_t *n_dev, int64_t n_max, int shift, int32_t *ctl, int pass, const uint32_t *__restrict__ gbase,
    const unsigned long long *__restrict__ kmin, uint64_t *__restrict__ status, int32_t *__restrict__ tile_ctr) {
    if (ctl[kCtlSkip + pass]) return;
    constexpr int kWaves = kSweepThreads / kWave;
    constexpr int kPerWave = kTileN / kWaves;  // contiguous slice of the tile per wavefront
    __shared__ union {
        uint64_t key[kTileN];  // the ranked tile, staged for the write-out
        struct {
            uint32_t wrun[kWaves][256];  // per-wave count, then per-wave offset, per digit
            uint32_t hist[256];
        } rank;
    } s_u;
    static_assert(sizeof(s_u.rank) <= sizeof(s_u.key), "ranking state must fit the staging buffer");
    __shared__ uint32_t s_val[kTileN];
    __shared__ uint32_t s_delta[256];  // destination start minus local start, per digit
    __shared__ uint32_t s_wave[kWaves];
    uint32_t *const s_hist = s_u.rank.hist;
    uint32_t (*const s_wrun)[256] = s_u.rank.wrun;
    uint64_t *const s_key = s_u.key;
    __shared__ int64_t s_tile;
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    const int lane = tid & (kWave - 1);
    const bool digit_owner = tid < 256;
    // one tile per workgroup, or (Persistent) tiles in ticket order until
    // none is left; a workgroup holds a ticket only while it works on that
    // tile, so every look-back waits on tiles that are running or done
    for (;;) {
        if (tid == 0) s_tile = atomicAdd(&tile_ctr[pass], 1);
        if (digit_owner) {
            s_hist[tid] = 0;
            for (int q = 0; q < kWaves; ++q) s_wrun[q][tid] = 0;
        }
        __syncthreads();
        const int64_t tile = s_tile;
        const int64_t n = live(n_dev, n_max);
        const int64_t base = tile * kTileN;
        if (base >= n) break;
        const bool src1 = ctl[kCtlSrc + pass] != 0;
        const uint64_t *ks = src1 ? k1 : k0;
        const uint32_t *vs = src1 ? v1 : v0;
        uint64_t *kd = src1 ? k0 : k1;
        uint32_t *vd = src1 ? v0 : v1;
        const int m = (int)(n - base < kTileN ? n - base : kTileN);
        const uint64_t kbase = *kmin;
        const int mode = ctl[kCtlMode + pass];
        const bool in32 = (mode & kModeIn32) != 0;
        const int nshift = ctl[kCtlBase];  // 32-bit keys hold key - kmin from this bit up
        // 64-bit keys are held as read; 32-bit keys are zero-extended
        auto digit = [&](uint64_t key) -> uint32_t {
            return in32 ? (uint32_t)(key >> (shift - nshift)) & 255u : (uint32_t)((key - kbase) >> shift) & 255u;
        };
        const uint32_t *ks32 = reinterpret_cast<const uint32_t *>(ks);

        // element (w, r, lane) is tile element w * kPerWave + r * 64 + lane, so
        // (wave, round, lane) order is index order; all loads in flight at once
        uint64_t kr[kSweepRounds];
    #pragma unroll
        for (int r = 0; r < kSweepRounds; ++r) {
            const int li = w * kPerWave + r * kWave + lane;
            kr[r] = li < m ? (in32 ? (uint64_t)ks32[base + li] : ks[base + li]) : 0ull;
        }
        // per element: its digit, later (wave-local rank << 8 | digit), later its
        // slot in the ranked tile (one register per element across the look-back)
        uint32_t dp[kSweepRounds];
    #pragma unroll
        for (int r = 0; r < kSweepRounds; ++r) {
            dp[r] = digit(kr[r]);
            if (w * kPerWave + r * kWave + lane < m) atomicAdd(&s_hist[dp[r]], 1u);
        }
        __syncthreads();
        const uint32_t cnt = digit_owner ? s_hist[tid] : 0u;

        // publish this tile's counts early, so later tiles' look-backs find them
        const uint64_t tag = (uint64_t)(pass + 1) << 56;
        if (digit_owner)
            __hip_atomic_store(&status[tile * 256 + tid], tag | (tile == 0 ? kFlagPre : kFlagAgg) | cnt,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        // wave-local ranking in index order: peers with the same digit by eight
        // ballots, a running count per digit in this wave's LDS row
        const uint64_t lt = lanemask_lt();
    #pragma unroll
        for (int r = 0; r < kSweepRounds; ++r) {
            const bool ok = w * kPerWave + r * kWave + lane < m;
            const uint32_t dg = dp[r];
            uint64_t peers = __ballot(ok);
    #pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (dg >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            const uint32_t rank = (uint32_t)__popcll(peers & lt);
            const uint32_t run = s_wrun[w][dg];
            dp[r] |= (run + rank) << 8;
            if (ok && rank == 0) s_wrun[w][dg] = run + (uint32_t)__popcll(peers);
        }

        // look-back: this tile's offset inside bucket `tid`.  The status words of
        // kWindow earlier tiles are read together; they are consumed newest
        // first until a prefix is found, waiting only on words not yet published.
        uint64_t excl = 0;
        if (digit_owner && tile > 0) {
            constexpr int kWindow = 4;
            const uint64_t ready_tag = (uint64_t)(pass + 1);
            int64_t t = tile - 1;
            int spins = 0;
            bool done = false;
            while (!done) {
                uint64_t v[kWindow];
    #pragma unroll
                for (int i = 0; i < kWindow; ++i)
                    v[i] = t - i >= 0 ? __hip_atomic_load(&status[(t - i) * 256 + tid], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : 0ull;  // never consumed: tile 0 always holds a prefix
    #pragma unroll
                for (int i = 0; i < kWindow; ++i) {
                    if (done) break;
                    uint64_t x = v[i];
                    while ((x >> 56) != ready_tag || (x & (kFlagAgg | kFlagPre)) == 0) {
                        if (++spins > kSpinLimit) {  // cannot happen while every earlier tile runs; bail out loudly
                            __hip_atomic_store(&ctl[kCtlError], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            x = ready_tag << 56 | kFlagPre;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        x = __hip_atomic_load(&status[(t - i) * 256 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    excl += x & kCountMask;
                    if (x & kFlagPre) done = true;
                }
                t -= kWindow;
            }
            __hip_atomic_store(&status[tile * 256 + tid], tag | kFlagPre | ((excl + cnt) & kCountMask),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();  // every wave's counts are final
        const uint32_t lo = block_excl_scan<kSweepThreads>(cnt, s_wave);
        if (digit_owner) {
            // per-wave offsets that start at the digit's local start, and the
            // distance from a staged slot to its destination
            uint32_t acc = lo;
    #pragma unroll
            for (int q = 0; q < kWaves; ++q) {
                const uint32_t c = s_wrun[q][tid];
                s_wrun[q][tid] = acc;
                acc += c;
            }
            s_delta[tid] = gbase[pass * 256 + tid] + (uint32_t)excl - lo;
        }
        __syncthreads();
    #pragma unroll
        for (int r = 0; r < kSweepRounds; ++r) {
            const uint32_t dg = dp[r] & 255u;
            dp[r] = (dp[r] >> 8) + s_wrun[w][dg];  // slot in the ranked tile
        }
        __syncthreads();  // the counts are read; their storage becomes the staged keys
        uint32_t vr[kSweepRounds];
    #pragma unroll
        for (int r = 0; r < kSweepRounds; ++r) {
            const int li = w * kPerWave + r * kWave + lane;
            vr[r] = li < m ? vs[base + li] : 0u;
        }
    #pragma unroll
        for (int r = 0; r < kSweepRounds; ++r) {
            if (w * kPerWave + r * kWave + lane < m) {
                s_key[dp[r]] = kr[r];
                s_val[dp[r]] = vr[r];
            }
        }
        __syncthreads();
        // leave in digit order: consecutive slots of one digit are consecutive destinations
    #pragma unroll
        for (int r = 0; r < kSweepRounds; ++r) {
            const int j = r * kSweepThreads + tid;
            if (j < m) {
                const uint64_t key = s_key[j];
                const uint32_t dg = digit(key);
                const uint32_t pos = s_delta[dg] + (uint32_t)j;
                if (mode & kModeOut32)
                    reinterpret_cast<uint32_t *>(kd)[pos] = in32 ? (uint32_t)key : (uint32_t)((key - kbase) >> nshift);
                else if (!(mode & kModeNoKeys))
                    kd[pos] = key;
                vd[pos] = s_val[j];
            }
        }
        if (!Persistent) break;
        __syncthreads();  // the staged tile is written out before the next tile reuses LDS
    }
}

}  // namespace

size_t sort_workspace(int64_t n_max, Carve &c, SortBuffers *b) {
    const int64_t tiles = (n_max + kTileN - 1) / kTileN > 0 ? (n_max + kTileN - 1) / kTileN : 1;
    SortBuffers x;
    x.keys[0] = c.take<uint64_t>(n_max);
    x.keys[1] = c.take<uint64_t>(n_max);
    x.vals[0] = c.take<uint32_t>(n_max);
    x.vals[1] = c.take<uint32_t>(n_max);
    x.status = c.take<uint64_t>(256 * tiles);
    x.n_status = 256 * tiles;
    x.ghist = c.take<uint32_t>(8 * 256);
    x.gbase = c.take<uint32_t>(8 * 256);
    x.tile_ctr = c.take<int32_t>(8);
    x.kmin = c.take<unsigned long long>(1);
    x.ctl = c.take<int32_t>(64);
    if (b) *b = x;
    return c.bytes();
}

int radix_sort_init(const SortBuffers &b, hipStream_t st) {
    JB_LAUNCH(k_sort_init, dim3(1), dim3(256), 0, st, b.ctl, b.ghist, b.tile_ctr, b.kmin);
    JB_LAUNCH_CHECK();
    int64_t blocks = (b.n_status + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    JB_LAUNCH(k_status_clear, dim3((unsigned)blocks), dim3(256), 0, st, b.status, b.n_status);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

int radix_global_hist(const SortBuffers &b, const int64_t *n_dev, int64_t n_max, hipStream_t st) {
    int64_t blocks = (n_max + kThreads * 8 - 1) / (kThreads * 8);
    int cap = device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    const int64_t min_blocks = (n_max + 1023) / 1024 < device_cu_count() ? (n_max + 1023) / 1024 : device_cu_count();
    JB_LAUNCH(k_key_min, dim3((unsigned)(min_blocks < 1 ? 1 : min_blocks)), dim3(1024), 0, st, b.keys[0], n_dev,
              n_max, b.kmin);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_global_hist, dim3((unsigned)blocks), dim3(kThreads), 0, st, b.keys[0], n_dev, n_max, b.kmin,
              b.ghist);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

namespace {
const char *pass_timer_name(const char *tag) {
    if (!tag || !tag[0]) return "k_onesweep";
    switch (tag[0]) {
        case 'g': return "k_onesweep_groups";
        case 'l': return "k_onesweep_large";
        case 'p': return "k_onesweep_points";
        case 'k': return "k_onesweep_kmeans";
        case 'r': return "k_onesweep_remap";
        default: return "k_onesweep_other";
    }
}
}  // namespace

int radix_sort_pairs(const SortBuffers &b, const int64_t *n_dev, int64_t n_max, hipStream_t st, const char *tag,
                     int key_form, bool sparse, int prefix_digits) {
    const bool main_sort = !tag || !tag[0];
    const int64_t tiles = (n_max + kTileN - 1) / kTileN > 0 ? (n_max + kTileN - 1) / kTileN : 1;
    JB_LAUNCH(k_plan, dim3(1), dim3(kThreads), 0, st, b.ghist, n_dev, n_max, key_form, prefix_digits, b.ctl,
              b.gbase);
    // A sparse sort's live count is far below its bound and known only on
    // the device: its passes run persistent workgroups, at most the resident
    // ones (three per compute unit), instead of one workgroup per possible
    // tile.
    const int64_t cap = (int64_t)device_cu_count() * 3;
    const int64_t grid = tiles < cap ? tiles : cap;
    JB_LAUNCH_CHECK();
    // the eight passes run back to back and are timed as one group of eight
    // launches, so the per-launch figure carries no event of its own
    KernelTimer timer(pass_timer_name(tag), st, 8);
    for (int pass = 0; pass < 8; ++pass) {
        hipLaunchKernelGGL(sparse ? (k_onesweep<1, true>) : main_sort ? (k_onesweep<0, false>) : (k_onesweep<1, false>),
                           dim3((unsigned)(sparse ? grid : tiles)), dim3(kSweepThreads), 0, st, b.keys[0], b.keys[1],
                           b.vals[0], b.vals[1], n_dev, n_max, 8 * pass, b.ctl, pass, b.gbase, b.kmin, b.status,
                           b.tile_ctr);
        JB_LAUNCH_CHECK();
    }
    return JABBA_OK;
}

}  // namespace jabba
