// Phase III of Alg. 1: global digitization with the two-stage aggregation of
// Sec. 5, and the dictionary of symbolic centers (Sec. 3.2).
//
// Data flow (N pieces, all counts stay on the device):
//   len/inc (canonical) --sum passes--> sigma_len, sigma_inc
//   --k_key--> (key bits, index) --radix sort--> sorted order (perm)
//   --k_gather--> sorted arrays key/x/y/len/inc (contiguous for Stage I)
//   --k_cuts--> blocks of B sorted pieces, cuts moved past equal keys
//   --k_stage1 (one wavefront per block)--> local start per piece, start flags,
//       per-start partial sums (count, len, inc)
//   --scan + k_compact_starts--> S: starting points in sorted order
//   --k_stage2--> global start per element of S, partial sums per global group
//   --scan--> symbol numbers; k_dict writes the dictionary; k_remap sends
//   each piece's symbol back to canonical order (label propagation).
//
// Decisions use binary64 with no contraction, in the order of the sequential
// definition, so local starts, blocks and symbols are bit-identical to it.
#include "common.h"

namespace jabba {

namespace {

constexpr int kTreeLeaves = 1024;  // leaves per workgroup in the pairwise sums
constexpr int kLdsBitWords = 1024; // 65,536 points per LDS bitmap

__device__ __forceinline__ int64_t live(const int64_t *n_dev, int64_t n_max) {
    int64_t n = *n_dev;
    return n < 0 ? 0 : (n > n_max ? n_max : n);
}

struct DigState {
    int32_t status[64];
    unsigned long long lsum[2];  // sum len, sum len^2
    double mean_inc;
    double sigma_len;
    double sigma_inc;
    int64_t n;  // live piece count (clamped)
};

__global__ void k_dig_prepare(DigState *ds, const int64_t *n_dev, int64_t n_max) {
    if (threadIdx.x == 0) {
        ds->status[0] = 0;
        ds->lsum[0] = 0;
        ds->lsum[1] = 0;
        int64_t n = *n_dev;
        if (n > n_max || n < 0) set_status(ds->status, kStOverflow);
        ds->n = n < 0 ? 0 : (n > n_max ? n_max : n);
    }
}

// Pairwise tree over 1024 leaves: 4 adjacent leaves per thread, then the
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

// level 0: leaves are inc (pass 1) or (inc - mean)^2 (pass 2); pass 1 also
// accumulates the exact integer sums of len and len^2.
template <int Pass>
__global__ __launch_bounds__(256) void k_sum_leaves(const int32_t *__restrict__ len, const double *__restrict__ inc,
                                                    DigState *ds, double *__restrict__ out) {
    const int64_t n = ds->n;
    const int64_t base = (int64_t)blockIdx.x * kTreeLeaves + 4 * threadIdx.x;
    double a[4];
    unsigned long long s1 = 0, s2 = 0;
    const double mean = Pass == 2 ? ds->mean_inc : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t idx = base + i;
        double v = 0.0;
        if (idx < n) {
            v = inc[idx];
            if (Pass == 2) {
                const double d = v - mean;
                v = d * d;
            } else {
                const unsigned long long l = (unsigned long long)len[idx];
                s1 += l;
                s2 += l * l;
            }
        }
        a[i] = v;
    }
    const double r = block_tree_1024(a[0], a[1], a[2], a[3]);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
    if (Pass == 1) {
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            s1 += __shfl_xor(s1, m);
            s2 += __shfl_xor(s2, m);
        }
        if (lane_id() == 0 && s1) {
            atomicAdd(&ds->lsum[0], s1);
            atomicAdd(&ds->lsum[1], s2);
        }
    }
}

// level l >= 1: groups of 1024 partial sums of level l-1, zero padded
__global__ __launch_bounds__(256) void k_sum_level(const double *__restrict__ in, const DigState *ds, int level,
                                                   double *__restrict__ out) {
    int64_t m = ds->n;
    for (int l = 0; l < level; ++l) m = (m + kTreeLeaves - 1) / kTreeLeaves;  // entries of level-1 output
    const int64_t base = (int64_t)blockIdx.x * kTreeLeaves + 4 * threadIdx.x;
    double a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = base + i < m ? in[base + i] : 0.0;
    const double r = block_tree_1024(a[0], a[1], a[2], a[3]);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
}

__global__ void k_mean(DigState *ds, const double *total) {
    if (threadIdx.x == 0) {
        const int64_t n = ds->n;
        ds->mean_inc = n > 0 ? (*total) / (double)n : 0.0;
    }
}

__global__ void k_sigma(DigState *ds, const double *total2, double scl, double alpha, double *params) {
    if (threadIdx.x != 0) return;
    const int64_t n = ds->n;
    double sl = 1.0, si = 1.0;
    if (n > 0) {
        const double mean_len = (double)(int64_t)ds->lsum[0] / (double)n;
        double var_len = (double)(int64_t)ds->lsum[1] / (double)n - mean_len * mean_len;
        if (var_len < 0.0) var_len = 0.0;
        sl = __dsqrt_rn(var_len);
        const double var_inc = (*total2) / (double)n;
        si = __dsqrt_rn(var_inc);
        if (!(sl > 0.0)) sl = 1.0;
        if (!(si > 0.0)) si = 1.0;
    }
    ds->sigma_len = sl;
    ds->sigma_inc = si;
    if (params) {
        params[0] = sl;
        params[1] = si;
        params[2] = scl;
        params[3] = alpha;
    }
}

__global__ void k_key(const int32_t *__restrict__ len, const double *__restrict__ inc, const DigState *ds, double scl,
                      uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t n = ds->n;
    const double sl = ds->sigma_len, si = ds->sigma_inc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const Scaled s = scale_piece(len[i], inc[i], scl, sl, si);
        keys[i] = (uint64_t)__double_as_longlong(piece_key(s));
        vals[i] = (uint32_t)i;
    }
}

__global__ void k_gather(const int32_t *__restrict__ len, const double *__restrict__ inc, const DigState *ds,
                         double scl, const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                         const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1, const int32_t *ctl,
                         double *__restrict__ sk, double *__restrict__ sx, double *__restrict__ sy,
                         int32_t *__restrict__ slen, double *__restrict__ sinc, uint32_t *__restrict__ perm) {
    const int64_t n = ds->n;
    const double sl = ds->sigma_len, si = ds->sigma_inc;
    const uint64_t *ks = ctl[0] ? k1 : k0;
    const uint32_t *vs = ctl[0] ? v1 : v0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = vs[p];
        const int32_t l = len[c];
        const double ic = inc[c];
        const Scaled s = scale_piece(l, ic, scl, sl, si);
        sk[p] = __longlong_as_double((long long)ks[p]);
        sx[p] = s.x;
        sy[p] = s.y;
        slen[p] = l;
        sinc[p] = ic;
        perm[p] = c;
    }
}

// cut j: first position >= j*B whose key differs from its predecessor
__global__ void k_cuts(const double *__restrict__ sk, const DigState *ds, int64_t B, int64_t nblk_max,
                       int64_t *__restrict__ cuts) {
    const int64_t n = ds->n;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= nblk_max;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t p = j * B;
        if (j == 0)
            p = 0;
        else if (p >= n)
            p = n;
        else
            while (p < n && sk[p] == sk[p - 1]) ++p;
        cuts[j] = p;
    }
}

// ------------------------------------------------------------ aggregation
struct LdsBits {
    uint64_t *w;
    __device__ uint64_t load(int64_t i) const { return w[i]; }
    __device__ void store(int64_t i, uint64_t v) const { w[i] = v; }
    __device__ void orw(int64_t i, uint64_t m) const { w[i] |= m; }
    __device__ void fence() const {}
};

struct GlobalBits {
    uint64_t *w;
    __device__ uint64_t load(int64_t i) const {
        return __hip_atomic_load(&w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void store(int64_t i, uint64_t v) const {
        __hip_atomic_store(&w[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void orw(int64_t i, uint64_t m) const {
        __hip_atomic_fetch_or(&w[i], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void fence() const { __threadfence(); }
};

// member weights: Stage I points weigh (1, len, inc); Stage II points are
// Stage I groups and carry their partial sums
struct PointWeights {
    const int32_t *len;
    const double *inc;
    __device__ int64_t cnt(int64_t) const { return 1; }
    __device__ int64_t ln(int64_t q) const { return len[q]; }
    __device__ double ic(int64_t q) const { return inc[q]; }
};
struct GroupWeights {
    const int64_t *c;
    const int64_t *l;
    const double *i;
    __device__ int64_t cnt(int64_t q) const { return c[q]; }
    __device__ int64_t ln(int64_t q) const { return l[q]; }
    __device__ double ic(int64_t q) const { return i[q]; }
};

// Greedy aggregation of the presorted points [lo, hi) by one wavefront.
// The wavefront scans a start's alpha-window 64 points at a time; the
// assigned set is a bitmap (bit r = point lo + r).  lab[q] <- start position,
// flag[q] <- 1 for starts, 0 for members; for every start p the partial sums
// of its members: count and len exactly, inc as the start's value followed
// by one pairwise wavefront sum per 64-point chunk, chunks in order.
template <class Bits, class Wt>
__device__ void aggregate_wave(int64_t lo, int64_t hi, const double *__restrict__ key, const double *__restrict__ x,
                               const double *__restrict__ y, Wt wt, double alpha, double a2, Bits bits,
                               int32_t *__restrict__ lab, uint32_t *__restrict__ flag, int64_t *__restrict__ ocnt,
                               int64_t *__restrict__ olen, double *__restrict__ oinc) {
    const int lane = lane_id();
    const int64_t n = hi - lo;
    const int64_t nw = (n + 63) >> 6;
    for (int64_t i = lane; i < nw; i += kWave) {
        uint64_t v = 0ull;
        if (i == nw - 1 && (n & 63)) v = ~0ull << (n & 63);
        bits.store(i, v);
    }
    bits.fence();
    int64_t p = lo;
    while (p < hi) {
        const double kp = key[p], xp = x[p], yp = y[p];
        int64_t cacc = wt.cnt(p), lacc = wt.ln(p);
        double iacc = wt.ic(p);
        if (lane == 0) {
            lab[p] = (int32_t)p;
            flag[p] = 1u;
            bits.orw((p - lo) >> 6, 1ull << ((p - lo) & 63));
        }
        bits.fence();
        for (int64_t q0 = p + 1; q0 < hi; q0 += kWave) {
            const int64_t q = q0 + lane;
            const bool inr = q < hi;
            const double kq = inr ? key[q] : 0.0;
            const bool inwin = inr && (kq - kp <= alpha);
            bool claim = false;
            if (inwin) {
                const int64_t r = q - lo;
                const bool taken = (bits.load(r >> 6) >> (r & 63)) & 1ull;
                if (!taken) {
                    const double dx = x[q] - xp;
                    const double dy = y[q] - yp;
                    const double dd = dx * dx;
                    const double ee = dy * dy;
                    claim = (dd + ee) <= a2;
                }
            }
            const uint64_t cm = ballot(claim);
            if (cm) {
                if (claim) {
                    lab[q] = (int32_t)p;
                    flag[q] = 0u;
                }
                if (lane == 0) {
                    const int64_t r0 = q0 - lo;
                    const int sh = (int)(r0 & 63);
                    bits.orw(r0 >> 6, cm << sh);
                    if (sh) {
                        const uint64_t hw = cm >> (64 - sh);
                        if (hw) bits.orw((r0 >> 6) + 1, hw);
                    }
                }
                bits.fence();
                cacc += wave_sum_i64(claim ? wt.cnt(q) : 0);
                lacc += wave_sum_i64(claim ? wt.ln(q) : 0);
                iacc = iacc + wave_tree_sum(claim ? wt.ic(q) : 0.0);
            }
            if (ballot(inr && !inwin) != 0ull) break;
        }
        if (lane == 0) {
            ocnt[p] = cacc;
            olen[p] = lacc;
            oinc[p] = iacc;
        }
        // next unassigned point after p
        const int64_t from = p + 1 - lo;
        p = hi;
        for (int64_t w0 = from >> 6; w0 < nw; w0 += kWave) {
            const int64_t wi = w0 + lane;
            uint64_t v = wi < nw ? bits.load(wi) : ~0ull;
            if (wi == (from >> 6) && (from & 63)) v |= ~0ull >> (64 - (from & 63));
            const uint64_t fz = ballot(v != ~0ull);
            if (fz) {
                const int l = ffs64(fz);
                const uint64_t vl = __shfl(v, l);
                p = lo + ((w0 + l) << 6) + __builtin_ctzll(~vl);
                break;
            }
        }
    }
}

__global__ __launch_bounds__(1024) void k_stage1(const int64_t *__restrict__ cuts, int64_t nblk_max,
                                                 const double *__restrict__ sk, const double *__restrict__ sx,
                                                 const double *__restrict__ sy, const int32_t *__restrict__ slen,
                                                 const double *__restrict__ sinc, double alpha, double a2,
                                                 uint64_t *__restrict__ gbits, int32_t *__restrict__ lab,
                                                 uint32_t *__restrict__ flag, int64_t *__restrict__ pcnt,
                                                 int64_t *__restrict__ plen, double *__restrict__ pinc) {
    extern __shared__ uint64_t lds_bits[];
    const int wave = threadIdx.x / kWave;
    const int64_t blk = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    if (blk >= nblk_max) return;
    const int64_t lo = cuts[blk], hi = cuts[blk + 1];
    if (lo >= hi) return;
    PointWeights wt{slen, sinc};
    if (hi - lo <= (int64_t)kLdsBitWords * 64) {
        LdsBits b{lds_bits + (size_t)wave * kLdsBitWords};
        aggregate_wave(lo, hi, sk, sx, sy, wt, alpha, a2, b, lab, flag, pcnt, plen, pinc);
    } else {
        GlobalBits b{gbits + (lo >> 6) + blk};
        aggregate_wave(lo, hi, sk, sx, sy, wt, alpha, a2, b, lab, flag, pcnt, plen, pinc);
    }
}

__global__ void k_compact_starts(const DigState *ds, const uint32_t *__restrict__ flag,
                                 const uint32_t *__restrict__ sidx, const double *__restrict__ sk,
                                 const double *__restrict__ sx, const double *__restrict__ sy,
                                 const int64_t *__restrict__ pcnt, const int64_t *__restrict__ plen,
                                 const double *__restrict__ pinc, double *__restrict__ gk, double *__restrict__ gx,
                                 double *__restrict__ gy, int64_t *__restrict__ gcnt, int64_t *__restrict__ glen,
                                 double *__restrict__ ginc, int64_t *__restrict__ g_count) {
    const int64_t n = ds->n;
    if (blockIdx.x == 0 && threadIdx.x == 0) *g_count = (int64_t)sidx[n];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[p]) continue;
        const uint32_t g = sidx[p];
        gk[g] = sk[p];
        gx[g] = sx[p];
        gy[g] = sy[p];
        gcnt[g] = pcnt[p];
        glen[g] = plen[p];
        ginc[g] = pinc[p];
    }
}

__global__ __launch_bounds__(64) void k_stage2(const int64_t *__restrict__ g_count, const double *__restrict__ gk,
                                               const double *__restrict__ gx, const double *__restrict__ gy,
                                               const int64_t *__restrict__ gcnt, const int64_t *__restrict__ glen,
                                               const double *__restrict__ ginc, double alpha, double a2,
                                               uint64_t *__restrict__ gbits, int32_t *__restrict__ glab,
                                               uint32_t *__restrict__ gflag, int64_t *__restrict__ ocnt,
                                               int64_t *__restrict__ olen, double *__restrict__ oinc) {
    __shared__ uint64_t lds_bits[kLdsBitWords];
    const int64_t G = *g_count;
    if (G <= 0) return;
    GroupWeights wt{gcnt, glen, ginc};
    if (G <= (int64_t)kLdsBitWords * 64) {
        LdsBits b{lds_bits};
        aggregate_wave((int64_t)0, G, gk, gx, gy, wt, alpha, a2, b, glab, gflag, ocnt, olen, oinc);
    } else {
        GlobalBits b{gbits};
        aggregate_wave((int64_t)0, G, gk, gx, gy, wt, alpha, a2, b, glab, gflag, ocnt, olen, oinc);
    }
}

__global__ void k_dict(const int64_t *__restrict__ g_count, const uint32_t *__restrict__ gflag,
                       const uint32_t *__restrict__ gsym, const int64_t *__restrict__ ocnt,
                       const int64_t *__restrict__ olen, const double *__restrict__ oinc, DigState *ds, double scl,
                       jabba_dict dict) {
    const int64_t G = *g_count;
    const double sl = ds->sigma_len, si = ds->sigma_inc;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t k = G > 0 ? (int64_t)gsym[G] : 0;
        *dict.k = k;
        if (k > dict.capacity) set_status(ds->status, kStCapacity);
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
        if (!gflag[g]) continue;
        const int64_t c = gsym[g];
        if (c >= dict.capacity) continue;
        const int64_t cnt = ocnt[g];
        const double cl = (double)olen[g] / (double)cnt;
        const double ci = oinc[g] / (double)cnt;
        dict.count[c] = cnt;
        dict.center_len[c] = cl;
        dict.center_inc[c] = ci;
        dict.cx[c] = scl * (cl / sl);
        dict.cy[c] = ci / si;
    }
}

__global__ void k_remap(const DigState *ds, const uint32_t *__restrict__ perm, const int32_t *__restrict__ lab,
                        const uint32_t *__restrict__ sidx, const int32_t *__restrict__ glab,
                        const uint32_t *__restrict__ gsym, int32_t *__restrict__ symbols) {
    const int64_t n = ds->n;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t g = sidx[lab[p]];
        symbols[perm[p]] = (int32_t)gsym[glab[g]];
    }
}

struct DigWs {
    DigState *ds;
    double *tree[2];
    SortBuffers sb;
    double *sk, *sx, *sy, *sinc;
    int32_t *slen;
    uint32_t *perm;
    int64_t *cuts;
    int32_t *lab;
    uint32_t *flag;
    uint32_t *sidx;
    int64_t *pcnt, *plen;
    double *pinc;
    double *gk, *gx, *gy, *ginc;
    int64_t *gcnt, *glen;
    int64_t *g_count;
    int32_t *glab;
    uint32_t *gflag;
    uint32_t *gsym;
    int64_t *ocnt, *olen;
    double *oinc;
    uint64_t *gbits;
    void *scan_ws;
    size_t bytes;
};

int64_t nblk_of(int64_t max_pieces, int64_t B) { return (max_pieces + B - 1) / B; }

DigWs carve_digitize(void *ws, int64_t max_pieces, int64_t B) {
    const int64_t N = max_pieces > 0 ? max_pieces : 1;
    const int64_t nblk = nblk_of(N, B);
    Carve c(ws);
    DigWs w;
    w.ds = c.take<DigState>(1);
    const int64_t t0 = (N + kTreeLeaves - 1) / kTreeLeaves;
    w.tree[0] = c.take<double>(t0 + 1);
    w.tree[1] = c.take<double>((t0 + kTreeLeaves - 1) / kTreeLeaves + 1);
    sort_workspace(N, c, &w.sb);
    w.sk = c.take<double>(N);
    w.sx = c.take<double>(N);
    w.sy = c.take<double>(N);
    w.sinc = c.take<double>(N);
    w.slen = c.take<int32_t>(N);
    w.perm = c.take<uint32_t>(N);
    w.cuts = c.take<int64_t>(nblk + 2);
    w.lab = c.take<int32_t>(N);
    w.flag = c.take<uint32_t>(N);
    w.sidx = c.take<uint32_t>(N + 1);
    w.pcnt = c.take<int64_t>(N);
    w.plen = c.take<int64_t>(N);
    w.pinc = c.take<double>(N);
    w.gk = c.take<double>(N);
    w.gx = c.take<double>(N);
    w.gy = c.take<double>(N);
    w.ginc = c.take<double>(N);
    w.gcnt = c.take<int64_t>(N);
    w.glen = c.take<int64_t>(N);
    w.g_count = c.take<int64_t>(1);
    w.glab = c.take<int32_t>(N);
    w.gflag = c.take<uint32_t>(N);
    w.gsym = c.take<uint32_t>(N + 1);
    w.ocnt = c.take<int64_t>(N);
    w.olen = c.take<int64_t>(N);
    w.oinc = c.take<double>(N);
    w.gbits = c.take<uint64_t>(N / 64 + nblk + 4);
    w.scan_ws = c.take<char>(scan_workspace(N + 1));
    w.bytes = c.bytes();
    return w;
}

unsigned grid_for(int64_t n, int per_cu = 8) {
    int64_t b = (n + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// sum of the level-0 leaves through all levels; returns the pointer holding
// the final value
int tree_sum_levels(const DigWs &w, int64_t N, double *level0, hipStream_t st, double **result) {
    int64_t m = (N + kTreeLeaves - 1) / kTreeLeaves;  // level-0 outputs
    double *in = level0;
    int which = 1;
    int level = 1;
    while (m > 1) {
        const int64_t blocks = (m + kTreeLeaves - 1) / kTreeLeaves;
        double *out = w.tree[which];
        JB_LAUNCH(k_sum_level, dim3((unsigned)blocks), dim3(256), 0, st, in, w.ds, level, out);
        JB_LAUNCH_CHECK();
        in = out;
        which ^= 1;
        m = blocks;
        ++level;
    }
    *result = in;
    return JABBA_OK;
}

}  // namespace

}  // namespace jabba

using namespace jabba;

extern "C" int jabba_digitize_workspace(int64_t max_pieces, int32_t B, size_t *bytes) {
    if (!bytes || max_pieces < 0 || B < 1) return JABBA_EINVAL;
    *bytes = carve_digitize(nullptr, max_pieces, B).bytes;
    return JABBA_OK;
}

extern "C" int jabba_digitize(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                              double alpha, double scl, int32_t B, const jabba_tuning *tuning, int32_t *symbols,
                              const jabba_dict *dict, void *workspace, size_t workspace_bytes, void *stream) {
    if (max_pieces < 0 || B < 1 || !n_pieces || !dict) return JABBA_EINVAL;
    if (!(alpha >= 0.0) || !(alpha <= 1.0e150) || !(scl >= 0.0) || !(scl <= 1.0e150)) return JABBA_EINVAL;
    if (max_pieces >= ((int64_t)1 << 31) - 1) return JABBA_EOVERFLOW;
    if (max_pieces > 0 && (!len || !inc || !symbols)) return JABBA_EINVAL;
    if (dict->capacity < 0 || !dict->k || (dict->capacity > 0 && (!dict->center_len || !dict->center_inc ||
                                                                  !dict->cx || !dict->cy || !dict->count)))
        return JABBA_EINVAL;
    const DigWs w0 = carve_digitize(nullptr, max_pieces, B);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    const DigWs w = carve_digitize(workspace, max_pieces, B);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = max_pieces > 0 ? max_pieces : 1;
    const int64_t nblk = nblk_of(N, B);
    int s1w = 4;
    if (tuning && tuning->stage1_waves) s1w = tuning->stage1_waves;
    if (s1w < 1 || s1w > 16) return JABBA_EINVAL;
    const double a2 = alpha * alpha;

    JB_LAUNCH(k_dig_prepare, dim3(1), dim3(64), 0, st, w.ds, n_pieces, max_pieces);
    JB_LAUNCH_CHECK();
    // scaling: two pairwise-sum passes over inc, exact integer sums of len
    const int64_t t0 = (N + kTreeLeaves - 1) / kTreeLeaves;
    JB_LAUNCH((k_sum_leaves<1>), dim3((unsigned)t0), dim3(256), 0, st, len, inc, w.ds, w.tree[0]);
    JB_LAUNCH_CHECK();
    double *tot = nullptr;
    int rc = tree_sum_levels(w, N, w.tree[0], st, &tot);
    if (rc) return rc;
    JB_LAUNCH(k_mean, dim3(1), dim3(64), 0, st, w.ds, tot);
    JB_LAUNCH_CHECK();
    JB_LAUNCH((k_sum_leaves<2>), dim3((unsigned)t0), dim3(256), 0, st, len, inc, w.ds, w.tree[0]);
    JB_LAUNCH_CHECK();
    rc = tree_sum_levels(w, N, w.tree[0], st, &tot);
    if (rc) return rc;
    JB_LAUNCH(k_sigma, dim3(1), dim3(64), 0, st, w.ds, tot, scl, alpha, dict->params);
    JB_LAUNCH_CHECK();

    // key and global sorting index
    rc = radix_sort_init(w.sb, st);
    if (rc) return rc;
    JB_LAUNCH(k_key, dim3(grid_for(N)), dim3(256), 0, st, len, inc, w.ds, scl, w.sb.keys[0], w.sb.vals[0]);
    JB_LAUNCH_CHECK();
    const int64_t *n_live = &w.ds->n;
    rc = radix_global_hist(w.sb, n_live, N, st);
    if (rc) return rc;
    rc = radix_sort_pairs(w.sb, n_live, N, st);
    if (rc) return rc;
    JB_LAUNCH(k_gather, dim3(grid_for(N)), dim3(256), 0, st, len, inc, w.ds, scl, w.sb.keys[0],
                       w.sb.keys[1], w.sb.vals[0], w.sb.vals[1], w.sb.ctl, w.sk, w.sx, w.sy, w.slen, w.sinc, w.perm);
    JB_LAUNCH_CHECK();

    // Stage I
    JB_LAUNCH(k_cuts, dim3(grid_for(nblk + 1)), dim3(256), 0, st, w.sk, w.ds, (int64_t)B, nblk, w.cuts);
    JB_LAUNCH_CHECK();
    const size_t lds = (size_t)s1w * kLdsBitWords * sizeof(uint64_t);
    JB_LAUNCH(k_stage1, dim3((unsigned)((nblk + s1w - 1) / s1w)), dim3(s1w * kWave), lds, st, w.cuts, nblk,
                       w.sk, w.sx, w.sy, w.slen, w.sinc, alpha, a2, w.gbits, w.lab, w.flag, w.pcnt, w.plen, w.pinc);
    JB_LAUNCH_CHECK();
    rc = scan_u32_to_u32(w.flag, w.sidx, n_live, N, w.scan_ws, st);
    if (rc) return rc;
    JB_LAUNCH(k_compact_starts, dim3(grid_for(N)), dim3(256), 0, st, w.ds, w.flag, w.sidx, w.sk, w.sx, w.sy,
                       w.pcnt, w.plen, w.pinc, w.gk, w.gx, w.gy, w.gcnt, w.glen, w.ginc, w.g_count);
    JB_LAUNCH_CHECK();

    // Stage II over the starting points, then numbering of global groups
    JB_LAUNCH(k_stage2, dim3(1), dim3(64), 0, st, w.g_count, w.gk, w.gx, w.gy, w.gcnt, w.glen, w.ginc, alpha,
                       a2, w.gbits, w.glab, w.gflag, w.ocnt, w.olen, w.oinc);
    JB_LAUNCH_CHECK();
    rc = scan_u32_to_u32(w.gflag, w.gsym, w.g_count, N, w.scan_ws, st);
    if (rc) return rc;
    JB_LAUNCH(k_dict, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.gflag, w.gsym, w.ocnt, w.olen,
                       w.oinc, w.ds, scl, *dict);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_remap, dim3(grid_for(N)), dim3(256), 0, st, w.ds, w.perm, w.lab, w.sidx, w.glab, w.gsym,
                       symbols);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

extern "C" int jabba_digitize_stats(const void *workspace, int64_t max_pieces, int32_t B, void *stream,
                                    int64_t *stats) {
    if (!workspace || !stats || max_pieces < 0 || B < 1) return JABBA_EINVAL;
    const DigWs w = carve_digitize(const_cast<void *>(workspace), max_pieces, B);
    JB_HIP(hipStreamSynchronize((hipStream_t)stream));
    DigState ds;
    int64_t G = 0;
    int32_t ctl[9] = {0};
    JB_HIP(hipMemcpy(&ds, w.ds, sizeof(DigState), hipMemcpyDeviceToHost));
    JB_HIP(hipMemcpy(&G, w.g_count, sizeof(int64_t), hipMemcpyDeviceToHost));
    JB_HIP(hipMemcpy(ctl, w.sb.ctl, sizeof(ctl), hipMemcpyDeviceToHost));
    uint32_t k = 0;
    if (G > 0) JB_HIP(hipMemcpy(&k, w.gsym + G, sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t active = 0;
    for (int d = 0; d < 8; ++d) active += ctl[1 + d] ? 0 : 1;
    stats[0] = ds.n;
    stats[1] = G;
    stats[2] = k;
    stats[3] = active;
    return JABBA_OK;
}
