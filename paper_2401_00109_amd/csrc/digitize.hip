// Phase III of Alg. 1: global digitization with the two-stage aggregation of
// Sec. 5, and the dictionary of symbolic centers (Sec. 3.2).
//
// Data flow (N pieces, all counts stay on the device):
//   len/inc (canonical) --sum passes--> sigma_len, sigma_inc
//   --k_key--> (key bits, index), piece records --radix passes over the
//       highest four varying digits--> pieces grouped by key prefix
//       --k_bucket_local (+ fallback for large groups)--> sorted arrays
//       key/x/y/len/inc/index (contiguous for Stage I)
//   --k_cuts--> blocks of B sorted pieces, cuts moved past equal keys
//   --k_stage1 (one wavefront per block)--> local start per piece, start flags,
//       per-start partial sums (count, len, inc)
//   --scan + k_compact_starts--> S: starting points in sorted order
//   --k_stage2--> global start per element of S, partial sums per global group
//   --scan--> symbol numbers; k_dict writes the dictionary; k_remap_pairs,
//   one radix pass and k_remap_scatter send each piece's symbol back to
//   canonical order (label propagation).
//
// Decisions use binary64 with no contraction, in the order of the sequential
// definition, so local starts, blocks and symbols are bit-identical to it.
#include "common.h"
#include "sort_plan.h"
#include "lane_ops.h"

namespace jabba {

namespace {

constexpr int kTreeLeaves = 1024;  // leaves per workgroup in the pairwise sums

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
    double var_len;   // before a zero deviation is replaced by 1
    double var_inc;
    double axis[2];   // unit principal axis (PCA key)
    int64_t n;  // live piece count (clamped)
    int64_t sort_passes;  // radix passes of the main sort that moved data
    int64_t sort_bytes;   // bytes per pair those passes read and wrote
    int64_t sort_large;   // pieces in prefix groups too large for the local sort
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


// level 0: leaves are inc (pass 1), (inc - mean_inc)^2 (pass 2) or
// (len - mean_len)*(inc - mean_inc) (pass 3, the PCA key's covariance); pass 1
// also accumulates the exact integer sums of len and len^2.
template <int Pass>
__global__ __launch_bounds__(256) void k_sum_leaves(const int32_t *__restrict__ len, const double *__restrict__ inc,
                                                    DigState *ds, double *__restrict__ out,
                                                    unsigned long long *__restrict__ lpart) {
    __shared__ unsigned long long ls[2][4];
    const int64_t n = ds->n;
    const int64_t base = (int64_t)blockIdx.x * kTreeLeaves + 4 * threadIdx.x;
    double a[4];
    unsigned long long s1 = 0, s2 = 0;
    bool bad = false;
    const double mean = Pass >= 2 ? ds->mean_inc : 0.0;
    const double mean_len = Pass == 3 && n > 0 ? (double)(int64_t)ds->lsum[0] / (double)n : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t idx = base + i;
        double v = 0.0;
        if (idx < n) {
            v = inc[idx];
            if (Pass == 2) {
                const double d = v - mean;
                v = d * d;
            } else if (Pass == 3) {
                const double dl = (double)len[idx] - mean_len;
                v = dl * (v - mean);
            } else {
                const unsigned long long l = (unsigned long long)len[idx];
                s1 += l;
                s2 += l * l;
                bad |= !isfinite(v);
            }
        }
        a[i] = v;
    }
    const double r = block_tree_1024(a[0], a[1], a[2], a[3]);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
    if (Pass == 1) {
        if (ballot(bad) && lane_id() == 0) set_status(ds->status, kStNonFinite);
        // exact integer partials per workgroup; reduced by k_sum_ints
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            s1 += __shfl_xor(s1, m);
            s2 += __shfl_xor(s2, m);
        }
        if (lane_id() == 0) {
            ls[0][threadIdx.x / kWave] = s1;
            ls[1][threadIdx.x / kWave] = s2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            lpart[2 * blockIdx.x] = ls[0][0] + ls[0][1] + ls[0][2] + ls[0][3];
            lpart[2 * blockIdx.x + 1] = ls[1][0] + ls[1][1] + ls[1][2] + ls[1][3];
        }
    }
}

__global__ __launch_bounds__(1024) void k_sum_ints(const unsigned long long *__restrict__ lpart, int64_t nparts,
                                                   DigState *ds) {
    __shared__ unsigned long long ls[2][16];
    unsigned long long s1 = 0, s2 = 0;
    for (int64_t i = threadIdx.x; i < nparts; i += 1024) {
        s1 += lpart[2 * i];
        s2 += lpart[2 * i + 1];
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        s1 += __shfl_xor(s1, m);
        s2 += __shfl_xor(s2, m);
    }
    if (lane_id() == 0) {
        ls[0][threadIdx.x / kWave] = s1;
        ls[1][threadIdx.x / kWave] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int wv = 0; wv < 16; ++wv) {
            a += ls[0][wv];
            b += ls[1][wv];
        }
        ds->lsum[0] = a;
        ds->lsum[1] = b;
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
        ds->var_len = var_len;
        ds->var_inc = var_inc;
    } else {
        ds->var_len = 0.0;
        ds->var_inc = 0.0;
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

// Principal axis of the scaled pieces (Sec. 5, PCA projection as the sort
// key).  By construction var(x) = scl^2 and var(y) = 1 (0 when the raw
// variance is 0) and cov(x, y) = scl*cov(len, inc)/(sigma_len*sigma_inc), with
// cov(len, inc) the pass-3 pairwise sum over N.  The eigenvector of the larger
// eigenvalue of [[a, c], [c, b]] is (h + r, c) or (c, r - h), h = (a - b)/2,
// r = sqrt(h^2 + c^2), whichever has no cancellation in its first entry;
// normalised and signed so its first nonzero entry is positive.  Only
// correctly rounded operations, in a fixed order.
__global__ void k_pca_axis(DigState *ds, const double *total3, double scl, double *axis_out) {
    if (threadIdx.x != 0) return;
    const int64_t n = ds->n;
    double a = 0.0, b = 0.0, c = 0.0;
    if (n > 0) {
        const double cov = (*total3) / (double)n;
        if (ds->var_len > 0.0) a = scl * scl;
        if (ds->var_inc > 0.0) b = 1.0;
        if (a > 0.0 && b > 0.0) c = scl * ((cov / ds->sigma_len) / ds->sigma_inc);
    }
    double ux, uy;
    if (c == 0.0) {
        ux = a >= b ? 1.0 : 0.0;
        uy = a >= b ? 0.0 : 1.0;
    } else {
        const double h = 0.5 * (a - b);
        const double r = __dsqrt_rn(h * h + c * c);
        double vx, vy;
        if (h >= 0.0) {
            vx = h + r;
            vy = c;
        } else {
            vx = c;
            vy = r - h;
        }
        if (vx < 0.0) {
            vx = -vx;
            vy = -vy;
        }
        const double nn = __dsqrt_rn(vx * vx + vy * vy);
        ux = vx / nn;
        uy = vy / nn;
    }
    ds->axis[0] = ux;
    ds->axis[1] = uy;
    if (axis_out) {
        axis_out[0] = ux;
        axis_out[1] = uy;
    }
}

// Sort keys as unsigned integers in the order of the doubles: -0 is taken as
// +0, a non-negative key gets its sign bit set, a negative one is inverted.
__device__ __forceinline__ uint64_t key_bits(double k) {
    const uint64_t b = (uint64_t)__double_as_longlong(k == 0.0 ? 0.0 : k);
    return (b >> 63) ? ~b : (b | ((uint64_t)1 << 63));
}
__device__ __forceinline__ double key_of_bits(uint64_t b) {
    return __longlong_as_double((long long)((b >> 63) ? (b & ~((uint64_t)1 << 63)) : ~b));
}

// key kinds
constexpr int kKeyNorm = 0;
constexpr int kKeyPca = 1;

// One piece as a 16-byte record, so that reading it in sorted (random)
// order touches one cache line instead of one per array.
struct __align__(16) PieceRec {
    double inc;
    int32_t len;
    int32_t pad;
};

// Sort key of one scaled piece (Sec. 5): its norm, or its projection on the
// principal axis (ux, uy); -0 is taken as +0.  The key kernel and the gather
// both evaluate it here, so the sorted keys the gather writes are the keys
// the sort ordered.
template <int Key>
__device__ __forceinline__ double sort_key(Scaled s, double ux, double uy) {
    double k;
    if (Key == kKeyPca) {
        const double px = ux * s.x;
        const double py = uy * s.y;
        k = px + py;
    } else {
        k = piece_key(s);
    }
    return k == 0.0 ? 0.0 : k;
}

template <int Key>
__global__ void k_key(const int32_t *__restrict__ len, const double *__restrict__ inc, const DigState *ds, double scl,
                      uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, PieceRec *__restrict__ rec) {
    const int64_t n = ds->n;
    const double sl = ds->sigma_len, si = ds->sigma_inc;
    const double ux = Key == kKeyPca ? ds->axis[0] : 0.0, uy = Key == kKeyPca ? ds->axis[1] : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = len[i];
        const double ic = inc[i];
        const Scaled s = scale_piece(l, ic, scl, sl, si);
        keys[i] = key_bits(sort_key<Key>(s, ux, uy));
        vals[i] = (uint32_t)i;
        PieceRec r;
        r.inc = ic;
        r.len = l;
        r.pad = 0;
        rec[i] = r;
    }
}

// ------------------------------------------------------------ bucket sort
//
// The radix passes order the pieces by the highest 32 varying bits of
// key - kmin only (the prefix), keeping canonical order inside a prefix
// group; they carry the order alone (canonical indices).  The order by
// (key, index) is finished per group: a workgroup takes the groups that
// start in its tile of kBucketTile positions, reads their piece records by
// index once and evaluates their keys again (with the key kernel's own
// function, so they are the keys sorted on), holds records, keys and indices
// in LDS (with the rest of the tile's last group, up to kBucketCap positions
// beyond the tile), and places each member at its group's start plus the
// number of members with a smaller (key, index), each lane ranking one
// piece.  Groups are contiguous and ordered by prefix, so this is the full
// order.  The sorted pieces then leave coalesced: key, x, y, len, inc and
// the canonical index.  A group that crosses the tile's end and reaches more
// than kBucketCap beyond its start (at most one per tile) is left to the
// fallback below, which sorts all such groups together with the general
// radix sort.
constexpr int kBucketTile = 1024;
constexpr int kBucketCap = 256;  // largest tail group finished locally (groups inside a tile always are)
constexpr int kBucketThreads = 256;
constexpr int kBucketSpan = kBucketTile + kBucketCap;
constexpr int kBucketExt = 64;  // positions past the tile read at a time while looking for the next group

__device__ __forceinline__ uint64_t prefix_of(uint64_t k, uint64_t kmin, int shift) {
    return shift >= 64 ? 0ull : (k - kmin) >> shift;
}

// key bits of the piece with canonical index c (as k_key computed them)
template <int Key>
__device__ __forceinline__ uint64_t piece_key_bits(const PieceRec *__restrict__ rec, uint32_t c, double scl, double sl,
                                                   double si, double ux, double uy) {
    const PieceRec r = rec[c];
    return key_bits(sort_key<Key>(scale_piece(r.len, r.inc, scl, sl, si), ux, uy));
}

template <int Key>
__global__ __launch_bounds__(kBucketThreads) void k_bucket_local(
    const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1, const PieceRec *__restrict__ rec,
    const int32_t *ctl, const unsigned long long *__restrict__ kmin_p, DigState *ds, double scl,
    double *__restrict__ sk, double *__restrict__ sx, double *__restrict__ sy, int32_t *__restrict__ slen,
    double *__restrict__ sinc, uint32_t *__restrict__ perm, int64_t *__restrict__ thead,
    int64_t *__restrict__ tlarge) {
    __shared__ uint64_t s_k[kBucketSpan + 1];  // keys of [b0 - 1, b1 + extension)
    __shared__ double s_inc[kBucketSpan + 1];  // their records and indices
    __shared__ int32_t s_len[kBucketSpan + 1];
    __shared__ uint32_t s_v[kBucketSpan + 1];
    __shared__ uint16_t s_slot[kBucketSpan];   // element of each sorted slot
    __shared__ unsigned long long s_red[3];
    const int64_t n = ds->n;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    if (t == 0 && tid == 0) {
        int64_t act = 0, bytes = 0;
        for (int d = 0; d < 8; ++d) {
            if (ctl[kSortCtlSkip + d]) continue;
            act += 1;
            bytes += sort_pass_bytes(ctl[kSortCtlMode + d]);
        }
        ds->sort_passes = act;
        ds->sort_bytes = bytes;
        if (ctl[kSortCtlError]) set_status(ds->status, kStInternal);  // a radix look-back wait ran out
    }
    const int64_t b0 = t * kBucketTile;
    if (b0 >= n) {
        if (tid == 0) {
            thead[t] = -1;
            tlarge[t] = -1;
        }
        return;
    }
    const int64_t b1 = b0 + kBucketTile < n ? b0 + kBucketTile : n;
    const int64_t e_lim = b1 + kBucketCap < n ? b1 + kBucketCap : n;
    const uint32_t *V = ctl[0] ? v1 : v0;
    const uint64_t kmin = *kmin_p;
    const int shift = ctl[kSortCtlPrefixShift];
    const double sl = ds->sigma_len, si = ds->sigma_inc;
    const double ux = Key == kKeyPca ? ds->axis[0] : 0.0, uy = Key == kKeyPca ? ds->axis[1] : 0.0;
    // position p is at slot p - b0 + 1; slot 0 holds the position before the
    // tile (or a copy of position 0 for the first tile, which starts a group)
    auto fetch = [&](int64_t p, int slot) {
        const uint32_t c = V[p];
        const PieceRec r = rec[c];
        s_v[slot] = c;
        s_len[slot] = r.len;
        s_inc[slot] = r.inc;
        s_k[slot] = key_bits(sort_key<Key>(scale_piece(r.len, r.inc, scl, sl, si), ux, uy));
    };
    {
        // all index loads of the thread first, then all record loads, so
        // the two dependent round trips overlap across its positions
        constexpr int kPer = (kBucketTile + kBucketThreads) / kBucketThreads;
        const int64_t f0 = (b0 > 0 ? b0 - 1 : 0) + tid;
        uint32_t cs[kPer];
        PieceRec rs[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = f0 + (int64_t)u * kBucketThreads;
            cs[u] = p < b1 ? V[p] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = f0 + (int64_t)u * kBucketThreads;
            if (p < b1) rs[u] = rec[cs[u]];
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = f0 + (int64_t)u * kBucketThreads;
            if (p < b1) {
                const int slot = (int)(p - b0) + 1;
                s_v[slot] = cs[u];
                s_len[slot] = rs[u].len;
                s_inc[slot] = rs[u].inc;
                s_k[slot] = key_bits(sort_key<Key>(scale_piece(rs[u].len, rs[u].inc, scl, sl, si), ux, uy));
            }
        }
    }
    if (tid == 0) {
        if (b0 == 0) fetch(0, 0);
        s_red[0] = ~0ull;
        s_red[1] = 0ull;
        s_red[2] = ~0ull;
    }
    __syncthreads();
    auto pre = [&](int slot) -> uint64_t { return prefix_of(s_k[slot], kmin, shift); };
    auto head = [&](int64_t p) -> bool {
        const int i = (int)(p - b0) + 1;
        return p == 0 || pre(i) != pre(i - 1);
    };
    // first and last group start in the tile: one LDS atomic per wavefront
    for (int64_t p0 = b0; p0 < b1; p0 += kBucketThreads) {
        const int64_t p = p0 + tid;
        const uint64_t bm = __ballot(p < b1 && head(p));
        if (bm && lane == 0) {
            const int64_t wb = p0 + (tid & ~(kWave - 1));
            atomicMin(&s_red[0], (unsigned long long)(wb + __builtin_ctzll(bm)));
            atomicMax(&s_red[1], (unsigned long long)(wb + 63 - __builtin_clzll(bm) + 1));
        }
    }
    __syncthreads();
    if (s_red[1] == 0) {  // no group starts here: the tile lies inside an earlier group
        if (tid == 0) {
            thead[t] = -1;
            tlarge[t] = -1;
        }
        return;
    }
    // the next group start after the tile: read kBucketExt positions at a time
    int64_t ext = b1;
    while (ext < e_lim && s_red[2] == ~0ull) {
        const int64_t x1 = ext + kBucketExt < e_lim ? ext + kBucketExt : e_lim;
        if (tid < x1 - ext) fetch(ext + tid, (int)(ext + tid - b0) + 1);
        __syncthreads();
        if (tid < kWave) {
            const int64_t p = ext + tid;
            const uint64_t bm = __ballot(p < x1 && head(p));
            if (bm && tid == 0) s_red[2] = (unsigned long long)(ext + __builtin_ctzll(bm));
        }
        ext = x1;
        __syncthreads();
    }
    const int64_t lo = (int64_t)s_red[0];
    const int64_t s_last = (int64_t)s_red[1] - 1;
    // end of the last group: the next start, n, or beyond the cap (large)
    const int64_t e = s_red[2] != ~0ull ? (int64_t)s_red[2] : (e_lim == n ? n : INT64_MAX);
    const bool large = e == INT64_MAX || e - s_last > kBucketCap;
    const int64_t hi = large ? s_last : e;
    if (tid == 0) {
        thead[t] = lo;
        tlarge[t] = large ? s_last : -1;
    }
    const int m = (int)(hi - lo);
    if (m <= 0) return;
    const int ofs = (int)(lo - b0) + 1;  // slot of range element 0
    // rank inside the group by (key, index): each lane finds its group's
    // bounds by walking to the neighbours with another prefix (groups hold
    // one or two pieces on average), then counts the smaller members
    for (int i = tid; i < m; i += kBucketThreads) {
        const uint64_t pi = pre(ofs + i);
        int a = i, b = i + 1;
        while (a > 0 && pre(ofs + a - 1) == pi) --a;
        while (b < m && pre(ofs + b) == pi) ++b;
        const uint64_t ki = s_k[ofs + i];
        const uint32_t vi = s_v[ofs + i];
        int r = a;
        for (int q = a; q < b; ++q) {
            const uint64_t kq = s_k[ofs + q];
            r += (kq < ki || (kq == ki && s_v[ofs + q] < vi)) ? 1 : 0;
        }
        s_slot[r] = (uint16_t)i;
    }
    __syncthreads();
    for (int j = tid; j < m; j += kBucketThreads) {
        const int i = ofs + s_slot[j];
        const int32_t len = s_len[i];
        const double inc = s_inc[i];
        const Scaled sc = scale_piece(len, inc, scl, sl, si);
        const int64_t p = lo + j;
        sk[p] = key_of_bits(s_k[i]);
        sx[p] = sc.x;
        sy[p] = sc.y;
        slen[p] = len;
        sinc[p] = inc;
        perm[p] = s_v[i];
    }
}

// Fallback plan, one workgroup: the large group recorded by tile t ends at
// the first group start of a later tile (or n); lsize[t] its size (0 when
// none); an exclusive scan of lsize (separate launch) gives each group's
// offset among all large-group pieces.
__global__ __launch_bounds__(1024) void k_large_plan(const int64_t *__restrict__ thead,
                                                     const int64_t *__restrict__ tlarge, const DigState *ds,
                                                     int64_t ntiles_max, int64_t *__restrict__ lsize) {
    const int64_t n = ds->n;
    const int64_t ntiles = (n + kBucketTile - 1) / kBucketTile;
    for (int64_t t = threadIdx.x; t < ntiles_max; t += blockDim.x) {
        int64_t sz = 0;
        if (t < ntiles && tlarge[t] >= 0) {
            int64_t e = n;
            for (int64_t u = t + 1; u < ntiles; ++u)
                if (thead[u] >= 0) {
                    e = thead[u];
                    break;
                }
            sz = e - tlarge[t];
        }
        lsize[t] = sz;
    }
}

// j-th piece (in prefix-sorted position order) of the large groups: its position
__device__ __forceinline__ int64_t large_position(int64_t j, const int64_t *__restrict__ loff,
                                                  const int64_t *__restrict__ tlarge, int64_t ntiles) {
    int64_t a = 0, b = ntiles;  // last tile with loff[t] <= j
    while (b - a > 1) {
        const int64_t mid = (a + b) >> 1;
        if (loff[mid] <= j)
            a = mid;
        else
            b = mid;
    }
    return tlarge[a] + (j - loff[a]);
}

// pieces of the large groups -> (key, prefix-sorted position) pairs for the general sort
template <int Key>
__global__ void k_large_collect(const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1,
                                const PieceRec *__restrict__ rec, const int32_t *ctl, const int64_t *__restrict__ loff,
                                const int64_t *__restrict__ tlarge, const DigState *ds, double scl,
                                uint64_t *__restrict__ okey, uint32_t *__restrict__ opos, int64_t *__restrict__ n_large) {
    const int64_t n = ds->n;
    const int64_t ntiles = (n + kBucketTile - 1) / kBucketTile;
    const int64_t total = ntiles > 0 ? loff[ntiles] : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_large = total;
    const uint32_t *V = ctl[0] ? v1 : v0;
    const double sl = ds->sigma_len, si = ds->sigma_inc;
    const double ux = Key == kKeyPca ? ds->axis[0] : 0.0, uy = Key == kKeyPca ? ds->axis[1] : 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = large_position(j, loff, tlarge, ntiles);
        okey[j] = piece_key_bits<Key>(rec, V[p], scl, sl, si, ux, uy);
        opos[j] = (uint32_t)p;
    }
}

// the large groups' pieces, sorted by (key, position) = (key, index), leave
// into the large groups' positions in order
template <int Key>
__global__ void k_large_emit(const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1,
                             const PieceRec *__restrict__ rec, const int32_t *ctl,
                             const uint32_t *__restrict__ sp0, const uint32_t *__restrict__ sp1,
                             const int32_t *sctl, const int64_t *__restrict__ loff,
                             const int64_t *__restrict__ tlarge, DigState *ds, double scl,
                             double *__restrict__ sk, double *__restrict__ sx, double *__restrict__ sy,
                             int32_t *__restrict__ slen, double *__restrict__ sinc, uint32_t *__restrict__ perm) {
    const int64_t n = ds->n;
    const int64_t ntiles = (n + kBucketTile - 1) / kBucketTile;
    const int64_t total = ntiles > 0 ? loff[ntiles] : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ds->sort_large = total;
        if (sctl[kSortCtlError]) set_status(ds->status, kStInternal);
    }
    const uint32_t *V = ctl[0] ? v1 : v0;
    const uint32_t *SP = sctl[0] ? sp1 : sp0;
    const double sl = ds->sigma_len, si = ds->sigma_inc;
    const double ux = Key == kKeyPca ? ds->axis[0] : 0.0, uy = Key == kKeyPca ? ds->axis[1] : 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = large_position(j, loff, tlarge, ntiles);
        const uint32_t c = V[SP[j]];
        const PieceRec r = rec[c];
        const Scaled sc = scale_piece(r.len, r.inc, scl, sl, si);
        sk[p] = sort_key<Key>(sc, ux, uy);
        sx[p] = sc.x;
        sy[p] = sc.y;
        slen[p] = r.len;
        sinc[p] = r.inc;
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
//
// Pull form of the greedy aggregation.  Visiting presorted points in order,
// the sequential greedy lets a start p claim every unassigned later q with
// key_q - key_p <= alpha and (x_q - x_p)^2 + (y_q - y_p)^2 <= alpha^2.  So a
// point belongs to the first (lowest-position) earlier start that covers it,
// and is itself a start when no earlier start does.  The wavefront takes 64
// consecutive points at a time: each lane tests its point against the active
// starts (the earlier starts still within alpha in key, oldest first), then
// the points no start covers are resolved among themselves lane by lane
// (the first becomes a start, covers later lanes, and so on).  Both give the
// sequential decisions exactly; the next 64 points are loaded while the
// current ones are tested.

constexpr int kActCap = 256;  // active starts cached in LDS per wavefront
constexpr int kStage = 4;     // batches of 64 points staged in LDS at a time

struct ActLds {
    double k[kActCap];
    double x[kActCap];
    double y[kActCap];
    int32_t p[kActCap];
};

// Active starts: an append-only list of positions (glist in global memory),
// the newest kActCap of them mirrored in LDS with their coordinates.  New
// entries go to LDS only; flush() copies them to glist once per staged
// chunk, before any of them can leave the mirror (a chunk pushes at most
// kStage * 64 = kActCap entries).  Reads of entries no longer mirrored take
// their own loop, so the common path (LDS only) never waits on memory.
struct Active {
    ActLds *c;
    int32_t *glist;
    int head, tail;

    // the lanes in `m`, in lane order, each with its own entry
    __device__ void push_lanes(uint64_t m, int32_t pos, double kp, double xp, double yp) {
        const int lane = lane_id();
        if ((m >> lane) & 1ull) {
            const int sl = (tail + __popcll(m & lanemask_lt())) % kActCap;
            c->k[sl] = kp;
            c->x[sl] = xp;
            c->y[sl] = yp;
            c->p[sl] = pos;
        }
        tail += __popcll(m);
    }
    // entries [from, tail) to glist
    __device__ void flush(int from) {
        for (int t = from + lane_id(); t < tail; t += kWave)
            __hip_atomic_store(&glist[t], c->p[t % kActCap], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ int first_cached() const { return tail - kActCap > head ? tail - kActCap : head; }
    // drop starts that no point with key >= k0 can reach
    __device__ void expire(double k0, double alpha, const double *key) {
        const int fc = first_cached();
        while (head < fc) {
            const double kh = key[__hip_atomic_load(&glist[head], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)];
            if (!(k0 - kh <= alpha)) ++head;
            else return;
        }
        while (head < tail && !(k0 - c->k[head % kActCap] <= alpha)) ++head;
    }
};

// Branch-free: both tests are always evaluated (pure comparisons, so the
// result equals the short-circuit form), which lets several candidates'
// FP64 chains overlap.
__device__ __forceinline__ bool covers(double kq, double xq, double yq, double kp, double xp, double yp, double alpha,
                                       double a2) {
    const bool in_window = kq - kp <= alpha;
    const double dx = xq - xp;
    const double dy = yq - yp;
    const double dd = dx * dx;
    const double ee = dy * dy;
    return in_window & ((dd + ee) <= a2);
}

// With separated length columns (one length step moves x by more than alpha,
// the test of k_col_keys) points of different lengths never cover each other
// (their fl(dx^2) alone exceeds alpha^2) and points of one length have
// bit-identical x, so the test is x equality, the key window and
// fl(dy^2) <= alpha^2 (fl(0 + dy^2) = fl(dy^2)): the same decisions with
// fewer FP64 operations.
template <bool Col>
__device__ __forceinline__ bool covers_t(double kq, double xq, double yq, double kp, double xp, double yp, double alpha,
                                         double a2) {
    if constexpr (Col) {
        const bool same = __double_as_longlong(xq) == __double_as_longlong(xp);
        const bool in_window = kq - kp <= alpha;
        const double dy = yq - yp;
        const double ee = dy * dy;
        return same & in_window & (ee <= a2);
    } else {
        return covers(kq, xq, yq, kp, xp, yp, alpha, a2);
    }
}

// whether the length columns are separated (see k_col_keys)
__device__ __forceinline__ bool columns_separated(const DigState *ds, double scl, double a2) {
    const double step = scl / ds->sigma_len;
    return step * step > a2 * (1.0 + 1e-9);
}

// Runs the greedy over positions [from, to) with the active list A as the
// state before `from`.  Owners are written to lab/flag when `write`.
// Points are staged kStage batches at a time (all loads of a chunk in flight
// together); within a batch each lane first tests its point against the
// active starts, oldest first, and the points no active start covers are
// then resolved among themselves in lane order (runs of lanes separated by
// key gaps above alpha side by side, one step per new start of a run).
template <bool Col>
__device__ void pull_range(int64_t from, int64_t to, Active &A, const double *__restrict__ key,
                           const double *__restrict__ x, const double *__restrict__ y, double alpha, double a2,
                           bool write, int32_t *__restrict__ lab, uint32_t *__restrict__ flag,
                           int32_t *__restrict__ start_tag = nullptr, int32_t tag = 0) {
    const int lane = lane_id();
    ActLds *L = A.c;
    for (int64_t c0 = from; c0 < to; c0 += kStage * kWave) {
        // the chunk's points in registers; batch r always reads slot 0 and
        // the slots rotate after each batch (static register indices)
        double kv[kStage], xv[kStage], yv[kStage];
        int32_t ov[kStage];
#pragma unroll
        for (int r = 0; r < kStage; ++r) {
            const int64_t p = c0 + r * kWave + lane;
            kv[r] = p < to ? key[p] : 0.0;
            xv[r] = p < to ? x[p] : 0.0;
            yv[r] = p < to ? y[p] : 0.0;
            ov[r] = -1;
        }
        const int64_t c1 = to < c0 + kStage * kWave ? to : c0 + kStage * kWave;
        const int tail0 = A.tail;
        for (int r = 0; r < kStage; ++r) {
            const int64_t b0 = c0 + (int64_t)r * kWave;
            const int64_t q = b0 + lane;
            const bool inr = q < to;
            const double kq = kv[0], xq = xv[0], yq = yv[0];
            int32_t owner = -1;
            if (b0 < c1) {
                // list entries that left the LDS mirror are read back from memory
                if (A.head < A.first_cached()) __threadfence();
                A.expire(readlane_f64(kq, 0), alpha, key);
                bool open = inr;
                int i = A.head;
                const int fc = A.first_cached();
                if (i < fc) {
                    for (; i < fc; ++i) {
                        if (ballot(open) == 0ull) break;
                        const int32_t pp = __hip_atomic_load(&A.glist[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (open && covers_t<Col>(kq, xq, yq, key[pp], x[pp], y[pp], alpha, a2)) {
                            owner = pp;
                            open = false;
                        }
                    }
                }
                if (i >= fc) {
                    // kGroup starts per step: their loads issue together, the
                    // tests run in list order, one ballot per step
                    constexpr int kGroup = 4;
                    for (; i < A.tail; i += kGroup) {
                        if (ballot(open) == 0ull) break;
                        double gk[kGroup], gx[kGroup], gy[kGroup];
                        int32_t gp[kGroup];
#pragma unroll
                        for (int u = 0; u < kGroup; ++u) {
                            const int e = (i + u) & (kActCap - 1);
                            gk[u] = L->k[e];
                            gx[u] = L->x[e];
                            gy[u] = L->y[e];
                            gp[u] = L->p[e];
                        }
                        bool hit[kGroup];
#pragma unroll
                        for (int u = 0; u < kGroup; ++u)
                            hit[u] = (i + u < A.tail) & covers_t<Col>(kq, xq, yq, gk[u], gx[u], gy[u], alpha, a2);
#pragma unroll
                        for (int u = 0; u < kGroup; ++u) {
                            if (open && hit[u]) {
                                owner = gp[u];
                                open = false;
                            }
                        }
                    }
                }
                // The points no active start covers, resolved in lane order.
                // A key more than alpha above the previous lane's starts a
                // new run of lanes: keys ascend, so no point reaches across
                // that gap, and the runs are resolved side by side.  At each
                // step the first pending lane of every run becomes a start
                // and covers the later lanes of its run; the batch's new
                // starts then enter the list in position order.
                uint64_t pend = ballot(open);
                if (pend) {
                    const double kprev = __shfl_up(kq, 1);
                    const uint64_t heads = ballot(lane == 0 || !(kq - kprev <= alpha));
                    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes [0, lane]
                    const int rh = 63 - __builtin_clzll(heads & upto);               // this lane's run head
                    const uint64_t run_before = lanemask_lt() & (~0ull << rh);       // lanes [rh, lane)
                    uint64_t starts = 0ull;
                    while (pend) {
                        const bool first = open && (pend & run_before) == 0ull;
                        starts |= ballot(first);
                        // this lane's run's start of the step (a lane below it when
                        // the lane is pending and not first)
                        const int sl = ffs64(pend & (~0ull << rh));
                        const double ks = __shfl(kq, sl), xs = __shfl(xq, sl), ys = __shfl(yq, sl);
                        if (first) {
                            owner = (int32_t)(b0 + lane);
                            open = false;
                        } else if (open && covers_t<Col>(kq, xq, yq, ks, xs, ys, alpha, a2)) {
                            owner = (int32_t)(b0 + sl);
                            open = false;
                        }
                        pend = ballot(open);
                    }
                    A.push_lanes(starts, (int32_t)(b0 + lane), kq, xq, yq);
                }
            }
#pragma unroll
            for (int i = 0; i + 1 < kStage; ++i) {
                kv[i] = kv[i + 1];
                xv[i] = xv[i + 1];
                yv[i] = yv[i + 1];
                ov[i] = ov[i + 1];
            }
            ov[kStage - 1] = owner;
        }
        // the chunk's owners and new list entries leave together
        A.flush(tail0);
        if (write) {
#pragma unroll
            for (int r = 0; r < kStage; ++r) {
                const int64_t q = c0 + r * kWave + lane;
                if (q < c1) {
                    const int32_t owner = ov[r];
                    lab[q] = owner;
                    flag[q] = owner == (int32_t)q ? 1u : 0u;
                    if (start_tag && owner == (int32_t)q) start_tag[q] = tag;
                }
            }
        }
    }
}

// Stage I: one wavefront per block of sorted pieces.
__global__ __launch_bounds__(1024) void k_stage1(const int64_t *__restrict__ cuts, int64_t nblk_max,
                                                 const double *__restrict__ sk, const double *__restrict__ sx,
                                                 const double *__restrict__ sy, double alpha, double a2,
                                                 const DigState *ds, double scl,
                                                 int32_t *__restrict__ glist, int32_t *__restrict__ lab,
                                                 uint32_t *__restrict__ flag, int32_t *__restrict__ start_blk) {
    extern __shared__ ActLds act_lds[];
    const int wave = threadIdx.x / kWave;
    // blocks in descending key order: the last blocks (large keys, sparse
    // points, many starts each) take the longest, and are started first so
    // that none of them is left to run alone at the end
    const int64_t idx = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    if (idx >= nblk_max) return;
    const int64_t blk = nblk_max - 1 - idx;
    const int64_t lo = cuts[blk], hi = cuts[blk + 1];
    if (lo >= hi) return;
    Active A{&act_lds[wave], glist + lo, 0, 0};
    if (columns_separated(ds, scl, a2))
        pull_range<true>(lo, hi, A, sk, sx, sy, alpha, a2, true, lab, flag, start_blk, (int32_t)blk);
    else
        pull_range<false>(lo, hi, A, sk, sx, sy, alpha, a2, true, lab, flag, start_blk, (int32_t)blk);
}

// Stage II runs on independent groups of starting points.  Two starting
// points can only interact when their keys are within alpha and their x
// within alpha.  x = scl*len/sigma_len grows with len, so when one length step
// already separates x by more than alpha (checked with a margin that covers
// rounding) the points of each length form their own column; otherwise all
// points share one column.  Inside a column, ordered by position (= key
// order), a key gap larger than alpha cuts the chain: no point before it can
// reach a point after it (FP subtraction is monotone).  The greedy of every
// resulting group, run in position order, makes exactly the decisions of the
// greedy over all starting points.
constexpr int64_t kLenCap = (int64_t)1 << 30;

__global__ void k_col_keys(const int64_t *__restrict__ g_count, const int32_t *__restrict__ spos,
                           const int32_t *__restrict__ slen, const DigState *ds, double scl, double a2,
                           uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t G = *g_count;
    const double step = scl / ds->sigma_len;
    const bool sep = step * step > a2 * (1.0 + 1e-9);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
        int64_t col = 0;
        if (sep) {
            col = slen[spos[g]];
            if (col > kLenCap) col = kLenCap;
        }
        keys[g] = (uint64_t)col;  // stable sort: equal columns keep g order
        vals[g] = (uint32_t)g;
    }
}

// group cut flags over the column-sorted order, and the gathered coordinates
__global__ void k_col_cuts(const int64_t *__restrict__ g_count, const uint64_t *__restrict__ k0,
                           const uint64_t *__restrict__ k1, const uint32_t *__restrict__ v0,
                           const uint32_t *__restrict__ v1, const int32_t *__restrict__ ctl,
                           const double *__restrict__ gk, const double *__restrict__ gx, const double *__restrict__ gy,
                           double alpha, uint32_t *__restrict__ cut, int32_t *__restrict__ ord,
                           double *__restrict__ ck, double *__restrict__ cx, double *__restrict__ cy) {
    const int64_t G = *g_count;
    const uint64_t *keys = ctl[0] ? k1 : k0;  // column
    const uint32_t *vals = ctl[0] ? v1 : v0;  // starting point
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < G; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t kj = keys[j];
        const int32_t g = (int32_t)vals[j];
        bool c = j == 0;
        if (!c) {
            const int32_t gp = (int32_t)vals[j - 1];
            c = kj != keys[j - 1] || !(gk[g] - gk[gp] <= alpha);
        }
        cut[j] = c ? 1u : 0u;
        ord[j] = g;
        ck[j] = gk[g];
        cx[j] = gx[g];
        cy[j] = gy[g];
    }
}

// group start positions (in the column-sorted order) from the cut flags
__global__ void k_col_groups(const int64_t *__restrict__ g_count, const uint32_t *__restrict__ cut,
                             const uint32_t *__restrict__ gid, int32_t *__restrict__ gstart,
                             int64_t *__restrict__ n_groups) {
    const int64_t G = *g_count;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t ng = G > 0 ? (int64_t)gid[G] : 0;
        *n_groups = ng;
        gstart[ng] = (int32_t)G;
    }
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < G; j += (int64_t)gridDim.x * blockDim.x)
        if (cut[j]) gstart[gid[j]] = (int32_t)j;
}

// one wavefront per group; owners are written back in starting-point positions
__global__ __launch_bounds__(256) void k_col_greedy(const int64_t *__restrict__ n_groups_p,
                                                    const int32_t *__restrict__ gstart, const int32_t *__restrict__ ord,
                                                    const double *__restrict__ ck, const double *__restrict__ cx,
                                                    const double *__restrict__ cy, double alpha, double a2,
                                                    const DigState *ds, double scl,
                                                    int32_t *__restrict__ glist, int32_t *__restrict__ own,
                                                    uint32_t *__restrict__ oflag, int32_t *__restrict__ glab,
                                                    uint32_t *__restrict__ gflag) {
    extern __shared__ ActLds act_lds[];
    const int wave = threadIdx.x / kWave;
    const int64_t ng = *n_groups_p;
    const bool sep = columns_separated(ds, scl, a2);
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t gi = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave; gi < ng; gi += waves) {
        const int64_t lo = gstart[gi], hi = gstart[gi + 1];
        Active A{&act_lds[wave], glist + lo, 0, 0};
        if (sep)
            pull_range<true>(lo, hi, A, ck, cx, cy, alpha, a2, true, own, oflag);
        else
            pull_range<false>(lo, hi, A, ck, cx, cy, alpha, a2, true, own, oflag);
        __threadfence();  // owners written by other lanes are read back below
        for (int64_t j = lo + lane_id(); j < hi; j += kWave) {
            const int32_t g = ord[j];
            glab[g] = ord[own[j]];
            gflag[g] = oflag[j];
        }
    }
}

// Per-start sums over the start's members (lab == start).
//
// Stage I groups never leave their block, so a block's sums need one pass
// over its points: k_block_sums takes one wavefront per block and keeps the
// block's accumulators in LDS (blocks with at most kBlkCap starts).  Each
// batch of 64 points is ordered by (local start, position) with a bitonic
// network across the lanes; a segmented scan then sums each start's members
// of the batch, and the segment's last lane adds that partial to the start's
// accumulator.  Batches are added in position order, so the floating-point
// order is fixed by the data alone.  Blocks with more starts take
// k_group_sums<true>, one wavefront per start scanning the start's
// alpha-window of keys in chunks of 64 positions added in order.
constexpr int kBlkCap = 512;  // starts per block summed in LDS
constexpr int kSumStage = 8;  // batches of 64 points loaded together

struct SumLds {
    unsigned long long len[kBlkCap];
    double inc[kBlkCap];
    uint32_t cnt[kBlkCap];
};

// lane ^ m for a stride m that the unrolled loops below fix at compile time
__device__ __forceinline__ uint32_t xor_lane_m(uint32_t v, int m) {
    switch (m) {
        case 1: return xor_lane<1>(v);
        case 2: return xor_lane<2>(v);
        case 4: return xor_lane<4>(v);
        case 8: return xor_lane<8>(v);
        case 16: return xor_lane<16>(v);
        default: return xor_lane<32>(v);
    }
}

// One step of the segmented inclusive scan: each lane takes the partial sums
// of the lane Ctrl selects and adds them when that lane is in its run (the
// keys are sorted, so runs are contiguous); lanes without a source read a
// segment that matches none.
template <int Ctrl, int RowMask>
__device__ __forceinline__ void seg_scan_step(uint32_t seg, double &v, long long &l, uint32_t &c) {
    const uint32_t ys = dpp_keep<Ctrl, RowMask>(0xFFFFFFFFu, seg);
    const uint32_t v0 = dpp_keep<Ctrl, RowMask>(0u, (uint32_t)__double2loint(v));
    const uint32_t v1 = dpp_keep<Ctrl, RowMask>(0u, (uint32_t)__double2hiint(v));
    const uint64_t lu = (uint64_t)l;
    const uint32_t l0 = dpp_keep<Ctrl, RowMask>(0u, (uint32_t)lu);
    const uint32_t l1 = dpp_keep<Ctrl, RowMask>(0u, (uint32_t)(lu >> 32));
    const uint32_t yc = dpp_keep<Ctrl, RowMask>(0u, c);
    if (ys == seg) {
        v = v + __hiloint2double((int)v1, (int)v0);
        l += (long long)(((uint64_t)l1 << 32) | l0);
        c += yc;
    }
}

__device__ __forceinline__ int64_t block_starts(const int64_t *__restrict__ cuts, const uint32_t *__restrict__ sidx,
                                                int64_t blk) {
    return (int64_t)sidx[cuts[blk + 1]] - (int64_t)sidx[cuts[blk]];
}

__global__ __launch_bounds__(256) void k_block_sums(const int64_t *__restrict__ cuts, int64_t nblk_max,
                                                    const uint32_t *__restrict__ sidx, const int32_t *__restrict__ lab,
                                                    const int32_t *__restrict__ slen, const double *__restrict__ sinc,
                                                    int64_t *__restrict__ ocnt, int64_t *__restrict__ olen,
                                                    double *__restrict__ oinc) {
    __shared__ SumLds sums_all[256 / kWave];
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const int64_t blk = (int64_t)blockIdx.x * (256 / kWave) + wave;
    if (blk >= nblk_max) return;
    const int64_t lo = cuts[blk], hi = cuts[blk + 1];
    if (lo >= hi) return;
    const uint32_t g0 = sidx[lo];
    const int64_t ns = (int64_t)sidx[hi] - (int64_t)g0;
    if (ns < 1 || ns > kBlkCap) return;
    SumLds &S = sums_all[wave];
    for (int j = lane; j < ns; j += kWave) {
        S.len[j] = 0ull;
        S.inc[j] = 0.0;
        S.cnt[j] = 0u;
    }
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    for (int64_t c0 = lo; c0 < hi; c0 += kSumStage * kWave) {
        int32_t own[kSumStage], lv[kSumStage];
        double iv[kSumStage];
        uint32_t key[kSumStage];
#pragma unroll
        for (int r = 0; r < kSumStage; ++r) {
            const int64_t q = c0 + r * kWave + lane;
            own[r] = q < hi ? lab[q] : -1;
            lv[r] = q < hi ? slen[q] : 0;
            iv[r] = q < hi ? sinc[q] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kSumStage; ++r) {
            key[r] = kNone;
            if (own[r] >= 0) {
                const int64_t li = (int64_t)sidx[own[r]] - (int64_t)g0;
                if (li >= 0 && li < ns) key[r] = ((uint32_t)li << 6) | (uint32_t)lane;
            }
        }
#pragma unroll
        for (int r = 0; r < kSumStage; ++r) {
            if (c0 + r * kWave >= hi) break;
            // ascending bitonic sort of the 64 keys across the lanes (the
            // partners move through DPP and the permlane swaps, not LDS)
            uint32_t k = key[r];
#pragma unroll
            for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
                for (int stride = size >> 1; stride > 0; stride >>= 1) {
                    const uint32_t o = xor_lane_m(k, stride);
                    const bool up = (lane & size) == 0 || size == kWave;
                    const bool low = (lane & stride) == 0;
                    k = (low == up) ? (k < o ? k : o) : (k < o ? o : k);
                }
            }
            const int src = (int)(k & 63u);
            const uint32_t seg = k >> 6;
            double v = __shfl(iv[r], src);
            long long l = (long long)__shfl(lv[r], src);
            uint32_t c = k != kNone ? 1u : 0u;
            // segmented inclusive scan over runs of equal seg: row shifts by
            // 1, 2, 4 and 8, then lane 15 of rows 0 and 2 into rows 1 and 3,
            // and lane 31 into rows 2 and 3
            seg_scan_step<0x111, 0xF>(seg, v, l, c);
            seg_scan_step<0x112, 0xF>(seg, v, l, c);
            seg_scan_step<0x114, 0xF>(seg, v, l, c);
            seg_scan_step<0x118, 0xF>(seg, v, l, c);
            seg_scan_step<0x142, 0xA>(seg, v, l, c);
            seg_scan_step<0x143, 0xC>(seg, v, l, c);
            const uint32_t nx = next_lane(seg, 0xFFFFFFFFu);  // the last lane ends its run
            if (k != kNone && nx != seg) {
                S.inc[seg] = S.inc[seg] + v;
                S.len[seg] += (unsigned long long)l;
                S.cnt[seg] += c;
            }
        }
    }
    for (int j = lane; j < ns; j += kWave) {
        ocnt[g0 + j] = (int64_t)S.cnt[j];
        olen[g0 + j] = (int64_t)S.len[j];
        oinc[g0 + j] = S.inc[j];
    }
}

template <bool Points>
__global__ __launch_bounds__(256) void k_group_sums(const int64_t *__restrict__ n_starts_p, int64_t n_pos_max,
                                                    const int64_t *__restrict__ n_pos_p,
                                                    const int32_t *__restrict__ start_pos,
                                                    const int32_t *__restrict__ start_blk,
                                                    const int64_t *__restrict__ cuts, const uint32_t *__restrict__ sidx,
                                                    const uint32_t *__restrict__ flag, const double *__restrict__ key,
                                                    const int32_t *__restrict__ lab, const int32_t *__restrict__ wlen32,
                                                    const int64_t *__restrict__ wcnt, const int64_t *__restrict__ wlen,
                                                    const double *__restrict__ winc, double alpha,
                                                    int64_t *__restrict__ ocnt, int64_t *__restrict__ olen,
                                                    double *__restrict__ oinc) {
    const int lane = lane_id();
    const int64_t n_starts = *n_starts_p;
    int64_t n_pos = *n_pos_p;
    if (n_pos > n_pos_max) n_pos = n_pos_max;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; g < n_starts; g += waves) {
        int64_t p, pend = n_pos;
        if (Points) {
            p = start_pos[g];
            const int64_t blk = start_blk[p];
            if (block_starts(cuts, sidx, blk) <= kBlkCap) continue;  // summed by k_block_sums
            pend = cuts[blk + 1];  // members never leave the start's block
        } else {
            if (!flag[g]) continue;
            p = g;
        }
        const double kp = key[p];
        int64_t c = 0, l = 0;
        double ic = 0.0;
        for (int64_t q0 = p; q0 < pend; q0 += kWave) {
            const int64_t q = q0 + lane;
            const bool inr = q < pend;
            const bool inwin = inr && (key[q] - kp <= alpha);
            const bool mem = inwin && lab[q] == (int32_t)p;
            int64_t cq = 0, lq = 0;
            double iq = 0.0;
            if (mem) {
                cq = Points ? 1 : wcnt[q];
                lq = Points ? (int64_t)wlen32[q] : wlen[q];
                iq = winc[q];
            }
            c += wave_sum_i64(cq);
            l += wave_sum_i64(lq);
            ic = ic + wave_tree_sum(iq);
            if (ballot(inr && !inwin) != 0ull) break;
        }
        if (lane == 0) {
            ocnt[g] = c;
            olen[g] = l;
            oinc[g] = ic;
        }
    }
}

// Stage II sums: the Stage I sums of every starting point added to its
// global owner.  The pairs (owner, starting point) are sorted by owner
// (stably, so each owner's members stay in position order), which makes each
// owner's members contiguous, and one wavefront per global start then adds
// only its own members, where a scan of the start's key window in position
// order reads every starting point of the window.  The increments are added
// as that scan adds them: a member q of start g sits at lane (q - g) mod 64 of
// chunk (q - g) / 64, each chunk is summed by the pairwise wavefront tree and
// the chunks are added in order (a chunk without members adds +0 there and
// is skipped here).
__global__ void k_owner_pairs(const int64_t *__restrict__ g_count, const int32_t *__restrict__ glab,
                              uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t G = *g_count;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
        keys[g] = (uint64_t)(uint32_t)glab[g];
        vals[g] = (uint32_t)g;
    }
}

// first position of each owner's members in the sorted pairs
__global__ void k_owner_heads(const int64_t *__restrict__ g_count, const uint64_t *__restrict__ k0,
                              const uint64_t *__restrict__ k1, const int32_t *__restrict__ ctl,
                              uint32_t *__restrict__ head) {
    const int64_t G = *g_count;
    const uint64_t *K = ctl[0] ? k1 : k0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G; i += (int64_t)gridDim.x * blockDim.x)
        if (i == 0 || K[i] != K[i - 1]) head[K[i]] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_owner_sums(const int64_t *__restrict__ g_count,
                                                    const uint32_t *__restrict__ gflag,
                                                    const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                                                    const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1,
                                                    const int32_t *__restrict__ ctl, const uint32_t *__restrict__ head,
                                                    const int64_t *__restrict__ wcnt, const int64_t *__restrict__ wlen,
                                                    const double *__restrict__ winc, int64_t *__restrict__ ocnt,
                                                    int64_t *__restrict__ olen, double *__restrict__ oinc) {
    const int lane = lane_id();
    const int64_t G = *g_count;
    const uint64_t *K = ctl[0] ? k1 : k0;
    const uint32_t *V = ctl[0] ? v1 : v0;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; g < G; g += waves) {
        if (!gflag[g]) continue;
        int64_t c = 0, l = 0;
        double ic = 0.0, chunk = 0.0;
        int64_t cur = -1;  // chunk being gathered in `chunk`
        for (int64_t i0 = head[g];; i0 += kWave) {
            const int64_t i = i0 + lane;
            const bool mem = i < G && K[i] == (uint64_t)g;
            const uint64_t mm = ballot(mem);
            int64_t cq = 0, lq = 0;
            double iq = 0.0;
            int64_t d = 0;  // the member's offset from its start
            if (mem) {
                const uint32_t q = V[i];
                cq = wcnt[q];
                lq = wlen[q];
                iq = winc[q];
                d = (int64_t)q - g;
            }
            c += wave_sum_i64(cq);
            l += wave_sum_i64(lq);
            // members ascend in position, so their chunks ascend in lane order
            uint64_t todo = mm;
            while (todo) {
                const int64_t ch = readlane_i64(d >> 6, ffs64(todo));
                if (ch != cur) {
                    if (cur >= 0) ic = ic + wave_tree_sum(chunk);
                    chunk = 0.0;
                    cur = ch;
                }
                const bool here = ((todo >> lane) & 1ull) && (d >> 6) == ch;
                const uint64_t hm = ballot(here);
                // lane t takes the member whose offset is t within the chunk
                uint64_t src = hm;
#pragma unroll
                for (int b = 0; b < 6; ++b) {
                    const uint64_t bb = ballot(here && ((d >> b) & 1));
                    src &= ((lane >> b) & 1) ? bb : ~bb;
                }
                const double v = __shfl(iq, src ? __builtin_ctzll(src) : 0);
                if (src) chunk = chunk + v;
                todo &= ~hm;
            }
            if (mm != ~0ull) break;  // the owner's members end in this batch
        }
        if (cur >= 0) ic = ic + wave_tree_sum(chunk);
        if (lane == 0) {
            ocnt[g] = c;
            olen[g] = l;
            oinc[g] = ic;
        }
    }
}

__global__ void k_compact_starts(const DigState *ds, const uint32_t *__restrict__ flag,
                                 const uint32_t *__restrict__ sidx, const double *__restrict__ sk,
                                 const double *__restrict__ sx, const double *__restrict__ sy,
                                 double *__restrict__ gk, double *__restrict__ gx, double *__restrict__ gy,
                                 int32_t *__restrict__ spos, int64_t *__restrict__ g_count) {
    const int64_t n = ds->n;
    if (blockIdx.x == 0 && threadIdx.x == 0) *g_count = (int64_t)sidx[n];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    auto emit = [&](int64_t p) {
        const uint32_t g = sidx[p];
        gk[g] = sk[p];
        gx[g] = sx[p];
        gy[g] = sy[p];
        spos[g] = (int32_t)p;
    };
    if (((uintptr_t)flag & 15) != 0) {
        for (int64_t p = tid; p < n; p += stride)
            if (flag[p]) emit(p);
        return;
    }
    // starts are sparse: four flags per lane in one 16-byte load, the rest
    // read only for the flagged positions
    const uint4 *flag4 = reinterpret_cast<const uint4 *>(flag);
    const int64_t n4 = (n + 3) >> 2;
    for (int64_t q = tid; q < n4; q += stride) {
        const int64_t p0 = q << 2;
        uint32_t f[4];
        if (p0 + 4 <= n) {
            const uint4 v = flag4[q];
            f[0] = v.x;
            f[1] = v.y;
            f[2] = v.z;
            f[3] = v.w;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) f[u] = p0 + u < n ? flag[p0 + u] : 0u;
        }
        if ((f[0] | f[1] | f[2] | f[3]) == 0u) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (f[u]) emit(p0 + u);
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

// Label propagation.  Writing each piece's symbol straight to its canonical
// index is a random 4-byte scatter over the whole symbol array; that is fast
// while the array stays in the caches (k_remap).  For larger arrays the
// (index, symbol) pairs of sorted positions are first grouped by the index's
// highest 16 bits with two radix passes.  The indices are a permutation of
// 0..n-1, so after the grouping window w of 2^wlog consecutive indices holds
// exactly its own pairs, at positions [w * 2^wlog, (w + 1) * 2^wlog): one
// workgroup scatters a window's symbols in LDS and writes the window out in
// order (k_remap_window), so every line of the symbol array is written once
// and whole.
__global__ void k_remap(const DigState *ds, const uint32_t *__restrict__ perm, const int32_t *__restrict__ lab,
                        const uint32_t *__restrict__ sidx, const int32_t *__restrict__ glab,
                        const uint32_t *__restrict__ gsym, int32_t *__restrict__ symbols) {
    const int64_t n = ds->n;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t g = sidx[lab[p]];
        symbols[perm[p]] = (int32_t)gsym[glab[g]];
    }
}

// The pairs' key is the canonical index shifted left by `sh` bits, so that
// the two highest radix digits hold the index's highest 16 bits; the keys
// are 32-bit words (the sort takes and keeps them at that width).
__global__ void k_remap_pairs(const DigState *ds, const uint32_t *__restrict__ perm, const int32_t *__restrict__ lab,
                              const uint32_t *__restrict__ sidx, const int32_t *__restrict__ glab,
                              const uint32_t *__restrict__ gsym, int sh, uint32_t *__restrict__ keys,
                              uint32_t *__restrict__ vals) {
    const int64_t n = ds->n;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t g = sidx[lab[p]];
        keys[p] = perm[p] << sh;
        vals[p] = gsym[glab[g]];
    }
}

// The keys are {i << sh : 0 <= i < n}, so the digit histograms the radix
// pass plans with follow from n and sh alone.  Digit d of i << sh is bits
// [a, a + 8) of i with a = 8d - sh when a >= 0: the value b on
// (n / 2^(a+8)) * 2^a + clamp(n mod 2^(a+8) - b * 2^a, 0, 2^a) keys.  For
// -8 < a < 0 the digit is (i mod 2^(8+a)) << -a: each multiple m << -a on
// (n / 2^(8+a)) + (m < n mod 2^(8+a)) keys, the other values on none; for
// a <= -8 it is 0 on every key.  Smallest key 0.
__global__ void k_remap_hist(const DigState *ds, int sh, uint32_t *__restrict__ ghist,
                             unsigned long long *__restrict__ kmin) {
    const uint64_t n = (uint64_t)ds->n;
    if (threadIdx.x == 0) *kmin = 0ull;
    const uint64_t b = threadIdx.x;
    for (int d = 0; d < 8; ++d) {
        const int a = 8 * d - sh;
        uint64_t cnt;
        if (a >= 0) {
            const bool full = a + 8 >= 64;  // 2^(a+8) exceeds every count
            const uint64_t S = 1ull << a;
            const uint64_t P = full ? 0ull : (S << 8);
            const uint64_t cycles = full ? 0ull : n / P;
            const uint64_t rem = full ? n : n % P;
            const uint64_t lo = b * S;
            const uint64_t part = rem > lo ? (rem - lo < S ? rem - lo : S) : 0ull;
            cnt = cycles * S + part;
        } else if (a > -8) {
            const uint64_t P = 1ull << (8 + a);
            const uint64_t step = 1ull << (-a);
            cnt = (b % step) ? 0ull : n / P + ((b / step) < n % P ? 1ull : 0ull);
        } else {  // the digit lies below the shift: 0 on every key
            cnt = b == 0 ? n : 0ull;
        }
        ghist[d * 256 + b] = (uint32_t)cnt;
    }
}

constexpr int kWindowMaxLog = 14;  // 16,384 symbols: 64 KB of LDS
constexpr int kWindowThreads = 1024;
constexpr int kWindowPer = (1 << kWindowMaxLog) / kWindowThreads;

__global__ __launch_bounds__(kWindowThreads) void k_remap_window(DigState *ds, const uint32_t *__restrict__ k0,
                                                                 const uint32_t *__restrict__ k1,
                                                                 const uint32_t *__restrict__ v0,
                                                                 const uint32_t *__restrict__ v1, const int32_t *ctl,
                                                                 int sh, int wlog, int32_t *__restrict__ symbols) {
    extern __shared__ int32_t s_sym[];
    const int64_t n = ds->n;
    const int64_t w0 = (int64_t)blockIdx.x << wlog;
    if (w0 >= n) return;
    const int m = (int)(n - w0 < ((int64_t)1 << wlog) ? n - w0 : ((int64_t)1 << wlog));
    const uint32_t *K = ctl[0] ? k1 : k0;
    const uint32_t *V = ctl[0] ? v1 : v0;
    uint32_t kr[kWindowPer];
    uint32_t vr[kWindowPer];
#pragma unroll
    for (int u = 0; u < kWindowPer; ++u) {
        const int i = u * kWindowThreads + (int)threadIdx.x;
        kr[u] = i < m ? K[w0 + i] : 0u;
        vr[u] = i < m ? V[w0 + i] : 0u;
    }
    bool bad = false;
#pragma unroll
    for (int u = 0; u < kWindowPer; ++u) {
        const int i = u * kWindowThreads + (int)threadIdx.x;
        if (i < m) {
            const int64_t li = (int64_t)(kr[u] >> sh) - w0;
            if (li >= 0 && li < m)
                s_sym[li] = (int32_t)vr[u];
            else
                bad = true;  // not a permutation: never expected
        }
    }
    if (bad) set_status(ds->status, kStInternal);
    __syncthreads();
    for (int i = (int)threadIdx.x; i < m; i += kWindowThreads) symbols[w0 + i] = s_sym[i];
}

// Fallback for windows above the LDS limit (more than 2^30 pieces): a scatter
// from the grouped pairs.
__global__ void k_remap_scatter(const DigState *ds, const uint32_t *__restrict__ k0, const uint32_t *__restrict__ k1,
                                const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1, const int32_t *ctl,
                                int sh, int32_t *__restrict__ symbols) {
    const int64_t n = ds->n;
    const uint32_t *K = ctl[0] ? k1 : k0;
    const uint32_t *V = ctl[0] ? v1 : v0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        symbols[K[q] >> sh] = (int32_t)V[q];
}

// ------------------------------------------------------------ raw 2-D points
//
// The aggregation on points as given (no scaling): the key and the gathered
// coordinates come from the points themselves; the sort, Stage I, Stage II
// (one column: no length structure) and the label propagation are the
// digitizer's kernels.  Centers are formed afterwards from the labels.
struct __align__(16) PointRec {
    double x;
    double y;
};
static_assert(sizeof(PointRec) == sizeof(PieceRec), "point records share the piece record slots");

__global__ void k_pts_prepare(DigState *ds) {
    if (threadIdx.x == 0) {
        ds->sigma_len = 1.0;
        ds->sigma_inc = 1.0;
    }
}

__global__ void k_pts_key(const double *__restrict__ px, const double *__restrict__ py, DigState *ds,
                          uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, PointRec *__restrict__ rec) {
    const int64_t n = ds->n;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = px[i], y = py[i];
        bad |= !(isfinite(x) && isfinite(y));
        const double xx = x * x;
        const double yy = y * y;
        keys[i] = key_bits(__dsqrt_rn(xx + yy));
        vals[i] = (uint32_t)i;
        PointRec r;
        r.x = x;
        r.y = y;
        rec[i] = r;
    }
    if (ballot(bad) && lane_id() == 0) set_status(ds->status, kStNonFinite);
}

__global__ void k_pts_gather(const PointRec *__restrict__ rec, DigState *ds, const uint64_t *__restrict__ k0,
                             const uint64_t *__restrict__ k1, const uint32_t *__restrict__ v0,
                             const uint32_t *__restrict__ v1, const int32_t *ctl, double *__restrict__ sk,
                             double *__restrict__ sx, double *__restrict__ sy, uint32_t *__restrict__ perm) {
    const int64_t n = ds->n;
    const uint64_t *ks = ctl[0] ? k1 : k0;
    const uint32_t *vs = ctl[0] ? v1 : v0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t act = 0;
        for (int d = 0; d < 8; ++d) act += ctl[1 + d] ? 0 : 1;
        ds->sort_passes = act;
        ds->sort_bytes = 24 * act;  // 64-bit keys and 32-bit values in and out
        if (ctl[32]) set_status(ds->status, kStInternal);
    }
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = vs[p];
        const PointRec r = rec[c];
        sk[p] = key_of_bits(ks[p]);
        sx[p] = r.x;
        sy[p] = r.y;
        perm[p] = c;
    }
}

// cluster count, and the sort pairs (label, index) for the per-cluster means
__global__ void k_pts_pairs(const int64_t *__restrict__ g_count, const uint32_t *__restrict__ gsym, DigState *ds,
                            const int32_t *__restrict__ labels, int64_t capacity, int64_t *__restrict__ k_out,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t n = ds->n;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t G = *g_count;
        const int64_t k = G > 0 ? (int64_t)gsym[G] : 0;
        *k_out = k;
        if (k > capacity) set_status(ds->status, kStCapacity);
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = (uint64_t)(uint32_t)labels[i];
        vals[i] = (uint32_t)i;
    }
}

// run [start, end) of every label in the label-sorted order
__global__ void k_pts_runs(const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                           const int32_t *__restrict__ ctl, const DigState *ds, int64_t *__restrict__ run_start,
                           int64_t *__restrict__ run_end) {
    const int64_t n = ds->n;
    const uint64_t *keys = ctl[0] ? k1 : k0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = keys[j];
        if (j == 0 || keys[j - 1] != c) run_start[c] = j;
        if (j == n - 1 || keys[j + 1] != c) run_end[c] = j + 1;
    }
}

// one wavefront per cluster: count, and the means of x and y with the members
// added one by one in input order (the stable sort keeps that order inside a
// label), the chain running lane by lane over chunks of 64 members
__global__ __launch_bounds__(256) void k_pts_centers(const double *__restrict__ px, const double *__restrict__ py,
                                                     const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1,
                                                     const int32_t *__restrict__ ctl, const int64_t *__restrict__ k_p,
                                                     int64_t capacity, const int64_t *__restrict__ run_start,
                                                     const int64_t *__restrict__ run_end, double *__restrict__ cx,
                                                     double *__restrict__ cy, int64_t *__restrict__ count) {
    const int lane = lane_id();
    const uint32_t *perm = ctl[0] ? v1 : v0;
    int64_t k = *k_p;
    if (k > capacity) k = capacity;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; c < k; c += waves) {
        const int64_t a = run_start[c], b = run_end[c];
        double sx = 0.0, sy = 0.0;
        for (int64_t j0 = a; j0 < b; j0 += kWave) {
            const int64_t j = j0 + lane;
            double vx = 0.0, vy = 0.0;
            if (j < b) {
                const uint32_t i = perm[j];
                vx = px[i];
                vy = py[i];
            }
            const int cnt = (int)((b - j0) < kWave ? (b - j0) : kWave);
            for (int u = 0; u < cnt; ++u) {
                sx = sx + readlane_f64(vx, u);
                sy = sy + readlane_f64(vy, u);
            }
        }
        if (lane == 0) {
            const double m = (double)(b - a);
            cx[c] = sx / m;
            cy[c] = sy / m;
            count[c] = b - a;
        }
    }
}

// level 0 of the SSE's pairwise tree: (x - cx)^2 + (y - cy)^2 in input order
__global__ __launch_bounds__(256) void k_pts_sse_leaves(const double *__restrict__ px, const double *__restrict__ py,
                                                        const int32_t *__restrict__ labels, const double *__restrict__ cx,
                                                        const double *__restrict__ cy, const int64_t *__restrict__ k_p,
                                                        int64_t capacity, const DigState *ds,
                                                        double *__restrict__ out) {
    const int64_t n = ds->n;
    const bool ok = *k_p <= capacity;
    const int64_t base = (int64_t)blockIdx.x * kTreeLeaves + 4 * threadIdx.x;
    double a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t idx = base + i;
        double v = 0.0;
        if (ok && idx < n) {
            const int32_t c = labels[idx];
            const double dx = px[idx] - cx[c];
            const double dy = py[idx] - cy[c];
            const double xx = dx * dx;
            const double yy = dy * dy;
            v = xx + yy;
        }
        a[i] = v;
    }
    const double r = block_tree_1024(a[0], a[1], a[2], a[3]);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
}

__global__ void k_pts_sse_out(const double *__restrict__ total, double *__restrict__ sse) {
    if (threadIdx.x == 0) *sse = *total;
}

// ------------------------------------------------------------ quality
//
// Squared deviation of every sorted piece from its symbol's scaled center.
__global__ void k_q_values(const DigState *ds, const double *__restrict__ sx, const double *__restrict__ sy,
                           const int32_t *__restrict__ lab, const uint32_t *__restrict__ sidx,
                           const int32_t *__restrict__ glab, const uint32_t *__restrict__ gsym, jabba_dict dict,
                           double *__restrict__ qx, double *__restrict__ qy) {
    const int64_t n = ds->n;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t g = sidx[lab[p]];
        const int64_t c = gsym[glab[g]];
        double ex2 = 0.0, ey2 = 0.0;
        if (c < dict.capacity) {
            const double ex = sx[p] - dict.cx[c];
            const double ey = sy[p] - dict.cy[c];
            ex2 = ex * ex;
            ey2 = ey * ey;
        }
        qx[p] = ex2;
        qy[p] = ey2;
    }
}

// per symbol: the mean squared deviations, and their sum for the SSE
__global__ void k_q_symbols(const int64_t *__restrict__ g_count, const uint32_t *__restrict__ gflag,
                            const uint32_t *__restrict__ gsym, const double *__restrict__ sum_x,
                            const double *__restrict__ sum_y, jabba_dict dict, double *__restrict__ var_len,
                            double *__restrict__ var_inc, double *__restrict__ per_symbol) {
    const int64_t G = *g_count;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
        if (!gflag[g]) continue;
        const int64_t c = gsym[g];
        if (c >= dict.capacity) continue;
        const double cnt = (double)dict.count[c];
        var_len[c] = sum_x[g] / cnt;
        var_inc[c] = sum_y[g] / cnt;
        per_symbol[c] = sum_x[g] + sum_y[g];
    }
}

// SSE = sum over symbols (each thread adds its strided symbols in order, then
// a fixed tree over the threads), and the largest variances
__global__ __launch_bounds__(1024) void k_q_totals(const int64_t *__restrict__ kp, int64_t capacity,
                                                   const double *__restrict__ per_symbol,
                                                   const double *__restrict__ var_len,
                                                   const double *__restrict__ var_inc, double *__restrict__ totals) {
    __shared__ double s_sum[1024 / kWave], s_ml[1024 / kWave], s_mi[1024 / kWave];
    int64_t k = *kp;
    k = k < 0 ? 0 : (k > capacity ? capacity : k);
    double acc = 0.0, ml = 0.0, mi = 0.0;
    for (int64_t c = threadIdx.x; c < k; c += blockDim.x) {
        acc = acc + per_symbol[c];
        ml = var_len[c] > ml ? var_len[c] : ml;
        mi = var_inc[c] > mi ? var_inc[c] : mi;
    }
    acc = wave_tree_sum(acc);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double yl = __shfl_xor(ml, o), yi = __shfl_xor(mi, o);
        ml = yl > ml ? yl : ml;
        mi = yi > mi ? yi : mi;
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s_sum[w] = acc;
        s_ml[w] = ml;
        s_mi[w] = mi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0, a = 0.0, b = 0.0;
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) {
            t = t + s_sum[q];
            a = s_ml[q] > a ? s_ml[q] : a;
            b = s_mi[q] > b ? s_mi[q] : b;
        }
        totals[0] = t;
        totals[1] = a;
        totals[2] = b;
    }
}

struct DigWs {
    DigState *ds;
    double *tree[2];
    unsigned long long *lpart;
    SortBuffers sb;
    SortBuffers sb2;  // the bucket sort's fallback for large prefix groups
    int64_t *thead, *tlarge, *lsize, *loff, *n_large;
    double *sk, *sx, *sy, *sinc;
    int32_t *slen;
    uint32_t *perm;
    PieceRec *rec;
    int64_t *cuts;
    int32_t *lab;
    uint32_t *flag;
    uint32_t *sidx;
    int32_t *glist;
    double *gk, *gx, *gy, *ginc;
    int64_t *gcnt, *glen;
    int32_t *spos;
    int64_t *g_count;
    int32_t *glab;
    uint32_t *gflag;
    uint32_t *gsym;
    int64_t *ocnt, *olen;
    double *oinc;
    uint32_t *cut;
    uint32_t *cgid;
    int32_t *ord;
    int32_t *gstart;
    int64_t *n_groups;
    double *ck, *cx, *cy;
    int32_t *own;
    uint32_t *oflag;
    int32_t *sblk;
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
    w.lpart = c.take<unsigned long long>(2 * t0 + 2);
    sort_workspace(N, c, &w.sb);
    sort_workspace(N, c, &w.sb2);
    const int64_t ntiles = (N + kBucketTile - 1) / kBucketTile;
    w.thead = c.take<int64_t>(ntiles);
    w.tlarge = c.take<int64_t>(ntiles);
    w.lsize = c.take<int64_t>(ntiles);
    w.loff = c.take<int64_t>(ntiles + 1);
    w.n_large = c.take<int64_t>(1);
    w.sk = c.take<double>(N);
    w.sx = c.take<double>(N);
    w.sy = c.take<double>(N);
    w.sinc = c.take<double>(N);
    w.slen = c.take<int32_t>(N);
    w.perm = c.take<uint32_t>(N);
    w.rec = c.take<PieceRec>(N);
    w.cuts = c.take<int64_t>(nblk + 2);
    w.lab = c.take<int32_t>(N);
    w.flag = c.take<uint32_t>(N);
    w.sidx = c.take<uint32_t>(N + 1);
    w.glist = c.take<int32_t>(N + 64);
    w.gk = c.take<double>(N);
    w.gx = c.take<double>(N);
    w.gy = c.take<double>(N);
    w.ginc = c.take<double>(N);
    w.gcnt = c.take<int64_t>(N);
    w.glen = c.take<int64_t>(N);
    w.spos = c.take<int32_t>(N);
    w.g_count = c.take<int64_t>(1);
    w.glab = c.take<int32_t>(N);
    w.gflag = c.take<uint32_t>(N);
    w.gsym = c.take<uint32_t>(N + 1);
    w.ocnt = c.take<int64_t>(N);
    w.olen = c.take<int64_t>(N);
    w.oinc = c.take<double>(N);
    w.cut = c.take<uint32_t>(N);
    w.cgid = c.take<uint32_t>(N + 1);
    w.ord = c.take<int32_t>(N);
    w.gstart = c.take<int32_t>(N + 1);
    w.n_groups = c.take<int64_t>(1);
    w.ck = c.take<double>(N);
    w.cx = c.take<double>(N);
    w.cy = c.take<double>(N);
    w.own = c.take<int32_t>(N);
    w.oflag = c.take<uint32_t>(N);
    w.sblk = c.take<int32_t>(N);
    w.scan_ws = c.take<char>(scan_workspace(N + 1 > ntiles + 1 ? N + 1 : ntiles + 1));
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

namespace jabba {
namespace {

constexpr int kPrefixDigits = 4;  // radix digits of the main sort; the rest is sorted per prefix group

// After the prefix passes: the local sort of every prefix group, and the
// general radix sort of the pieces in groups too large for it.
template <int Key>
int bucket_sort(const DigWs &w, int64_t N, double scl, hipStream_t st) {
    const int64_t ntiles = (N + kBucketTile - 1) / kBucketTile;
    JB_LAUNCH_NAMED("k_bucket_local", k_bucket_local<Key>, dim3((unsigned)ntiles), dim3(kBucketThreads), 0, st,
                    w.sb.vals[0], w.sb.vals[1], w.rec, w.sb.ctl, w.sb.kmin, w.ds, scl, w.sk, w.sx, w.sy, w.slen,
                    w.sinc, w.perm, w.thead, w.tlarge);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_large_plan, dim3(1), dim3(1024), 0, st, w.thead, w.tlarge, w.ds, ntiles, w.lsize);
    JB_LAUNCH_CHECK();
    int rc = scan_i64_to_i64(w.lsize, w.loff, nullptr, ntiles, w.scan_ws, st);
    if (rc) return rc;
    rc = radix_sort_init(w.sb2, st);
    if (rc) return rc;
    JB_LAUNCH_NAMED("k_large_collect", k_large_collect<Key>, dim3(grid_for(N, 4)), dim3(256), 0, st, w.sb.vals[0],
                    w.sb.vals[1], w.rec, w.sb.ctl, w.loff, w.tlarge, w.ds, scl, w.sb2.keys[0], w.sb2.vals[0],
                    w.n_large);
    JB_LAUNCH_CHECK();
    rc = radix_global_hist(w.sb2, w.n_large, N, st);
    if (rc) return rc;
    rc = radix_sort_pairs(w.sb2, w.n_large, N, st, "large", kSortOrderOnly, /*sparse=*/true);
    if (rc) return rc;
    JB_LAUNCH_NAMED("k_large_emit", k_large_emit<Key>, dim3(grid_for(N, 4)), dim3(256), 0, st, w.sb.vals[0],
                    w.sb.vals[1], w.rec, w.sb.ctl, w.sb2.vals[0], w.sb2.vals[1], w.sb2.ctl, w.loff, w.tlarge, w.ds,
                    scl, w.sk, w.sx, w.sy, w.slen, w.sinc, w.perm);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

// label propagation (symbols in canonical order), see k_remap_pairs
constexpr int64_t kRemapDirectMax = (int64_t)1 << 26;  // 256 MB of symbols

int remap(const DigWs &w, int64_t N, int32_t *symbols, hipStream_t st) {
    if (N <= kRemapDirectMax) {
        JB_LAUNCH(k_remap, dim3(grid_for(N)), dim3(256), 0, st, w.ds, w.perm, w.lab, w.sidx, w.glab, w.gsym, symbols);
        JB_LAUNCH_CHECK();
        return JABBA_OK;
    }
    int rc = radix_sort_init(w.sb, st);
    if (rc) return rc;
    // indices below 2^bits; the two sorted digits are the index's top 16 bits
    // (the keys are shifted to end at bit 32), windows of 2^(bits - 16)
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < N) ++bits;
    const int wlog = bits - 16;
    const bool window = wlog <= kWindowMaxLog;
    const int sh = window ? 32 - bits : 0;
    JB_LAUNCH(k_remap_pairs, dim3(grid_for(N)), dim3(256), 0, st, w.ds, w.perm, w.lab, w.sidx, w.glab, w.gsym, sh,
              reinterpret_cast<uint32_t *>(w.sb.keys[0]), w.sb.vals[0]);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_remap_hist, dim3(1), dim3(256), 0, st, w.ds, sh, w.sb.ghist, w.sb.kmin);
    JB_LAUNCH_CHECK();
    rc = radix_sort_pairs(w.sb, &w.ds->n, N, st, "remap", kSortKeep32, /*sparse=*/false, /*prefix_digits=*/2);
    if (rc) return rc;
    if (window) {
        const int64_t nwin = (N + ((int64_t)1 << wlog) - 1) >> wlog;
        JB_LAUNCH(k_remap_window, dim3((unsigned)nwin), dim3(kWindowThreads), (size_t)4 << wlog, st, w.ds,
                  reinterpret_cast<const uint32_t *>(w.sb.keys[0]), reinterpret_cast<const uint32_t *>(w.sb.keys[1]),
                  w.sb.vals[0], w.sb.vals[1], w.sb.ctl, sh, wlog, symbols);
    } else {
        JB_LAUNCH(k_remap_scatter, dim3(grid_for(N)), dim3(256), 0, st, w.ds,
                  reinterpret_cast<const uint32_t *>(w.sb.keys[0]), reinterpret_cast<const uint32_t *>(w.sb.keys[1]),
                  w.sb.vals[0], w.sb.vals[1], w.sb.ctl, sh, symbols);
    }
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

int digitize_impl(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces, double alpha,
                  double scl, int32_t B, const jabba_tuning *tuning, int32_t *symbols, const jabba_dict *dict,
                  int key_kind, double *axis_out, void *workspace, size_t workspace_bytes, void *stream) {
    if (max_pieces < 0 || B < 1 || !n_pieces || !dict) return JABBA_EINVAL;
    if (!(alpha >= 0.0) || !(alpha <= 1.0e150) || !(scl >= 0.0) || !(scl <= 1.0e150)) return JABBA_EINVAL;
    if (max_pieces >= ((int64_t)1 << 31) - 1) return JABBA_EOVERFLOW;
    if (max_pieces > 0 && (!len || !inc || !symbols)) return JABBA_EINVAL;
    if (dict->capacity < 0 || !dict->k || (dict->capacity > 0 && (!dict->center_len || !dict->center_inc ||
                                                                  !dict->cx || !dict->cy || !dict->count)))
        return JABBA_EINVAL;
    const DigWs w0 = carve_digitize(nullptr, max_pieces, B);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    const DigWs w = carve_digitize(workspace, max_pieces, B);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = max_pieces > 0 ? max_pieces : 1;
    const int64_t nblk = nblk_of(N, B);
    int s1w = 4;
    if (tuning && tuning->stage1_waves) s1w = tuning->stage1_waves;
    if (s1w < 1 || s1w > 16) return JABBA_EINVAL;
    while (s1w > 1 && (size_t)s1w * sizeof(ActLds) > 65536) s1w >>= 1;  // keep the workgroup's LDS <= 64 KB
    const double a2 = alpha * alpha;

    JB_LAUNCH(k_dig_prepare, dim3(1), dim3(64), 0, st, w.ds, n_pieces, max_pieces);
    JB_LAUNCH_CHECK();
    // scaling: two pairwise-sum passes over inc, exact integer sums of len
    const int64_t t0 = (N + kTreeLeaves - 1) / kTreeLeaves;
    JB_LAUNCH((k_sum_leaves<1>), dim3((unsigned)t0), dim3(256), 0, st, len, inc, w.ds, w.tree[0], w.lpart);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_sum_ints, dim3(1), dim3(1024), 0, st, w.lpart, t0, w.ds);
    JB_LAUNCH_CHECK();
    double *tot = nullptr;
    int rc = tree_sum_levels(w, N, w.tree[0], st, &tot);
    if (rc) return rc;
    JB_LAUNCH(k_mean, dim3(1), dim3(64), 0, st, w.ds, tot);
    JB_LAUNCH_CHECK();
    JB_LAUNCH((k_sum_leaves<2>), dim3((unsigned)t0), dim3(256), 0, st, len, inc, w.ds, w.tree[0], w.lpart);
    JB_LAUNCH_CHECK();
    rc = tree_sum_levels(w, N, w.tree[0], st, &tot);
    if (rc) return rc;
    JB_LAUNCH(k_sigma, dim3(1), dim3(64), 0, st, w.ds, tot, scl, alpha, dict->params);
    JB_LAUNCH_CHECK();
    if (key_kind == kKeyPca) {
        // third pairwise-sum pass: covariance of len and inc, then the axis
        JB_LAUNCH((k_sum_leaves<3>), dim3((unsigned)t0), dim3(256), 0, st, len, inc, w.ds, w.tree[0], w.lpart);
        JB_LAUNCH_CHECK();
        rc = tree_sum_levels(w, N, w.tree[0], st, &tot);
        if (rc) return rc;
        JB_LAUNCH(k_pca_axis, dim3(1), dim3(64), 0, st, w.ds, tot, scl, axis_out);
        JB_LAUNCH_CHECK();
    }

    // key and global sorting index
    rc = radix_sort_init(w.sb, st);
    if (rc) return rc;
    if (key_kind == kKeyPca)
        JB_LAUNCH_NAMED("k_key_pca", (k_key<kKeyPca>), dim3(grid_for(N)), dim3(256), 0, st, len, inc, w.ds, scl,
                        w.sb.keys[0], w.sb.vals[0], w.rec);
    else
        JB_LAUNCH_NAMED("k_key", (k_key<kKeyNorm>), dim3(grid_for(N)), dim3(256), 0, st, len, inc, w.ds, scl,
                        w.sb.keys[0], w.sb.vals[0], w.rec);
    JB_LAUNCH_CHECK();
    const int64_t *n_live = &w.ds->n;
    rc = radix_global_hist(w.sb, n_live, N, st);
    if (rc) return rc;
    // radix passes over the highest four varying digits (the order alone),
    // then every prefix group is put in (key, index) order and leaves as the
    // sorted arrays
    rc = radix_sort_pairs(w.sb, n_live, N, st, "", kSortOrderOnly, /*sparse=*/false, kPrefixDigits);
    if (rc) return rc;
    rc = key_kind == kKeyPca ? bucket_sort<kKeyPca>(w, N, scl, st) : bucket_sort<kKeyNorm>(w, N, scl, st);
    if (rc) return rc;

    // Stage I: blocks of B sorted pieces, one wavefront each
    JB_LAUNCH(k_cuts, dim3(grid_for(nblk + 1)), dim3(256), 0, st, w.sk, w.ds, (int64_t)B, nblk, w.cuts);
    JB_LAUNCH_CHECK();
    const size_t lds = (size_t)s1w * sizeof(ActLds);
    JB_LAUNCH(k_stage1, dim3((unsigned)((nblk + s1w - 1) / s1w)), dim3(s1w * kWave), lds, st, w.cuts, nblk, w.sk,
              w.sx, w.sy, alpha, a2, w.ds, scl, w.glist, w.lab, w.flag, w.sblk);
    JB_LAUNCH_CHECK();
    rc = scan_u32_to_u32(w.flag, w.sidx, n_live, N, w.scan_ws, st);
    if (rc) return rc;
    JB_LAUNCH(k_compact_starts, dim3(grid_for(N)), dim3(256), 0, st, w.ds, w.flag, w.sidx, w.sk, w.sx, w.sy, w.gk,
              w.gx, w.gy, w.spos, w.g_count);
    JB_LAUNCH_CHECK();
    // sums of every local group: per block in LDS, per start for crowded blocks
    JB_LAUNCH(k_block_sums, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, st, w.cuts, nblk, w.sidx, w.lab,
              w.slen, w.sinc, w.gcnt, w.glen, w.ginc);
    JB_LAUNCH_CHECK();
    JB_LAUNCH((k_group_sums<true>), dim3(grid_for(N * kWave, 16)), dim3(256), 0, st, w.g_count, N, n_live, w.spos,
              w.sblk, w.cuts, w.sidx, w.flag, w.sk, w.lab, w.slen, (const int64_t *)nullptr, (const int64_t *)nullptr,
              w.sinc, alpha, w.gcnt, w.glen, w.ginc);
    JB_LAUNCH_CHECK();

    // Stage II over the starting points: independent groups (length column,
    // key gaps), one wavefront per group
    rc = radix_sort_init(w.sb, st);
    if (rc) return rc;
    JB_LAUNCH(k_col_keys, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.spos, w.slen, w.ds, scl, a2,
              w.sb.keys[0], w.sb.vals[0]);
    JB_LAUNCH_CHECK();
    rc = radix_global_hist(w.sb, w.g_count, N, st);
    if (rc) return rc;
    rc = radix_sort_pairs(w.sb, w.g_count, N, st, "groups", kSortKeep64, /*sparse=*/true);
    if (rc) return rc;
    JB_LAUNCH(k_col_cuts, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.sb.keys[0], w.sb.keys[1], w.sb.vals[0],
              w.sb.vals[1], w.sb.ctl, w.gk,
              w.gx, w.gy, alpha, w.cut, w.ord, w.ck, w.cx, w.cy);
    JB_LAUNCH_CHECK();
    rc = scan_u32_to_u32(w.cut, w.cgid, w.g_count, N, w.scan_ws, st);
    if (rc) return rc;
    JB_LAUNCH(k_col_groups, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.cut, w.cgid, w.gstart, w.n_groups);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_col_greedy, dim3(grid_for(N * kWave / 4 + 1, 32)), dim3(4 * kWave), 4 * sizeof(ActLds), st,
              w.n_groups, w.gstart, w.ord, w.ck, w.cx, w.cy, alpha, a2, w.ds, scl, w.glist, w.own, w.oflag, w.glab,
              w.gflag);
    JB_LAUNCH_CHECK();
    rc = scan_u32_to_u32(w.gflag, w.gsym, w.g_count, N, w.scan_ws, st);
    if (rc) return rc;
    // Stage II sums by owner (the column sort's buffers are free again)
    rc = radix_sort_init(w.sb, st);
    if (rc) return rc;
    JB_LAUNCH(k_owner_pairs, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.glab, w.sb.keys[0], w.sb.vals[0]);
    JB_LAUNCH_CHECK();
    rc = radix_global_hist(w.sb, w.g_count, N, st);
    if (rc) return rc;
    rc = radix_sort_pairs(w.sb, w.g_count, N, st, "owners", kSortKeep64, /*sparse=*/true);
    if (rc) return rc;
    JB_LAUNCH(k_owner_heads, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.sb.keys[0], w.sb.keys[1], w.sb.ctl,
              w.cgid);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_owner_sums, dim3(grid_for(N * kWave, 16)), dim3(256), 0, st, w.g_count, w.gflag, w.sb.keys[0],
              w.sb.keys[1], w.sb.vals[0], w.sb.vals[1], w.sb.ctl, w.cgid, w.gcnt, w.glen, w.ginc, w.ocnt, w.olen,
              w.oinc);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_dict, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.gflag, w.gsym, w.ocnt, w.olen, w.oinc, w.ds,
              scl, *dict);
    JB_LAUNCH_CHECK();
    rc = remap(w, N, symbols, st);
    if (rc) return rc;
    return JABBA_OK;
}

}  // namespace
}  // namespace jabba

extern "C" int jabba_digitize(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                              double alpha, double scl, int32_t B, const jabba_tuning *tuning, int32_t *symbols,
                              const jabba_dict *dict, void *workspace, size_t workspace_bytes, void *stream) {
    return digitize_impl(len, inc, n_pieces, max_pieces, alpha, scl, B, tuning, symbols, dict, kKeyNorm, nullptr,
                         workspace, workspace_bytes, stream);
}

extern "C" int jabba_aggregate_points(const double *x, const double *y, const int64_t *n_points, int64_t max_points,
                                      double alpha, int32_t B, int32_t *labels, int64_t capacity, double *cx,
                                      double *cy, int64_t *count, int64_t *k, double *sse, void *workspace,
                                      size_t workspace_bytes, void *stream) {
    if (max_points < 0 || B < 1 || !n_points || !k || capacity < 0) return JABBA_EINVAL;
    if (!(alpha >= 0.0) || !(alpha <= 1.0e150)) return JABBA_EINVAL;
    if (max_points >= ((int64_t)1 << 31) - 1) return JABBA_EOVERFLOW;
    if (max_points > 0 && (!x || !y || !labels)) return JABBA_EINVAL;
    if (capacity > 0 && (!cx || !cy || !count)) return JABBA_EINVAL;
    const DigWs w0 = carve_digitize(nullptr, max_points, B);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    const DigWs w = carve_digitize(workspace, max_points, B);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = max_points > 0 ? max_points : 1;
    const int64_t nblk = nblk_of(N, B);
    int s1w = 4;
    while (s1w > 1 && (size_t)s1w * sizeof(ActLds) > 65536) s1w >>= 1;
    const double a2 = alpha * alpha;
    PointRec *rec = reinterpret_cast<PointRec *>(w.rec);
    const int64_t *n_live = &w.ds->n;

    JB_LAUNCH(k_dig_prepare, dim3(1), dim3(64), 0, st, w.ds, n_points, max_points);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_pts_prepare, dim3(1), dim3(64), 0, st, w.ds);
    JB_LAUNCH_CHECK();
    int rc = radix_sort_init(w.sb, st);
    if (rc) return rc;
    JB_LAUNCH(k_pts_key, dim3(grid_for(N)), dim3(256), 0, st, x, y, w.ds, w.sb.keys[0], w.sb.vals[0], rec);
    JB_LAUNCH_CHECK();
    rc = radix_global_hist(w.sb, n_live, N, st);
    if (rc) return rc;
    rc = radix_sort_pairs(w.sb, n_live, N, st);
    if (rc) return rc;
    JB_LAUNCH(k_pts_gather, dim3(grid_for(N)), dim3(256), 0, st, rec, w.ds, w.sb.keys[0], w.sb.keys[1],
              w.sb.vals[0], w.sb.vals[1], w.sb.ctl, w.sk, w.sx, w.sy, w.perm);
    JB_LAUNCH_CHECK();

    // Stage I
    JB_LAUNCH(k_cuts, dim3(grid_for(nblk + 1)), dim3(256), 0, st, w.sk, w.ds, (int64_t)B, nblk, w.cuts);
    JB_LAUNCH_CHECK();
    const size_t lds = (size_t)s1w * sizeof(ActLds);
    JB_LAUNCH(k_stage1, dim3((unsigned)((nblk + s1w - 1) / s1w)), dim3(s1w * kWave), lds, st, w.cuts, nblk, w.sk,
              w.sx, w.sy, alpha, a2, w.ds, 0.0, w.glist, w.lab, w.flag, w.sblk);
    JB_LAUNCH_CHECK();
    rc = scan_u32_to_u32(w.flag, w.sidx, n_live, N, w.scan_ws, st);
    if (rc) return rc;
    JB_LAUNCH(k_compact_starts, dim3(grid_for(N)), dim3(256), 0, st, w.ds, w.flag, w.sidx, w.sk, w.sx, w.sy, w.gk,
              w.gx, w.gy, w.spos, w.g_count);
    JB_LAUNCH_CHECK();

    // Stage II: one column (scl = 0 switches the length columns off), groups
    // cut at key gaps larger than alpha
    rc = radix_sort_init(w.sb, st);
    if (rc) return rc;
    JB_LAUNCH(k_col_keys, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.spos, w.slen, w.ds, 0.0, a2,
              w.sb.keys[0], w.sb.vals[0]);
    JB_LAUNCH_CHECK();
    rc = radix_global_hist(w.sb, w.g_count, N, st);
    if (rc) return rc;
    rc = radix_sort_pairs(w.sb, w.g_count, N, st, "groups", kSortKeep64, /*sparse=*/true);
    if (rc) return rc;
    JB_LAUNCH(k_col_cuts, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.sb.keys[0], w.sb.keys[1], w.sb.vals[0],
              w.sb.vals[1], w.sb.ctl, w.gk, w.gx, w.gy, alpha, w.cut, w.ord, w.ck, w.cx, w.cy);
    JB_LAUNCH_CHECK();
    rc = scan_u32_to_u32(w.cut, w.cgid, w.g_count, N, w.scan_ws, st);
    if (rc) return rc;
    JB_LAUNCH(k_col_groups, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.cut, w.cgid, w.gstart, w.n_groups);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_col_greedy, dim3(grid_for(N * kWave / 4 + 1, 32)), dim3(4 * kWave), 4 * sizeof(ActLds), st,
              w.n_groups, w.gstart, w.ord, w.ck, w.cx, w.cy, alpha, a2, w.ds, 0.0, w.glist, w.own, w.oflag, w.glab,
              w.gflag);
    JB_LAUNCH_CHECK();
    rc = scan_u32_to_u32(w.gflag, w.gsym, w.g_count, N, w.scan_ws, st);
    if (rc) return rc;
    rc = remap(w, N, labels, st);
    if (rc) return rc;

    // centers: labels sorted stably, one wavefront per cluster
    rc = radix_sort_init(w.sb, st);
    if (rc) return rc;
    JB_LAUNCH(k_pts_pairs, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.gsym, w.ds, labels, capacity, k,
              w.sb.keys[0], w.sb.vals[0]);
    JB_LAUNCH_CHECK();
    rc = radix_global_hist(w.sb, n_live, N, st);
    if (rc) return rc;
    rc = radix_sort_pairs(w.sb, n_live, N, st, "points");
    if (rc) return rc;
    JB_LAUNCH(k_pts_runs, dim3(grid_for(N)), dim3(256), 0, st, w.sb.keys[0], w.sb.keys[1], w.sb.ctl, w.ds, w.ocnt,
              w.olen);
    JB_LAUNCH_CHECK();
    if (capacity > 0) {
        JB_LAUNCH(k_pts_centers, dim3(grid_for(capacity * kWave, 32)), dim3(256), 0, st, x, y, w.sb.vals[0],
                  w.sb.vals[1], w.sb.ctl, k, capacity, w.ocnt, w.olen, cx, cy, count);
        JB_LAUNCH_CHECK();
    }
    if (sse) {
        const int64_t t0 = (N + kTreeLeaves - 1) / kTreeLeaves;
        JB_LAUNCH(k_pts_sse_leaves, dim3((unsigned)t0), dim3(256), 0, st, x, y, labels, cx, cy, k, capacity, w.ds,
                  w.tree[0]);
        JB_LAUNCH_CHECK();
        double *tot = nullptr;
        rc = tree_sum_levels(w, N, w.tree[0], st, &tot);
        if (rc) return rc;
        JB_LAUNCH(k_pts_sse_out, dim3(1), dim3(64), 0, st, tot, sse);
        JB_LAUNCH_CHECK();
    }
    return JABBA_OK;
}

extern "C" int jabba_axis_tolerances(double alpha_len, double alpha_inc, double scl_in, double *alpha,
                                     double *scl) {
    if (!alpha || !scl) return JABBA_EINVAL;
    if (!(alpha_len > 0.0) || !(alpha_len <= 1.0e150) || !(alpha_inc > 0.0) || !(alpha_inc <= 1.0e150) ||
        !(scl_in >= 0.0) || !(scl_in <= 1.0e150))
        return JABBA_EINVAL;
    *alpha = alpha_inc;
    *scl = scl_in * (alpha_inc / alpha_len);
    return JABBA_OK;
}

extern "C" int jabba_digitize_pca(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                                  double alpha, double scl, int32_t B, const jabba_tuning *tuning, int32_t *symbols,
                                  const jabba_dict *dict, double *axis, void *workspace, size_t workspace_bytes,
                                  void *stream) {
    return digitize_impl(len, inc, n_pieces, max_pieces, alpha, scl, B, tuning, symbols, dict, kKeyPca, axis,
                         workspace, workspace_bytes, stream);
}

extern "C" int jabba_digitize_stats(const void *workspace, int64_t max_pieces, int32_t B, void *stream,
                                    int64_t *stats) {
    if (!workspace || !stats || max_pieces < 0 || B < 1) return JABBA_EINVAL;
    const DigWs w = carve_digitize(const_cast<void *>(workspace), max_pieces, B);
    JB_HIP(hipStreamSynchronize((hipStream_t)stream));
    DigState ds;
    int64_t G = 0;
    JB_HIP(hipMemcpy(&ds, w.ds, sizeof(DigState), hipMemcpyDeviceToHost));
    JB_HIP(hipMemcpy(&G, w.g_count, sizeof(int64_t), hipMemcpyDeviceToHost));
    uint32_t k = 0;
    if (G > 0) JB_HIP(hipMemcpy(&k, w.gsym + G, sizeof(uint32_t), hipMemcpyDeviceToHost));
    const int64_t active = ds.sort_passes;
    stats[0] = ds.n;
    stats[1] = G;
    stats[2] = k;
    stats[3] = active;
    int64_t ng = 0;
    JB_HIP(hipMemcpy(&ng, w.n_groups, sizeof(int64_t), hipMemcpyDeviceToHost));
    stats[4] = ng;
    stats[5] = ds.sort_bytes;
    stats[6] = ds.sort_large;
    return JABBA_OK;
}

// Quality of the digitization held by the workspace: the squared deviations
// are summed per Stage I group and then per symbol by the same kernels and in
// the same order as the centers.  Scratch: arrays the digitization no longer
// needs (piece records, Stage II column copies, the final group sums).
extern "C" int jabba_digitize_quality(const int32_t *len, const double *inc, const int64_t *n_pieces,
                                      int64_t max_pieces, double alpha, int32_t B, const jabba_dict *dict,
                                      double *var_len, double *var_inc, double *totals, void *workspace,
                                      size_t workspace_bytes, void *stream) {
    if (max_pieces < 0 || B < 1 || !n_pieces || !dict || !var_len || !var_inc || !totals) return JABBA_EINVAL;
    if (!(alpha >= 0.0) || !(alpha <= 1.0e150)) return JABBA_EINVAL;
    if (max_pieces >= ((int64_t)1 << 31) - 1) return JABBA_EOVERFLOW;
    if (max_pieces > 0 && (!len || !inc)) return JABBA_EINVAL;
    if (dict->capacity < 1 || !dict->k || !dict->cx || !dict->cy || !dict->count) return JABBA_EINVAL;
    const DigWs w0 = carve_digitize(nullptr, max_pieces, B);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    const DigWs w = carve_digitize(workspace, max_pieces, B);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = max_pieces > 0 ? max_pieces : 1;
    const int64_t nblk = nblk_of(N, B);
    const int64_t *n_live = &w.ds->n;
    double *qx = reinterpret_cast<double *>(w.rec);  // 2N doubles of dead piece records
    double *qy = qx + N;
    JB_LAUNCH(k_q_values, dim3(grid_for(N)), dim3(256), 0, st, w.ds, w.sx, w.sy, w.lab, w.sidx, w.glab, w.gsym,
              *dict, qx, qy);
    JB_LAUNCH_CHECK();
    double *q[2] = {qx, qy};
    double *stage1[2] = {w.ck, w.cx};   // per Stage I group
    double *stage2[2] = {w.cy, w.oinc}; // per symbol (indexed by its global start)
    for (int a = 0; a < 2; ++a) {
        JB_LAUNCH(k_block_sums, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, st, w.cuts, nblk, w.sidx, w.lab,
                  w.slen, q[a], w.ocnt, w.olen, stage1[a]);
        JB_LAUNCH_CHECK();
        JB_LAUNCH((k_group_sums<true>), dim3(grid_for(N * kWave, 16)), dim3(256), 0, st, w.g_count, N, n_live,
                  w.spos, w.sblk, w.cuts, w.sidx, w.flag, w.sk, w.lab, w.slen, (const int64_t *)nullptr,
                  (const int64_t *)nullptr, q[a], alpha, w.ocnt, w.olen, stage1[a]);
        JB_LAUNCH_CHECK();
        JB_LAUNCH((k_group_sums<false>), dim3(grid_for(N * kWave, 16)), dim3(256), 0, st, w.g_count, N, w.g_count,
                  (const int32_t *)nullptr, (const int32_t *)nullptr, (const int64_t *)nullptr,
                  (const uint32_t *)nullptr, w.gflag, w.gk, w.glab, (const int32_t *)nullptr, w.gcnt, w.glen,
                  stage1[a], alpha, w.ocnt, w.olen, stage2[a]);
        JB_LAUNCH_CHECK();
    }
    double *per_symbol = w.gy;
    JB_LAUNCH(k_q_symbols, dim3(grid_for(N)), dim3(256), 0, st, w.g_count, w.gflag, w.gsym, stage2[0], stage2[1],
              *dict, var_len, var_inc, per_symbol);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_q_totals, dim3(1), dim3(1024), 0, st, dict->k, dict->capacity, per_symbol, var_len, var_inc, totals);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}
