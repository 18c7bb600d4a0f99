// Nearest-center digitization against a resident dictionary (Sec. 3.2:
// c* = argmin_c ||p - c||_2, f_d(p) = I_d(c*)), ties to the lowest symbol.
//
// The k scaled centers are ordered by (cx, cy, symbol) in one workgroup and
// grouped into columns of equal cx.  A piece binary-searches its x among the
// column abscissae and visits columns outwards in both directions; within a
// column (one rounded dx^2 for all its centers) it binary-searches its y and
// walks outwards in cy.  A walk stops at the first center whose rounded
// distance fl(fl(dx^2) + fl(dy^2)) already exceeds the best, and a direction
// of columns stops at the first column whose fl(dx^2) does: the rounded
// distance grows with |dx| and with |dy| along every walk, so each skipped
// center is strictly farther than the best.  The result is the argmin over
// all k centers with the same rounded distances as a full scan, ties (equal
// rounded distance) to the lowest symbol.  The distance is plain FP64 VALU
// work: the exact rounded d2 decides, so it is not recast as a matrix
// product.
#include "common.h"

#include <mutex>

namespace jabba {
namespace {

constexpr int kThreads = 256;
constexpr int kSortLds = 2048;     // centers sorted in LDS; larger dictionaries sort in global memory
constexpr int kLdsCenters = 2048;  // centers and columns staged in LDS for the search up to this capacity

// order-preserving unsigned image of a double (total order for non-NaN
// values); -0.0 is taken as +0.0 so that equal values share one key
__device__ __forceinline__ uint64_t dkey(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v == 0.0 ? 0.0 : v);
    return (b >> 63) ? ~b : (b | (1ull << 63));
}

struct CKey {
    uint64_t x, y;
    int32_t id;
};

__device__ __forceinline__ bool less_key(const CKey &a, const CKey &b) {
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.id < b.id;
}

// bitonic sort of (cx key, cy key, id) over P = 2^m slots, one workgroup
__device__ void bitonic(uint64_t *kx, uint64_t *ky, int32_t *id, int P, bool global) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const CKey a{kx[lo], ky[lo], id[lo]}, b{kx[hi], ky[hi], id[hi]};
                const bool swap = up ? less_key(b, a) : less_key(a, b);
                if (swap) {
                    kx[lo] = b.x;
                    ky[lo] = b.y;
                    id[lo] = b.id;
                    kx[hi] = a.x;
                    ky[hi] = a.y;
                    id[hi] = a.id;
                }
            }
            if (global) __threadfence_block();
            __syncthreads();
        }
    }
}

// Sorts the centers and builds the columns: col_x[c] is the abscissa of
// column c, its centers are [col_start[c], col_start[c + 1]) in cy order.
__global__ __launch_bounds__(1024) void k_enc_sort(const int64_t *__restrict__ kp, int64_t capacity, int P_max,
                                                   const double *__restrict__ cx, const double *__restrict__ cy,
                                                   uint64_t *__restrict__ gkx, uint64_t *__restrict__ gky,
                                                   int32_t *__restrict__ gid, double *__restrict__ scy,
                                                   int32_t *__restrict__ sid, double *__restrict__ col_x,
                                                   int32_t *__restrict__ col_start, int32_t *__restrict__ n_col) {
    __shared__ uint64_t lkx[kSortLds];
    __shared__ uint64_t lky[kSortLds];
    __shared__ int32_t lid[kSortLds];
    __shared__ int32_t wave_cnt[1024 / kWave];
    __shared__ int32_t carry_s;
    int64_t k = *kp;
    k = k < 0 ? 0 : (k > capacity ? capacity : k);
    int P = 1;
    while (P < k) P <<= 1;
    if (P > P_max) P = P_max;
    const bool lds = P <= kSortLds;
    uint64_t *kx = lds ? lkx : gkx;
    uint64_t *ky = lds ? lky : gky;
    int32_t *id = lds ? lid : gid;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        kx[i] = i < k ? dkey(cx[i]) : ~0ull;
        ky[i] = i < k ? dkey(cy[i]) : ~0ull;
        id[i] = i < k ? i : 0x7fffffff;
    }
    if (!lds) __threadfence_block();
    __syncthreads();
    bitonic(kx, ky, id, P, !lds);
    // heads of the runs of equal cx, numbered by a block-wide scan
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    for (int64_t base = 0; base < k; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool head = i < k && (i == 0 || kx[i] != kx[i - 1]);
        const uint64_t hm = __ballot(head);
        if (lane == 0) wave_cnt[wave] = __popcll(hm);
        __syncthreads();
        int off = carry_s;
        for (int q = 0; q < wave; ++q) off += wave_cnt[q];
        if (i < k) {
            const int32_t c = id[i];
            sid[i] = c;
            scy[i] = cy[c];
            if (head) {
                const int ci = off + __popcll(hm & lanemask_lt());
                col_start[ci] = (int32_t)i;
                col_x[ci] = cx[c];
            }
        }
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) {
            int tot = carry_s;
            for (int q = 0; q < (int)(blockDim.x / kWave); ++q) tot += wave_cnt[q];
            carry_s = tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *n_col = carry_s;
        col_start[carry_s] = (int32_t)k;
    }
}

// best (d2, symbol) over column c, walking outwards from the nearest cy
__device__ __forceinline__ void scan_column(double sx, double sy, double dd, int32_t lo, int32_t hi,
                                            const double *__restrict__ scy, const int32_t *__restrict__ sid,
                                            int32_t &best, double &bd) {
    int32_t a = lo, b = hi;  // first center with cy >= sy
    while (a < b) {
        const int32_t m = (a + b) >> 1;
        if (scy[m] < sy)
            a = m + 1;
        else
            b = m;
    }
    for (int32_t j = a; j < hi; ++j) {
        const double dy = sy - scy[j];
        const double ee = dy * dy;
        const double d2 = dd + ee;
        if (best >= 0 && d2 > bd) break;
        const int32_t c = sid[j];
        if (best < 0 || d2 < bd || (d2 == bd && c < best)) {
            best = c;
            bd = d2;
        }
    }
    for (int32_t j = a - 1; j >= lo; --j) {
        const double dy = sy - scy[j];
        const double ee = dy * dy;
        const double d2 = dd + ee;
        if (best >= 0 && d2 > bd) break;
        const int32_t c = sid[j];
        if (best < 0 || d2 < bd || (d2 == bd && c < best)) {
            best = c;
            bd = d2;
        }
    }
}

template <bool Lds>
__global__ __launch_bounds__(kThreads) void k_encode(const int32_t *__restrict__ len, const double *__restrict__ inc,
                                                     const int64_t *__restrict__ n_dev, int64_t n_max,
                                                     const double *__restrict__ params, const int64_t *__restrict__ kp,
                                                     int64_t capacity, const double *__restrict__ gcy,
                                                     const int32_t *__restrict__ gid,
                                                     const double *__restrict__ gcol_x,
                                                     const int32_t *__restrict__ gcol_start,
                                                     const int32_t *__restrict__ n_col_p,
                                                     int32_t *__restrict__ symbols) {
    __shared__ double lcy[Lds ? kLdsCenters : 1];
    __shared__ int32_t lid[Lds ? kLdsCenters : 1];
    __shared__ double lcx[Lds ? kLdsCenters : 1];
    __shared__ int32_t lcs[Lds ? kLdsCenters + 1 : 1];
    int64_t n = *n_dev;
    n = n < 0 ? 0 : (n > n_max ? n_max : n);
    int64_t k = *kp;
    k = k < 0 ? 0 : (k > capacity ? capacity : k);
    const int32_t ncol = *n_col_p;
    const double *scy = gcy;
    const int32_t *sid = gid;
    const double *col_x = gcol_x;
    const int32_t *col_start = gcol_start;
    if (Lds) {
        for (int64_t i = threadIdx.x; i < k; i += kThreads) {
            lcy[i] = gcy[i];
            lid[i] = gid[i];
        }
        for (int i = threadIdx.x; i <= ncol; i += kThreads) {
            lcs[i] = gcol_start[i];
            if (i < ncol) lcx[i] = gcol_x[i];
        }
        __syncthreads();
        scy = lcy;
        sid = lid;
        col_x = lcx;
        col_start = lcs;
    }
    const double sl = params[0], si = params[1], scl = params[2];
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const Scaled s = scale_piece(len[i], inc[i], scl, sl, si);
        // first column with cx >= x
        int32_t lo = 0, hi = ncol;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (col_x[mid] < s.x)
                lo = mid + 1;
            else
                hi = mid;
        }
        int32_t best = -1;
        double bd = 0.0;
        for (int32_t c = lo; c < ncol; ++c) {
            const double dx = s.x - col_x[c];
            const double dd = dx * dx;
            if (best >= 0 && dd > bd) break;
            scan_column(s.x, s.y, dd, col_start[c], col_start[c + 1], scy, sid, best, bd);
        }
        for (int32_t c = lo - 1; c >= 0; --c) {
            const double dx = s.x - col_x[c];
            const double dd = dx * dx;
            if (best >= 0 && dd > bd) break;
            scan_column(s.x, s.y, dd, col_start[c], col_start[c + 1], scy, sid, best, bd);
        }
        symbols[i] = best;
    }
}

struct EncWs {
    uint64_t *kx, *ky;
    int32_t *id;
    double *scy;
    int32_t *sid;
    double *col_x;
    int32_t *col_start;
    int32_t *n_col;
    size_t bytes;
    int P;
};

EncWs carve_enc(void *ws, int64_t capacity) {
    int P = 1;
    while (P < capacity) P <<= 1;
    Carve c(ws);
    EncWs w;
    w.P = P;
    w.kx = c.take<uint64_t>(P);
    w.ky = c.take<uint64_t>(P);
    w.id = c.take<int32_t>(P);
    w.scy = c.take<double>(P);
    w.sid = c.take<int32_t>(P);
    w.col_x = c.take<double>(P);
    w.col_start = c.take<int32_t>(P + 1);
    w.n_col = c.take<int32_t>(1);
    w.bytes = c.bytes();
    return w;
}

}  // namespace

// ----------------------------------------------------------- allocation-free
// Scratch of jabba_encode_noalloc: the encode workspace of a dictionary of
// JABBA_ENCODE_NOALLOC_MAX_CAPACITY centers, held in a file-scope device
// array.  Every device the library runs on holds its own copy, at its own
// address, until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in symbol); it passes the
// device address that hipGetSymbolAddress returned for the current device.
constexpr size_t kNoallocScratchBytes = 3u << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch, looked up once per device with
// that device current.  JABBA_EHIP when the runtime cannot resolve it.
int scratch_address(void **out) {
    int dev = -1;
    JB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return JABBA_EHIP;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        JB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return JABBA_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return JABBA_OK;
}

int encode_launch(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                  const jabba_dict *dict, int32_t *symbols, void *workspace, hipStream_t st) {
    JB_DEVICE_CHECK();
    const EncWs w = carve_enc(workspace, dict->capacity);
    JB_LAUNCH(k_enc_sort, dim3(1), dim3(1024), 0, st, dict->k, dict->capacity, w.P, dict->cx, dict->cy, w.kx, w.ky,
              w.id, w.scy, w.sid, w.col_x, w.col_start, w.n_col);
    JB_LAUNCH_CHECK();
    int64_t blocks = (max_pieces + kThreads - 1) / kThreads;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (blocks > cap) blocks = cap;
    if (dict->capacity <= kLdsCenters)
        JB_LAUNCH(k_encode<true>, dim3((unsigned)blocks), dim3(kThreads), 0, st, len, inc, n_pieces, max_pieces,
                  dict->params, dict->k, dict->capacity, w.scy, w.sid, w.col_x, w.col_start, w.n_col, symbols);
    else
        JB_LAUNCH(k_encode<false>, dim3((unsigned)blocks), dim3(kThreads), 0, st, len, inc, n_pieces, max_pieces,
                  dict->params, dict->k, dict->capacity, w.scy, w.sid, w.col_x, w.col_start, w.n_col, symbols);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

int encode_check(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                 const jabba_dict *dict, int32_t *symbols) {
    if (!dict || !n_pieces || max_pieces < 0) return JABBA_EINVAL;
    if (max_pieces == 0) return JABBA_OK;
    if (!len || !inc || !symbols || !dict->params || !dict->k || dict->capacity < 1 || !dict->cx || !dict->cy)
        return JABBA_EINVAL;
    if (dict->capacity > (1 << 30)) return JABBA_EINVAL;
    return JABBA_OK;
}
}  // namespace
}  // namespace jabba

using namespace jabba;

extern "C" int jabba_encode_workspace(int64_t capacity, size_t *bytes) {
    if (!bytes || capacity < 1 || capacity > (1 << 30)) return JABBA_EINVAL;
    *bytes = carve_enc(nullptr, capacity).bytes;
    return JABBA_OK;
}

extern "C" int jabba_encode(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                            const jabba_dict *dict, int32_t *symbols, void *workspace, size_t workspace_bytes,
                            void *stream) {
    const int rc = encode_check(len, inc, n_pieces, max_pieces, dict, symbols);
    if (rc != JABBA_OK || max_pieces == 0) return rc;
    if (!workspace || workspace_bytes < carve_enc(nullptr, dict->capacity).bytes) return JABBA_ENOMEM;
    return encode_launch(len, inc, n_pieces, max_pieces, dict, symbols, workspace, (hipStream_t)stream);
}

extern "C" int jabba_encode_noalloc(const int32_t *len, const double *inc, const int64_t *n_pieces,
                                    int64_t max_pieces, const jabba_dict *dict, int32_t *symbols, void *stream) {
    const int rc = encode_check(len, inc, n_pieces, max_pieces, dict, symbols);
    if (rc != JABBA_OK || max_pieces == 0) return rc;
    if (dict->capacity > JABBA_ENCODE_NOALLOC_MAX_CAPACITY) return JABBA_ELIMIT;
    if (carve_enc(nullptr, dict->capacity).bytes > kNoallocScratchBytes) return JABBA_ELIMIT;
    JB_DEVICE_CHECK();
    void *ws = nullptr;
    const int ra = scratch_address(&ws);
    if (ra != JABBA_OK) return ra;
    return encode_launch(len, inc, n_pieces, max_pieces, dict, symbols, ws, (hipStream_t)stream);
}
