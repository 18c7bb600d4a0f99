// Nearest-center digitization against a resident dictionary (Sec. 3.2:
// c* = argmin_c ||p - c||_2, f_d(p) = I_d(c*)), ties to the lowest symbol.
//
// The k scaled centers are first ordered by cx (ties by symbol) in one
// workgroup.  Each piece then binary-searches its x among the sorted cx and
// walks outwards in both directions, keeping the best (d2, symbol) pair; a
// walk stops at the first center whose fl(dx^2) already exceeds the best d2.
// Because fl(dx^2 + dy^2) >= fl(dx^2) and |dx| only grows along the walk,
// every center not visited is strictly farther than the best, so the result
// is the argmin over all k centers with the same rounded distances as a full
// scan (which a sequential evaluation performs).  The distance is plain FP64
// VALU work: the exact rounded d2 decides, so it is not recast as a matrix
// product.
#include "common.h"

namespace jabba {
namespace {

constexpr int kThreads = 256;
constexpr int kSortLds = 4096;  // centers sorted in LDS; larger dictionaries sort in global memory

// order-preserving unsigned image of a double (total order for non-NaN values)
__device__ __forceinline__ uint64_t dkey(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | (1ull << 63));
}

__device__ __forceinline__ bool less_pair(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// bitonic sort of (key, id) over P = 2^m slots, one workgroup
__device__ void bitonic(uint64_t *key, int32_t *id, int P, bool global) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = key[lo], b = key[hi];
                const int32_t ia = id[lo], ib = id[hi];
                const bool swap = up ? less_pair(b, ib, a, ia) : less_pair(a, ia, b, ib);
                if (swap) {
                    key[lo] = b;
                    key[hi] = a;
                    id[lo] = ib;
                    id[hi] = ia;
                }
            }
            if (global) __threadfence_block();
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(1024) void k_enc_sort(const int64_t *__restrict__ kp, int64_t capacity, int P_max,
                                                   const double *__restrict__ cx, const double *__restrict__ cy,
                                                   uint64_t *__restrict__ gkey, int32_t *__restrict__ gid,
                                                   double *__restrict__ scx, double *__restrict__ scy,
                                                   int32_t *__restrict__ sid) {
    __shared__ uint64_t lkey[kSortLds];
    __shared__ int32_t lid[kSortLds];
    int64_t k = *kp;
    k = k < 0 ? 0 : (k > capacity ? capacity : k);
    int P = 1;
    while (P < k) P <<= 1;
    if (P > P_max) P = P_max;
    const bool lds = P <= kSortLds;
    uint64_t *key = lds ? lkey : gkey;
    int32_t *id = lds ? lid : gid;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        key[i] = i < k ? dkey(cx[i]) : ~0ull;
        id[i] = i < k ? i : 0x7fffffff;
    }
    if (!lds) __threadfence_block();
    __syncthreads();
    bitonic(key, id, P, !lds);
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const int32_t c = id[i];
        sid[i] = c;
        scx[i] = cx[c];
        scy[i] = cy[c];
    }
}

__global__ __launch_bounds__(kThreads) void k_encode(const int32_t *__restrict__ len, const double *__restrict__ inc,
                                                     const int64_t *__restrict__ n_dev, int64_t n_max,
                                                     const double *__restrict__ params, const int64_t *__restrict__ kp,
                                                     int64_t capacity, const double *__restrict__ scx,
                                                     const double *__restrict__ scy, const int32_t *__restrict__ sid,
                                                     int32_t *__restrict__ symbols) {
    int64_t n = *n_dev;
    n = n < 0 ? 0 : (n > n_max ? n_max : n);
    int64_t k = *kp;
    k = k < 0 ? 0 : (k > capacity ? capacity : k);
    const double sl = params[0], si = params[1], scl = params[2];
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const Scaled s = scale_piece(len[i], inc[i], scl, sl, si);
        // first sorted center with cx >= x
        int64_t lo = 0, hi = k;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (scx[mid] < s.x)
                lo = mid + 1;
            else
                hi = mid;
        }
        int32_t best = -1;
        double bd = 0.0;
        for (int64_t j = lo; j < k; ++j) {
            const double dx = s.x - scx[j];
            const double dd = dx * dx;
            if (best >= 0 && dd > bd) break;
            const double dy = s.y - scy[j];
            const double ee = dy * dy;
            const double d2 = dd + ee;
            const int32_t c = sid[j];
            if (best < 0 || d2 < bd || (d2 == bd && c < best)) {
                best = c;
                bd = d2;
            }
        }
        for (int64_t j = lo - 1; j >= 0; --j) {
            const double dx = s.x - scx[j];
            const double dd = dx * dx;
            if (best >= 0 && dd > bd) break;
            const double dy = s.y - scy[j];
            const double ee = dy * dy;
            const double d2 = dd + ee;
            const int32_t c = sid[j];
            if (best < 0 || d2 < bd || (d2 == bd && c < best)) {
                best = c;
                bd = d2;
            }
        }
        symbols[i] = best;
    }
}

struct EncWs {
    uint64_t *key;
    int32_t *id;
    double *scx, *scy;
    int32_t *sid;
    size_t bytes;
    int P;
};

EncWs carve_enc(void *ws, int64_t capacity) {
    int P = 1;
    while (P < capacity) P <<= 1;
    Carve c(ws);
    EncWs w;
    w.P = P;
    w.key = c.take<uint64_t>(P);
    w.id = c.take<int32_t>(P);
    w.scx = c.take<double>(P);
    w.scy = c.take<double>(P);
    w.sid = c.take<int32_t>(P);
    w.bytes = c.bytes();
    return w;
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
    if (!dict || !n_pieces || max_pieces < 0) return JABBA_EINVAL;
    if (max_pieces == 0) return JABBA_OK;
    if (!len || !inc || !symbols || !dict->params || !dict->k || dict->capacity < 1 || !dict->cx || !dict->cy)
        return JABBA_EINVAL;
    if (dict->capacity > (1 << 30)) return JABBA_EINVAL;
    const EncWs w0 = carve_enc(nullptr, dict->capacity);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    const EncWs w = carve_enc(workspace, dict->capacity);
    hipStream_t st = (hipStream_t)stream;
    JB_LAUNCH(k_enc_sort, dim3(1), dim3(1024), 0, st, dict->k, dict->capacity, w.P, dict->cx, dict->cy, w.key, w.id,
              w.scx, w.scy, w.sid);
    JB_LAUNCH_CHECK();
    int64_t blocks = (max_pieces + kThreads - 1) / kThreads;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (blocks > cap) blocks = cap;
    JB_LAUNCH(k_encode, dim3((unsigned)blocks), dim3(kThreads), 0, st, len, inc, n_pieces, max_pieces, dict->params,
              dict->k, dict->capacity, w.scx, w.scy, w.sid, symbols);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}
