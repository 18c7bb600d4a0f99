// Nearest-center digitization against a resident dictionary (Sec. 3.2:
// c* = argmin_c ||p - c||_2, f_d(p) = I_d(c*)).
//
// The scaled centers (cx, cy) are staged through LDS in tiles of kTileC
// entries; each thread scans every center for its piece, keeping the first
// strict minimum, so ties go to the lowest symbol exactly as a sequential
// scan does.  k distance evaluations per piece: plain FP64 VALU work (the
// comparison needs the exact rounded distances, so it is not recast as a
// matrix product).
#include "common.h"

namespace jabba {
namespace {

constexpr int kThreads = 256;
constexpr int kTileC = 4096;  // 64 KB of (cx, cy) per tile

__global__ __launch_bounds__(kThreads) void k_encode(const int32_t *__restrict__ len, const double *__restrict__ inc,
                                                     const int64_t *__restrict__ n_dev, int64_t n_max,
                                                     const double *__restrict__ params, const int64_t *__restrict__ kp,
                                                     int64_t capacity, const double *__restrict__ cx,
                                                     const double *__restrict__ cy, int32_t *__restrict__ symbols) {
    __shared__ double2 c_lds[kTileC];
    int64_t n = *n_dev;
    n = n < 0 ? 0 : (n > n_max ? n_max : n);
    int64_t k = *kp;
    k = k < 0 ? 0 : (k > capacity ? capacity : k);
    const double sl = params[0], si = params[1], scl = params[2];
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < n; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool ok = i < n;
        Scaled s{0.0, 0.0};
        if (ok) s = scale_piece(len[i], inc[i], scl, sl, si);
        int32_t best = -1;
        double bd = 0.0;
        for (int64_t c0 = 0; c0 < k; c0 += kTileC) {
            const int64_t m = (k - c0) < kTileC ? (k - c0) : kTileC;
            __syncthreads();
            for (int64_t t = threadIdx.x; t < m; t += kThreads) c_lds[t] = make_double2(cx[c0 + t], cy[c0 + t]);
            __syncthreads();
            if (ok) {
                for (int t = 0; t < (int)m; ++t) {
                    const double2 cc = c_lds[t];
                    const double dx = s.x - cc.x;
                    const double dy = s.y - cc.y;
                    const double dd = dx * dx;
                    const double ee = dy * dy;
                    const double d2 = dd + ee;
                    if (best < 0 || d2 < bd) {
                        best = (int32_t)(c0 + t);
                        bd = d2;
                    }
                }
            }
        }
        if (ok) symbols[i] = best;
    }
}

}  // namespace
}  // namespace jabba

using namespace jabba;

extern "C" int jabba_encode(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                            const jabba_dict *dict, int32_t *symbols, void *stream) {
    if (!dict || !n_pieces || max_pieces < 0) return JABBA_EINVAL;
    if (max_pieces == 0) return JABBA_OK;
    if (!len || !inc || !symbols || !dict->params || !dict->k || dict->capacity < 1 || !dict->cx || !dict->cy)
        return JABBA_EINVAL;
    int64_t blocks = (max_pieces + kThreads - 1) / kThreads;
    const int64_t cap = (int64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    JB_LAUNCH(k_encode, dim3((unsigned)blocks), dim3(kThreads), 0, (hipStream_t)stream, len, inc, n_pieces,
                       max_pieces, dict->params, dict->k, dict->capacity, dict->cx, dict->cy, symbols);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}
