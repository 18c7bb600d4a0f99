// Inverse symbolization (Sec. 3.3): inverse digitization (symbol -> center),
// quantization of the lengths (Eq. repolygon) and inverse compression.
//
// Pieces are taken 64 at a time (one chunk per wavefront step).
//  * Quantization: the carry rule keeps sum(len^_1..j) = round(sum(len~_1..j)),
//    halves away from zero.  Every center length >= 1 is an integer multiple
//    of 2^-52, so the running sums are exact unsigned 128-bit integers at
//    scale 2^52: a wavefront inclusive scan plus a carry from the previous
//    chunk, then S_j = (C_j + 2^51) >> 52 and len^_j = S_j - S_{j-1}.  When
//    every center length of a chunk is below 2^25 the scan runs on three
//    32-bit limbs (integer part, two 26-bit halves of the fraction), whose
//    64-lane sums cannot overflow.
//  * Values: V_j = V_{j-1} + inc~_j is a sequential binary64 recurrence; the
//    wavefront walks it one lane per step (a DPP shift and one addition), so
//    every V_j has the bits of the plain left-to-right evaluation.
//  * Fill: V_{j-1} + (inc~_j / len^_j) * q for 0 < q < len^_j, then V_j.
#include "common.h"

namespace jabba {
namespace {

typedef unsigned __int128 u128;

__device__ __forceinline__ u128 shfl_up_u128(u128 v, int d) {
    unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    lo = __shfl_up(lo, d);
    hi = __shfl_up(hi, d);
    return ((u128)hi << 64) | lo;
}
// DPP step on the four 32-bit limbs of a u128
template <int Ctrl, int RowMask>
__device__ __forceinline__ u128 dpp_u128(u128 v) {
    const uint32_t a = dpp_u32<Ctrl, RowMask>((uint32_t)v);
    const uint32_t b = dpp_u32<Ctrl, RowMask>((uint32_t)(v >> 32));
    const uint32_t c = dpp_u32<Ctrl, RowMask>((uint32_t)(v >> 64));
    const uint32_t d = dpp_u32<Ctrl, RowMask>((uint32_t)(v >> 96));
    return ((u128)d << 96) | ((u128)c << 64) | ((u128)b << 32) | (u128)a;
}

// inclusive scan of a u128 across the 64 lanes (exact integer sums): row
// shifts by 1, 2, 4, 8 scan each row of 16 lanes, then lane 15 of rows 0 and
// 2 is added to rows 1 and 3, and lane 31 to rows 2 and 3
__device__ __forceinline__ u128 wave_incl_scan_u128(u128 x) {
    x += dpp_u128<0x111, 0xf>(x);
    x += dpp_u128<0x112, 0xf>(x);
    x += dpp_u128<0x114, 0xf>(x);
    x += dpp_u128<0x118, 0xf>(x);
    x += dpp_u128<0x142, 0xa>(x);
    x += dpp_u128<0x143, 0xc>(x);
    return x;
}

// inclusive scan of a u32 across the 64 lanes, the same steps as above
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    x += dpp_u32<0x111, 0xf>(x);
    x += dpp_u32<0x112, 0xf>(x);
    x += dpp_u32<0x114, 0xf>(x);
    x += dpp_u32<0x118, 0xf>(x);
    x += dpp_u32<0x142, 0xa>(x);
    x += dpp_u32<0x143, 0xc>(x);
    return x;
}

// lane l receives lane l-1's v and lane 0 receives `first` (DPP wave shift
// right by one lane; the source of lane 0 is out of range, so it keeps the
// old value)
__device__ __forceinline__ double wave_shr1_f64(double v, double first) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(first), __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(first), __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t wave_shr1_i64(int64_t v, int64_t first) {
    const int lo = __builtin_amdgcn_update_dpp((int)first, (int)v, 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(first >> 32), (int)(v >> 32), 0x138, 0xf, 0xf, false);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// value of lane l, l uniform across the wavefront (scalar reads, no LDS)
__device__ __forceinline__ u128 readlane_u128(u128 v, int l) {
    const uint64_t lo = (uint64_t)readlane_i64((int64_t)(uint64_t)v, l);
    const uint64_t hi = (uint64_t)readlane_i64((int64_t)(uint64_t)(v >> 64), l);
    return ((u128)hi << 64) | lo;
}

__device__ __forceinline__ u128 shfl_u128(u128 v, int l) {
    unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    lo = __shfl(lo, l);
    hi = __shfl(hi, l);
    return ((u128)hi << 64) | lo;
}
__device__ __forceinline__ u128 xor_u128(u128 v, int m) {
    unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    lo = __shfl_xor(lo, m);
    hi = __shfl_xor(hi, m);
    return ((u128)hi << 64) | lo;
}

// d * 2^52 as an exact integer; ok = false when d is negative, not finite or
// not a multiple of 2^-52 (never the case for means of integer lengths >= 1)
__device__ __forceinline__ u128 to_fixed(double d, bool &ok) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(d);
    const int e = (int)((b >> 52) & 0x7FF);
    if ((b >> 63) || e == 0x7FF) {
        ok = false;
        return 0;
    }
    if (e == 0) return 0;  // zero or subnormal: below 2^-52 unless zero
    const unsigned long long m = (b & ((1ull << 52) - 1)) | (1ull << 52);
    const int sh = e - 1023;  // d * 2^52 = m * 2^(e - 1023)
    if (sh >= 0) {
        if (sh > 60) {
            ok = false;
            return 0;
        }
        return (u128)m << sh;
    }
    if (sh < -52 || (m & ((1ull << -sh) - 1))) {
        ok = false;
        return 0;
    }
    return (u128)(m >> -sh);
}

__device__ __forceinline__ int64_t fixed_round(u128 c) { return (int64_t)((c + ((u128)1 << 51)) >> 52); }

struct Src {
    // dictionary form: symbols + centers; raw form: len/inc (centers == null)
    const int32_t *sym;
    const double *center_len;
    const double *center_inc;
    int64_t k;
    const int32_t *len;
    const double *inc;
    // first load of piece j: its symbol (dictionary form) or nothing
    __device__ int32_t tag(int64_t j) const { return center_len ? sym[j] : 0; }
    // second load: the piece's raw length and increment
    struct Raw {
        double l;
        double it;
        int32_t li;
        bool bad;
    };
    __device__ Raw load(int64_t j, int32_t c) const {
        Raw r{0.0, 0.0, 0, false};
        if (center_len) {
            if (c < 0 || c >= k) {
                r.bad = true;
            } else {
                r.l = center_len[c];
                r.it = center_inc[c];
            }
        } else {
            r.li = len[j];
            r.it = inc[j];
        }
        return r;
    }
    // the length as a fixed-point integer (an invalid symbol reads as length 1, increment 0)
    __device__ void convert(const Raw &r, u128 &lt, double &it, bool &ok) const {
        if (center_len) {
            if (r.bad) {
                ok = false;
                lt = (u128)1 << 52;
                it = 0.0;
                return;
            }
            lt = to_fixed(r.l, ok);
            it = r.it;
        } else {
            lt = (u128)(uint32_t)r.li << 52;
            it = r.it;
        }
    }
    __device__ void get(int64_t j, u128 &lt, double &it, bool &ok) const { convert(load(j, tag(j)), lt, it, ok); }
    // Branch-free forms of tag() and load() for a prefetch pipeline: every
    // load is issued (indices are clamped by the caller, an invalid symbol
    // reads center 0 and is flagged), so the loaded registers are the
    // loop-carried ones and nothing waits for them before their use.
    // Dictionary form needs k >= 1.
    template <bool Dict>
    __device__ int32_t tag_at(int64_t j) const {
        return Dict ? sym[j] : 0;
    }
    template <bool Dict>
    __device__ Raw fetch(int64_t j, int32_t c) const {
        Raw r{0.0, 0.0, 0, false};
        if (Dict) {
            r.bad = c < 0 || c >= k;
            const int64_t cc = r.bad ? 0 : c;
            r.l = center_len[cc];
            r.it = center_inc[cc];
        } else {
            r.li = len[j];
            r.it = inc[j];
        }
        return r;
    }
};

__global__ __launch_bounds__(256) void k_recon_count(Src src, const int64_t *__restrict__ piece_off,
                                                     const int64_t *__restrict__ series_off, int64_t n_series,
                                                     const int32_t *__restrict__ order, int64_t *__restrict__ cnt,
                                                     int32_t *status) {
    const int lane = lane_id();
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < n_series; i += waves) {
        const int64_t s = order[i];
        const int64_t a = piece_off[s], b = piece_off[s + 1];
        if (b <= a) {
            if (lane == 0) cnt[s] = (series_off[s + 1] - series_off[s]) >= 1 ? 1 : 0;
            continue;
        }
        // exact integer sum, so any order: four chunks' loads are issued
        // before any is used (symbols, then their centers)
        constexpr int kAhead = 4;
        u128 acc = 0;
        bool ok = true;
        for (int64_t j0 = a + lane; j0 < b; j0 += kAhead * kWave) {
            int32_t c[kAhead];
            Src::Raw r[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                const int64_t j = j0 + (int64_t)u * kWave;
                c[u] = j < b ? src.tag(j) : 0;
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                const int64_t j = j0 + (int64_t)u * kWave;
                r[u] = j < b ? src.load(j, c[u]) : Src::Raw{0.0, 0.0, 0, false};
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                if (j0 + (int64_t)u * kWave < b) {
                    u128 lt;
                    double it;
                    src.convert(r[u], lt, it, ok);
                    acc += lt;
                }
            }
        }
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) acc += xor_u128(acc, m);
        if (ballot(!ok) && lane == 0) set_status(status, kStInvalid);
        if (lane == 0) cnt[s] = 1 + fixed_round(acc);
    }
}

// One workgroup per series, the series taken in the order given (longest
// first).  Wavefront 0 produces chunks of 64 pieces (the fixed-point scan of
// the lengths and the sequential values) into LDS while the next chunks'
// loads are in flight; wavefront 1 fills the points of the
// previous chunk, one point per thread (coalesced stores), with the original
// values for the squared error loaded four points at a time.  The two LDS
// buffers alternate, one barrier per chunk.
struct ReconChunk {
    int64_t beg[kWave];  // S_{j-1}: offset of the piece's first point (its predecessor's end)
    int64_t end[kWave];  // S_j
    double vme[kWave];   // V_j
    double slope[kWave];
    double vin;          // V before the chunk's first piece
};

constexpr int kReconThreads = 128;
constexpr int kFillThreads = kReconThreads - kWave;

// With `values`, the filler also accumulates the squared error against the
// original series over the common prefix m = min(n, n^): each filler thread
// sums its own points in order, and the 64 partials are added by one fixed
// tree per series (deterministic).
template <bool Dict>
__global__ __launch_bounds__(kReconThreads, 4) void k_recon(Src src, const int64_t *__restrict__ piece_off,
                                                         const int64_t *__restrict__ out_off, int64_t n_series,
                                                         const double *__restrict__ t0, double *__restrict__ out,
                                                         int64_t *__restrict__ lhat,
                                                         const int64_t *__restrict__ series_off,
                                                         const double *__restrict__ values,
                                                         double *__restrict__ sse, int64_t *__restrict__ sse_cnt,
                                                         const int32_t *__restrict__ order) {
    __shared__ ReconChunk buf[2];
    const int lane = lane_id();
    // uniform per wavefront, and known to be: the roles branch on a scalar
    const bool producer = __builtin_amdgcn_readfirstlane(threadIdx.x) < kWave;
    for (int64_t i = blockIdx.x; i < n_series; i += gridDim.x) {
        const int64_t s = order[i];
        const int64_t a = piece_off[s], b = piece_off[s + 1];
        const int64_t o = out_off[s];
        const int64_t nch = b > a ? (b - a + kWave - 1) / kWave : 0;
        // squared-error state (filler threads)
        int64_t m_err = 0, vo = 0;
        double err = 0.0;
        if (values && !producer) {
            vo = series_off[s];
            const int64_t n = series_off[s + 1] - vo, nh = out_off[s + 1] - o;
            m_err = n < nh ? n : nh;
            if (threadIdx.x == kWave && m_err > 0) {
                const double d = values[vo] - t0[s];
                err = d * d;
            }
        }
        int64_t carryH = 0, carryS = 0;
        uint64_t carryL = 0;
        double V = 0.0;
        // loads of the next chunk (raw_n) and of the symbols two chunks
        // ahead (tag_n); indices past the series' last piece are clamped to
        // it and their results never used
        auto clampj = [&](int64_t j) -> int64_t { return j < b ? j : b - 1; };
        // symbols are loaded kTagAhead chunks ahead (from HBM), the centers
        // they select one chunk ahead (from the cache-resident dictionary)
        constexpr int kTagAhead = 3;
        Src::Raw raw_n{0.0, 0.0, 0, false};
        int32_t tg0 = 0, tg1 = 0, tg2 = 0, tg3 = 0;
        if (producer) {
            V = t0[s];
            if (lane == 0 && out_off[s + 1] > o) out[o] = V;
            if (nch > 0) {
                const int64_t j = a + lane;
                raw_n = src.fetch<Dict>(clampj(j), src.tag_at<Dict>(clampj(j)));
                tg1 = src.tag_at<Dict>(clampj(j + kWave));
                tg2 = src.tag_at<Dict>(clampj(j + 2 * kWave));
                tg3 = src.tag_at<Dict>(clampj(j + 3 * kWave));
            }
        }
        // chunk t: cur holds its loads, tnext the symbols of chunk t + 1; the
        // step loads chunk t + 1 into nxt and the symbols of chunk
        // t + 1 + kTagAhead into tload (the register that held chunk t's).
        // The loop below rotates the register sets, so a load lands in a
        // register nothing reads until it is due.
        auto step = [&](int64_t t, const Src::Raw &cur, Src::Raw &nxt, const int32_t &tnext, int32_t &tload) {
            if (producer && t < nch) {
                const int64_t j0 = a + t * kWave;
                const int64_t j = j0 + lane;
                u128 lt = 0;
                double it = 0.0;
                nxt = src.fetch<Dict>(clampj(j + kWave), tnext);
                tload = src.tag_at<Dict>(clampj(j + (1 + kTagAhead) * kWave));
                if (j < b) {
                    bool ok = true;
                    src.convert(cur, lt, it, ok);
                }
                const int cnt = (int)((b - j0) < kWave ? (b - j0) : kWave);
                ReconChunk &B = buf[t & 1];
                // inclusive scan of the fixed-point center lengths on top of
                // the carry carryH * 2^52 + carryL (carryL < 2^52)
                constexpr uint64_t kFrac = (1ull << 52) - 1;
                int64_t S;
                if (!ballot((lt >> 77) != 0)) {
                    // limbs of lt = h * 2^52 + m * 2^26 + q, h < 2^25 and
                    // m, q < 2^26: the scans stay below 2^32
                    const uint32_t hs = wave_incl_scan_u32((uint32_t)(lt >> 52));
                    const uint32_t ms = wave_incl_scan_u32((uint32_t)(lt >> 26) & ((1u << 26) - 1));
                    const uint32_t qs = wave_incl_scan_u32((uint32_t)lt & ((1u << 26) - 1));
                    const uint64_t low = ((uint64_t)ms << 26) + qs + carryL;  // below 2^59
                    S = carryH + (int64_t)hs + (int64_t)((low + (1ull << 51)) >> 52);
                    const uint64_t lowc = (uint64_t)readlane_i64((int64_t)low, cnt - 1);
                    carryH += (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)hs, cnt - 1) + (int64_t)(lowc >> 52);
                    carryL = lowc & kFrac;
                } else {
                    const u128 C = wave_incl_scan_u128(lt) + (((u128)(uint64_t)carryH << 52) | carryL);
                    S = fixed_round(C);
                    const u128 Cc = readlane_u128(C, cnt - 1);
                    carryH = (int64_t)(Cc >> 52);
                    carryL = (uint64_t)Cc & kFrac;
                }
                const int64_t Sp = wave_shr1_i64(S, carryS);
                const int64_t lh = S - Sp;
                B.beg[lane] = Sp;
                B.end[lane] = S;
                carryS = readlane_i64(S, cnt - 1);
                // sequential running value, V_j on lane j: every step moves
                // each lane's value one lane up (lane 0 takes V before the
                // chunk) and adds the lane's own increment.  After cnt steps
                // lanes 0..cnt-1 hold V_0..V_{cnt-1}, each the one binary64
                // addition V_{j-1} + inc~_j of the left-to-right evaluation.
                if (lane == 0) B.vin = V;
                // (prev keeps V on lane 0 from one step to the next, so the
                // shift writes it in place)
                double Vl = V, prev = V;
                int l = 0;
                for (; l + 4 <= cnt; l += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        prev = wave_shr1_f64(Vl, prev);
                        Vl = prev + it;
                    }
                }
                for (; l < cnt; ++l) {
                    prev = wave_shr1_f64(Vl, prev);
                    Vl = prev + it;
                }
                B.vme[lane] = Vl;
                V = readlane_f64(Vl, cnt - 1);
                B.slope[lane] = it / (double)lh;
            }
            if (!producer && t > 0) {
                const int64_t tc = t - 1;
                const int64_t j0 = a + tc * kWave;
                const int cnt = (int)((b - j0) < kWave ? (b - j0) : kWave);
                const ReconChunk &B = buf[tc & 1];
                const int64_t lo = B.beg[0], hi = B.end[cnt - 1];
                const int f = threadIdx.x - kWave;
                constexpr int kAhead = 4;  // points per thread whose originals are loaded together
                for (int64_t r0 = lo + 1 + f; r0 <= hi; r0 += kAhead * kFillThreads) {
                    double orig[kAhead];
#pragma unroll
                    for (int u = 0; u < kAhead; ++u) {
                        const int64_t r = r0 + (int64_t)u * kFillThreads;
                        orig[u] = (r <= hi && r < m_err) ? values[vo + r] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < kAhead; ++u) {
                        const int64_t r = r0 + (int64_t)u * kFillThreads;
                        if (r > hi) break;
                        // first piece whose end is at or after point r: the
                        // ends do not decrease and lanes past the chunk's
                        // last piece hold its end (hi >= r), so a fixed
                        // six-step search over all 64 entries finds it
                        int L = 0;
#pragma unroll
                        for (int step = kWave / 2; step > 0; step >>= 1)
                            L += B.end[L + step - 1] < r ? step : 0;
                        const double vprev = L > 0 ? B.vme[L - 1] : B.vin;
                        // the offset inside a piece is below 2^31 (a series' point count)
                        const double vr = (r == B.end[L]) ? B.vme[L]
                                                          : vprev + B.slope[L] * (double)(int32_t)(r - B.beg[L]);
                        out[o + r] = vr;
                        if (r < m_err) {  // each thread adds its points in increasing r
                            const double d = orig[u] - vr;
                            err = err + d * d;
                        }
                    }
                }
                if (lhat)
                    for (int l = f; l < cnt; l += kFillThreads) lhat[j0 + l] = B.end[l] - B.beg[l];
            }
            __syncthreads();
        };
        Src::Raw raw_b{0.0, 0.0, 0, false};
        static_assert(kTagAhead == 3, "the rotation below holds four symbol registers");
        for (int64_t t = 0; t <= nch; t += 4) {
            step(t, raw_n, raw_b, tg1, tg0);
            if (t + 1 <= nch) step(t + 1, raw_b, raw_n, tg2, tg1);
            if (t + 2 <= nch) step(t + 2, raw_n, raw_b, tg3, tg2);
            if (t + 3 <= nch) step(t + 3, raw_b, raw_n, tg0, tg3);
        }
        if (values && !producer) {
            const double tot = wave_tree_sum(err);
            if (threadIdx.x == kWave) {
                sse[s] = tot;
                sse_cnt[s] = m_err;
            }
        }
    }
}

__global__ void k_recon_prep(int32_t *status) {
    if (threadIdx.x == 0) status[0] = 0;
}

// Series order for the per-series kernels: the longest first.  One workgroup
// (or wavefront) per series is started as earlier ones end, so a long series
// started late sets the kernel's end; taking the series by descending
// power-of-two class of their 64-piece chunk count bounds that tail by the
// shortest class.  A counting sort: class counts, then each series a slot in
// its class's range (the order inside a class depends on timing; nothing
// computed depends on it, since every series writes only its own outputs).
constexpr int kOrderClasses = 34;  // 1 + floor(log2(chunks)) below 2^32, and one for series without pieces
constexpr int kOrderThreads = 256;

// class 32 - floor(log2(chunks)) (0 beyond 2^32 chunks), the last for none
__device__ __forceinline__ int order_class(const int64_t *__restrict__ piece_off, int64_t s) {
    const int64_t nch = (piece_off[s + 1] - piece_off[s] + kWave - 1) / kWave;
    if (nch <= 0) return kOrderClasses - 1;
    const int lg = 63 - __clzll((unsigned long long)nch);
    return lg < 32 ? 32 - lg : 0;
}

__global__ void k_order_prep(uint32_t *hist, uint32_t *cursor) {
    if (threadIdx.x < kOrderClasses) {
        hist[threadIdx.x] = 0u;
        cursor[threadIdx.x] = 0u;
    }
}

__global__ __launch_bounds__(kOrderThreads) void k_order_count(const int64_t *__restrict__ piece_off,
                                                               int64_t n_series, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[kOrderClasses];
    if (threadIdx.x < kOrderClasses) h[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t s = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x; s < n_series;
         s += (int64_t)gridDim.x * kOrderThreads)
        atomicAdd(&h[order_class(piece_off, s)], 1u);
    __syncthreads();
    if (threadIdx.x < kOrderClasses && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// one series per thread: its rank among the workgroup's series of its class
// (LDS), the workgroup's range in the class (one global atomic per class)
__global__ __launch_bounds__(kOrderThreads) void k_order_scatter(const int64_t *__restrict__ piece_off,
                                                                 int64_t n_series, const uint32_t *__restrict__ hist,
                                                                 uint32_t *__restrict__ cursor,
                                                                 int32_t *__restrict__ order) {
    __shared__ uint32_t base[kOrderClasses];
    __shared__ uint32_t h[kOrderClasses];
    __shared__ uint32_t at[kOrderClasses];
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int c = 0; c < kOrderClasses; ++c) {
            base[c] = run;
            run += hist[c];
        }
    }
    for (int64_t s0 = (int64_t)blockIdx.x * kOrderThreads; s0 < n_series; s0 += (int64_t)gridDim.x * kOrderThreads) {
        if (threadIdx.x < kOrderClasses) h[threadIdx.x] = 0u;
        __syncthreads();
        const int64_t s = s0 + threadIdx.x;
        int c = 0;
        uint32_t r = 0;
        if (s < n_series) {
            c = order_class(piece_off, s);
            r = atomicAdd(&h[c], 1u);
        }
        __syncthreads();
        if (threadIdx.x < kOrderClasses && h[threadIdx.x])
            at[threadIdx.x] = base[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]);
        __syncthreads();
        if (s < n_series) order[at[c] + r] = (int32_t)s;
        __syncthreads();
    }
}

// The grids below hold one wavefront (k_recon_count) or one workgroup
// (k_recon) per series and no more than that: series lengths can differ by
// orders of magnitude, and the dispatcher starting each workgroup as an
// earlier one ends balances the load, where a fixed share of series per
// workgroup would leave the kernel waiting on the few workgroups that drew the
// longest series.  (The kernels still stride, so any grid is correct.)
constexpr int64_t kMaxGrid = ((int64_t)1 << 31) - 1;

unsigned waves_grid(int64_t n_series) {
    int64_t blocks = (n_series * kWave + 255) / 256;
    if (blocks > kMaxGrid) blocks = kMaxGrid;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

unsigned series_grid(int64_t n_series) {
    int64_t blocks = n_series;
    if (blocks > kMaxGrid) blocks = kMaxGrid;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

struct ReconWs {
    int32_t *status;
    int64_t *cnt;
    void *scan_ws;
    uint32_t *hist, *cursor;
    int32_t *order;
    size_t bytes;
};

ReconWs carve_recon(void *ws, int64_t n_series) {
    Carve c(ws);
    ReconWs w;
    w.status = c.take<int32_t>(64);
    w.cnt = c.take<int64_t>(n_series + 1);
    w.scan_ws = c.take<char>(scan_workspace(n_series + 1));
    w.hist = c.take<uint32_t>(64);
    w.cursor = c.take<uint32_t>(64);
    w.order = c.take<int32_t>(n_series);
    w.bytes = c.bytes();
    return w;
}

// w.order <- the series, longest class first
int series_order(const ReconWs &w, const int64_t *piece_off, int64_t n_series, hipStream_t st) {
    if (n_series <= 0) return JABBA_OK;
    int64_t blocks = (n_series + kOrderThreads - 1) / kOrderThreads;
    const int64_t cap = (int64_t)device_cu_count() * 4;
    if (blocks > cap) blocks = cap;
    JB_LAUNCH(k_order_prep, dim3(1), dim3(64), 0, st, w.hist, w.cursor);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_order_count, dim3((unsigned)blocks), dim3(kOrderThreads), 0, st, piece_off, n_series, w.hist);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_order_scatter, dim3((unsigned)blocks), dim3(kOrderThreads), 0, st, piece_off, n_series, w.hist,
              w.cursor, w.order);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

int sizes(const Src &src, const int64_t *piece_off, const int64_t *series_off, int64_t n_series, int64_t *out_off,
          void *workspace, size_t workspace_bytes, hipStream_t st) {
    if (n_series < 0 || !piece_off || !series_off || !out_off) return JABBA_EINVAL;
    const ReconWs w0 = carve_recon(nullptr, n_series);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    const ReconWs w = carve_recon(workspace, n_series);
    JB_LAUNCH(k_recon_prep, dim3(1), dim3(64), 0, st, w.status);
    JB_LAUNCH_CHECK();
    if (n_series > 0) {
        const int rc = series_order(w, piece_off, n_series, st);
        if (rc) return rc;
        JB_LAUNCH(k_recon_count, dim3(waves_grid(n_series)), dim3(256), 0, st, src, piece_off, series_off,
                           n_series, w.order, w.cnt, w.status);
        JB_LAUNCH_CHECK();
    }
    return scan_i64_to_i64(w.cnt, out_off, nullptr, n_series, w.scan_ws, st);
}

// Mean squared error over all series (Sec. 3.3): the per-series squared
// errors summed by a balanced pairwise tree over the series (leaves in series
// order, zero-padded to a power of two, adjacent leaves paired first), the
// point counts summed exactly, then one division.  One workgroup: each
// thread sums a power-of-two run of leaves (a binary counter of partial sums
// merges equal-size neighbours, which is the same tree), then the threads'
// sums are paired level by level.
constexpr int kMseThreads = 1024;
__global__ __launch_bounds__(kMseThreads) void k_mse(const double *__restrict__ sse, const int64_t *__restrict__ cnt,
                                                     int64_t n_series, double *__restrict__ mse) {
    __shared__ double s_v[kMseThreads];
    __shared__ unsigned long long s_c[kMseThreads];
    int64_t per = 1;
    while (per * kMseThreads < n_series) per <<= 1;
    const int64_t lo = (int64_t)threadIdx.x * per;
    double part[64];
    int depth = 0;
    unsigned long long c = 0;
    for (int64_t i = 0; i < per; ++i) {
        const int64_t j = lo + i;
        double x = j < n_series ? sse[j] : 0.0;
        if (j < n_series) c += (unsigned long long)cnt[j];
        for (int64_t k = i + 1; (k & 1) == 0; k >>= 1) x = part[--depth] + x;
        part[depth++] = x;
    }
    s_v[threadIdx.x] = part[0];
    s_c[threadIdx.x] = c;
    __syncthreads();
    for (int h = 1; h < kMseThreads; h <<= 1) {
        if ((threadIdx.x & (2 * h - 1)) == 0) {
            s_v[threadIdx.x] = s_v[threadIdx.x] + s_v[threadIdx.x + h];
            s_c[threadIdx.x] += s_c[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) mse[0] = s_c[0] ? s_v[0] / (double)s_c[0] : 0.0;
}

}  // namespace
}  // namespace jabba

using namespace jabba;

extern "C" int jabba_reconstruct_mse(const double *sse, const int64_t *cnt, int64_t n_series, double *mse,
                                     void *stream) {
    if (n_series < 0 || !mse || (n_series > 0 && (!sse || !cnt))) return JABBA_EINVAL;
    JB_DEVICE_CHECK();
    JB_LAUNCH(k_mse, dim3(1), dim3(kMseThreads), 0, (hipStream_t)stream, sse, cnt, n_series, mse);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

extern "C" int jabba_reconstruct_workspace(int64_t n_series, size_t *bytes) {
    if (!bytes || n_series < 0) return JABBA_EINVAL;
    *bytes = carve_recon(nullptr, n_series).bytes;
    return JABBA_OK;
}

extern "C" int jabba_reconstruct_size(const int32_t *symbols, const int64_t *piece_off, const int64_t *series_off,
                                      int64_t n_series, const jabba_dict *dict, int64_t *out_off, void *workspace,
                                      size_t workspace_bytes, void *stream) {
    if (!dict || !dict->center_len || !dict->center_inc) return JABBA_EINVAL;
    Src src{symbols, dict->center_len, dict->center_inc, dict->capacity, nullptr, nullptr};
    return sizes(src, piece_off, series_off, n_series, out_off, workspace, workspace_bytes, (hipStream_t)stream);
}

extern "C" int jabba_reconstruct(const int32_t *symbols, const int64_t *piece_off, const int64_t *series_off,
                                 int64_t n_series, const double *t0, const jabba_dict *dict, const int64_t *out_off,
                                 double *out, int64_t *lhat, const double *values, double *sse, int64_t *cnt,
                                 void *workspace, size_t workspace_bytes, void *stream) {
    if (!dict || !dict->center_len || !dict->center_inc || n_series < 0 || !piece_off || !out_off) return JABBA_EINVAL;
    if (dict->capacity < 1) return JABBA_EINVAL;
    if (n_series == 0) return JABBA_OK;
    if (!t0 || !out || !series_off) return JABBA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Src src{symbols, dict->center_len, dict->center_inc, dict->capacity, nullptr, nullptr};
    if (values && (!sse || !cnt)) return JABBA_EINVAL;
    if (!workspace || workspace_bytes < carve_recon(nullptr, n_series).bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    const ReconWs w = carve_recon(workspace, n_series);
    const int rc = series_order(w, piece_off, n_series, st);
    if (rc) return rc;
    JB_LAUNCH_NAMED("k_recon", k_recon<true>, dim3(series_grid(n_series)), dim3(kReconThreads), 0, st, src, piece_off,
                    out_off, n_series, t0, out, lhat, series_off, values, sse, cnt, w.order);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

extern "C" int jabba_reconstruct_pieces(const int32_t *len, const double *inc, const int64_t *piece_off,
                                        const int64_t *series_off, int64_t n_series, const double *t0,
                                        int64_t *out_off, double *out, void *workspace, size_t workspace_bytes,
                                        void *stream) {
    hipStream_t st = (hipStream_t)stream;
    Src src{nullptr, nullptr, nullptr, 0, len, inc};
    int rc = sizes(src, piece_off, series_off, n_series, out_off, workspace, workspace_bytes, st);
    if (rc || n_series == 0) return rc;
    if (!t0 || !out) return JABBA_EINVAL;
    // the size pass above left the series order in the workspace
    JB_LAUNCH_NAMED("k_recon_pieces", k_recon<false>, dim3(series_grid(n_series)), dim3(kReconThreads), 0, st, src,
                    piece_off, out_off, n_series, t0, out, (int64_t *)nullptr, series_off, (const double *)nullptr,
                    (double *)nullptr, (int64_t *)nullptr, carve_recon(workspace, n_series).order);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}
