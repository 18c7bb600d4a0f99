// Phase I (domain construction) and Phase II (parallel compression) of
// Alg. 1, with the greedy ABBA compression of Sec. 3.1 (Eq. compress).
//
// Layout in HBM
//   values  f64[total_points]                 (input, series concatenated)
//   doms    {start i64, nint i32, series i32}  one per domain, canonical order
//   queue   i32[n_dom]                         domain ids, longest first
//   staging len i32 / inc f64 indexed by the domain's first point: domain d
//           writes its pieces at [start_d, start_d + count_d); since
//           count_d <= nint_d = start_{d+1} - start_d the regions never overlap
//   output  len i32[N], inc f64[N]             canonical (series, domain, position)
//
// compress_kernel: W lanes test W consecutive candidate end points of one
// domain together (W = 64: one wavefront per domain, the form that tests 64
// candidates per round; W = 1: every lane grows its own domain).  Each lane
// accumulates its candidate's squared error in ascending k exactly as the
// sequential definition does, so the decision bits are identical for every W.
// A round is decided as soon as the smallest failing candidate has finished
// its sum and every smaller candidate has finished too (early exit); a ballot
// over the group finds that candidate.  Groups pull the next domain from an
// atomic work queue ordered by domain length (longest first), so the launch
// is persistent and balances uneven series.
#include "common.h"
#include "compress_filter.h"
#include "compress_repair.h"

namespace jabba {

constexpr int32_t kMinSegment = 32;       // smallest segment (workspace sizing)
constexpr int32_t kDefaultSegment = 128;  // intervals per segment by default

namespace {

__global__ void k_series_domains(const int64_t *__restrict__ series_off, int64_t n_series, int32_t D, int32_t G,
                                 int32_t *__restrict__ ndom, int32_t *status) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_series) return;
    int64_t n = series_off[s + 1] - series_off[s];
    if (n < 0) {
        set_status(status, kStOverflow);
        n = 0;
    }
    if (n < 2) {
        ndom[s] = 0;
        return;
    }
    const int64_t nd = (n - 1 + D - 1) / D;
    const int32_t last = (int32_t)((n - 1) - (nd - 1) * D);
    ndom[s] = (int32_t)((nd - 1) * n_segments(D, G) + n_segments(last, G));
}

// One wavefront per series; its lanes write the series' work units (every
// domain of D intervals, the last one shorter, each cut into segments of G).
__global__ void k_fill_domains(const int64_t *__restrict__ series_off, const int64_t *__restrict__ dom_off,
                               int64_t n_series, int32_t D, int32_t G, Dom *__restrict__ doms,
                               unsigned long long *__restrict__ len_hist) {
    __shared__ unsigned long long cnt_lds[2];
    const int lane = lane_id();
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    // full-length domains and full-length segments all fall in two bins: their
    // counts are gathered over the whole loop and added once per workgroup
    unsigned long long full = 0, fullseg = 0;
    if (threadIdx.x < 2) cnt_lds[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; s < n_series; s += waves) {
        const int64_t lo = series_off[s], n = series_off[s + 1] - series_off[s];
        if (n < 2) continue;
        const int64_t d0 = dom_off[s];
        const int64_t nd = (n - 1 + D - 1) / D;
        const int32_t last = (int32_t)((n - 1) - (nd - 1) * D);
        const int32_t spd = n_segments(D, G);  // segments of a full domain
        const int64_t n_full = (nd - 1) * spd;
        const int32_t nsl = n_segments(last, G);
        for (int64_t u = lane; u < n_full + nsl; u += kWave) {
            int64_t dom;
            int32_t k, ns, nint_d;
            if (u < n_full) {
                dom = u / spd;
                k = (int32_t)(u - dom * spd);
                ns = spd;
                nint_d = D;
            } else {
                dom = nd - 1;
                k = (int32_t)(u - n_full);
                ns = nsl;
                nint_d = last;
            }
            const int64_t a = dom * D + (int64_t)k * (ns > 1 ? G : 0);
            const int64_t b = k == ns - 1 ? dom * D + nint_d : a + G;
            Dom x;
            x.start = lo + a;
            x.nint = (int32_t)(b - a);
            x.series = (int32_t)s;
            x.seg = k;
            x.nseg = ns;
            doms[d0 + u] = x;
            if (len_hist) {
                if (x.nint == D)
                    ++full;
                else if (x.nint == G)
                    ++fullseg;
                else
                    atomicAdd(&len_hist[D - x.nint], 1ull);
            }
        }
    }
    if (len_hist) {
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            full += __shfl_xor(full, m);
            fullseg += __shfl_xor(fullseg, m);
        }
        if (lane == 0 && full) atomicAdd(&cnt_lds[0], full);
        if (lane == 0 && fullseg) atomicAdd(&cnt_lds[1], fullseg);
    }
    __syncthreads();
    if (len_hist && threadIdx.x == 0) {
        if (cnt_lds[0]) atomicAdd(&len_hist[0], cnt_lds[0]);
        if (cnt_lds[1]) atomicAdd(&len_hist[D - G], cnt_lds[1]);
    }
}

// queue position by descending length (counting sort; order inside a bin is
// irrelevant to the results).  Lanes of a wavefront that share a bin take
// their positions with one atomic.
__global__ void k_queue_scatter(const Dom *__restrict__ doms, const int64_t *__restrict__ n_dom_p, int64_t max_dom,
                                int32_t D, unsigned long long *__restrict__ cursor, int32_t *__restrict__ queue) {
    const int64_t n_dom = *n_dom_p;
    const int64_t lim = n_dom < max_dom ? n_dom : max_dom;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < lim; i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const bool ok = i < lim;
        const int bin = ok ? D - doms[i].nint : -1;
        bool pending = ok;
        while (__ballot(pending)) {
            const int lead = __builtin_ctzll(__ballot(pending));
            const int lb = __shfl(bin, lead);
            const bool mine = pending && bin == lb;
            const uint64_t m = __ballot(mine);
            unsigned long long base = 0;
            if (lane_id() == lead) base = atomicAdd(&cursor[lb], (unsigned long long)__popcll(m));
            base = __shfl(base, lead);
            if (mine) {
                queue[base + __popcll(m & lanemask_lt())] = (int32_t)i;
                pending = false;
            }
        }
    }
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Per-series z-normalisation statistics: mean = T(v)/n and
// std = sqrt(T((v - mean)^2)/n) (population), a zero (or n <= 1) deviation
// replaced by 1 so the series is only centred.  T is the balanced pairwise sum
// over the series' points zero-padded to a power of two P, taken as 1024-leaf
// subtrees aligned to the series start, then a tree over up to 1024 subtree
// sums, then over up to 1024 of those (zero subtrees add +0 exactly, so this
// is the tree over P).  One workgroup of 256 threads per series.
constexpr int64_t kZnMaxBlocks = (int64_t)1 << 20;  // series of up to 2^30 points

template <int Pass>
__device__ double zn_tree(const double *__restrict__ v, int64_t n, double mean, double *lvl1, double *lvl2) {
    const int64_t nb = (n + 1023) / 1024;
    double total = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        double a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t idx = b * 1024 + 4 * threadIdx.x + i;
            double x = 0.0;
            if (idx < n) {
                x = v[idx];
                if (Pass == 2) {
                    const double d = x - mean;
                    x = d * d;
                }
            }
            a[i] = x;
        }
        const double r = block_tree_1024(a[0], a[1], a[2], a[3]);
        if (nb == 1) {
            total = r;
            break;
        }
        if (threadIdx.x == 0) lvl1[b & 1023] = r;
        const bool sb_end = (b & 1023) == 1023 || b == nb - 1;
        if (sb_end) {
            __syncthreads();
            const int64_t cnt = (b & 1023) + 1;
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = 4 * threadIdx.x + i < cnt ? lvl1[4 * threadIdx.x + i] : 0.0;
            const double sb = block_tree_1024(a[0], a[1], a[2], a[3]);
            if (nb <= 1024) {
                total = sb;
            } else if (threadIdx.x == 0) {
                lvl2[b >> 10] = sb;
            }
            __syncthreads();
        }
    }
    if (nb > 1024) {
        __syncthreads();
        const int64_t cnt = (nb + 1023) >> 10;
        double a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = 4 * threadIdx.x + i < cnt ? lvl2[4 * threadIdx.x + i] : 0.0;
        total = block_tree_1024(a[0], a[1], a[2], a[3]);
    }
    return total;
}

__global__ __launch_bounds__(256) void k_zn_stats(const double *__restrict__ values,
                                                  const int64_t *__restrict__ series_off, int64_t n_series,
                                                  double *__restrict__ zmean, double *__restrict__ zstd,
                                                  int32_t *status) {
    __shared__ double lvl1[1024];
    __shared__ double lvl2[1024];
    for (int64_t sr = blockIdx.x; sr < n_series; sr += gridDim.x) {
        const int64_t a = series_off[sr];
        const int64_t n = series_off[sr + 1] - a;
        if (n <= 0 || (n + 1023) / 1024 > kZnMaxBlocks) {
            if (threadIdx.x == 0) {
                zmean[sr] = 0.0;
                zstd[sr] = 1.0;
                if (n > 0) set_status(status, kStOverflow);
            }
            continue;
        }
        const double mean = zn_tree<1>(values + a, n, 0.0, lvl1, lvl2) / (double)n;
        const double var = zn_tree<2>(values + a, n, mean, lvl1, lvl2) / (double)n;
        double sd = __dsqrt_rn(var);
        if (!(sd > 0.0)) sd = 1.0;
        if (threadIdx.x == 0) {
            zmean[sr] = mean;
            zstd[sr] = sd;
        }
    }
}

__global__ void k_prepare(int32_t *status, int32_t *q_head) {
    if (threadIdx.x == 0) {
        status[0] = 0;
        *q_head = 0;
    }
}

// Lane exchanges inside a group of W lanes.  For W <= 16 they are DPP moves
// (quad permutations for W <= 4, row shifts for W = 8, 16): register to
// register, no LDS round trip on the round's critical path.
template <int Ctrl>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), Ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), Ctrl, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// value of lane (j - O) of the group (only read where j >= O)
template <int W, int O>
__device__ __forceinline__ double group_up(double v) {
    if constexpr (W == 2) return dpp_f64<0xA0>(v);                 // quad_perm(0,0,2,2)
    else if constexpr (W == 4 && O == 1) return dpp_f64<0x90>(v);  // quad_perm(0,0,1,2)
    else if constexpr (W == 4 && O == 2) return dpp_f64<0x44>(v);  // quad_perm(0,1,0,1)
    else if constexpr (W == 8 || W == 16) return dpp_f64<0x110 + O>(v);  // row_shr:O
    else return __shfl_up(v, O, W);
}

// value of the group's last lane
template <int W>
__device__ __forceinline__ double group_last(double v, int leader) {
    if constexpr (W == 1) return v;
    else if constexpr (W == 2) return dpp_f64<0xF5>(v);  // quad_perm(1,1,3,3)
    else if constexpr (W == 4) return dpp_f64<0xFF>(v);  // quad_perm(3,3,3,3)
    else return __shfl(v, leader + W - 1);
}

// Ring of staged points per group (positions p live in slot p & (R - 1)).
// Small rings keep every group of a launch resident at once (the LDS of a
// compute unit holds ~160 groups of 64 points); the next Q points are always
// in flight in registers, so a refill only moves them into the ring.
template <int W>
struct RingShape {
    static constexpr int R = W >= 8 ? 128 : (W >= 2 ? 64 : 32);
    static constexpr int Q = R / 2;  // refill granularity
    static_assert(W <= R - Q, "a refill must not overwrite the window a round reads");
    static_assert(Q % W == 0, "each lane stages Q / W points per refill");
};

template <int W>
size_t compress_lds_per_wave() {
    return (size_t)(kWave / W) * (RingShape<W>::R + 1) * sizeof(double);
}

// Norm: every value is read as (t - mean[series]) / std[series], so the
// z-normalised series is compressed without being written anywhere.
template <int W, bool Norm>
__global__ __launch_bounds__(1024) void k_compress(const double *__restrict__ t, const Dom *__restrict__ doms,
                                                   const int32_t *__restrict__ queue,
                                                   const int64_t *__restrict__ n_dom_p, int32_t *__restrict__ q_head,
                                                   int64_t direct_base, int64_t direct_end, double tol2,
                                                   int32_t max_len, int32_t *__restrict__ st_len,
                                                   double *__restrict__ st_inc, int32_t *__restrict__ dom_count,
                                                   int32_t *status, const double *__restrict__ zmean,
                                                   const double *__restrict__ zstd) {
    constexpr int R = RingShape<W>::R;
    constexpr int Q = RingShape<W>::Q;
    extern __shared__ double ring_all[];
    const int lane = lane_id();
    const int j = lane & (W - 1);
    const int leader = lane - j;
    const uint64_t gmask = (W == 64) ? ~0ull : (((1ull << W) - 1ull) << leader);
    // one ring per group; the stride of R + 1 doubles puts the same slot of
    // neighbouring groups in different LDS banks (domains of equal length
    // keep their groups' slots in step)
    double *ring = ring_all + ((size_t)(threadIdx.x / kWave) * (kWave / W) + (size_t)(lane / W)) * (R + 1);
    const int64_t n_dom = *n_dom_p;
    const bool direct = direct_base >= 0;
    const int64_t wave_g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;

    // group state, replicated over the group's lanes
    int32_t dom = -1;
    bool exhausted = false;
    int64_t s = 0, e = 0, obase = 0, le = 0;
    int32_t np = 0;
    double ts = 0.0;
    int32_t c0 = 2;
    double S2c = 0.0, S1c = 0.0;  // sums over the terms of candidates below c0
    double pre[Q / W];            // points [le, le + Q), loaded ahead of the refill that stages them
    double zm = 0.0, zs = 1.0;    // the domain's series mean and deviation (Norm)

    auto value = [&](int64_t p) -> double {
        if constexpr (Norm) {
            const double d = t[p] - zm;
            return d / zs;
        } else {
            return t[p];
        }
    };
    // requests [le, le + Q): lane j holds points le + r * W + j
    auto prefetch = [&]() {
#pragma unroll
        for (int r = 0; r < Q / W; ++r) {
            const int64_t p = le + r * W + j;
            pre[r] = p <= e ? value(p) : 0.0;
        }
    };

    auto start_domain = [&](int32_t d) {
        dom = d;
        const Dom x = doms[dom];
        s = x.start;
        e = x.start + x.nint;
        obase = x.start;
        le = x.start;
        np = 0;
        if constexpr (Norm) {
            zm = zmean[x.series];
            zs = zstd[x.series];
        }
        ts = value(s);
        if (j == 0 && !isfinite(ts)) set_status(status, kStNonFinite);
        c0 = 2;
        S2c = 0.0;
        S1c = 0.0;
        prefetch();
    };
    // The ring holds positions [le - R, le).  A round reads only the window
    // [s + c0 - 1, s + c0 + W - 1], which the refill keeps staged, so the
    // round's own reads never wait on global memory (and so never on the
    // output stores still in flight).  Only the exact evaluation of an
    // undecided candidate may reach below the ring, and reads memory there.
    auto at = [&](int64_t p) -> double { return ring[p & (R - 1)]; };
    auto at_far = [&](int64_t p) -> double { return p >= le - R ? ring[p & (R - 1)] : value(p); };

    if (direct) {
        const int64_t d = direct_base + wave_g * (kWave / W) + lane / W;
        exhausted = true;
        if (d < direct_end && d < n_dom) start_domain((int32_t)d);
    }

    for (;;) {
        if (!direct) {
            const bool need = (j == 0) && dom < 0 && !exhausted;
            const uint64_t nm = ballot(need);
            if (nm) {
                const int first = ffs64(nm);
                int base = 0;
                if (lane == first) base = atomicAdd(q_head, (int)__popcll(nm));
                base = shfl_i(base, first);
                int got = dom;
                bool ex = exhausted;
                if (need) {
                    const int64_t qp = (int64_t)base + __popcll(nm & lanemask_lt());
                    if (qp < n_dom)
                        got = queue[qp];
                    else
                        ex = true;
                }
                got = shfl_i(got, leader);
                ex = shfl_i((int)ex, leader) != 0;
                if (got >= 0 && dom < 0) start_domain(got);
                exhausted = ex;
            }
        }
        const bool act = dom >= 0;
        if (ballot(act || !exhausted) == 0ull) break;

        int verdict = -1;  // per lane: +1 accept, -1 reject
        int32_t c = 0;
        double S2 = 0.0, S1 = 0.0;
        if (act) {
            // stage the points this round reads: [s + c0 - 1, s + c0 + W - 1]
            int64_t need_hi = s + c0 + W - 1;
            if (need_hi > e) need_hi = e;
            // refill Q points at a time from the registers loaded ahead,
            // then request the next Q.  Overwritten slots hold
            // [le - R, le - R + Q), below the window because W <= R - Q.
            while (le <= need_hi) {
#pragma unroll
                for (int r = 0; r < Q / W; ++r) ring[(le + r * W + j) & (R - 1)] = pre[r];
                le += Q;
                prefetch();
            }
            c = c0 + j;
            const int64_t pk = s + c - 1;  // the term this candidate adds: k = c - 1
            double a2 = 0.0, a1 = 0.0;
            if (pk <= e) {
                const double d = at(pk) - ts;
                a2 = d * d;
                a1 = (double)(c - 1) * d;
            }
            S2 = a2;
            S1 = a1;
            if constexpr (W >= 2) {
                const double y2 = group_up<W, 1>(S2), y1 = group_up<W, 1>(S1);
                if (j >= 1) { S2 += y2; S1 += y1; }
            }
            if constexpr (W >= 4) {
                const double y2 = group_up<W, 2>(S2), y1 = group_up<W, 2>(S1);
                if (j >= 2) { S2 += y2; S1 += y1; }
            }
            if constexpr (W >= 8) {
                const double y2 = group_up<W, 4>(S2), y1 = group_up<W, 4>(S1);
                if (j >= 4) { S2 += y2; S1 += y1; }
            }
            if constexpr (W >= 16) {
                const double y2 = group_up<W, 8>(S2), y1 = group_up<W, 8>(S1);
                if (j >= 8) { S2 += y2; S1 += y1; }
            }
            if constexpr (W >= 32) {
                const double y2 = group_up<W, 16>(S2), y1 = group_up<W, 16>(S1);
                if (j >= 16) { S2 += y2; S1 += y1; }
            }
            if constexpr (W >= 64) {
                const double y2 = group_up<W, 32>(S2), y1 = group_up<W, 32>(S1);
                if (j >= 32) { S2 += y2; S1 += y1; }
            }
            S2 += S2c;
            S1 += S1c;
            const bool valid = (s + c <= e) && (max_len <= 0 || c <= max_len);
            if (valid) {
                const double te = at(s + c);
                const double b = (te - ts) / (double)c;
                const double thr = (double)(c - 1) * tol2;
                verdict = filter_decide(S2, S1, b, ts, c, thr);
                if (verdict == 0) {
                    // undecided by the bound: evaluate the definition itself
                    double acc = 0.0;
                    for (int32_t k = 1; k < c; ++k) {
                        double v = b * (double)k;
                        v = ts + v;
                        const double r = v - at_far(s + k);
                        acc = acc + r * r;
                    }
                    verdict = (acc <= thr) ? 1 : -1;
                }
            }
        }
        const uint64_t fm = ballot(act && verdict < 0) & gmask;
        const double S2last = group_last<W>(S2, leader);
        const double S1last = group_last<W>(S1, leader);
        if (!act) continue;
        if (fm) {
            // the first rejected candidate ends the piece at the last accepted length
            const int32_t L = c0 + (ffs64(fm) - leader) - 1;
            const double tend = at(s + L);
            if (j == 0) {
                if (!isfinite(tend)) set_status(status, kStNonFinite);
                st_len[obase + np] = L;
                st_inc[obase + np] = tend - ts;
            }
            ++np;
            s += L;
            ts = tend;
            c0 = 2;
            S2c = 0.0;
            S1c = 0.0;
            if (s >= e) {
                if (j == 0) dom_count[dom] = np;
                dom = -1;
            }
        } else {
            // all W candidates accepted: the next round extends the sums
            c0 += W;
            S2c = S2last;
            S1c = S1last;
        }
    }
}

// One lane per domain (W = 1) with refills on a common schedule.  A lane's
// round tests one candidate c and needs one point it has not read before:
// point s + c - 1 (the new term of the sums) was the previous round's end
// point, and whether the candidate is accepted (c + 1) or ends the piece at
// c - 1 (the next piece starts there, at its c = 2), the next round's end
// point is the one after this round's.  So every lane takes exactly one new
// point per round, and all lanes of the wavefront refill their rings at the
// same rounds, every kQ1 rounds, each with the kQ1 points it loaded (one
// cache line) at the refill before.  Those loads are a whole refill period
// old when they are stored, where a per-lane refill schedule makes the
// wavefront wait on whichever lane refilled last.  A lane that starts a
// domain stages its first points itself, sized so that it falls into step
// with the schedule.  The arithmetic, the certified filter and the exact
// evaluation are those of k_compress with W = 1.
constexpr int kR1 = 32;           // ring of staged points per lane
constexpr int kQ1 = kR1 / 2;      // points per refill, and rounds between refills

size_t compress1_lds_per_wave() { return (size_t)kWave * (kR1 + 1) * sizeof(double); }

template <bool Norm, bool Grouped>
__global__ __launch_bounds__(1024) void k_compress1(const double *__restrict__ t, const Dom *__restrict__ doms,
                                                    const int32_t *__restrict__ queue,
                                                    const int64_t *__restrict__ n_dom_p, int32_t *__restrict__ q_head,
                                                    int64_t direct_base, int64_t direct_end, double tol2,
                                                    int32_t max_len, int32_t *__restrict__ st_len,
                                                    double *__restrict__ st_inc, int32_t *__restrict__ dom_count,
                                                    int32_t *status, const double *__restrict__ zmean,
                                                    const double *__restrict__ zstd) {
    extern __shared__ double ring_all[];
    const int lane = lane_id();
    // the stride of kR1 + 1 doubles puts the same slot of neighbouring lanes
    // in different LDS banks
    double *ring = ring_all + (size_t)threadIdx.x * (kR1 + 1);
    const int64_t n_dom = *n_dom_p;
    const bool direct = direct_base >= 0;
    const int64_t wave_g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;

    int32_t dom = -1;
    bool exhausted = false;
    int64_t s = 0, e = 0, obase = 0;
    int64_t le = 0;     // the ring holds points [le - kR1, le)
    int32_t np = 0;
    int32_t c = 2;
    double ts = 0.0;    // point s (the piece's start)
    double tpk = 0.0;   // point s + c - 1
    double tend = 0.0;  // point s + c (the candidate's end; any value past e)
    double S2c = 0.0, S1c = 0.0;  // sums over the terms below k = c - 1
    double zm = 0.0, zs = 1.0;
    double pre[kQ1];    // points [le, le + kQ1), stored at the next refill
    uint32_t rr = 0;    // iteration count, the same on every lane
    // Grouped: pieces are kept in groups of four staging slots aligned to the
    // slot index and leave as one 16-byte store of lengths and two of
    // increments when a group is complete; a domain's first and last groups,
    // which share their slots with its neighbours, leave slot by slot.  That
    // takes the piece stores from two to three-quarters of an instruction per
    // piece, which pays when there are at least as many domains as lanes (the
    // vector-memory pipeline bounds the kernel then); with fewer domains the
    // per-round latency does, and each piece is stored at once.
    int32_t gl0 = 0, gl1 = 0, gl2 = 0, gl3 = 0;
    double gi0 = 0.0, gi1 = 0.0, gi2 = 0.0, gi3 = 0.0;
    int gfirst = 0;     // first slot of the current group that is this domain's

    auto value = [&](int64_t p) -> double {
        if constexpr (Norm) {
            const double d = t[p] - zm;
            return d / zs;
        } else {
            return t[p];
        }
    };
    auto at = [&](int64_t p) -> double { return ring[p & (kR1 - 1)]; };
    auto at_far = [&](int64_t p) -> double { return p >= le - kR1 ? ring[p & (kR1 - 1)] : value(p); };
    auto load_pre = [&]() {
#pragma unroll
        for (int r = 0; r < kQ1; ++r) {
            const int64_t p = le + r;
            pre[r] = value(p <= e ? p : e);
        }
    };
    // The round of iteration rr reads point q = s + c + 1, one further each
    // round; a refill at the start of each iteration with rr % kQ1 == 0
    // stores pre[] at [le, le + kQ1).  A domain started at iteration rr0 reads
    // q0 = s + 3 first and meets its first refill k = (kQ1 - rr0 % kQ1) % kQ1
    // rounds later, when it reads q1 = q0 + k.  Staging [s + 1, L) with any L
    // in [q1, q1 + kQ1] keeps every q it reads inside [le - kR1, le) from then on
    // (right after a refill kQ1 <= le - q <= kR1, just before one
    // 1 <= le - q <= kQ1 + 1), and a refill overwrites only points below the
    // next q.  L is taken as a multiple of kQ1, so that every refill loads
    // kQ1 points of one aligned 128-byte line.
    auto start_domain = [&](int32_t d) {
        dom = d;
        const Dom x = doms[dom];
        s = x.start;
        e = x.start + x.nint;
        obase = x.start;
        np = 0;
        gfirst = (int)(obase & 3);
        if constexpr (Norm) {
            zm = zmean[x.series];
            zs = zstd[x.series];
        }
        ts = value(s);
        tpk = value(s + 1);
        tend = value(s + 2 <= e ? s + 2 : e);
        if (!isfinite(ts)) set_status(status, kStNonFinite);
        c = 2;
        S2c = 0.0;
        S1c = 0.0;
        const int k = (int)((kQ1 - (rr & (kQ1 - 1))) & (kQ1 - 1));
        const int64_t q0 = s + 3;
        le = (q0 + k + kQ1 - 1) & ~(int64_t)(kQ1 - 1);
        // from s + 1: the exact evaluation reads points s + 1 .. q - 2 through
        // the ring wherever they lie in its window (le - (s + 1) <= kR1)
        for (int64_t p = s + 1; p < le; ++p) ring[p & (kR1 - 1)] = value(p <= e ? p : e);
        load_pre();
    };

    if (direct) {
        exhausted = true;
        const int64_t d = direct_base + wave_g * kWave + lane;
        if (d < direct_end && d < n_dom) start_domain((int32_t)d);
    }

    for (;;) {
        if (!direct) {
            const bool need = dom < 0 && !exhausted;
            const uint64_t nm = ballot(need);
            if (nm) {
                const int first = ffs64(nm);
                int base = 0;
                if (lane == first) base = atomicAdd(q_head, (int)__popcll(nm));
                base = shfl_i(base, first);
                if (need) {
                    const int64_t qp = (int64_t)base + __popcll(nm & lanemask_lt());
                    if (qp < n_dom)
                        start_domain(queue[qp]);
                    else
                        exhausted = true;
                }
            }
        }
        const bool act = dom >= 0;
        if (ballot(act || !exhausted) == 0ull) break;
        if ((rr & (kQ1 - 1)) == 0 && act) {
#pragma unroll
            for (int r = 0; r < kQ1; ++r) ring[(le + r) & (kR1 - 1)] = pre[r];
            le += kQ1;
            load_pre();
        }
        ++rr;
        if (!act) continue;

        // the next round's end point
        const double tnext = at(s + c + 1);
        const double d = tpk - ts;
        const double S2 = d * d + S2c;
        const double S1 = (double)(c - 1) * d + S1c;
        int verdict = -1;
        if ((s + c <= e) && (max_len <= 0 || c <= max_len)) {
            const double b = (tend - ts) / (double)c;
            const double thr = (double)(c - 1) * tol2;
            verdict = filter_decide(S2, S1, b, ts, c, thr);
            if (verdict == 0) {
                // undecided by the bound: evaluate the definition itself
                double acc = 0.0;
                for (int32_t k = 1; k < c; ++k) {
                    double v = b * (double)k;
                    v = ts + v;
                    const double r = v - at_far(s + k);
                    acc = acc + r * r;
                }
                verdict = (acc <= thr) ? 1 : -1;
            }
        }
        if (verdict < 0) {
            // the piece ends at the last accepted length, on point s + c - 1
            const int32_t L = c - 1;
            if (!isfinite(tpk)) set_status(status, kStNonFinite);
            const int64_t idx = obase + np;
            const int slot = (int)(idx & 3);
            const double iv = tpk - ts;
            if constexpr (!Grouped) {
                st_len[idx] = L;
                st_inc[idx] = iv;
            }
            gl0 = slot == 0 ? L : gl0;
            gl1 = slot == 1 ? L : gl1;
            gl2 = slot == 2 ? L : gl2;
            gl3 = slot == 3 ? L : gl3;
            gi0 = slot == 0 ? iv : gi0;
            gi1 = slot == 1 ? iv : gi1;
            gi2 = slot == 2 ? iv : gi2;
            gi3 = slot == 3 ? iv : gi3;
            ++np;
            s += L;
            ts = tpk;
            c = 2;
            S2c = 0.0;
            S1c = 0.0;
            const bool last = s >= e;
            if (Grouped && (slot == 3 || last)) {
                const int64_t g0 = idx - slot;
                if (gfirst == 0 && slot == 3) {
                    *reinterpret_cast<int4 *>(st_len + g0) = make_int4(gl0, gl1, gl2, gl3);
                    *reinterpret_cast<double2 *>(st_inc + g0) = make_double2(gi0, gi1);
                    *reinterpret_cast<double2 *>(st_inc + g0 + 2) = make_double2(gi2, gi3);
                } else {
                    if (gfirst <= 0 && slot >= 0) {
                        st_len[g0] = gl0;
                        st_inc[g0] = gi0;
                    }
                    if (gfirst <= 1 && slot >= 1) {
                        st_len[g0 + 1] = gl1;
                        st_inc[g0 + 1] = gi1;
                    }
                    if (gfirst <= 2 && slot >= 2) {
                        st_len[g0 + 2] = gl2;
                        st_inc[g0 + 2] = gi2;
                    }
                    if (gfirst <= 3 && slot >= 3) {
                        st_len[g0 + 3] = gl3;
                        st_inc[g0 + 3] = gi3;
                    }
                }
                gfirst = 0;
            }
            if (last) {
                dom_count[dom] = np;
                dom = -1;
            }
        } else {
            ++c;
            S2c = S2;
            S1c = S1;
        }
        tpk = tend;
        tend = tnext;
    }
}

// ------------------------------------------------------------ segment repair
//
// Segments were compressed as if each were a domain, so every segment's
// chain of pieces starts at the segment start and its last piece is cut at
// the segment end.  The domain's true chain is recovered per domain, one lane
// walking its segments in order: from the true chain's position it takes the
// greedy's own pieces until it lands on a start of the segment's chain (from
// there the two chains coincide, being the same greedy from the same point),
// keeps the segment's pieces up to its last one, and recomputes that last
// piece without the segment end.  Each segment's staging region is rewritten
// in place to hold exactly the true pieces that start inside it, so the
// compaction that follows is the one of the plain domains.  Decisions come
// from the same certified filter with the same exact fallback as the
// kernel's, so they are the definition's.
template <bool Norm>
struct Values {
    const double *t;
    double zm, zs;
    __device__ double operator()(int64_t p) const {
        if constexpr (Norm) {
            const double d = t[p] - zm;
            return d / zs;
        } else {
            return t[p];
        }
    }
};

template <bool Norm>
__global__ void k_repair(const Dom *__restrict__ doms, const int64_t *__restrict__ n_dom_p,
                         const double *__restrict__ t, const double *__restrict__ zmean,
                         const double *__restrict__ zstd, double tol2, int32_t max_len, int32_t *__restrict__ st_len,
                         double *__restrict__ st_inc, int32_t *__restrict__ dom_count, int32_t *__restrict__ first,
                         int32_t *status) {
    const int64_t n_dom = *n_dom_p;
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n_dom;
         d += (int64_t)gridDim.x * blockDim.x) {
        const Dom x = doms[d];
        if (x.seg != 0 || x.nseg <= 1) continue;
        Values<Norm> v{t, 0.0, 1.0};
        if constexpr (Norm) {
            v.zm = zmean[x.series];
            v.zs = zstd[x.series];
        }
        bool nonfinite = false;
        if (repair_domain(v, doms, d, tol2, max_len, st_len, st_inc, dom_count, first, &nonfinite))
            set_status(status, kStInternal);
        if (nonfinite) set_status(status, kStNonFinite);
    }
}

__global__ void k_compact(const Dom *__restrict__ doms, const int64_t *__restrict__ n_dom_p,
                          const int32_t *__restrict__ dom_count, const int64_t *__restrict__ dom_poff,
                          const int32_t *__restrict__ st_len, const double *__restrict__ st_inc,
                          const int32_t *__restrict__ first, int32_t *__restrict__ len, double *__restrict__ inc) {
    const int64_t n_dom = *n_dom_p;
    const int lane = lane_id();
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t d = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; d < n_dom; d += waves) {
        const Dom x = doms[d];
        const int64_t src = x.start + (x.nseg > 1 ? first[d] : 0);
        const int64_t dst = dom_poff[d];
        const int32_t cnt = dom_count[d];
        for (int32_t i = lane; i < cnt; i += kWave) {
            len[dst + i] = st_len[src + i];
            inc[dst + i] = st_inc[src + i];
        }
    }
}

__global__ void k_piece_off(const int64_t *__restrict__ dom_off, const int64_t *__restrict__ dom_poff,
                            int64_t n_series, int64_t *__restrict__ piece_off, int64_t *__restrict__ n_pieces) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_series) return;
    int64_t v = dom_poff[dom_off[s]];
    piece_off[s] = v;
    if (s == n_series) *n_pieces = v;
}

struct CompressWs {
    int32_t *status;
    int32_t *q_head;
    int32_t *ndom;
    int64_t *dom_off;
    Dom *doms;
    unsigned long long *len_hist;
    int64_t *bin_off;
    int32_t *queue;
    int32_t *dom_count;
    int32_t *dom_first;
    int64_t *dom_poff;
    int32_t *st_len;
    double *st_inc;
    void *scan_ws;
    size_t bytes;
};

// work units (segments of domains) for any segment length >= kMinSegment
int64_t max_domains(int64_t n_series, int64_t total_points, int32_t D) {
    const int64_t G = D < kMinSegment ? D : kMinSegment;
    return total_points / G + total_points / D + n_series + 1;
}

CompressWs carve_compress(void *ws, int64_t n_series, int64_t total_points, int32_t D) {
    const int64_t md = max_domains(n_series, total_points, D);
    Carve c(ws);
    CompressWs w;
    w.status = c.take<int32_t>(64);
    w.q_head = c.take<int32_t>(64);
    w.ndom = c.take<int32_t>(n_series + 1);
    w.dom_off = c.take<int64_t>(n_series + 2);
    w.doms = c.take<Dom>(md);
    w.len_hist = c.take<unsigned long long>((size_t)D + 2);
    w.bin_off = c.take<int64_t>((size_t)D + 3);
    w.queue = c.take<int32_t>(md);
    w.dom_count = c.take<int32_t>(md);
    w.dom_first = c.take<int32_t>(md);
    w.dom_poff = c.take<int64_t>(md + 1);
    w.st_len = c.take<int32_t>(total_points);
    w.st_inc = c.take<double>(total_points);
    int64_t scan_n = md > n_series + 1 ? md : n_series + 1;
    if (scan_n < D + 2) scan_n = D + 2;
    w.scan_ws = c.take<char>(scan_workspace(scan_n));
    w.bytes = c.bytes();
    return w;
}

int validate(const double *values, const int64_t *series_off, int64_t n_series, int64_t total_points, int32_t D,
             double tol, int32_t max_len, int32_t *len, double *inc, int64_t *piece_off, int64_t *n_pieces) {
    if (n_series < 0 || total_points < 0 || D < 1 || max_len < 0) return JABBA_EINVAL;
    if (!(tol >= 0.0) || !(tol <= 1.0e150)) return JABBA_EINVAL;
    if (total_points - n_series >= (int64_t)1 << 31) return JABBA_EOVERFLOW;
    if (max_domains(n_series, total_points, D) >= ((int64_t)1 << 31) - 65536) return JABBA_EOVERFLOW;
    if (!series_off || !piece_off || !n_pieces) return JABBA_EINVAL;
    if (total_points > 0 && (!values || !len || !inc)) return JABBA_EINVAL;
    return JABBA_OK;
}

int domain_table(const CompressWs &w, const int64_t *series_off, int64_t n_series, int64_t total_points, int32_t D,
                 int32_t G, bool want_queue, hipStream_t st) {
    const int64_t md = max_domains(n_series, total_points, D);
    const unsigned sb = (unsigned)((n_series + 255) / 256 > 0 ? (n_series + 255) / 256 : 1);
    JB_LAUNCH(k_prepare, dim3(1), dim3(64), 0, st, w.status, w.q_head);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_series_domains, dim3(sb), dim3(256), 0, st, series_off, n_series, D, G, w.ndom, w.status);
    JB_LAUNCH_CHECK();
    int rc = scan_i32_to_i64(w.ndom, w.dom_off, nullptr, n_series, w.scan_ws, st);
    if (rc) return rc;
    if (want_queue) {
        JB_LAUNCH(k_zero_u64, dim3((unsigned)((D + 2 + 255) / 256)), dim3(256), 0, st, w.len_hist,
                           (int64_t)D + 2);
        JB_LAUNCH_CHECK();
    }
    {
        int64_t fb = (n_series * kWave + 255) / 256;
        const int64_t cap = (int64_t)device_cu_count() * 2;
        if (fb > cap) fb = cap;
        if (fb < 1) fb = 1;
        JB_LAUNCH(k_fill_domains, dim3((unsigned)fb), dim3(256), 0, st, series_off, w.dom_off, n_series, D, G, w.doms,
                  want_queue ? w.len_hist : nullptr);
    }
    JB_LAUNCH_CHECK();
    if (want_queue) {
        rc = scan_i64_to_i64(reinterpret_cast<const int64_t *>(w.len_hist), w.bin_off, nullptr, (int64_t)D + 1,
                             w.scan_ws, st);
        if (rc) return rc;
        int64_t blocks = (md + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        JB_LAUNCH(k_queue_scatter, dim3((unsigned)blocks), dim3(256), 0, st, w.doms, w.dom_off + n_series,
                           md, D, reinterpret_cast<unsigned long long *>(w.bin_off), w.queue);
        JB_LAUNCH_CHECK();
    }
    return JABBA_OK;
}

int finish(const CompressWs &w, int64_t n_series, int64_t total_points, int32_t D, int32_t *len, double *inc,
           int64_t *piece_off, int64_t *n_pieces, hipStream_t st) {
    const int64_t md = max_domains(n_series, total_points, D);
    const int64_t *n_dom_p = w.dom_off + n_series;
    int rc = scan_i32_to_i64(w.dom_count, w.dom_poff, n_dom_p, md, w.scan_ws, st);
    if (rc) return rc;
    int64_t blocks = (md * kWave + 255) / 256;
    int cap = device_cu_count() * 16;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    JB_LAUNCH(k_compact, dim3((unsigned)blocks), dim3(256), 0, st, w.doms, n_dom_p, w.dom_count, w.dom_poff,
                       w.st_len, w.st_inc, w.dom_first, len, inc);
    JB_LAUNCH_CHECK();
    JB_LAUNCH(k_piece_off, dim3((unsigned)((n_series + 1 + 255) / 256)), dim3(256), 0, st, w.dom_off,
                       w.dom_poff, n_series, piece_off, n_pieces);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

// units: the host's upper bound on the work units (domains or segments)
template <int W>
void launch_w(dim3 g, dim3 b, hipStream_t st, const double *t, const CompressWs &w, const int64_t *n_dom_p,
              int64_t dbase, int64_t dend, double tol2, int32_t max_len, const double *zmean, const double *zstd,
              int64_t units) {
    if constexpr (W == 1) {
        const size_t lds = compress1_lds_per_wave() * (b.x / kWave);
        const bool grouped = units >= (int64_t)g.x * b.x;  // at least one unit per lane
        if (zmean) {
            if (grouped)
                JB_LAUNCH_NAMED("k_compress_znorm", (k_compress1<true, true>), g, b, lds, st, t, w.doms, w.queue,
                                n_dom_p, w.q_head, dbase, dend, tol2, max_len, w.st_len, w.st_inc, w.dom_count,
                                w.status, zmean, zstd);
            else
                JB_LAUNCH_NAMED("k_compress_znorm", (k_compress1<true, false>), g, b, lds, st, t, w.doms, w.queue,
                                n_dom_p, w.q_head, dbase, dend, tol2, max_len, w.st_len, w.st_inc, w.dom_count,
                                w.status, zmean, zstd);
        } else {
            if (grouped)
                JB_LAUNCH_NAMED("k_compress<W>", (k_compress1<false, true>), g, b, lds, st, t, w.doms, w.queue,
                                n_dom_p, w.q_head, dbase, dend, tol2, max_len, w.st_len, w.st_inc, w.dom_count,
                                w.status, zmean, zstd);
            else
                JB_LAUNCH_NAMED("k_compress<W>", (k_compress1<false, false>), g, b, lds, st, t, w.doms, w.queue,
                                n_dom_p, w.q_head, dbase, dend, tol2, max_len, w.st_len, w.st_inc, w.dom_count,
                                w.status, zmean, zstd);
        }
    } else {
        const size_t lds = compress_lds_per_wave<W>() * (b.x / kWave);
        if (zmean)
            JB_LAUNCH_NAMED("k_compress_znorm", (k_compress<W, true>), g, b, lds, st, t, w.doms, w.queue, n_dom_p,
                            w.q_head, dbase, dend, tol2, max_len, w.st_len, w.st_inc, w.dom_count, w.status, zmean,
                            zstd);
        else
            JB_LAUNCH_NAMED("k_compress<W>", (k_compress<W, false>), g, b, lds, st, t, w.doms, w.queue, n_dom_p,
                            w.q_head, dbase, dend, tol2, max_len, w.st_len, w.st_inc, w.dom_count, w.status, zmean,
                            zstd);
    }
}

int launch_repair(const CompressWs &w, const int64_t *n_dom_p, int64_t n_series, int64_t total_points, int32_t D,
                  const double *t, double tol2, int32_t max_len, const double *zmean, const double *zstd,
                  hipStream_t st) {
    const int64_t md = max_domains(n_series, total_points, D);
    int64_t blocks = (md + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    if (zmean)
        JB_LAUNCH(k_repair<true>, dim3((unsigned)blocks), dim3(256), 0, st, w.doms, n_dom_p, t, zmean, zstd, tol2,
                  max_len, w.st_len, w.st_inc, w.dom_count, w.dom_first, w.status);
    else
        JB_LAUNCH(k_repair<false>, dim3((unsigned)blocks), dim3(256), 0, st, w.doms, n_dom_p, t, zmean, zstd, tol2,
                  max_len, w.st_len, w.st_inc, w.dom_count, w.dom_first, w.status);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

// units: an upper bound on the work units the launch takes (domains or
// segments), which picks between forms of the one-lane kernel
int launch_compress(int W, dim3 g, dim3 b, hipStream_t st, const double *t, const CompressWs &w,
                    const int64_t *n_dom_p, int64_t dbase, int64_t dend, double tol2, int32_t max_len,
                    const double *zmean, const double *zstd, int64_t units);

// segments: one group per work unit, assigned statically (segments are of
// nearly equal length, so no queue is needed)
int launch_segments(int W, int wpb, hipStream_t st, const double *t, const CompressWs &w, const int64_t *n_dom_p,
                    int64_t n_series, int64_t total_points, int32_t D, int32_t G, double tol2, int32_t max_len,
                    const double *zmean, const double *zstd) {
    const int64_t md = max_domains(n_series, total_points, D);
    const int64_t groups_per_block = (int64_t)wpb * (kWave / W);
    int64_t blocks = (md + groups_per_block - 1) / groups_per_block;
    if (blocks < 1) blocks = 1;
    if (blocks > ((int64_t)1 << 31) - 1) return JABBA_EOVERFLOW;
    return launch_compress(W, dim3((unsigned)blocks), dim3((unsigned)(wpb * kWave)), st, t, w, n_dom_p, 0, md, tol2,
                           max_len, zmean, zstd, total_points / G + total_points / D + n_series);
}

// Segment length from the tuning: negative = whole domains; 0 = the default,
// which segments only when the domains are fewer than a quarter of the
// compute units.  With more domains the repair's sequential walks (the two
// chains can stay out of step for hundreds of rounds on noisy data) cost
// more than the extra parallelism saves; the autotuner tries both.
constexpr int64_t kFewDomainsDivisor = 4;

int32_t segment_of(const jabba_tuning *tuning, int64_t n_series, int64_t total_points, int32_t D, int *rc) {
    int32_t G = kDefaultSegment;
    if (tuning && tuning->segment_intervals) {
        G = tuning->segment_intervals;
    } else {
        const int64_t domains = total_points / D + n_series;
        if (domains * kFewDomainsDivisor >= (int64_t)device_cu_count()) return D;
    }
    if (G < 0) return D;
    if (G < kMinSegment) {
        *rc = JABBA_EINVAL;
        return D;
    }
    return G < D ? G : D;
}

size_t lds_per_wave(int W) {
    switch (W) {
        case 1: return compress1_lds_per_wave();
        case 2: return compress_lds_per_wave<2>();
        case 4: return compress_lds_per_wave<4>();
        case 8: return compress_lds_per_wave<8>();
        case 16: return compress_lds_per_wave<16>();
        case 32: return compress_lds_per_wave<32>();
        default: return compress_lds_per_wave<64>();
    }
}

int launch_compress(int W, dim3 g, dim3 b, hipStream_t st, const double *t, const CompressWs &w,
                    const int64_t *n_dom_p, int64_t dbase, int64_t dend, double tol2, int32_t max_len,
                    const double *zmean, const double *zstd, int64_t units) {
    switch (W) {
        case 1: launch_w<1>(g, b, st, t, w, n_dom_p, dbase, dend, tol2, max_len, zmean, zstd, units); break;
        case 2: launch_w<2>(g, b, st, t, w, n_dom_p, dbase, dend, tol2, max_len, zmean, zstd, units); break;
        case 4: launch_w<4>(g, b, st, t, w, n_dom_p, dbase, dend, tol2, max_len, zmean, zstd, units); break;
        case 8: launch_w<8>(g, b, st, t, w, n_dom_p, dbase, dend, tol2, max_len, zmean, zstd, units); break;
        case 16: launch_w<16>(g, b, st, t, w, n_dom_p, dbase, dend, tol2, max_len, zmean, zstd, units); break;
        case 32: launch_w<32>(g, b, st, t, w, n_dom_p, dbase, dend, tol2, max_len, zmean, zstd, units); break;
        case 64: launch_w<64>(g, b, st, t, w, n_dom_p, dbase, dend, tol2, max_len, zmean, zstd, units); break;
        default: return JABBA_EINVAL;
    }
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

}  // namespace

// defaults (the autotuner may pick others; results never change).  One lane
// per domain keeps 64 domains per wavefront: with short pieces most rounds
// end a piece, so wider groups mostly test candidates past the first failure.
constexpr int kDefaultW = 1;
constexpr int kDefaultWavesPerBlock = 4;
constexpr int kDefaultBlocksPerCu = 4;

}  // namespace jabba

using namespace jabba;

extern "C" int jabba_compress_workspace(int64_t n_series, int64_t total_points, int32_t D, size_t *bytes) {
    if (!bytes || n_series < 0 || total_points < 0 || D < 1) return JABBA_EINVAL;
    *bytes = carve_compress(nullptr, n_series, total_points, D).bytes;
    return JABBA_OK;
}

extern "C" int jabba_compress(const double *values, const int64_t *series_off, int64_t n_series, int64_t total_points,
                              int32_t D, double tol, int32_t max_len, const jabba_tuning *tuning, int32_t *len,
                              double *inc, int64_t *piece_off, int64_t *n_pieces, void *workspace,
                              size_t workspace_bytes, void *stream) {
    int rc = validate(values, series_off, n_series, total_points, D, tol, max_len, len, inc, piece_off, n_pieces);
    if (rc) return rc;
    CompressWs w0 = carve_compress(nullptr, n_series, total_points, D);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    CompressWs w = carve_compress(workspace, n_series, total_points, D);
    hipStream_t st = (hipStream_t)stream;
    int W = kDefaultW, wpb = kDefaultWavesPerBlock, bpc = kDefaultBlocksPerCu;
    if (tuning) {
        if (tuning->lanes_per_domain) W = tuning->lanes_per_domain;
        if (tuning->waves_per_block) wpb = tuning->waves_per_block;
        if (tuning->blocks_per_cu) bpc = tuning->blocks_per_cu;
    }
    if (wpb < 1 || wpb > 16 || bpc < 1 || bpc > 32) return JABBA_EINVAL;
    if (W != 1 && W != 2 && W != 4 && W != 8 && W != 16 && W != 32 && W != 64) return JABBA_EINVAL;
    // a workgroup's ring buffers stay within 64 KB of LDS
    const size_t lw = lds_per_wave(W);
    const int max_wpb = lw ? (int)(65536 / lw) : 16;
    if (wpb > max_wpb) wpb = max_wpb < 1 ? 1 : max_wpb;
    const int32_t G = segment_of(tuning, n_series, total_points, D, &rc);
    if (rc) return rc;
    rc = domain_table(w, series_off, n_series, total_points, D, G, G >= D, st);
    if (rc) return rc;
    const int64_t *n_dom_p = w.dom_off + n_series;
    rc = G < D ? launch_segments(W, wpb, st, values, w, n_dom_p, n_series, total_points, D, G, tol * tol, max_len,
                                 nullptr, nullptr)
               : launch_compress(W, dim3((unsigned)(device_cu_count() * bpc)), dim3((unsigned)(wpb * kWave)), st,
                                 values, w, n_dom_p, -1, 0, tol * tol, max_len, nullptr, nullptr,
                                 total_points / D + n_series);
    if (rc) return rc;
    if (G < D) {
        rc = launch_repair(w, n_dom_p, n_series, total_points, D, values, tol * tol, max_len, nullptr, nullptr, st);
        if (rc) return rc;
    }
    return finish(w, n_series, total_points, D, len, inc, piece_off, n_pieces, st);
}

extern "C" int jabba_compress_znorm(const double *values, const int64_t *series_off, int64_t n_series,
                                    int64_t total_points, int32_t D, double tol, int32_t max_len,
                                    const jabba_tuning *tuning, int32_t *len, double *inc, int64_t *piece_off,
                                    int64_t *n_pieces, double *mean, double *std_dev, void *workspace,
                                    size_t workspace_bytes, void *stream) {
    int rc = validate(values, series_off, n_series, total_points, D, tol, max_len, len, inc, piece_off, n_pieces);
    if (rc) return rc;
    if (n_series > 0 && (!mean || !std_dev)) return JABBA_EINVAL;
    CompressWs w0 = carve_compress(nullptr, n_series, total_points, D);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    CompressWs w = carve_compress(workspace, n_series, total_points, D);
    hipStream_t st = (hipStream_t)stream;
    int W = kDefaultW, wpb = kDefaultWavesPerBlock, bpc = kDefaultBlocksPerCu;
    if (tuning) {
        if (tuning->lanes_per_domain) W = tuning->lanes_per_domain;
        if (tuning->waves_per_block) wpb = tuning->waves_per_block;
        if (tuning->blocks_per_cu) bpc = tuning->blocks_per_cu;
    }
    if (wpb < 1 || wpb > 16 || bpc < 1 || bpc > 32) return JABBA_EINVAL;
    if (W != 1 && W != 2 && W != 4 && W != 8 && W != 16 && W != 32 && W != 64) return JABBA_EINVAL;
    const size_t lw = lds_per_wave(W);
    const int max_wpb = lw ? (int)(65536 / lw) : 16;
    if (wpb > max_wpb) wpb = max_wpb < 1 ? 1 : max_wpb;
    const int32_t G = segment_of(tuning, n_series, total_points, D, &rc);
    if (rc) return rc;
    rc = domain_table(w, series_off, n_series, total_points, D, G, G >= D, st);
    if (rc) return rc;
    if (n_series > 0) {
        int64_t blocks = n_series;
        const int64_t cap = (int64_t)device_cu_count() * 16;
        if (blocks > cap) blocks = cap;
        JB_LAUNCH(k_zn_stats, dim3((unsigned)blocks), dim3(256), 0, st, values, series_off, n_series, mean, std_dev,
                  w.status);
        JB_LAUNCH_CHECK();
    }
    const int64_t *n_dom_p = w.dom_off + n_series;
    const double *zm = n_series > 0 ? mean : nullptr;
    rc = G < D ? launch_segments(W, wpb, st, values, w, n_dom_p, n_series, total_points, D, G, tol * tol, max_len, zm,
                                 std_dev)
               : launch_compress(W, dim3((unsigned)(device_cu_count() * bpc)), dim3((unsigned)(wpb * kWave)), st,
                                 values, w, n_dom_p, -1, 0, tol * tol, max_len, zm, std_dev,
                                 total_points / D + n_series);
    if (rc) return rc;
    if (G < D && n_series > 0) {
        rc = launch_repair(w, n_dom_p, n_series, total_points, D, values, tol * tol, max_len, mean, std_dev, st);
        if (rc) return rc;
    }
    return finish(w, n_series, total_points, D, len, inc, piece_off, n_pieces, st);
}

extern "C" int jabba_compress_plain(const double *values, const int64_t *series_off, const int64_t *series_off_host,
                                    int64_t n_series, int32_t D, double tol, int32_t max_len, int32_t *len,
                                    double *inc, int64_t *piece_off, int64_t *n_pieces, void *workspace,
                                    size_t workspace_bytes, void *stream) {
    if (!series_off_host) return JABBA_EINVAL;
    const int64_t total_points = n_series >= 0 ? series_off_host[n_series] : -1;
    int rc = validate(values, series_off, n_series, total_points, D, tol, max_len, len, inc, piece_off, n_pieces);
    if (rc) return rc;
    CompressWs w0 = carve_compress(nullptr, n_series, total_points, D);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    CompressWs w = carve_compress(workspace, n_series, total_points, D);
    hipStream_t st = (hipStream_t)stream;
    rc = domain_table(w, series_off, n_series, total_points, D, D, false, st);
    if (rc) return rc;
    const int64_t *n_dom_p = w.dom_off + n_series;
    int64_t d0 = 0;
    for (int64_t s = 0; s < n_series; ++s) {
        const int64_t n = series_off_host[s + 1] - series_off_host[s];
        const int64_t nd = n >= 2 ? (n - 1 + D - 1) / D : 0;
        if (nd > 0) {
            rc = launch_compress(64, dim3((unsigned)nd), dim3(kWave), st, values, w, n_dom_p, d0, d0 + nd,
                                 tol * tol, max_len, nullptr, nullptr, nd);
            if (rc) return rc;
        }
        d0 += nd;
    }
    return finish(w, n_series, total_points, D, len, inc, piece_off, n_pieces, st);
}

extern "C" int jabba_workspace_status(const void *workspace, void *stream, int32_t *status) {
    if (!workspace || !status) return JABBA_EINVAL;
    int32_t bits = 0;
    JB_HIP(hipStreamSynchronize((hipStream_t)stream));
    JB_HIP(hipMemcpy(&bits, workspace, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (bits & kStNonFinite)
        *status = JABBA_ENONFINITE;
    else if (bits & kStCapacity)
        *status = JABBA_ECAPACITY;
    else if (bits & kStOverflow)
        *status = JABBA_EOVERFLOW;
    else if (bits & kStInvalid)
        *status = JABBA_EINVAL;
    else if (bits & kStInternal)
        *status = JABBA_EHIP;
    else
        *status = JABBA_OK;
    return JABBA_OK;
}
