// Segment repair for the compression, shared by the kernel and its host-side
// model test.  Plain C++ so the host compiler can build it too.
//
// A domain (Sec. 4.1.1) of many intervals is compressed as several segments
// in parallel, each as if it were a domain: a segment's chain of pieces starts
// at the segment start and its last piece is cut at the segment end.  The
// domain's own chain is then recovered by one walk over its segments in
// order.  From the true chain's position the walk takes the greedy's pieces
// until it lands on a start of the segment's chain; from there the two chains
// coincide (the same greedy from the same point) except for the segment's
// last piece, which is recomputed without the segment end.  Every segment's
// staging region is rewritten in place to hold exactly the true pieces that
// start inside it (there are never more of them than the segment has
// intervals), so the compaction of plain domains applies unchanged.
#pragma once

#include <math.h>
#include <stdint.h>

#include "compress_filter.h"

namespace jabba {

// A unit of work for the compression kernel: a domain, or segment seg of the
// nseg segments of one.
struct Dom {
    int64_t start;
    int32_t nint;
    int32_t series;
    int32_t seg;
    int32_t nseg;
};

// segments of a domain of nint intervals for segment length G
JB_HD inline int32_t n_segments(int32_t nint, int32_t G) { return nint <= G ? 1 : (nint + G - 1) / G; }

// Length of the greedy piece from s inside a domain that ends at point e:
// candidate c = 2, 3, ... is accepted while the definition's sum is within
// (c-1)*tol^2 (decided by filter_decide, else by the sum itself), until the
// domain end or max_len.  v(p) returns point p.
template <class V>
JB_HD int32_t greedy_piece(const V &v, int64_t s, int64_t e, double ts, double tol2, int32_t max_len) {
    double S2 = 0.0, S1 = 0.0;
    for (int32_t c = 2;; ++c) {
        if (s + c > e || (max_len > 0 && c > max_len)) return c - 1;
        const double d = v(s + c - 1) - ts;
        S2 = S2 + d * d;
        S1 = S1 + (double)(c - 1) * d;
        const double te = v(s + c);
        const double b = (te - ts) / (double)c;
        const double thr = (double)(c - 1) * tol2;
        int verdict = filter_decide(S2, S1, b, ts, c, thr);
        if (verdict == 0) {
            double acc = 0.0;
            for (int32_t k = 1; k < c; ++k) {
                double w = b * (double)k;
                w = ts + w;
                const double r = w - v(s + k);
                acc = acc + r * r;
            }
            verdict = (acc <= thr) ? 1 : -1;
        }
        if (verdict < 0) return c - 1;
    }
}

// Repairs the segments doms[d .. d + nseg) of one domain (doms[d].seg == 0).
// On entry st_len/st_inc hold each segment's pieces from its start position
// on and dom_count their number.  On return segment j's true pieces are the
// dom_count[j] entries from index doms[j].start + first[j] (first[j] may be
// negative: free slots after the previous segment's pieces are borrowed), in
// order, and the segments' pieces follow each other inside the domain's
// region.  The kept run of a segment's own pieces is moved only when the
// pieces recomputed in front of it do not fit before it.  Returns 0, or 1 if
// the walk did not end at the domain end (never expected).  *nonfinite is set
// when a recomputed piece ends on a NaN or infinite value.
constexpr int kRepairCache = 8;  // recomputed pieces kept in registers per segment

template <class V>
JB_HD int repair_domain(const V &v, const Dom *doms, int64_t d, double tol2, int32_t max_len, int32_t *st_len,
                        double *st_inc, int32_t *dom_count, int32_t *first, bool *nonfinite) {
    const int32_t nseg = doms[d].nseg;
    const int64_t e = doms[d + nseg - 1].start + doms[d + nseg - 1].nint;
    int64_t pos = doms[d].start;    // start of the next true piece
    int64_t floor = doms[d].start;  // first staging index not holding an earlier true piece
    for (int32_t k = 0; k < nseg; ++k) {
        const int64_t j = d + k;
        const int64_t ps = doms[j].start, pe = ps + doms[j].nint;
        const int32_t cnt = dom_count[j];
        if (pos >= pe) {
            dom_count[j] = 0;
            first[j] = 0;
            continue;
        }
        // p: start of the segment's piece i (pe once i == cnt), the first at or after pos
        int32_t i = 0;
        int64_t p = ps;
        while (i < cnt && p < pos) p += st_len[ps + i++];
        // true pieces from pos until they land on a segment start or leave the segment
        int32_t a = 0;
        int64_t q = pos;
        int32_t cl[kRepairCache];
        double ci[kRepairCache];
        while (q < pe && q != p) {
            const double tq = v(q);
            const int32_t L = greedy_piece(v, q, e, tq, tol2, max_len);
            if (a < kRepairCache) {
                const double tend = v(q + L);
                if (!isfinite(tend)) *nonfinite = true;
                cl[a] = L;
                ci[a] = tend - tq;
            }
            q += L;
            ++a;
            while (i < cnt && p < q) p += st_len[ps + i++];
        }
        const bool synced = q < pe && q == p && i < cnt;
        const int32_t run = synced ? cnt - 1 - i : 0;  // the segment's pieces kept as they are
        const int32_t n_new = synced ? a + run + 1 : a;
        const int64_t p_last = synced ? pe - st_len[ps + cnt - 1] : 0;
        // where the a recomputed pieces go: right before the kept run if there is room
        int64_t dst = ps + i - a;
        if (!synced || dst < floor) dst = floor;
        if (synced && dst + a != ps + i) {
            // move the run (always to the right: dst + a > ps + i here)
            for (int32_t r = run - 1; r >= 0; --r) {
                st_len[dst + a + r] = st_len[ps + i + r];
                st_inc[dst + a + r] = st_inc[ps + i + r];
            }
        }
        int64_t w = pos;
        for (int32_t r = 0; r < a; ++r) {
            int32_t L;
            double dv;
            if (r < kRepairCache) {
                L = cl[r];
                dv = ci[r];
            } else {
                const double tw = v(w);
                L = greedy_piece(v, w, e, tw, tol2, max_len);
                const double tend = v(w + L);
                if (!isfinite(tend)) *nonfinite = true;
                dv = tend - tw;
            }
            st_len[dst + r] = L;
            st_inc[dst + r] = dv;
            w += L;
        }
        if (synced) {
            // the segment's last piece again, free to run past the segment end
            const double tl = v(p_last);
            const int32_t L = greedy_piece(v, p_last, e, tl, tol2, max_len);
            const double tend = v(p_last + L);
            if (!isfinite(tend)) *nonfinite = true;
            st_len[dst + a + run] = L;
            st_inc[dst + a + run] = tend - tl;
            pos = p_last + L;
        } else {
            pos = q;
        }
        dom_count[j] = n_new;
        first[j] = (int32_t)(dst - ps);
        floor = dst + n_new;
    }
    return pos == e ? 0 : 1;
}

}  // namespace jabba
