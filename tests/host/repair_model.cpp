// Host model of the segmented compression: every domain is cut into segments
// of G intervals, each segment compressed as its own domain with the kernel's
// greedy_piece, then repaired with the kernel's repair_domain and compacted.
// The result must be the domain-by-domain compression.
#include <stdint.h>

#include <vector>

#include "compress_repair.h"

using jabba::Dom;

namespace {
struct HostValues {
    const double *t;
    double operator()(int64_t p) const { return t[p]; }
};
}  // namespace

extern "C" int64_t seg_compress(const double *vals, const int64_t *off, int64_t ns, int32_t D, int32_t G, double tol,
                                int32_t max_len, int32_t *len, double *inc, int64_t *n_repaired) {
    const double tol2 = tol * tol;
    std::vector<Dom> doms;
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t lo = off[s], n = off[s + 1] - off[s];
        for (int64_t a = 0; a + 1 < n; a += D) {
            const int64_t b = a + D < n - 1 ? a + D : n - 1;
            const int32_t nint = (int32_t)(b - a);
            const int32_t nseg = jabba::n_segments(nint, G);
            for (int32_t k = 0; k < nseg; ++k) {
                const int64_t sa = a + (int64_t)k * G;
                const int64_t sb = k == nseg - 1 ? b : sa + G;
                doms.push_back(Dom{lo + sa, (int32_t)(sb - sa), (int32_t)s, k, nseg});
            }
        }
    }
    const int64_t total = off[ns];
    std::vector<int32_t> st_len(total > 0 ? total : 1);
    std::vector<double> st_inc(total > 0 ? total : 1);
    std::vector<int32_t> cnt(doms.size());
    std::vector<int32_t> first(doms.size(), 0);
    HostValues v{vals};
    for (size_t j = 0; j < doms.size(); ++j) {
        int64_t p = doms[j].start;
        const int64_t e = p + doms[j].nint;
        int32_t np = 0;
        while (p < e) {
            const double ts = v(p);
            const int32_t L = jabba::greedy_piece(v, p, e, ts, tol2, max_len);
            st_len[doms[j].start + np] = L;
            st_inc[doms[j].start + np] = v(p + L) - ts;
            ++np;
            p += L;
        }
        cnt[j] = np;
    }
    *n_repaired = 0;
    for (size_t j = 0; j < doms.size(); ++j) {
        if (doms[j].seg != 0 || doms[j].nseg <= 1) continue;
        bool nonfinite = false;
        if (jabba::repair_domain(v, doms.data(), (int64_t)j, tol2, max_len, st_len.data(), st_inc.data(), cnt.data(),
                                 first.data(), &nonfinite))
            return -1;
        ++*n_repaired;
    }
    int64_t o = 0;
    for (size_t j = 0; j < doms.size(); ++j) {
        const int64_t src = doms[j].start + (doms[j].nseg > 1 ? first[j] : 0);
        for (int32_t i = 0; i < cnt[j]; ++i) {
            len[o] = st_len[src + i];
            inc[o] = st_inc[src + i];
            ++o;
        }
    }
    return o;
}
