// Host model of the compression kernel's per-group decision procedure, built
// with the product's own decision header: W emulated lanes test candidates
// c0..c0+W-1 of a piece, running sums S2/S1 come from an inclusive lane scan
// plus the carry of earlier rounds, undecided candidates fall back to the
// sequential sum, and the first rejected candidate ends the piece.  Test
// infrastructure: compared against the oracle on the CPU.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "compress_filter.h"

extern "C" {
static long n_undecided = 0, n_cand = 0;
/* emulate one group of W lanes on domain [a, b] (points), returns #pieces */
int64_t sim_domain(const double *t, int64_t a, int64_t e, double tol, int32_t max_len, int W, int32_t *len, double *inc) {
    double tol2 = tol * tol;
    int64_t s = a, np = 0;
    double ts = t[s];
    int32_t c0 = 2;
    double S2c = 0, S1c = 0;
    double S2[64], S1[64];
    int verdict[64];
    while (s < e) {
        /* lanes */
        for (int j = 0; j < W; j++) {
            int32_t c = c0 + j;
            int64_t pk = s + c - 1;
            double a2 = 0, a1 = 0;
            if (pk <= e) { double d = t[pk] - ts; a2 = d * d; a1 = (double)(c - 1) * d; }
            S2[j] = a2; S1[j] = a1;
        }
        /* inclusive scan (Hillis-Steele like the shuffles) */
        for (int o = 1; o < W; o <<= 1) {
            double n2[64], n1[64];
            for (int j = 0; j < W; j++) { n2[j] = S2[j]; n1[j] = S1[j]; if (j >= o) { n2[j] = S2[j] + S2[j - o]; n1[j] = S1[j] + S1[j - o]; } }
            for (int j = 0; j < W; j++) { S2[j] = n2[j]; S1[j] = n1[j]; }
        }
        for (int j = 0; j < W; j++) {
            S2[j] += S2c; S1[j] += S1c;
            int32_t c = c0 + j;
            int valid = (s + c <= e) && (max_len <= 0 || c <= max_len);
            verdict[j] = -1;
            if (valid) {
                double te = t[s + c];
                double b = (te - ts) / (double)c;
                double thr = (double)(c - 1) * tol2;
                n_cand++;
                verdict[j] = filter_decide(S2[j], S1[j], b, ts, c, thr);
                if (verdict[j] == 0) {
                    n_undecided++;
                    double acc = 0;
                    for (int32_t k = 1; k < c; k++) { double v = b * (double)k; v = ts + v; double r = v - t[s + k]; acc = acc + r * r; }
                    verdict[j] = acc <= thr ? 1 : -1;
                }
            }
        }
        int f = -1;
        for (int j = 0; j < W; j++) if (verdict[j] < 0) { f = j; break; }
        if (f >= 0) {
            int32_t L = c0 + f - 1;
            double tend = t[s + L];
            len[np] = L; inc[np] = tend - ts; np++;
            s += L; ts = tend; c0 = 2; S2c = 0; S1c = 0;
        } else { c0 += W; S2c = S2[W - 1]; S1c = S1[W - 1]; }
    }
    return np;
}
int64_t sim_compress(const double *t, const int64_t *off, int64_t ns, int32_t D, double tol, int32_t max_len, int W, int32_t *len, double *inc) {
    int64_t np = 0;
    for (int64_t s = 0; s < ns; s++) {
        int64_t lo = off[s], n = off[s + 1] - off[s];
        for (int64_t a = 0; a + 1 < n; a += D) {
            int64_t b = a + D < n - 1 ? a + D : n - 1;
            np += sim_domain(t, lo + a, lo + b, tol, max_len, W, len + np, inc + np);
        }
    }
    return np;
}
long get_undecided(void) { return n_undecided; }
long get_cand(void) { return n_cand; }
void reset_counts(void) { n_undecided = 0; n_cand = 0; }
}
