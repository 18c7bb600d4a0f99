// Decision rule for one candidate piece, shared by the compression kernel and
// its host-side model test.  Plain C++ so the host compiler can build it too.
//
// For a piece starting at s the sequential definition accepts candidate
// length c iff acc <= thr, where acc adds (t_s + b*k - t_{s+k})^2 for
// k = 1..c-1 left to right, b = fl(fl(t_{s+c} - t_s)/c), thr = fl((c-1)*tol^2).
//
// Here the same decision is taken from running sums instead:
//   S2 ~ sum_{k<c} d_k^2 and S1 ~ sum_{k<c} k*d_k with d_k = t_{s+k} - t_s,
//   E  = S2 - 2*b*S1 + b^2*K2 with K2 = sum_{k<c} k^2,
// which equals A = sum (t_s + b*k - t_{s+k})^2 in real arithmetic.
//   errE   bounds |E - A|: rounding of d_k, of the products and of the sums
//          (depth <= c), and of the three-term combination (8u * magnitudes);
//          the cross term uses |b| sum k|d_k| <= (b^2 K2 + S2)/2.
//   accErr bounds |acc - A|: recursive-summation error gamma_{c-2}, the
//          rounding of each square, and per-term errors of the chord value and
//          residual, at most u*(|t_s| + (2+u)|b|k) + u|rho_k| each; summing with
//          Cauchy-Schwarz and AM-GM gives <= u((c+2.05)A + 1.003(c-1)H^2)
//          <= 4cu(A + (c-1)H^2), H = |t_s| + 2|b|(c-1).
// Both are inflated by 1.25 (rounding of the bound itself) plus an absolute
// floor (underflow).  When thr lies outside [E - m, E + m] the verdict is
// certain; otherwise (or for non-finite values) the caller evaluates the
// definition itself.  u = 2^-53.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define JB_HD __host__ __device__
#else
#define JB_HD
#endif

// +1 accept, -1 reject, 0 undecided
JB_HD inline int filter_decide(double S2, double S1, double b, double ts, int32_t c, double thr) {
    const double u = 1.1102230246251565e-16;
    const double cm1 = (double)(c - 1);
    const double cd = (double)c;
    // K2 = sum_{k<c} k^2, an exact integer below c = 2^20 (rounded once to
    // double past 2^53; that relative error u is inside the 8u*ME term)
    double K2;
    if (c <= 1024) {  // the product stays below 2^32
        const uint32_t ci = (uint32_t)c;
        K2 = (double)((ci - 1u) * ci * (2u * ci - 1u) / 6u);
    } else if (c <= (1 << 20)) {
        const int64_t ci = c;
        K2 = (double)((ci - 1) * ci * (2 * ci - 1) / 6);
    } else {
        K2 = cm1 * cd * (2.0 * cd - 1.0) / 6.0;
    }
    const double T1 = (2.0 * b) * S1;
    const double T2 = (b * b) * K2;
    const double E = (S2 - T1) + T2;
    const double ME = S2 + fabs(T1) + T2;
    const double errE = 8.0 * u * ME + (cd + 4.0) * u * (2.0 * S2 + T2);
    double Aup = E + errE;
    Aup = Aup > 0.0 ? Aup : 0.0;
    const double H = fabs(ts) + 2.0000001 * fabs(b) * cm1;
    const double accErr = 4.0 * cd * u * (Aup + cm1 * (H * H));
    const double m = 1.25 * (errE + accErr) + 1e-290;
    const double hi = E + m, lo = E - m;
    if (hi <= thr) return 1;
    if (lo > thr) return -1;
    return 0;
}
