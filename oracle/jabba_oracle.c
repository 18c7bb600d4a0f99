/*
 * CPU oracle for the joint symbolic approximation (JABBA) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product links or calls this file;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
 * is a plain, slow, single-threaded FP64 transcription of the method, written
 * from the paper (arXiv 2401.00109) and sharing no code with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (no fused multiply-add, no reassociation: every FP operation below is one
 * IEEE-754 binary64 operation, rounded to nearest, in the order written).
 *
 * Where the paper is silent or garbled, the reading used here is stated at
 * the function; all readings are listed together in the design notes.
 *
 * Parity pins: every function here is checked by tests against closed forms,
 * brute force with exact rational arithmetic, library routines or invariants
 * the paper states; none is "parity unpinned" except where noted at the
 * function (Stage II block rule, see jo_digitize).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define JO_OK 0
#define JO_EINVAL (-1)
#define JO_ENOMEM (-2)
#define JO_ENONFINITE (-5)
#define JO_ECAPACITY (-4)

typedef __int128 i128;

/* ------------------------------------------------------------------------ */
/* Phase I: domain construction (Alg. 1, Phase I; Sec. 4.1.1).                */
/*                                                                          */
/* Series s holds points t_0..t_{n-1}.  Its n-1 unit intervals are cut into   */
/* chunks of D intervals; chunk d covers points [d*D, min((d+1)*D, n-1)], so  */
/* consecutive chunks share their end point (s_{k+1} = e_k in Sec. 4.1.1).    */
/* A series with n <= 1 has no interval and therefore no domain.              */
/* ------------------------------------------------------------------------ */
int64_t jo_count_domains(const int64_t *series_off, int64_t n_series, int32_t D)
{
    int64_t total = 0;
    for (int64_t s = 0; s < n_series; s++) {
        int64_t n = series_off[s + 1] - series_off[s];
        if (n >= 2) total += (n - 1 + D - 1) / D;
    }
    return total;
}

int jo_domains(const int64_t *series_off, int64_t n_series, int32_t D,
               int64_t *dom_series, int64_t *dom_start, int64_t *dom_nint)
{
    if (D < 1) return JO_EINVAL;
    int64_t m = 0;
    for (int64_t s = 0; s < n_series; s++) {
        int64_t n = series_off[s + 1] - series_off[s];
        if (n < 2) continue;
        for (int64_t a = 0; a < n - 1; a += D) {
            int64_t b = a + D < n - 1 ? a + D : n - 1;
            dom_series[m] = s;
            dom_start[m] = series_off[s] + a;
            dom_nint[m] = b - a;
            m++;
        }
    }
    return JO_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase II: greedy compression of one domain (Sec. 3.1, Eq. compress).       */
/*                                                                          */
/* From the current piece start s the piece is grown one point at a time.     */
/* A candidate piece of length c (end point s+c) is accepted when the squared */
/* distance of the interior points from the chord t_s -> t_{s+c} is at most   */
/* (c-1)*tol^2.  The piece ends just before the first rejected candidate      */
/* ("first failure"); a length-1 piece is always accepted (empty sum).        */
/*                                                                          */
/* Readings: the chord value at offset k is t_s + slope*k with               */
/* slope = (t_{s+c} - t_s)/c (the paper's fraction, slope taken first); the   */
/* sum runs over the interior offsets k = 1..c-1 in ascending order (the two  */
/* end terms vanish exactly in the paper's formula); acceptance is            */
/* acc <= (c-1)*(tol*tol); a domain end or max_len > 0 also stops a piece.    */
/* inc = t_{s+L} - t_s (Sec. 3.1, after Eq. compress).                        */
/* ------------------------------------------------------------------------ */
static int64_t compress_domain(const double *t, int64_t a, int64_t b, double tol, int32_t max_len,
                               int32_t *len, double *inc)
{
    const double tol2 = tol * tol;
    int64_t np = 0;
    int64_t s = a;
    while (s < b) {
        int64_t L = 1;
        for (;;) {
            int64_t c = L + 1;
            if (s + c > b) break;
            if (max_len > 0 && c > max_len) break;
            double slope = (t[s + c] - t[s]) / (double)c;
            double acc = 0.0;
            for (int64_t k = 1; k < c; k++) {
                double v = slope * (double)k;
                v = t[s] + v;
                double r = v - t[s + k];
                acc = acc + r * r;
            }
            double thr = (double)(c - 1) * tol2;
            if (acc <= thr)
                L = c;
            else
                break;
        }
        len[np] = (int32_t)L;
        inc[np] = t[s + L] - t[s];
        np++;
        s += L;
    }
    return np;
}

/*
 * Compress every series: domains in order, pieces of a series concatenated in
 * domain order (Sec. 4.1.3, P = P^(1) (+) ... (+) P^(M)).  len/inc must hold
 * sum(max(n_s - 1, 0)) entries; piece_off gets n_series + 1 offsets.
 * Returns the number of pieces, or a negative status.
 */
int64_t jo_compress(const double *t, const int64_t *series_off, int64_t n_series, int32_t D, double tol,
                    int32_t max_len, int32_t *len, double *inc, int64_t *piece_off)
{
    if (D < 1 || !(tol >= 0.0) || max_len < 0) return JO_EINVAL;
    for (int64_t i = 0; i < series_off[n_series]; i++)
        if (!isfinite(t[i])) return JO_ENONFINITE;
    int64_t np = 0;
    for (int64_t s = 0; s < n_series; s++) {
        piece_off[s] = np;
        int64_t lo = series_off[s], n = series_off[s + 1] - series_off[s];
        for (int64_t a = 0; a + 1 < n; a += D) {
            int64_t b = a + D < n - 1 ? a + D : n - 1;
            np += compress_domain(t, lo + a, lo + b, tol, max_len, len + np, inc + np);
        }
    }
    piece_off[n_series] = np;
    return np;
}

/* ------------------------------------------------------------------------ */
/* Sums.                                                                      */
/* ------------------------------------------------------------------------ */

/*
 * Balanced binary (pairwise) sum: the leaves a[0..n) are zero-padded to the
 * next power of two P and the sum is sum(a[0:P/2]) + sum(a[P/2:P]), applied
 * recursively.  This is the fixed summation order used for the standard
 * deviation of the increments, so that the result does not depend on how the
 * work is split.
 */
static double tree_rec(const double *a, int64_t n, int64_t lo, int64_t size)
{
    if (lo >= n) return 0.0;
    if (size == 1) return a[lo];
    int64_t h = size / 2;
    double l = tree_rec(a, n, lo, h);
    double r = tree_rec(a, n, lo + h, h);
    return l + r;
}

double jo_tree_sum(const double *a, int64_t n)
{
    if (n <= 0) return 0.0;
    int64_t P = 1;
    while (P < n) P <<= 1;
    return tree_rec(a, n, 0, P);
}

/*
 * Series z-normalisation ahead of compression: per series of n points
 * mean = T(v)/n and std = sqrt(T((v - mean)^2)/n) (population deviation, T the
 * pairwise sum above), a zero deviation (n = 1, a constant series) replaced
 * by 1 so the series is only centred; z_i = (v_i - mean)/std.  An empty
 * series has mean 0 and std 1.
 */
int jo_znorm(const double *values, const int64_t *series_off, int64_t n_series, double *mean, double *std_dev,
             double *out)
{
    for (int64_t s = 0; s < n_series; s++) {
        const int64_t a = series_off[s], n = series_off[s + 1] - a;
        if (n <= 0) {
            mean[s] = 0.0;
            std_dev[s] = 1.0;
            continue;
        }
        double m = jo_tree_sum(values + a, n) / (double)n;
        double *sq = (double *)malloc((size_t)n * sizeof(double));
        if (!sq) return JO_ENOMEM;
        for (int64_t i = 0; i < n; i++) {
            double d = values[a + i] - m;
            sq[i] = d * d;
        }
        double var = jo_tree_sum(sq, n) / (double)n;
        free(sq);
        double sd = sqrt(var);
        if (!(sd > 0.0)) sd = 1.0;
        mean[s] = m;
        std_dev[s] = sd;
        for (int64_t i = 0; i < n; i++) out[a + i] = (values[a + i] - m) / sd;
    }
    return JO_OK;
}

/*
 * Exact sum rounded once to binary64: the running sum is kept as a list of
 * non-overlapping partials updated with error-free two-sum steps (Shewchuk,
 * "Adaptive precision floating-point arithmetic", 1997), then the partials
 * are added from the largest down with a final half-way correction.  The
 * partials update and the half-way correction follow CPython's math.fsum,
 * which implements the same method and which the tests pin this sum against.
 * Used for the dictionary means, whose reference value is the mean of the
 * members.
 */
typedef struct {
    double *p;
    int64_t n, cap;
} expansion;

static int exp_add(expansion *e, double x)
{
    int64_t i = 0;
    for (int64_t j = 0; j < e->n; j++) {
        double y = e->p[j];
        if (fabs(x) < fabs(y)) {
            double tmp = x;
            x = y;
            y = tmp;
        }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0) e->p[i++] = lo;
        x = hi;
    }
    if (i >= e->cap) {
        int64_t nc = e->cap ? 2 * e->cap : 16;
        double *np = (double *)realloc(e->p, (size_t)nc * sizeof(double));
        if (!np) return JO_ENOMEM;
        e->p = np;
        e->cap = nc;
    }
    e->p[i++] = x;
    e->n = i;
    return JO_OK;
}

static double exp_round(const expansion *e)
{
    int64_t n = e->n;
    if (n == 0) return 0.0;
    double hi = e->p[--n];
    double lo = 0.0;
    while (n > 0) {
        double x = hi;
        double y = e->p[--n];
        hi = x + y;
        double yr = hi - x;
        lo = y - yr;
        if (lo != 0.0) break;
    }
    /* Half-way case: the remaining partials decide the direction. */
    if (n > 0 && ((lo < 0.0 && e->p[n - 1] < 0.0) || (lo > 0.0 && e->p[n - 1] > 0.0))) {
        double y = lo * 2.0;
        double x = hi + y;
        double yr = x - hi;
        if (y == yr) hi = x;
    }
    return hi;
}

double jo_exact_sum(const double *a, int64_t n)
{
    expansion e = {0, 0, 0};
    for (int64_t i = 0; i < n; i++)
        if (exp_add(&e, a[i]) != JO_OK) {
            free(e.p);
            return NAN;
        }
    double r = exp_round(&e);
    free(e.p);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Phase III-a: scaling (Sec. 3.2, Eq. tupseq2).                               */
/*                                                                          */
/* sigma_len and sigma_inc are population standard deviations (ddof 0).       */
/* Lengths: exact integer sums S1 = sum len, S2 = sum len^2, then             */
/*   var = S2/N - (S1/N)^2 (clamped at 0).                                    */
/* Increments: two passes with the balanced pairwise sum above,              */
/*   mean = T(inc)/N, var = T((inc - mean)^2)/N.                              */
/* A zero deviation (and N <= 1) is replaced by 1.  Every piece is scaled the */
/* same way: x = scl*(len/sigma_len), y = inc/sigma_inc (the garbled subscripts */
/* of Eq. tupseq2 are read as "all N pieces").  The sort key is the 2-norm    */
/* key = sqrt(x*x + y*y) (Sec. 5 names the norm as one choice of key).        */
/* ------------------------------------------------------------------------ */
int jo_scaling(const int32_t *len, const double *inc, int64_t N, double scl, double *sigma_len,
               double *sigma_inc, double *x, double *y, double *key)
{
    double sl = 1.0, si = 1.0;
    if (N > 0) {
        int64_t S1 = 0, S2 = 0;
        for (int64_t i = 0; i < N; i++) {
            S1 += len[i];
            S2 += (int64_t)len[i] * (int64_t)len[i];
        }
        double mean_len = (double)S1 / (double)N;
        double var_len = (double)S2 / (double)N - mean_len * mean_len;
        if (var_len < 0.0) var_len = 0.0;
        sl = sqrt(var_len);

        double mean_inc = jo_tree_sum(inc, N) / (double)N;
        double *sq = (double *)malloc((size_t)N * sizeof(double));
        if (!sq) return JO_ENOMEM;
        for (int64_t i = 0; i < N; i++) {
            double d = inc[i] - mean_inc;
            sq[i] = d * d;
        }
        double var_inc = jo_tree_sum(sq, N) / (double)N;
        free(sq);
        si = sqrt(var_inc);
        if (!(sl > 0.0)) sl = 1.0;
        if (!(si > 0.0)) si = 1.0;
    }
    *sigma_len = sl;
    *sigma_inc = si;
    if (x)
        for (int64_t i = 0; i < N; i++) {
            double xi = scl * ((double)len[i] / sl);
            double yi = inc[i] / si;
            x[i] = xi;
            y[i] = yi;
            key[i] = sqrt(xi * xi + yi * yi);
        }
    return JO_OK;
}

/* ------------------------------------------------------------------------ */
/* PCA sort key (Sec. 5 allows the projection on a principal axis in place of  */
/* the norm).  The points are the scaled pieces p_i = (x_i, y_i).  Their       */
/* population covariance follows from the scaling itself:                    */
/*   var(x)    = scl^2 * var_len / sigma_len^2  = scl^2 (0 when var_len = 0), */
/*   var(y)    = var_inc / sigma_inc^2          = 1     (0 when var_inc = 0), */
/*   cov(x, y) = scl * cov(len, inc) / (sigma_len * sigma_inc),               */
/* where cov(len, inc) = T((len_i - S1/N) * (inc_i - T(inc)/N)) / N with the   */
/* pairwise tree T of the increment deviation (and 0 when either variance is  */
/* 0).  For the symmetric matrix [[a, c], [c, b]] the larger eigenvalue is     */
/* l = (a + b)/2 + r, r = sqrt(((a - b)/2)^2 + c^2); an eigenvector is         */
/* (l - b, c) = (h + r, c) and also (c, l - a) = (c, r - h), h = (a - b)/2;    */
/* the form whose first entry has no cancellation is taken (h >= 0: the       */
/* first), normalised, and signed so that its first nonzero entry is          */
/* positive.  c = 0 gives the coordinate axis of the larger variance (x on a  */
/* tie).  The key is u_x*x_i + u_y*y_i, with -0 taken as +0.  Only +, -, *, / */
/* and sqrt appear, all correctly rounded.                                    */
/* ------------------------------------------------------------------------ */
int jo_pca_axis(const int32_t *len, const double *inc, int64_t N, double scl, double *axis)
{
    double a = 0.0, b = 0.0, c = 0.0;
    if (N > 0) {
        int64_t S1 = 0, S2 = 0;
        for (int64_t i = 0; i < N; i++) {
            S1 += len[i];
            S2 += (int64_t)len[i] * (int64_t)len[i];
        }
        double mean_len = (double)S1 / (double)N;
        double var_len = (double)S2 / (double)N - mean_len * mean_len;
        if (var_len < 0.0) var_len = 0.0;
        double sl = sqrt(var_len);
        double mean_inc = jo_tree_sum(inc, N) / (double)N;
        double *t = (double *)malloc((size_t)N * sizeof(double));
        if (!t) return JO_ENOMEM;
        for (int64_t i = 0; i < N; i++) {
            double d = inc[i] - mean_inc;
            t[i] = d * d;
        }
        double var_inc = jo_tree_sum(t, N) / (double)N;
        for (int64_t i = 0; i < N; i++) t[i] = ((double)len[i] - mean_len) * (inc[i] - mean_inc);
        double cov = jo_tree_sum(t, N) / (double)N;
        free(t);
        double si = sqrt(var_inc);
        if (var_len > 0.0 && sl > 0.0) a = scl * scl;
        if (var_inc > 0.0 && si > 0.0) b = 1.0;
        if (a > 0.0 && b > 0.0) c = scl * ((cov / sl) / si);
    }
    double ux, uy;
    if (c == 0.0) {
        ux = a >= b ? 1.0 : 0.0;
        uy = a >= b ? 0.0 : 1.0;
    } else {
        double h = 0.5 * (a - b);
        double r = sqrt(h * h + c * c);
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
        double n = sqrt(vx * vx + vy * vy);
        ux = vx / n;
        uy = vy / n;
    }
    axis[0] = ux;
    axis[1] = uy;
    return JO_OK;
}

/* ------------------------------------------------------------------------ */
/* Sort (Sec. 5: one global sorting index).  Ascending key; equal keys keep   */
/* the canonical piece order.                                                 */
/* ------------------------------------------------------------------------ */
static const double *g_sort_key;
static int cmp_key_idx(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    double ka = g_sort_key[a], kb = g_sort_key[b];
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (a > b) - (a < b);
}

void jo_sort_order(const double *key, int64_t N, int64_t *perm)
{
    for (int64_t i = 0; i < N; i++) perm[i] = i;
    g_sort_key = key;
    qsort(perm, (size_t)N, sizeof(int64_t), cmp_key_idx);
}

/*
 * Contiguous blocks of the sorted order (Sec. 5, Stage I).  The paper splits
 * the sorted pieces into M contiguous blocks without a sizing rule; here a
 * block holds B pieces, and each nominal cut j*B is moved forward past any run
 * of equal keys so that equal keys never straddle two blocks.  Cuts that
 * collapse onto an earlier cut or onto N are dropped.
 * Writes block starts into bstart[0..M] (bstart[M] = N); returns M.
 */
int64_t jo_blocks(const double *skey, int64_t N, int64_t B, int64_t *bstart)
{
    if (N == 0) {
        bstart[0] = 0;
        return 0;
    }
    int64_t M = 0;
    bstart[M++] = 0;
    for (int64_t j = 1; j * B < N; j++) {
        int64_t p = j * B;
        while (p < N && skey[p] == skey[p - 1]) p++;
        if (p < N && p > bstart[M - 1]) bstart[M++] = p;
    }
    bstart[M] = N;
    return M;
}

/*
 * Greedy aggregation of presorted points (fABBA's aggregation, Sec. 3.2 and
 * the pruning rule of Sec. 5).  Points are visited in the given (sorted)
 * order; an unassigned point p opens a group; the points q after p are
 * scanned while key[q] - key[p] <= alpha (the early stop), and an unassigned
 * q joins p's group when (x_q - x_p)^2 + (y_q - y_p)^2 <= alpha^2.
 * lab[i] receives the position (within [lo, hi)) of the group's start.
 */
static void aggregate_range(const double *sx, const double *sy, const double *skey, int64_t lo, int64_t hi,
                            double alpha, int64_t *lab)
{
    const double a2 = alpha * alpha;
    for (int64_t i = lo; i < hi; i++) lab[i] = -1;
    for (int64_t p = lo; p < hi; p++) {
        if (lab[p] != -1) continue;
        lab[p] = p;
        for (int64_t q = p + 1; q < hi; q++) {
            if (!(skey[q] - skey[p] <= alpha)) break;
            if (lab[q] != -1) continue;
            double dx = sx[q] - sx[p];
            double dy = sy[q] - sy[p];
            double d2 = dx * dx + dy * dy;
            if (d2 <= a2) lab[q] = p;
        }
    }
}

/* Serial greedy aggregation over arrays already in sorted order. */
void jo_aggregate_sorted(const double *sx, const double *sy, const double *skey, int64_t n, double alpha,
                         int64_t *lab)
{
    aggregate_range(sx, sy, skey, 0, n, alpha, lab);
}

/*
 * Steps 2-4 of Phase III on points that are already in their final
 * coordinates: global sort by key (ties by index), Stage I in every block,
 * Stage II over the starting points, label propagation.  Returns k or
 * JO_ENOMEM; the optional outputs are those of jo_digitize.
 */
static int64_t two_stage(const double *x, const double *y, const double *key, int64_t N, double alpha, int64_t B,
                         int32_t *symbols, int64_t *perm_out, int64_t *local_start_out, int64_t *n_starts_out,
                         int64_t *gmap_out, int64_t *n_blocks_out)
{
    int64_t k = 0, rc = JO_ENOMEM;
    double *sx = malloc((size_t)(N + 1) * sizeof(double));
    double *sy = malloc((size_t)(N + 1) * sizeof(double));
    double *sk = malloc((size_t)(N + 1) * sizeof(double));
    int64_t *perm = malloc((size_t)(N + 1) * sizeof(int64_t));
    int64_t *lab = malloc((size_t)(N + 1) * sizeof(int64_t));
    int64_t *bstart = malloc((size_t)(N + 2) * sizeof(int64_t));
    int64_t *sidx = malloc((size_t)(N + 1) * sizeof(int64_t));
    double *gx = calloc((size_t)(N + 1), sizeof(double));
    double *gy = calloc((size_t)(N + 1), sizeof(double));
    double *gk = calloc((size_t)(N + 1), sizeof(double));
    int64_t *glab = malloc((size_t)(N + 1) * sizeof(int64_t));
    int64_t *gsym = malloc((size_t)(N + 1) * sizeof(int64_t));
    if (!sx || !sy || !sk || !perm || !lab || !bstart || !sidx || !gx || !gy || !gk || !glab || !gsym) goto done;

    jo_sort_order(key, N, perm);
    for (int64_t i = 0; i < N; i++) {
        sx[i] = x[perm[i]];
        sy[i] = y[perm[i]];
        sk[i] = key[perm[i]];
    }

    /* Stage I */
    int64_t M = jo_blocks(sk, N, B, bstart);
    if (n_blocks_out) *n_blocks_out = M;
    for (int64_t b = 0; b < M; b++) aggregate_range(sx, sy, sk, bstart[b], bstart[b + 1], alpha, lab);

    /* starting points in sorted order */
    int64_t G = 0;
    for (int64_t i = 0; i < N; i++) {
        if (lab[i] == i) {
            sidx[i] = G;
            gx[G] = sx[i];
            gy[G] = sy[i];
            gk[G] = sk[i];
            G++;
        } else
            sidx[i] = -1;
    }
    if (n_starts_out) *n_starts_out = G;

    /* Stage II */
    aggregate_range(gx, gy, gk, 0, G, alpha, glab);
    for (int64_t g = 0; g < G; g++) gsym[g] = (glab[g] == g) ? k++ : -1;
    for (int64_t g = 0; g < G; g++) gsym[g] = gsym[glab[g]];
    if (gmap_out)
        for (int64_t g = 0; g < G; g++) gmap_out[g] = gsym[g];

    /* label propagation */
    for (int64_t i = 0; i < N; i++) {
        int64_t sym = gsym[sidx[lab[i]]];
        symbols[perm[i]] = (int32_t)sym;
    }
    if (perm_out)
        for (int64_t i = 0; i < N; i++) perm_out[i] = perm[i];
    if (local_start_out)
        for (int64_t i = 0; i < N; i++) local_start_out[i] = lab[i];

    rc = k;
done:
    free(sx);
    free(sy);
    free(sk);
    free(perm);
    free(lab);
    free(bstart);
    free(sidx);
    free(gx);
    free(gy);
    free(gk);
    free(glab);
    free(gsym);
    return rc;
}

/*
 * Phase III: two-stage digitization (Sec. 5) and the dictionary.
 *
 *  1. scaling and key (jo_scaling; with key_kind 1 the projection on the
 *     principal axis of jo_pca_axis), global sort (jo_sort_order);
 *  2. Stage I: aggregation inside every block of B sorted pieces;
 *  3. Stage II: the same aggregation over the collected starting points,
 *     which are a subsequence of the sorted order and so already sorted;
 *  4. label propagation: a piece's symbol is the global group of its local
 *     group's start (Eq. l_i = l~_g), with no second distance pass;
 *  5. dictionary: per symbol the member count, exact integer length sum and
 *     the exact increment sum; center = mean of the members' raw (len, inc)
 *     (Sec. 3.2, "aggregated group means"), scaled centers
 *     cx = scl*(center_len/sigma_len), cy = center_inc/sigma_inc.
 *
 * Local groups and global symbols are numbered in increasing sorted position
 * of their starts.  The block rule (B pieces, cuts moved past equal keys) and
 * "Stage II merges starting points" are readings of Sec. 5; beyond the two
 * reductions pinned by tests (B >= N and, with distinct keys, B = 1 both equal
 * the serial aggregation) the block rule is parity unpinned against the paper.
 *
 * Outputs (any may be NULL except symbols and k):
 *   symbols[N]          symbol per piece, canonical order
 *   perm[N]             sorted position -> canonical index
 *   local_start[N]      per sorted position, sorted position of its local start
 *   n_starts            G, number of Stage I starting points
 *   gmap[N]             per Stage I start (numbered 0..G-1), its global symbol
 *   sigma[2]            sigma_len, sigma_inc
 *   center_len/inc, cx, cy, count: capacity entries
 * Returns k (number of symbols) or a negative status.
 */
int64_t jo_digitize_key(const int32_t *len, const double *inc, int64_t N, double alpha, double scl, int64_t B,
                        int key_kind, double *axis_out, int64_t capacity, int32_t *symbols, int64_t *perm_out,
                        int64_t *local_start_out, int64_t *n_starts_out, int64_t *gmap_out, double *sigma,
                        double *center_len, double *center_inc, double *cx, double *cy, int64_t *count,
                        int64_t *n_blocks_out)
{
    if (key_kind != 0 && key_kind != 1) return JO_EINVAL;
    if (!(alpha >= 0.0) || !(scl >= 0.0) || B < 1 || N < 0) return JO_EINVAL;
    for (int64_t i = 0; i < N; i++)
        if (!isfinite(inc[i]) || len[i] < 1) return JO_EINVAL;
    int rc = JO_ENOMEM;
    int64_t k = 0;
    double sl = 1.0, si = 1.0;
    double *x = malloc((size_t)(N + 1) * sizeof(double));
    double *y = malloc((size_t)(N + 1) * sizeof(double));
    double *key = malloc((size_t)(N + 1) * sizeof(double));
    if (!x || !y || !key) goto done;

    rc = jo_scaling(len, inc, N, scl, &sl, &si, x, y, key);
    if (rc != JO_OK) goto done;
    if (key_kind == 1) {
        double u[2];
        rc = jo_pca_axis(len, inc, N, scl, u);
        if (rc != JO_OK) goto done;
        for (int64_t i = 0; i < N; i++) {
            double kv = u[0] * x[i] + u[1] * y[i];
            key[i] = kv == 0.0 ? 0.0 : kv;
        }
        if (axis_out) {
            axis_out[0] = u[0];
            axis_out[1] = u[1];
        }
    }
    if (sigma) {
        sigma[0] = sl;
        sigma[1] = si;
    }
    k = two_stage(x, y, key, N, alpha, B, symbols, perm_out, local_start_out, n_starts_out, gmap_out, n_blocks_out);
    if (k < 0) {
        rc = (int)k;
        goto done;
    }

    /* dictionary */
    rc = JO_OK;
    if (k > capacity) {
        rc = JO_ECAPACITY;
    } else if (count) {
        int64_t *slen = calloc((size_t)(k + 1), sizeof(int64_t));
        int64_t *cnt = calloc((size_t)(k + 1), sizeof(int64_t));
        expansion *ex = calloc((size_t)(k + 1), sizeof(expansion));
        if (!slen || !cnt || !ex) rc = JO_ENOMEM;
        for (int64_t i = 0; rc == JO_OK && i < N; i++) {
            int64_t c = symbols[i];
            cnt[c] += 1;
            slen[c] += len[i];
            rc = exp_add(&ex[c], inc[i]);
        }
        for (int64_t c = 0; rc == JO_OK && c < k; c++) {
            double cl = (double)slen[c] / (double)cnt[c];
            double ci = exp_round(&ex[c]) / (double)cnt[c];
            count[c] = cnt[c];
            center_len[c] = cl;
            center_inc[c] = ci;
            cx[c] = scl * (cl / sl);
            cy[c] = ci / si;
        }
        if (ex)
            for (int64_t c = 0; c < k; c++) free(ex[c].p);
        free(slen);
        free(cnt);
        free(ex);
    }
done:
    free(x);
    free(y);
    free(key);
    return rc == JO_OK ? k : rc;
}

/*
 * Two-stage aggregation of 2-D points as given (Sec. 5; the Gaussian-blob
 * experiment of Sec. 7.1 aggregates raw points and compares the two-stage
 * result with the serial greedy aggregation, which is the case B >= N).
 * key = sqrt(x*x + y*y); labels by steps 2-4 of Phase III.  Centers: the
 * member count and the means of x and of y with the members added one by
 * one in input order.  SSE (Eq. sse): the exact sum over the points of
 * (x - cx)^2 + (y - cy)^2, each term rounded as written.
 * Returns k, JO_ECAPACITY when k > capacity (labels and k still valid), or
 * another negative status.
 */
int64_t jo_aggregate_points(const double *x, const double *y, int64_t N, double alpha, int64_t B, int64_t capacity,
                            int32_t *labels, double *cx, double *cy, int64_t *count, double *sse, int64_t *n_starts_out,
                            int64_t *n_blocks_out)
{
    if (!(alpha >= 0.0) || B < 1 || N < 0) return JO_EINVAL;
    for (int64_t i = 0; i < N; i++)
        if (!isfinite(x[i]) || !isfinite(y[i])) return JO_EINVAL;
    double *key = malloc((size_t)(N + 1) * sizeof(double));
    if (!key) return JO_ENOMEM;
    for (int64_t i = 0; i < N; i++) key[i] = sqrt(x[i] * x[i] + y[i] * y[i]);
    int64_t k = two_stage(x, y, key, N, alpha, B, labels, NULL, NULL, n_starts_out, NULL, n_blocks_out);
    free(key);
    if (k < 0) return k;
    if (k > capacity) return JO_ECAPACITY;
    for (int64_t c = 0; c < k; c++) {
        cx[c] = 0.0;
        cy[c] = 0.0;
        count[c] = 0;
    }
    for (int64_t i = 0; i < N; i++) {
        int64_t c = labels[i];
        cx[c] = cx[c] + x[i];
        cy[c] = cy[c] + y[i];
        count[c] += 1;
    }
    for (int64_t c = 0; c < k; c++) {
        cx[c] = cx[c] / (double)count[c];
        cy[c] = cy[c] / (double)count[c];
    }
    if (sse) {
        double *t = malloc((size_t)(N + 1) * sizeof(double));
        if (!t) return JO_ENOMEM;
        for (int64_t i = 0; i < N; i++) {
            const double dx = x[i] - cx[labels[i]];
            const double dy = y[i] - cy[labels[i]];
            t[i] = dx * dx + dy * dy;
        }
        *sse = jo_exact_sum(t, N);
        free(t);
    }
    return k;
}

/* The two-stage digitization with the norm key. */
int64_t jo_digitize(const int32_t *len, const double *inc, int64_t N, double alpha, double scl, int64_t B,
                    int64_t capacity, int32_t *symbols, int64_t *perm_out, int64_t *local_start_out,
                    int64_t *n_starts_out, int64_t *gmap_out, double *sigma, double *center_len,
                    double *center_inc, double *cx, double *cy, int64_t *count, int64_t *n_blocks_out)
{
    return jo_digitize_key(len, inc, N, alpha, scl, B, 0, NULL, capacity, symbols, perm_out, local_start_out,
                           n_starts_out, gmap_out, sigma, center_len, center_inc, cx, cy, count, n_blocks_out);
}

/* ------------------------------------------------------------------------ */
/* Inverse symbolization (Sec. 3.3).                                          */
/*                                                                          */
/* Inverse digitization: each symbol is replaced by its center              */
/* (len~_j, inc~_j).  Quantization: len^_1 = round(len~_1), e = len~_1 -      */
/* len^_1, then len^_j = round(len~_j + e) and the carry becomes              */
/* e = (len~_j + e) - len^_j (the paper prints the carry with the opposite    */
/* sign; this reading keeps sum(len^) equal to round(sum(len~)) at every      */
/* step).  The carry is held exactly: a center length >= 1 is an integer      */
/* multiple of 2^-52, so every quantity is an exact 128-bit fixed-point       */
/* number at scale 2^52, and round() sends halves away from zero.  Inverse    */
/* compression starts at t_0; V_j = V_{j-1} + inc^_j (sequential), the piece's */
/* interior points are V_{j-1} + (inc^_j/len^_j)*k for 0 < k < len^_j, and the */
/* piece ends at V_j.  The output has 1 + sum(len^) points per series with     */
/* pieces, one point (t_0) for a single-point series and none for an empty    */
/* one.                                                                       */
/* ------------------------------------------------------------------------ */
#define FIX_SHIFT 52

static int to_fixed(double v, i128 *out)
{
    if (!isfinite(v) || v < 0.0) return JO_EINVAL;
    if (v == 0.0) {
        *out = 0;
        return JO_OK;
    }
    int e;
    double m = frexp(v, &e);                 /* v = m * 2^e, 0.5 <= m < 1 */
    int64_t mi = (int64_t)ldexp(m, 53);      /* exact 53-bit significand  */
    int sh = e - 53 + FIX_SHIFT;             /* v * 2^52 = mi * 2^sh      */
    if (sh < 0) {
        if (mi & (((int64_t)1 << -sh) - 1)) return JO_EINVAL; /* not a multiple of 2^-52 */
        *out = (i128)(mi >> -sh);
    } else {
        if (sh > 60) return JO_EINVAL;
        *out = (i128)mi << sh;
    }
    return JO_OK;
}

/* round-half-away-from-zero of a non-negative fixed-point value, as integer */
static int64_t fixed_round(i128 v)
{
    return (int64_t)((v + ((i128)1 << (FIX_SHIFT - 1))) >> FIX_SHIFT);
}

/*
 * Per-series output sizes.  out_off gets n_series + 1 offsets.
 * Returns JO_OK or a negative status.
 */
int jo_reconstruct_size(const int32_t *symbols, const int64_t *piece_off, const int64_t *series_off,
                        int64_t n_series, const double *center_len, int64_t k, int64_t *out_off)
{
    int64_t o = 0;
    for (int64_t s = 0; s < n_series; s++) {
        out_off[s] = o;
        int64_t a = piece_off[s], b = piece_off[s + 1];
        if (b == a) {
            o += (series_off[s + 1] - series_off[s]) >= 1 ? 1 : 0;
            continue;
        }
        i128 e = 0;
        int64_t total = 0;
        for (int64_t j = a; j < b; j++) {
            if (symbols[j] < 0 || symbols[j] >= k) return JO_EINVAL;
            i128 lt;
            if (to_fixed(center_len[symbols[j]], &lt) != JO_OK) return JO_EINVAL;
            i128 v = lt + e;
            int64_t lh = fixed_round(v);
            e = v - ((i128)lh << FIX_SHIFT);
            total += lh;
        }
        o += 1 + total;
    }
    out_off[n_series] = o;
    return JO_OK;
}

/*
 * Reconstruct every series into out[out_off[s] .. out_off[s+1]).
 * lhat (optional, N entries) receives the quantized lengths; sse/cnt
 * (optional, n_series entries) the squared error against the original
 * series over its first min(n, n^) points (Sec. 3.3, MSE).
 */
int jo_reconstruct(const int32_t *symbols, const int64_t *piece_off, const int64_t *series_off,
                   int64_t n_series, const double *t0, const double *center_len, const double *center_inc,
                   int64_t k, const int64_t *out_off, double *out, int64_t *lhat, const double *orig,
                   double *sse, int64_t *cnt)
{
    for (int64_t s = 0; s < n_series; s++) {
        int64_t a = piece_off[s], b = piece_off[s + 1];
        int64_t o = out_off[s];
        int64_t n_out = out_off[s + 1] - o;
        if (n_out > 0) out[o] = t0[s];
        i128 e = 0;
        int64_t pos = 0;
        double V = t0[s];
        for (int64_t j = a; j < b; j++) {
            if (symbols[j] < 0 || symbols[j] >= k) return JO_EINVAL;
            double it = center_inc[symbols[j]];
            i128 lt;
            if (to_fixed(center_len[symbols[j]], &lt) != JO_OK) return JO_EINVAL;
            i128 v = lt + e;
            int64_t lh = fixed_round(v);
            e = v - ((i128)lh << FIX_SHIFT);
            if (lhat) lhat[j] = lh;
            double slope = it / (double)lh;
            for (int64_t q = 1; q < lh; q++) out[o + pos + q] = V + slope * (double)q;
            V = V + it;
            pos += lh;
            out[o + pos] = V;
        }
        if (orig && sse && cnt) {
            int64_t n = series_off[s + 1] - series_off[s];
            int64_t m = n < n_out ? n : n_out;
            double acc = 0.0;
            for (int64_t i = 0; i < m; i++) {
                double d = orig[series_off[s] + i] - out[o + i];
                acc = acc + d * d;
            }
            sse[s] = acc;
            cnt[s] = m;
        }
    }
    return JO_OK;
}

/*
 * Inverse compression directly from the raw pieces (Sec. 3.1: the chain is
 * recovered from t_0 and the tuples).  Same fill rule as above with the
 * integer lengths; out_off is derived from piece lengths by the caller.
 */
int jo_reconstruct_pieces(const int32_t *len, const double *inc, const int64_t *piece_off, int64_t n_series,
                          const double *t0, const int64_t *out_off, double *out)
{
    for (int64_t s = 0; s < n_series; s++) {
        int64_t a = piece_off[s], b = piece_off[s + 1];
        int64_t o = out_off[s];
        if (out_off[s + 1] > o) out[o] = t0[s];
        double V = t0[s];
        int64_t pos = 0;
        for (int64_t j = a; j < b; j++) {
            int64_t lh = len[j];
            double slope = inc[j] / (double)lh;
            for (int64_t q = 1; q < lh; q++) out[o + pos + q] = V + slope * (double)q;
            V = V + inc[j];
            pos += lh;
            out[o + pos] = V;
        }
    }
    return JO_OK;
}

/* ------------------------------------------------------------------------ */
/* Digitization against a fixed dictionary (Sec. 3.2: nearest symbolic      */
/* center, c* = argmin ||p - c||, f_d(p) = I_d(c*)).  The piece is scaled     */
/* with the dictionary's sigma and scl; ties go to the lowest symbol.         */
/* ------------------------------------------------------------------------ */
int jo_encode(const int32_t *len, const double *inc, int64_t N, double sigma_len, double sigma_inc, double scl,
              const double *cx, const double *cy, int64_t k, int32_t *symbols)
{
    if (k < 1 && N > 0) return JO_EINVAL;
    for (int64_t i = 0; i < N; i++) {
        double x = scl * ((double)len[i] / sigma_len);
        double y = inc[i] / sigma_inc;
        int64_t best = -1;
        double bd = 0.0;
        for (int64_t c = 0; c < k; c++) {
            double dx = x - cx[c];
            double dy = y - cy[c];
            double d2 = dx * dx + dy * dy;
            if (best < 0 || d2 < bd) {
                best = c;
                bd = d2;
            }
        }
        symbols[i] = (int32_t)best;
    }
    return JO_OK;
}

/* ------------------------------------------------------------------------ */
/* Quality of a digitization (Sec. 3.2: the VQ objective, Eq. sse, and the  */
/* per-cluster variances, Eq. Var).  Pieces are scaled as the aggregation   */
/* scales them, x_i = scl*(len_i/sigma_len), y_i = inc_i/sigma_inc, and     */
/* compared with their symbol's scaled center (cx, cy), which is the mean   */
/* of the members; so for symbol c with members S_c                         */
/*   var_len[c] = (1/|S_c|) sum_{i in S_c} (x_i - cx_c)^2,                  */
/*   var_inc[c] = (1/|S_c|) sum_{i in S_c} (y_i - cy_c)^2,                  */
/*   SSE        = sum_c sum_{i in S_c} ((x_i - cx_c)^2 + (y_i - cy_c)^2).   */
/* Each squared deviation is one rounded binary64 value; every sum is the   */
/* exact sum of those values, rounded once (non-overlapping partials).      */
/* count[c] = |S_c|.  A symbol outside [0, k) is an error.                  */
/* ------------------------------------------------------------------------ */
int jo_quality(const int32_t *len, const double *inc, const int32_t *symbols, int64_t N, double sigma_len,
               double sigma_inc, double scl, const double *cx, const double *cy, int64_t k, double *var_len,
               double *var_inc, int64_t *count, double *sse)
{
    if (N < 0 || k < 0) return JO_EINVAL;
    for (int64_t i = 0; i < N; i++)
        if (symbols[i] < 0 || symbols[i] >= k) return JO_EINVAL;
    int rc = JO_ENOMEM;
    int64_t *start = calloc((size_t)(k + 1), sizeof(int64_t));
    int64_t *order = malloc((size_t)(N + 1) * sizeof(int64_t));
    double *dx2 = malloc((size_t)(N + 1) * sizeof(double));
    double *dy2 = malloc((size_t)(N + 1) * sizeof(double));
    double *both = malloc((size_t)(2 * N + 1) * sizeof(double));
    if (!start || !order || !dx2 || !dy2 || !both) goto done;
    /* members of each symbol, in canonical order (counting sort) */
    for (int64_t i = 0; i < N; i++) start[symbols[i] + 1]++;
    for (int64_t c = 0; c < k; c++) start[c + 1] += start[c];
    {
        int64_t *fill = calloc((size_t)(k + 1), sizeof(int64_t));
        if (!fill) goto done;
        for (int64_t i = 0; i < N; i++) {
            const int64_t c = symbols[i];
            order[start[c] + fill[c]++] = i;
        }
        free(fill);
    }
    for (int64_t c = 0; c < k; c++) {
        const int64_t a = start[c], b = start[c + 1];
        for (int64_t j = a; j < b; j++) {
            const int64_t i = order[j];
            const double x = scl * ((double)len[i] / sigma_len);
            const double y = inc[i] / sigma_inc;
            const double ex = x - cx[c];
            const double ey = y - cy[c];
            dx2[j] = ex * ex;
            dy2[j] = ey * ey;
            both[2 * j] = dx2[j];
            both[2 * j + 1] = dy2[j];
        }
        count[c] = b - a;
        var_len[c] = b > a ? jo_exact_sum(dx2 + a, b - a) / (double)(b - a) : 0.0;
        var_inc[c] = b > a ? jo_exact_sum(dy2 + a, b - a) / (double)(b - a) : 0.0;
    }
    *sse = jo_exact_sum(both, 2 * N);
    rc = JO_OK;
done:
    free(start);
    free(order);
    free(dx2);
    free(dy2);
    free(both);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* k-means digitization with a given number of symbols (Sec. 3.2: Lloyd's   */
/* algorithm minimises the VQ objective; Alg. 1 takes the symbol count as   */
/* its parameter C).  Pieces are scaled as in jo_digitize with the given    */
/* sigma and scl; the k initial centers (cx, cy) are inputs.  Each iteration */
/*   1. assigns every piece to its nearest center (ties to the lowest       */
/*      index, as in jo_encode), and stops when no assignment changed;      */
/*   2. moves every center to the mean of its members: center_len = exact   */
/*      integer sum of len / count, center_inc = sum of inc in canonical    */
/*      piece order, left to right, / count; a center with no member stays. */
/* After max_iter assignments the last assignment and its means are        */
/* returned.  Reading: the paper fixes neither the summation order nor the  */
/* initialisation; both are stated here and in the design notes.            */
/* ------------------------------------------------------------------------ */
int jo_kmeans(const int32_t *len, const double *inc, int64_t N, double sigma_len, double sigma_inc, double scl,
              int64_t k, int64_t max_iter, double *cx, double *cy, double *center_len, double *center_inc,
              int64_t *count, int32_t *symbols, int64_t *iters_done)
{
    if (k < 1 || N < 0 || max_iter < 1) return JO_EINVAL;
    int rc = JO_ENOMEM;
    int64_t *slen = malloc((size_t)k * sizeof(int64_t));
    double *sinc = malloc((size_t)k * sizeof(double));
    int32_t *prev = malloc((size_t)(N + 1) * sizeof(int32_t));
    if (!slen || !sinc || !prev) goto done;
    for (int64_t c = 0; c < k; c++) {
        center_len[c] = 0.0;
        center_inc[c] = 0.0;
        count[c] = 0;
    }
    int64_t it = 0;
    for (; it < max_iter; it++) {
        rc = jo_encode(len, inc, N, sigma_len, sigma_inc, scl, cx, cy, k, symbols);
        if (rc != JO_OK) goto done;
        if (it > 0) {
            int64_t changed = 0;
            for (int64_t i = 0; i < N; i++) changed += symbols[i] != prev[i];
            if (changed == 0) break;
        }
        for (int64_t c = 0; c < k; c++) {
            slen[c] = 0;
            sinc[c] = 0.0;
            count[c] = 0;
        }
        for (int64_t i = 0; i < N; i++) {
            const int32_t c = symbols[i];
            slen[c] += len[i];
            sinc[c] = sinc[c] + inc[i];
            count[c] += 1;
            prev[i] = c;
        }
        for (int64_t c = 0; c < k; c++) {
            if (count[c] == 0) continue;
            center_len[c] = (double)slen[c] / (double)count[c];
            center_inc[c] = sinc[c] / (double)count[c];
            cx[c] = scl * (center_len[c] / sigma_len);
            cy[c] = center_inc[c] / sigma_inc;
        }
    }
    *iters_done = it < max_iter ? it + 1 : max_iter;
    rc = JO_OK;
done:
    free(slen);
    free(sinc);
    free(prev);
    return rc;
}
