/*
 * jabba.h — C ABI of the MI355X (gfx950) joint-symbolic-approximation library.
 *
 * The calls follow the statement of the problem in arXiv 2401.00109:
 * Algorithm 1 takes a collection of series, a compression tolerance and a
 * digitization method and returns symbols plus a shared dictionary; Table 1
 * (table:ABBA) fixes the objects: series T, pieces P = [(len, inc)], symbols A,
 * and the inverse chain P~ -> P^ -> T^.
 *
 *   compress(series, tol)      -> pieces            (Sec. 3.1, Eq. compress; Sec. 4.1)
 *   digitize(pieces, alpha)    -> dictionary, symbols (Sec. 3.2; Sec. 5 two-stage)
 *   encode(pieces, dictionary) -> symbols           (Sec. 3.2, nearest center)
 *   reconstruct(symbols, dictionary, t0) -> series  (Sec. 3.3)
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers are DEVICE pointers unless the argument name ends in "_host".
 *    The caller allocates and owns every buffer, including workspaces and the
 *    dictionary arrays; nothing on these paths allocates device memory.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the legacy
 *    default stream).  A return of JABBA_OK means the work was enqueued.
 *  - Counts produced on the device (number of pieces, symbols, output points)
 *    stay in device memory; no call synchronises the host, except
 *    jabba_workspace_status and the plan/tuning helpers that say so.
 *  - Host-detected errors are returned immediately and nothing is enqueued.
 *    Every call that enqueues work first checks, after its arguments, that
 *    the current device is a gfx950 (JABBA_ENODEV otherwise, also when no
 *    device is visible).
 *    Device-detected errors (a non-finite input value, a dictionary that is
 *    too small) are OR-ed into a status word held in the call's workspace;
 *    read it with jabba_workspace_status after the stream has run.
 *  - Layouts: values of all series concatenated, series s occupying
 *    [series_off[s], series_off[s+1]); pieces of all series concatenated in
 *    canonical order (series, domain, position), series s occupying
 *    [piece_off[s], piece_off[s+1]).  len is int32, inc/values are binary64.
 *  - Arithmetic is binary64 everywhere a decision is taken (piece ends,
 *    groups, symbols), with no fused multiply-add, in the operation order
 *    documented at each call, so results are bit-identical to a plain
 *    sequential CPU evaluation of the same formulas.
 *  - Limits: fewer than 2^31 pieces per call; series lengths < 2^31.
 *  - Thread safety: calls on distinct streams with distinct buffers (and
 *    distinct workspaces) may run concurrently.
 *  - No C++ exception crosses this interface.
 */
#ifndef JABBA_H
#define JABBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JABBA_ABI_VERSION 4

enum jabba_status {
    JABBA_OK = 0,
    JABBA_EINVAL = -1,      /* bad argument (sizes, tolerances, null pointers)          */
    JABBA_ENOMEM = -2,      /* workspace smaller than the size query returned            */
    JABBA_EHIP = -3,        /* a HIP runtime call failed (or, from jabba_workspace_status,
                               a bounded device-side wait ran out)                       */
    JABBA_ECAPACITY = -4,   /* device: more symbols than the dictionary capacity         */
    JABBA_ENONFINITE = -5,  /* device: a series value is NaN or infinite                 */
    JABBA_EOVERFLOW = -6,   /* a count exceeds the 2^31 limit                            */
    JABBA_ENODEV = -7,      /* no gfx950 device is current                               */
    JABBA_ELIMIT = -8       /* a size exceeds the fixed maximum of an allocation-free call */
};

/* Library ABI version (JABBA_ABI_VERSION of the build). */
int jabba_abi_version(void);

/* Static, human-readable text for a status code. */
const char *jabba_status_str(int status);

/*
 * Launch-shape knobs.  They never change results, only speed (the autotuner
 * checks that every variant it times returns bit-identical outputs).
 * A zero field means "library default".  Pass NULL for all defaults.
 */
typedef struct jabba_tuning {
    int32_t lanes_per_domain; /* compress: lanes that test candidate end points of one
                                 domain together; 1, 2, 4, 8, 16, 32 or 64 (64 = one
                                 wavefront per domain)                                  */
    int32_t waves_per_block;  /* compress: wavefronts per workgroup, 1..16 (lowered when
                                 the workgroup's staging buffers would exceed 64 KB)   */
    int32_t blocks_per_cu;    /* compress: persistent workgroups per compute unit, 1..32 */
    int32_t stage1_waves;     /* digitize Stage I: wavefronts per workgroup (one block
                                 of sorted pieces per wavefront), 1..16 (halved until
                                 the workgroup's LDS fits in 64 KB, i.e. at most 4)     */
    int32_t segment_intervals; /* compress: domains are compressed as segments of this
                                 many intervals in parallel, then repaired into the
                                 domain's own pieces; >= 32, or -1 for whole domains;
                                 0 = default: segments of 128 when the domains are
                                 fewer than a quarter of the compute units, else
                                 whole domains                                          */
    int32_t reserved[3];
} jabba_tuning;

/*
 * Dictionary (Sec. 3.2: the symbolic centers; Alg. 1 output D).  All arrays
 * are caller-allocated device memory with `capacity` entries.
 *   params[0] = sigma_len, params[1] = sigma_inc  (population std of the
 *               training pieces, a zero deviation replaced by 1),
 *   params[2] = scl, params[3] = alpha.
 *   k[0]      = number of symbols (written by jabba_digitize).
 *   center_len[c], center_inc[c] = mean (len, inc) of the members of symbol c;
 *   cx[c] = scl*(center_len/sigma_len), cy[c] = center_inc/sigma_inc;
 *   count[c] = number of member pieces.
 */
typedef struct jabba_dict {
    int64_t capacity;
    double *params;
    int64_t *k;
    double *center_len;
    double *center_inc;
    double *cx;
    double *cy;
    int64_t *count;
} jabba_dict;

/* ------------------------------------------------------------------------ */
/* Compression: Alg. 1 Phases I-II (Sec. 4.1) with the ABBA compression of    */
/* Sec. 3.1 (Eq. compress).                                                   */
/* ------------------------------------------------------------------------ */

/*
 * Workspace bytes for jabba_compress / jabba_compress_plain with these sizes.
 * n_series >= 0, total_points = series_off[n_series] >= 0, D >= 1.
 */
int jabba_compress_workspace(int64_t n_series, int64_t total_points, int32_t D, size_t *bytes);

/*
 * Phase I: every series is cut into domains of D unit intervals; domain d of
 * a series with n points covers points [d*D, min((d+1)*D, n-1)], so adjacent
 * domains share an end point (Sec. 4.1.1).  Phase II: each domain is
 * compressed independently (Sec. 4.1.2) by greedy first-failure growth: from
 * piece start s, candidate length c = 2, 3, ... is accepted while
 *     sum_{k=1}^{c-1} (t_s + slope*k - t_{s+k})^2 <= (c-1)*(tol*tol),
 *     slope = (t_{s+c} - t_s)/c, terms added in ascending k,
 * and the piece ends just before the first rejected candidate, at the domain
 * end, or at max_len (> 0).  Each piece is (len, inc = t_{s+len} - t_s).
 * Pieces are concatenated in canonical order (Sec. 4.1.3).
 *
 *  values[total_points], series_off[n_series+1] (non-decreasing, [0] = 0)
 *  len, inc: capacity sum_s max(n_s - 1, 0) (the worst case; <= total_points)
 *  piece_off[n_series+1]: out, piece offsets per series
 *  n_pieces[1]: out, total number of pieces (int64)
 *  tuning: NULL or launch knobs; tol >= 0 finite; max_len >= 0 (0 = none).
 * Device status: JABBA_ENONFINITE if a value is NaN/Inf (pieces are then
 * unspecified).  Returns JABBA_EINVAL for bad sizes, JABBA_ENOMEM if
 * workspace_bytes is below jabba_compress_workspace.
 */
int jabba_compress(const double *values, const int64_t *series_off, int64_t n_series, int64_t total_points,
                   int32_t D, double tol, int32_t max_len, const jabba_tuning *tuning, int32_t *len, double *inc,
                   int64_t *piece_off, int64_t *n_pieces, void *workspace, size_t workspace_bytes, void *stream);

/*
 * jabba_compress on the z-normalised series, without writing them: per series
 * of n points mean = T(v)/n and std = sqrt(T((v - mean)^2)/n) (population
 * deviation; T the balanced pairwise sum over the series' points in order,
 * zero-padded to a power of two), a zero deviation (n = 1, a constant series)
 * replaced by 1 so the series is only centred, an empty series mean 0 and
 * std 1; the compression then reads every value as (v - mean)/std.  Pieces
 * are in normalised units (reconstruct, then multiply by std and add mean).
 *  mean, std_dev: device, n_series entries each, out.
 * Other arguments, workspace size and device status as jabba_compress; a
 * series longer than 2^30 points sets JABBA_EOVERFLOW.
 */
int jabba_compress_znorm(const double *values, const int64_t *series_off, int64_t n_series, int64_t total_points,
                         int32_t D, double tol, int32_t max_len, const jabba_tuning *tuning, int32_t *len,
                         double *inc, int64_t *piece_off, int64_t *n_pieces, double *mean, double *std_dev,
                         void *workspace, size_t workspace_bytes, void *stream);

/*
 * The same computation launched the plain way: one kernel launch per series
 * (grid = that series' domains, one wavefront per domain, 64 candidate end
 * points per round), no work queue.  Kept as the per-domain-launch baseline
 * the batched form is compared with.  series_off_host is a host copy of
 * series_off.  Same outputs, bit for bit, as jabba_compress.
 */
int jabba_compress_plain(const double *values, const int64_t *series_off, const int64_t *series_off_host,
                         int64_t n_series, int32_t D, double tol, int32_t max_len, int32_t *len, double *inc,
                         int64_t *piece_off, int64_t *n_pieces, void *workspace, size_t workspace_bytes,
                         void *stream);

/* ------------------------------------------------------------------------ */
/* Digitization: Alg. 1 Phase III with the two-stage aggregation of Sec. 5.   */
/* ------------------------------------------------------------------------ */

/* Workspace bytes for jabba_digitize with at most max_pieces pieces. */
int jabba_digitize_workspace(int64_t max_pieces, int32_t B, size_t *bytes);

/*
 * 1. Scaling (Sec. 3.2, Eq. tupseq2): sigma_len from exact int64 sums of len
 *    and len^2 (var = S2/N - (S1/N)^2, clamped at 0); sigma_inc by two passes
 *    of a balanced pairwise sum (leaves in canonical order, zero-padded to a
 *    power of two); zero deviations replaced by 1;
 *    x = scl*(len/sigma_len), y = inc/sigma_inc, key = sqrt(x*x + y*y).
 * 2. Sort: ascending key, ties by canonical index (Sec. 5, global sorting
 *    index).
 * 3. Blocks: B sorted pieces per block, each cut moved forward past equal
 *    keys (Sec. 5, "M contiguous blocks").
 * 4. Stage I: in every block, greedy aggregation in sorted order: an
 *    unassigned piece p starts a group; later pieces q are scanned while
 *    key_q - key_p <= alpha, and an unassigned q joins when
 *    (x_q - x_p)^2 + (y_q - y_p)^2 <= alpha*alpha.
 * 5. Stage II: the same aggregation over all Stage I starting points, which
 *    are already in sorted order.
 * 6. Label propagation (Eq. l_i = l~_g): symbol of a piece = global group of
 *    its local start.  Symbols are numbered by sorted position of the global
 *    start.
 * 7. Dictionary: count and exact int64 length sum per symbol; center_len =
 *    sum/count (correctly rounded); center_inc = increment sum / count with
 *    the sum taken in a fixed order (deterministic; within ~1e-15 relative of
 *    the exact mean); cx, cy as in jabba_dict.
 *
 *  len, inc: pieces, n_pieces[0] of them (device count, <= max_pieces)
 *  alpha >= 0, scl >= 0 finite; B >= 1 pieces per block (a method parameter:
 *  it changes results); symbols[max_pieces]: out.
 *  dict: out; dict->capacity symbols.  Device status JABBA_ECAPACITY when k >
 *  capacity (k is still written; only the first capacity centers are);
 *  JABBA_ENONFINITE when an increment is NaN or infinite (results are then
 *  unspecified).
 */
int jabba_digitize(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces, double alpha,
                   double scl, int32_t B, const jabba_tuning *tuning, int32_t *symbols, const jabba_dict *dict,
                   void *workspace, size_t workspace_bytes, void *stream);

/*
 * jabba_digitize with a PCA projection as the sort key (Sec. 5 names the norm
 * or a PCA projection as the scalar the pieces are sorted by).  Step 1 also
 * forms the population covariance of the scaled points:
 *   var(x) = scl^2 (0 when var_len = 0), var(y) = 1 (0 when var_inc = 0),
 *   cov(x, y) = scl*((cov(len, inc)/sigma_len)/sigma_inc), 0 unless both
 *   variances are positive, with cov(len, inc) = T((len - S1/N)*(inc - T(inc)/N))/N
 *   and T the pairwise sum of step 1;
 * the key is u_x*x + u_y*y (no fused multiply-add; -0 taken as +0), u the unit
 * eigenvector of the larger eigenvalue of that 2x2 matrix in closed form
 * ((h + r, c) if h >= 0 else (c, r - h), h = (var(x) - var(y))/2,
 * r = sqrt(h^2 + cov^2), normalised), signed so its first nonzero entry is
 * positive; a zero covariance gives (1, 0) if var(x) >= var(y), else (0, 1).
 * Keys may be negative.  Steps 2-7 are those of jabba_digitize; the pruning
 * in steps 4-5 stays sound because a projection on a unit vector never
 * exceeds the distance.
 *  axis: device, 2 doubles, out (may be NULL): u_x, u_y.
 * Arguments, workspace size, errors and device status as jabba_digitize.
 */
int jabba_digitize_pca(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                       double alpha, double scl, int32_t B, const jabba_tuning *tuning, int32_t *symbols,
                       const jabba_dict *dict, double *axis, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Two-stage greedy aggregation of 2-D points as given, with no scaling
 * (Sec. 5; the Gaussian-blob experiment of Sec. 7.1 runs the two-stage
 * method on raw points and compares it with the serial greedy aggregation,
 * which is B >= n).  key = sqrt(x*x + y*y); steps 2-6 of jabba_digitize
 * (sort, blocks of B, Stage I, Stage II, label propagation) give labels
 * numbered by sorted position of the global start.  Then per label: count,
 * and the means of x and of y with the members added one by one in input
 * order; and SSE (Eq. sse) = sum of (x - cx)^2 + (y - cy)^2 over the points,
 * a pairwise tree in input order (within ~1e-15 relative of the exact sum).
 *  x, y: n_points[0] points (device count, <= max_points), finite.
 *  alpha >= 0; B >= 1 points per block.
 *  labels[max_points]: out.  cx, cy, count: capacity entries, out.
 *  k: device, 1 entry, out (written also when k > capacity; then device
 *  status JABBA_ECAPACITY, centers beyond capacity and the SSE are not
 *  written).  sse: device, 1 entry, out (may be NULL).
 *  workspace: jabba_digitize_workspace(max_points, B) bytes.
 * Non-finite points set device status JABBA_ENONFINITE.
 */
int jabba_aggregate_points(const double *x, const double *y, const int64_t *n_points, int64_t max_points,
                           double alpha, int32_t B, int32_t *labels, int64_t capacity, double *cx, double *cy,
                           int64_t *count, int64_t *k, double *sse, void *workspace, size_t workspace_bytes,
                           void *stream);

/*
 * Separate digitization tolerances for length and increment (Sec. 3.2,
 * alpha_len and alpha_inc of Eq. Var1).  A piece joins a start when
 *   ((x - x_s)/alpha_len)^2 + ((y - y_s)/alpha_inc)^2 <= 1,
 * which is the aggregation's test when alpha_len = alpha_inc = alpha.  The
 * same test is the aggregation's disc test of radius alpha_inc after x is
 * multiplied by alpha_inc/alpha_len, so this host function only returns the
 * jabba_digitize (or jabba_digitize_pca) arguments that run it:
 *   *alpha = alpha_inc,  *scl = scl_in*(alpha_inc/alpha_len)
 * and the test evaluated is that rescaled disc test.  With one block every
 * symbol then has Var_len <= alpha_len^2 (x in units of scl_in*len/sigma_len)
 * and Var_inc <= alpha_inc^2, hence Eq. Var1.  alpha_len, alpha_inc > 0 and
 * scl_in >= 0, all finite, else JABBA_EINVAL.  No device work.
 */
int jabba_axis_tolerances(double alpha_len, double alpha_inc, double scl_in, double *alpha, double *scl);

/*
 * Counters of the last jabba_digitize that used `workspace` (same max_pieces
 * and B): stats[0] = N pieces, stats[1] = G Stage I starting points,
 * stats[2] = k symbols, stats[3] = radix passes of the global sort that
 * moved data (the highest four varying digits of the key; digits equal in
 * every key are skipped), stats[4] = number of independent groups Stage II
 * ran on, stats[5] = bytes per piece those radix passes read and wrote
 * together (keys narrow to 32 bits after the first), stats[6] = pieces
 * whose prefix group was too large for the local sort (sorted by the general
 * radix sort instead).
 * stats holds 7 entries.
 * Synchronises `stream`.
 */
int jabba_digitize_stats(const void *workspace, int64_t max_pieces, int32_t B, void *stream, int64_t *stats);

/*
 * Quality of the digitization the workspace holds (Sec. 3.2: the vector
 * quantization objective, Eq. sse, and the per-cluster variances, Eq. Var).
 * Call after jabba_digitize with the same len, inc, n_pieces, max_pieces,
 * alpha, B, dictionary and workspace, on the same stream, before the
 * workspace is used again (this call overwrites parts of it that the
 * digitization no longer needs).  With x = scl*(len/sigma_len) and
 * y = inc/sigma_inc, the scaled coordinates the aggregation uses, and the
 * symbol's scaled center (cx, cy):
 *   var_len[c] = mean over the members of c of (x - cx_c)^2,
 *   var_inc[c] = mean over the members of c of (y - cy_c)^2,
 *   totals[0] = SSE, the sum over all pieces of (x - cx)^2 + (y - cy)^2,
 *   totals[1] = max_c var_len[c], totals[2] = max_c var_inc[c].
 * var_len, var_inc: device, dict->capacity entries (symbols >= capacity are
 * skipped); totals: device, 3 entries.  Each squared deviation is one rounded
 * binary64 value; they are summed per Stage I group in position order and
 * per symbol over its groups, the same fixed order as the centers, and the
 * SSE adds the per-symbol sums in a fixed order, so the results are
 * deterministic.
 */
int jabba_digitize_quality(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                           double alpha, int32_t B, const jabba_dict *dict, double *var_len, double *var_inc,
                           double *totals, void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes for jabba_encode with a dictionary of this capacity. */
int jabba_encode_workspace(int64_t capacity, size_t *bytes);

/*
 * Nearest-center digitization against an existing dictionary (Sec. 3.2,
 * c* = argmin_c ||p - c||, f_d = I_d(c*)): x = params[2]*(len/params[0]),
 * y = inc/params[1], symbol = argmin_c (x - cx_c)^2 + (y - cy_c)^2 over all
 * k symbols (each distance rounded as written), ties to the lowest symbol; -1
 * when the dictionary is empty.  The centers are ordered by cx in the
 * workspace and every piece walks outward from its x until the remaining
 * centers are provably farther, which returns the same symbol as a full scan.
 * symbols[max_pieces]: out.
 */
int jabba_encode(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                 const jabba_dict *dict, int32_t *symbols, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Largest dictionary capacity jabba_encode_noalloc accepts.  Its scratch is a
 * fixed 3 MiB device array per GPU (jabba_encode_workspace of this capacity
 * fits in it).
 */
#define JABBA_ENCODE_NOALLOC_MAX_CAPACITY 65536

/*
 * jabba_encode without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, serving loops that
 * forbid allocation, harnesses that ban hipMalloc.  Same arguments, result
 * and errors as jabba_encode, bit for bit.  The call allocates nothing: its
 * scratch (the ordered centers and columns) is a file-scope device array of
 * the library, one per GPU, resolved on the first call on each device and
 * kept until the process ends.
 *   dict->capacity > JABBA_ENCODE_NOALLOC_MAX_CAPACITY -> JABBA_ELIMIT,
 *   nothing enqueued.
 * Every call on one GPU shares that GPU's scratch, which holds the last
 * call's contents (each call rewrites all it reads): calls that overlap on
 * one GPU (different streams, or different host threads) race and must be
 * serialised by the caller.
 */
int jabba_encode_noalloc(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                         const jabba_dict *dict, int32_t *symbols, void *stream);

/*
 * Workspace bytes for jabba_kmeans with at most max_pieces pieces and a
 * dictionary of this capacity.
 */
int jabba_kmeans_workspace(int64_t max_pieces, int64_t capacity, size_t *bytes);

/*
 * k-means digitization with a given number of symbols (Sec. 3.2: Lloyd's
 * algorithm for the vector quantization objective; the symbol count is the
 * parameter C of Alg. 1).  Pieces are scaled as jabba_digitize scales them,
 * x = scl*(len/sigma_len), y = inc/sigma_inc, with
 *   dict->params[0..2] = sigma_len, sigma_inc, scl (device; e.g. as written
 *   by a previous jabba_digitize), *dict->k = the number of centers k
 *   (device, 1..capacity), dict->cx/cy = the k initial scaled centers.
 * Each iteration assigns every piece to its nearest center exactly as
 * jabba_encode does (rounded distances, ties to the lowest symbol), stops
 * when no assignment changed, and otherwise moves every center to the mean of
 * its members: center_len = exact integer sum of len / count, center_inc =
 * the members' inc added one by one in canonical piece order / count,
 * cx = scl*(center_len/sigma_len), cy = center_inc/sigma_inc; a center with
 * no member keeps its position (count 0).  At most max_iter assignments.
 * Outputs: symbols (device, max_pieces), the dictionary's cx, cy,
 * center_len, center_inc, count (the means of the final assignment), and
 * *iterations (device int64, assignments made).  center_len/center_inc of a
 * center that never had a member are 0.  Synchronises `stream` once per
 * iteration for the convergence check.  Ownership: all buffers belong to the
 * caller; the workspace is reused between calls.
 */
int jabba_kmeans(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces, int32_t max_iter,
                 const jabba_dict *dict, int32_t *symbols, int64_t *iterations, void *workspace,
                 size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Inverse symbolization (Sec. 3.3).                                          */
/* ------------------------------------------------------------------------ */

/* Workspace bytes for the reconstruct calls. */
int jabba_reconstruct_workspace(int64_t n_series, size_t *bytes);

/*
 * Output sizes.  Quantization (Eq. repolygon) keeps the running sum of the
 * integer lengths equal to the rounded running sum of the center lengths
 * (halves away from zero); it is evaluated exactly in 128-bit fixed point at
 * scale 2^52 (every center length >= 1 is a multiple of 2^-52).
 * Series s gets 1 + sum(len^) points if it has pieces, otherwise
 * min(n_s, 1) points.  out_off[n_series+1]: out (device); the total is
 * out_off[n_series].
 */
int jabba_reconstruct_size(const int32_t *symbols, const int64_t *piece_off, const int64_t *series_off,
                           int64_t n_series, const jabba_dict *dict, int64_t *out_off, void *workspace,
                           size_t workspace_bytes, void *stream);

/*
 * Inverse digitization, quantization and inverse compression: V_0 = t0[s],
 * V_j = V_{j-1} + center_inc (sequential per series), interior points
 * V_{j-1} + (center_inc/len^_j)*q for 0 < q < len^_j, end point V_j.
 * out[out_off[n_series]]: out.  lhat[max pieces]: optional out (may be NULL).
 * values/series_off: optional originals; when values is non-NULL, sse[s] and
 * cnt[s] receive the squared error over the first min(n_s, n^_s) points
 * (Sec. 3.3, MSE = sum(sse)/sum(cnt)).  dict->capacity >= 1, else
 * JABBA_EINVAL; a symbol outside [0, capacity) reads as length 1, increment 0
 * (jabba_reconstruct_size flags it in the device status).
 * workspace: jabba_reconstruct_workspace(n_series) bytes (JABBA_ENOMEM if
 * smaller; the one given to jabba_reconstruct_size may be passed again, its
 * status word is kept); it holds the order in which series are taken, the
 * longest first, which changes no output.
 */
int jabba_reconstruct(const int32_t *symbols, const int64_t *piece_off, const int64_t *series_off, int64_t n_series,
                      const double *t0, const jabba_dict *dict, const int64_t *out_off, double *out, int64_t *lhat,
                      const double *values, double *sse, int64_t *cnt, void *workspace, size_t workspace_bytes,
                      void *stream);

/*
 * Mean squared error of a reconstruction (Sec. 3.3): mse[0] (device) =
 * sum(sse) / sum(cnt) over the n_series per-series outputs of
 * jabba_reconstruct.  The squared errors are added by a balanced pairwise
 * tree over the series (leaves in series order, zero-padded to a power of
 * two), the counts exactly; 0 when no point was compared.
 */
int jabba_reconstruct_mse(const double *sse, const int64_t *cnt, int64_t n_series, double *mse, void *stream);

/*
 * Inverse compression straight from (len, inc) (Sec. 3.1: the polygonal
 * chain is recovered from t_0 and the tuples).  out_off[n_series+1] is
 * written (1 + sum(len) per series with pieces); same fill rule as above.
 */
int jabba_reconstruct_pieces(const int32_t *len, const double *inc, const int64_t *piece_off,
                             const int64_t *series_off, int64_t n_series, const double *t0, int64_t *out_off,
                             double *out, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Status.                                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Synchronises `stream`, then copies the device status word of a workspace
 * used by a previous call on that stream into *status (JABBA_OK or the first
 * device-detected error code).  Returns JABBA_OK or JABBA_EHIP.
 */
int jabba_workspace_status(const void *workspace, void *stream, int32_t *status);

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                               */
/* ------------------------------------------------------------------------ */

/*
 * quot[i] = a[i] / b[i] and root[i] = sqrt(a[i]) evaluated with exactly the
 * device code the library's kernels use for the scaling and the sort key
 * (Sec. 3.2, Eq. tupseq2).  Lets a caller confirm that both are correctly
 * rounded binary64 operations on the device at hand, which the bit-exact
 * decisions rely on.  n >= 0 elements, device arrays.
 */
int jabba_fp64_selftest(const double *a, const double *b, double *quot, double *root, int64_t n, void *stream);

/*
 * Per-kernel timing for benchmarks.  While enabled, every kernel launch of
 * the library is bracketed by two HIP events recorded on the stream the
 * kernel is launched on; durations accumulate per kernel name.  The eight
 * radix passes of a sort run back to back and are bracketed together (one
 * event pair, counted as eight launches).  Enabling
 * clears the accumulators.  Must be off while a plan is being captured.
 * jabba_timing_get synchronises on the recorded events; *launches is the
 * number of timed launches of `name` (0 if none).  jabba_timing_names writes
 * the kernel names seen so far, comma-separated, into buf (truncated to
 * buf_len - 1 characters).
 */
int jabba_timing_enable(int enable);
int jabba_timing_get(const char *name, double *total_ms, int64_t *launches);
int jabba_timing_names(char *buf, size_t buf_len);

/* ------------------------------------------------------------------------ */
/* Batched plan: the whole compress + digitize path captured once into a HIP  */
/* graph (persistent compression kernel with a work queue ordered by domain   */
/* length, every later kernel sized from upper bounds and device counters)   */
/* and replayed with one graph launch per batch.                              */
/* ------------------------------------------------------------------------ */

typedef struct jabba_plan jabba_plan;

typedef struct jabba_plan_desc {
    /* inputs */
    const double *values;
    const int64_t *series_off;
    int64_t n_series;
    int64_t total_points;
    int32_t D;
    double tol;
    int32_t max_len;
    double alpha;
    double scl;
    int32_t B;
    int64_t max_pieces; /* upper bound on the piece count, as given to jabba_digitize_workspace */
    /* outputs (device) */
    int32_t *len;
    double *inc;
    int64_t *piece_off;
    int64_t *n_pieces;
    int32_t *symbols;
    jabba_dict dict;
    /* workspaces (device) sized by the two workspace queries */
    void *compress_ws;
    size_t compress_ws_bytes;
    void *digitize_ws;
    size_t digitize_ws_bytes;
    /* launch shapes; NULL = autotuned by jabba_plan_create */
    const jabba_tuning *tuning;
} jabba_plan_desc;

/*
 * Captures the path for the buffers and sizes in *desc (they are bound to the
 * plan) on an internal stream and instantiates the graph.  Synchronous.
 *
 * With desc->tuning NULL the launch shapes are chosen first, on the plan's
 * own buffers and inputs: the compression is timed over lanes per domain
 * {1, 2, 4} x wavefronts per workgroup {1, 2, 4} x workgroups per compute
 * unit {2, 4, 8}, then the digitization over Stage I wavefronts {1, 2, 4}
 * (best of two runs each).  Every variant's output is compared on the device
 * with the default launch's (pieces, offsets and count, using the digitize
 * workspace for the copy; symbols, using the compress workspace) whenever
 * that workspace can hold the copy, and a variant that differs is never
 * chosen.  The inputs are read and the outputs written during the search,
 * which costs a few dozen runs of the path.  jabba_plan_tuning reports the
 * choice.
 */
int jabba_plan_create(const jabba_plan_desc *desc, jabba_plan **plan);

/* The launch shapes the plan was captured with (the caller's or the autotuned ones). */
int jabba_plan_tuning(const jabba_plan *plan, jabba_tuning *tuning);

/* Replays the captured graph on `stream` (asynchronous). */
int jabba_plan_run(jabba_plan *plan, void *stream);

/* Frees the graph; buffers stay with the caller.  The plan is freed in every
 * case; JABBA_EHIP if the runtime reported an error while destroying it. */
int jabba_plan_destroy(jabba_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* JABBA_H */
