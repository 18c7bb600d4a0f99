"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign or index, a
transposed operand, a skipped step) in a copy of the oracle's C source, builds
it on the CPU, and runs the oracle pin tests against that copy: at least one
pin has to fail.  The real oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "jabba_oracle.c")
PINS = ["tests/test_oracle_compress.py", "tests/test_oracle_digitize.py", "tests/test_oracle_reconstruct.py",
        "tests/test_oracle_quality.py", "tests/test_oracle_kmeans.py", "tests/test_oracle_pca.py",
        "tests/test_oracle_points.py", "tests/test_oracle_znorm.py"]

MUTANTS = {
    "square_dropped": ("acc = acc + r * r;", "acc = acc + r;"),
    "last_interior_term_dropped": ("for (int64_t k = 1; k < c; k++) {", "for (int64_t k = 1; k < c - 1; k++) {"),
    "threshold_index": ("double thr = (double)(c - 1) * tol2;", "double thr = (double)(c) * tol2;"),
    "residual_index": ("double r = v - t[s + k];", "double r = v - t[s + k - 1];"),
    "inc_sign": ("inc[np] = t[s + L] - t[s];", "inc[np] = t[s] - t[s + L];"),
    "var_len_sign": ("(double)S2 / (double)N - mean_len * mean_len", "(double)S2 / (double)N + mean_len * mean_len"),
    "y_scaled_by_sigma_len": ("double yi = inc[i] / si;", "double yi = inc[i] / sl;"),
    "tree_overlap": ("double r = tree_rec(a, n, lo + h, h);", "double r = tree_rec(a, n, lo + h - 1, h);"),
    "window_too_narrow": ("if (!(skey[q] - skey[p] <= alpha)) break;", "if (!(skey[q] - skey[p] <= 0.5 * alpha)) break;"),
    "radius_too_wide": ("if (d2 <= a2) lab[q] = p;", "if (d2 <= 4.0 * a2) lab[q] = p;"),
    "dy_transposed": ("double dy = sy[q] - sy[p];", "double dy = sx[q] - sy[p];"),
    "stage2_skipped": ("aggregate_range(gx, gy, gk, 0, G, alpha, glab);",
                       "for (int64_t g = 0; g < G; g++) glab[g] = g;"),
    "blocks_split_ties": ("while (p < N && skey[p] == skey[p - 1]) p++;", ""),
    "center_len_count": ("double cl = (double)slen[c] / (double)cnt[c];",
                         "double cl = (double)slen[c] / (double)(cnt[c] + 1);"),
    "carry_dropped": ("e = v - ((i128)lh << FIX_SHIFT);", "e = 0;"),
    "fill_index": ("out[o + pos + q] = V + slope * (double)q;", "out[o + pos + q] = V + slope * (double)(q + 1);"),
    "encode_ties_high": ("if (best < 0 || d2 < bd) {", "if (best < 0 || d2 <= bd) {"),
    "exact_sum_lossy": ("double lo = y - (hi - x);", "double lo = 0.0;"),
    "quality_var_divisor": ("var_len[c] = b > a ? jo_exact_sum(dx2 + a, b - a) / (double)(b - a) : 0.0;",
                            "var_len[c] = b > a ? jo_exact_sum(dx2 + a, b - a) / (double)(b - a + 1) : 0.0;"),
    "quality_dy_from_x": ("const double ey = y - cy[c];", "const double ey = x - cy[c];"),
    "quality_sse_half": ("*sse = jo_exact_sum(both, 2 * N);", "*sse = jo_exact_sum(both, N);"),
    "kmeans_inc_mean_divisor": ("center_inc[c] = sinc[c] / (double)count[c];",
                                "center_inc[c] = sinc[c] / (double)(count[c] + 1);"),
    "kmeans_stops_early": ("if (changed == 0) break;", "if (changed < 3) break;"),
    "pca_cov_uncentered": ("t[i] = ((double)len[i] - mean_len) * (inc[i] - mean_inc);",
                           "t[i] = (double)len[i] * inc[i];"),
    "pca_cov_sign": ("c = scl * ((cov / sl) / si);", "c = -scl * ((cov / sl) / si);"),
    "pca_var_x_unsquared": ("a = scl * scl;", "a = scl;"),
    "pca_minor_axis": ("vx = h + r;", "vx = h - r;"),
    "pca_key_transposed": ("double kv = u[0] * x[i] + u[1] * y[i];", "double kv = u[1] * x[i] + u[0] * y[i];"),
    "points_cy_from_x": ("cy[c] = cy[c] + y[i];", "cy[c] = cy[c] + x[i];"),
    "points_key_without_y": ("for (int64_t i = 0; i < N; i++) key[i] = sqrt(x[i] * x[i] + y[i] * y[i]);",
                             "for (int64_t i = 0; i < N; i++) key[i] = fabs(x[i]);"),
    "points_sse_dy_dropped": ("t[i] = dx * dx + dy * dy;", "t[i] = dx * dx;"),
    "znorm_sample_variance": ("double var = jo_tree_sum(sq, n) / (double)n;",
                              "double var = jo_tree_sum(sq, n) / (double)(n > 1 ? n - 1 : 1);"),
    "znorm_not_centred": ("for (int64_t i = 0; i < n; i++) out[a + i] = (values[a + i] - m) / sd;",
                          "for (int64_t i = 0; i < n; i++) out[a + i] = values[a + i] / sd;"),
    "round_floor": ("return (int64_t)((v + ((i128)1 << (FIX_SHIFT - 1))) >> FIX_SHIFT);",
                    "return (int64_t)(v >> FIX_SHIFT);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mut = src.replace(old, new)
    c_path = tmp_path / "mutant.c"
    so_path = tmp_path / "mutant.so"
    c_path.write_text(mut)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-shared", "-fPIC",
                    "-o", str(so_path), str(c_path), "-lm"], check=True)
    env = dict(os.environ, JABBA_ORACLE_SO=str(so_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught mutant {name}:\n{r.stdout[-2000:]}"
