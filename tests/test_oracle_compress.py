"""Pins for the oracle's compression (Sec. 3.1 Eq. compress; Sec. 4.1 domains).

The oracle is checked against things other than itself:
  * exact rational arithmetic over the paper's literal sum (end points
    included) on small inputs, with first-failure growth done by brute force;
  * closed forms: straight lines, integer piecewise-linear data at tol = 0;
  * invariants the paper states: every piece's error <= (len-1) tol^2, the
    pieces tile the series, domain boundaries cut pieces (Sec. 4.1.3).
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle as O


# ---------------------------------------------------------------- helpers
def exact_err(t, s, c):
    """Paper's Eq. (compress) sum over i = s..s+c inclusive, exact rationals."""
    ts, te = t[s], t[s + c]
    return sum((ts + (te - ts) * F(k, c) - t[s + k]) ** 2 for k in range(0, c + 1))


def exact_segmentation(t, a, b, tol2, max_len=0):
    """First-failure greedy on exact arithmetic; returns [(len, inc)]."""
    out = []
    s = a
    while s < b:
        L = 1
        while s + L + 1 <= b and (max_len == 0 or L + 1 <= max_len) and exact_err(t, s, L + 1) <= (L) * tol2:
            L += 1
        out.append((L, t[s + L] - t[s]))
        s += L
    return out


def min_gap(t, a, b, tol2):
    """Smallest relative distance of any candidate's error from its threshold."""
    g = float("inf")
    for s in range(a, b):
        for c in range(2, b - s + 1):
            thr = (c - 1) * tol2
            e = exact_err(t, s, c)
            g = min(g, abs(float(e - thr)) / max(float(thr), 1e-300))
    return g


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_exact_rational(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 15))
    # dyadic values: exactly representable, small denominators
    vals = rng.integers(-12, 13, n) / 4.0
    if seed % 3 == 0:
        vals = np.cumsum(rng.integers(-3, 4, n)).astype(float)
    tol = float(rng.choice([0.3, 0.55, 0.8, 1.1, 1.7, 2.3]))
    tol2 = F(tol) * F(tol)
    t = [F(v) for v in vals]
    if min_gap(t, 0, n - 1, tol2) < 1e-9:
        pytest.skip("near-tie between an error and its threshold")
    ln, inc, po = O.compress(vals, np.array([0, n]), D=n, tol=tol)
    exp = exact_segmentation(t, 0, n - 1, tol2)
    assert [int(x) for x in ln] == [L for L, _ in exp]
    assert [F(float(x)) for x in inc] == [i for _, i in exp]
    assert po.tolist() == [0, len(exp)]


@pytest.mark.parametrize("max_len", [1, 2, 3, 5])
def test_bruteforce_max_len(max_len):
    vals = np.arange(12, dtype=float) * 0.5  # a straight line: only max_len stops pieces
    ln, inc, _ = O.compress(vals, np.array([0, 12]), D=100, tol=0.1, max_len=max_len)
    exp = exact_segmentation([F(v) for v in vals], 0, 11, F(0.1) ** 2, max_len)
    assert ln.tolist() == [L for L, _ in exp]
    assert all(L <= max_len for L in ln)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n,D", [(2, 1), (10, 3), (1000, 999), (1000, 100), (1001, 100), (5000, 4999), (777, 50)])
@pytest.mark.parametrize("tol", [0.0, 0.05])
def test_straight_line_one_piece_per_domain(n, D, tol):
    vals = 3.0 + 0.25 * np.arange(n)  # dyadic slope: every residual is exactly 0
    ln, inc, po = O.compress(vals, np.array([0, n]), D=D, tol=tol)
    ndom = -(-(n - 1) // D)
    assert ln.size == ndom                     # boundary-induced pieces, Sec. 4.1.3
    assert int(ln.sum()) == n - 1
    starts = np.concatenate(([0], np.cumsum(ln)[:-1]))
    np.testing.assert_array_equal(inc, vals[starts + ln] - vals[starts])
    # each piece is exactly one domain
    assert all(L == min(D, n - 1 - d * D) for d, L in enumerate(ln))


@pytest.mark.parametrize("seed", range(10))
def test_integer_pwl_tol0_recovers_breakpoints(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(50, 400))
    n_knots = int(rng.integers(1, 12))
    knots = np.sort(rng.choice(np.arange(1, n - 1), n_knots, replace=False))
    bps = np.concatenate(([0], knots, [n - 1]))
    slopes = []
    for _ in range(bps.size - 1):
        s = int(rng.integers(-4, 5))
        while slopes and s == slopes[-1]:
            s = int(rng.integers(-4, 5))
        slopes.append(s)
    vals = np.zeros(n)
    for i in range(bps.size - 1):
        a, b = bps[i], bps[i + 1]
        vals[a + 1:b + 1] = vals[a] + slopes[i] * np.arange(1, b - a + 1)
    D = int(rng.choice([n, 37, 100]))
    ln, inc, po = O.compress(vals, np.array([0, n]), D=D, tol=0.0)
    ends = np.cumsum(ln)
    dom_ends = set(range(D, n - 1, D))
    expected = sorted(set(bps[1:].tolist()) | dom_ends)
    assert ends.tolist() == expected


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("tol", [0.02, 0.05, 0.1, 0.4])
def test_error_bound_and_first_failure(tol):
    rng = np.random.default_rng(7)
    vals = np.cumsum(rng.standard_normal(600))
    vals = (vals - vals.mean()) / vals.std()
    D = 250
    ln, inc, po = O.compress(vals, np.array([0, vals.size]), D=D, tol=tol)
    t = [F(v) for v in vals]
    tol2 = F(tol) ** 2
    assert int(ln.sum()) == vals.size - 1
    s = 0
    dom_end = lambda p: min((p // D + 1) * D, vals.size - 1)  # noqa: E731
    for L in ln.tolist():
        e = exact_err(t, s, L) if L >= 2 else F(0)
        assert float(e) <= float((L - 1) * tol2) * (1 + 1e-9) + 1e-300
        # first failure: the next candidate exceeds the bound (or the domain ends)
        if s + L + 1 <= dom_end(s):
            e2 = exact_err(t, s, L + 1)
            assert float(e2) >= float(L * tol2) * (1 - 1e-9)
        s += L


def test_domain_independence_and_concatenation():
    rng = np.random.default_rng(3)
    vals = np.cumsum(rng.standard_normal(5001))
    D = 700
    ln, inc, po = O.compress(vals, np.array([0, vals.size]), D=D, tol=0.3)
    parts = []
    for a in range(0, vals.size - 1, D):
        b = min(a + D, vals.size - 1)
        l2, i2, _ = O.compress(vals[a:b + 1], np.array([0, b - a + 1]), D=10**9, tol=0.3)
        parts.append((l2, i2))
    np.testing.assert_array_equal(ln, np.concatenate([p[0] for p in parts]))
    np.testing.assert_array_equal(inc, np.concatenate([p[1] for p in parts]))


def test_multi_series_offsets_and_degenerate_lengths():
    rng = np.random.default_rng(5)
    lens = [0, 1, 2, 3, 17, 1, 0, 250]
    ser = [rng.standard_normal(n) for n in lens]
    off = np.concatenate(([0], np.cumsum(lens))).astype(np.int64)
    vals = np.concatenate(ser)
    ln, inc, po = O.compress(vals, off, D=10, tol=0.2)
    for s, n in enumerate(lens):
        a, b = po[s], po[s + 1]
        assert int(ln[a:b].sum()) == max(n - 1, 0)
        if n <= 1:
            assert a == b
        # series alone gives the same pieces
        l1, i1, _ = O.compress(ser[s], np.array([0, n]), D=10, tol=0.2)
        np.testing.assert_array_equal(ln[a:b], l1)
        np.testing.assert_array_equal(inc[a:b], i1)
    assert O.count_domains(off, 10) == sum(-(-(n - 1) // 10) for n in lens if n >= 2)


def test_domain_table():
    off = np.array([0, 1, 11, 12, 1012], dtype=np.int64)
    ds, st, ni = O.domains(off, 300)
    assert ds.tolist() == [1, 3, 3, 3, 3]
    assert st.tolist() == [1, 12, 312, 612, 912]
    assert ni.tolist() == [9, 300, 300, 300, 99]


def test_nonfinite_rejected():
    vals = np.array([0.0, 1.0, np.nan, 2.0])
    with pytest.raises(O.OracleError):
        O.compress(vals, np.array([0, 4]), D=10, tol=0.1)
    with pytest.raises(O.OracleError):
        O.compress(np.array([0.0, np.inf]), np.array([0, 2]), D=10, tol=0.1)
