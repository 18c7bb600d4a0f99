"""Pins for the oracle's sums, scaling, sort, blocks, two-stage aggregation and
dictionary (Sec. 3.2 Eqs. tupseq2, sse, Var; Sec. 5 Stage I / II / label
propagation).

Independent references used: math.fsum and numpy (std, lexsort, argmin),
exact rational arithmetic (fractions), an unpruned pure-Python greedy, the
paper's variance / SSE bounds and the triangle inequality.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle as O

U = 2.0 ** -53


# ---------------------------------------------------------------- sums
def test_exact_sum_matches_fsum():
    rng = np.random.default_rng(0)
    for n in [0, 1, 2, 3, 10, 1000, 33333]:
        a = rng.standard_normal(n) * 10.0 ** rng.integers(-12, 12, n)
        assert O.exact_sum(a) == math.fsum(a)
    a = np.array([1e100, 1.0, -1e100, 1e-100, 3.0])
    assert O.exact_sum(a) == math.fsum(a)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 1023, 1024, 1025, 4097, 100_000])
def test_tree_sum_error_bound(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal(n) * np.exp(rng.uniform(-5, 5, n))
    m = max(1, math.ceil(math.log2(n)))
    gamma = m * U / (1 - m * U)
    assert abs(O.tree_sum(a) - math.fsum(a)) <= gamma * math.fsum(np.abs(a)) + 1e-300


def test_tree_sum_is_not_sequential():
    # 1 followed by 2^20 copies of 2^-53: a left-to-right sum stays at 1.0,
    # a balanced pairwise sum must be within its log2(n) error bound of the truth.
    a = np.full(2 ** 20 + 1, 2.0 ** -53)
    a[0] = 1.0
    exact = math.fsum(a)
    seq = 0.0
    for v in a[:4]:
        seq += v
    assert seq == 1.0 and exact > 1.0
    m = math.ceil(math.log2(a.size))
    assert abs(O.tree_sum(a) - exact) <= m * U * math.fsum(a)


def test_tree_sum_exact_on_integers():
    rng = np.random.default_rng(1)
    a = rng.integers(-1000, 1000, 77777).astype(float)
    assert O.tree_sum(a) == float(a.sum())


# ---------------------------------------------------------------- scaling
def test_scaling_closed_forms():
    sl, si, x, y, k = O.scaling(np.array([1, 3], np.int32), np.array([-1.0, 1.0]), scl=1.0)
    assert sl == 1.0 and si == 1.0
    assert x.tolist() == [1.0, 3.0] and y.tolist() == [-1.0, 1.0]
    assert k.tolist() == [math.sqrt(2.0), math.sqrt(10.0)]
    # zero deviation is replaced by 1
    sl, si, *_ = O.scaling(np.array([2, 2, 2], np.int32), np.array([0.5, 0.5, 0.5]))
    assert sl == 1.0 and si == 1.0
    # scl = 0 drops the length coordinate
    sl, si, x, y, k = O.scaling(np.array([1, 5], np.int32), np.array([0.0, 2.0]), scl=0.0)
    assert x.tolist() == [0.0, 0.0]


def test_scaling_matches_numpy_std():
    rng = np.random.default_rng(2)
    ln = rng.integers(1, 40, 50_000).astype(np.int32)
    inc = rng.standard_normal(50_000) * 0.7 + 0.1
    sl, si, x, y, k = O.scaling(ln, inc, scl=1.0)
    assert abs(sl - np.std(ln.astype(float))) <= 1e-13 * sl
    assert abs(si - np.std(inc)) <= 1e-13 * si
    np.testing.assert_array_equal(x, 1.0 * (ln / sl))
    np.testing.assert_array_equal(y, inc / si)
    np.testing.assert_allclose(k, np.hypot(x, y), rtol=4 * U, atol=0)


# ---------------------------------------------------------------- sort and blocks
def test_sort_matches_lexsort_with_ties():
    rng = np.random.default_rng(3)
    key = rng.integers(0, 50, 20_000) * 0.125
    perm = O.sort_order(key)
    np.testing.assert_array_equal(perm, np.lexsort((np.arange(key.size), key)))


@pytest.mark.parametrize("B", [1, 2, 7, 64, 1000, 10**6])
def test_blocks_never_split_equal_keys(B):
    rng = np.random.default_rng(B)
    sk = np.sort(rng.integers(0, 300, 5000) * 0.5)
    bs = O.blocks(sk, B)
    N = sk.size
    assert bs[0] == 0 and bs[-1] == N
    assert np.all(np.diff(bs) > 0)
    # brute force: cut j is the first p >= j*B whose key differs from its predecessor
    cuts = set()
    for j in range(1, -(-N // B)):
        p = j * B
        while p < N and sk[p] == sk[p - 1]:
            p += 1
        if p < N:
            cuts.add(p)
    assert bs[1:-1].tolist() == sorted(cuts)
    for c in bs[1:-1]:
        assert sk[c] != sk[c - 1]


# ---------------------------------------------------------------- aggregation
def unpruned_greedy(x, y, alpha):
    """Serial greedy aggregation without the sorted-key early stop (O(n^2))."""
    n = len(x)
    lab = [-1] * n
    a2 = alpha * alpha
    for p in range(n):
        if lab[p] != -1:
            continue
        lab[p] = p
        for q in range(p + 1, n):
            if lab[q] == -1:
                dx, dy = x[q] - x[p], y[q] - y[p]
                if dx * dx + dy * dy <= a2:
                    lab[q] = p
    return lab


@pytest.mark.parametrize("seed", range(25))
def test_pruned_greedy_equals_unpruned(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 300))
    x = rng.integers(0, 24, n) * 0.125
    y = rng.integers(-24, 24, n) * 0.125
    alpha = float(rng.choice([0.2, 0.3, 0.45, 0.7]))
    key = np.sqrt(x * x + y * y)
    perm = np.lexsort((np.arange(n), key))
    sx, sy, sk = x[perm], y[perm], key[perm]
    lab = O.aggregate_sorted(sx, sy, sk, alpha)
    assert lab.tolist() == unpruned_greedy(sx.tolist(), sy.tolist(), alpha)


def _pieces(seed, n=3000):
    rng = np.random.default_rng(seed)
    vals = np.cumsum(rng.standard_normal(n * 4))
    vals = (vals - vals.mean()) / vals.std()
    ln, inc, _ = O.compress(vals, np.array([0, vals.size]), D=500, tol=0.05)
    return ln, inc


def _exact_d2(x1, y1, x2, y2):
    return (F(x1) - F(x2)) ** 2 + (F(y1) - F(y2)) ** 2


@pytest.mark.parametrize("B", [64, 512, 4096])
@pytest.mark.parametrize("alpha", [0.05, 0.2])
def test_stage_invariants(B, alpha):
    ln, inc = _pieces(11)
    d = O.digitize(ln, inc, alpha=alpha, scl=1.0, B=B)
    sl, si, x, y, key = O.scaling(ln, inc)
    N = ln.size
    perm, lst = d.perm, d.local_start
    a2 = F(alpha) ** 2
    # Stage I: every member within alpha of its local start (exact arithmetic)
    for i in range(N):
        p = lst[i]
        assert p <= i
        if p != i:
            assert _exact_d2(x[perm[i]], y[perm[i]], x[perm[p]], y[perm[p]]) <= a2 * (1 + F(1, 10**9))
    # Var per local group <= alpha^2 (Eq. Var2), SSE <= alpha^2 (N - k_local)
    groups = {}
    for i in range(N):
        groups.setdefault(lst[i], []).append(perm[i])
    sse = 0.0
    for members in groups.values():
        gx, gy = x[members], y[members]
        assert np.var(gx) <= alpha ** 2 * (1 + 1e-9) and np.var(gy) <= alpha ** 2 * (1 + 1e-9)
        sse += float(((gx - gx.mean()) ** 2 + (gy - gy.mean()) ** 2).sum())
    assert sse <= alpha ** 2 * (N - len(groups)) * (1 + 1e-9)
    assert len(groups) == d.n_starts
    # Final groups: within 2 alpha of the global start (triangle inequality)
    start_of_sym = {}
    for i in range(N):
        if lst[i] == i:
            s = d.symbols[perm[i]]
            start_of_sym.setdefault(s, i)  # smallest sorted position = global start
    for i in range(N):
        g = start_of_sym[d.symbols[perm[i]]]
        dd = _exact_d2(x[perm[i]], y[perm[i]], x[perm[g]], y[perm[g]])
        assert dd <= 4 * a2 * (1 + F(1, 10**9))
    assert d.k <= d.n_starts
    assert sorted(set(d.symbols.tolist())) == list(range(d.k))


def _serial_symbols(ln, inc, alpha, scl=1.0):
    sl, si, x, y, key = O.scaling(ln, inc, scl)
    perm = np.lexsort((np.arange(ln.size), key))
    lab = O.aggregate_sorted(x[perm], y[perm], key[perm], alpha)
    sym_of_start = {}
    out = np.zeros(ln.size, np.int32)
    for i in range(ln.size):
        if lab[i] == i:
            sym_of_start[i] = len(sym_of_start)
        out[perm[i]] = sym_of_start[lab[i]]
    return out


@pytest.mark.parametrize("alpha", [0.02, 0.05, 0.3])
def test_single_block_equals_serial_aggregation(alpha):
    ln, inc = _pieces(21)
    d = O.digitize(ln, inc, alpha=alpha, B=10**9)
    assert d.n_blocks == 1
    np.testing.assert_array_equal(d.symbols, _serial_symbols(ln, inc, alpha))
    assert d.k == d.n_starts  # Stage II is the identity on mutually distant starts


@pytest.mark.parametrize("alpha", [0.02, 0.05, 0.3])
def test_unit_blocks_equal_serial_aggregation_when_keys_distinct(alpha):
    ln, inc = _pieces(31, n=1500)
    _, _, _, _, key = O.scaling(ln, inc)
    assert np.unique(key).size == key.size
    d = O.digitize(ln, inc, alpha=alpha, B=1)
    assert d.n_starts == ln.size
    np.testing.assert_array_equal(d.symbols, _serial_symbols(ln, inc, alpha))


@pytest.mark.parametrize("B", [1, 3, 50, 4096])
def test_identical_pieces_get_identical_symbols(B):
    ln, inc = _pieces(41, n=800)
    rng = np.random.default_rng(B)
    src = rng.integers(0, ln.size, 300)
    dst = rng.integers(0, ln.size + 300, 300)
    ln2, inc2 = ln.tolist(), inc.tolist()
    for s, d_ in zip(src, dst):
        ln2.insert(int(d_), int(ln[s]))
        inc2.insert(int(d_), float(inc[s]))
    ln2 = np.array(ln2, np.int32)
    inc2 = np.array(inc2)
    d = O.digitize(ln2, inc2, alpha=0.05, B=B)
    seen = {}
    for i in range(ln2.size):
        key = (int(ln2[i]), float(inc2[i]))
        if key in seen:
            assert d.symbols[i] == seen[key]
        seen[key] = d.symbols[i]


def test_dictionary_means():
    ln, inc = _pieces(51)
    d = O.digitize(ln, inc, alpha=0.05, B=512)
    for c in range(d.k):
        m = d.symbols == c
        cnt = int(m.sum())
        assert d.count[c] == cnt
        assert d.center_len[c] == int(ln[m].astype(np.int64).sum()) / cnt  # correctly rounded int / int
        assert d.center_inc[c] == math.fsum(inc[m]) / cnt
    np.testing.assert_array_equal(d.cx, 1.0 * (d.center_len / d.sigma_len))
    np.testing.assert_array_equal(d.cy, d.center_inc / d.sigma_inc)


def test_degenerate_digitize():
    d = O.digitize(np.zeros(0, np.int32), np.zeros(0), alpha=0.1)
    assert d.k == 0 and d.symbols.size == 0
    d = O.digitize(np.array([3], np.int32), np.array([0.5]), alpha=0.0)
    assert d.k == 1 and d.center_len[0] == 3.0 and d.center_inc[0] == 0.5
    # alpha = 0: only identical scaled pieces share a symbol
    ln, inc = _pieces(61, n=500)
    d = O.digitize(ln, inc, alpha=0.0, B=64)
    pairs = set(zip(ln.tolist(), inc.tolist()))
    assert d.k == len(pairs)
    with pytest.raises(O.OracleError):
        O.digitize(np.array([1, 2], np.int32), np.array([0.0, np.nan]), alpha=0.1)
    with pytest.raises(O.OracleError):
        O.digitize(np.array([1, 2], np.int32), np.array([0.0, 1.0]), alpha=0.1, capacity=1)


# ---------------------------------------------------------------- encode
def test_encode_matches_numpy_argmin():
    ln, inc = _pieces(71)
    d = O.digitize(ln, inc, alpha=0.05, B=4096)
    rng = np.random.default_rng(9)
    q_ln = rng.integers(1, 30, 5000).astype(np.int32)
    q_inc = rng.standard_normal(5000)
    sym = O.encode(q_ln, q_inc, d.sigma_len, d.sigma_inc, 1.0, d.cx, d.cy)
    x = 1.0 * (q_ln / d.sigma_len)
    y = q_inc / d.sigma_inc
    dx = x[:, None] - d.cx[None, :]
    dy = y[:, None] - d.cy[None, :]
    np.testing.assert_array_equal(sym, np.argmin(dx * dx + dy * dy, axis=1))


def test_encode_centers_map_to_themselves_and_ties_go_low():
    cx = np.array([1.0, 2.0, 2.0, 3.0])
    cy = np.array([0.0, 0.5, 0.5, -1.0])
    ln = np.array([1, 2, 3], np.int32)
    inc = np.array([0.0, 0.5, -1.0])
    sym = O.encode(ln, inc, 1.0, 1.0, 1.0, cx, cy)
    assert sym.tolist() == [0, 1, 3]
