"""Pins for the oracle's two-stage aggregation of raw 2-D points (Sec. 5 and
the Gaussian-blob experiment of Sec. 7.1).

One block is the serial greedy aggregation: checked against a brute-force
greedy that scans every later point (no sorted-key pruning at all), so the
pruning of the sorted scan is pinned too.  Centers are member means, the SSE
is Eq. sse evaluated in numpy and stays under the paper's bound
alpha^2 (N - k) for the serial case; blocks of one point with distinct keys
reduce to the serial result as well.
"""
import numpy as np
import pytest

import oracle as O


def _blobs(seed, n, k=6, spread=0.3):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-3, 3, (k, 2))
    pick = rng.integers(0, k, n)
    p = centers[pick] + rng.normal(0, spread, (n, 2))
    return p[:, 0].copy(), p[:, 1].copy()


def _greedy_no_pruning(x, y, alpha):
    # sort by norm (ties by index); each unassigned point in that order
    # starts a group and takes every later unassigned point within alpha
    n = x.size
    key = np.sqrt(x * x + y * y)
    order = sorted(range(n), key=lambda i: (key[i], i))
    lab = -np.ones(n, np.int64)
    k = 0
    for a, i in enumerate(order):
        if lab[i] >= 0:
            continue
        lab[i] = k
        for j in order[a + 1:]:
            if lab[j] < 0 and (x[j] - x[i]) ** 2 + (y[j] - y[i]) ** 2 <= alpha * alpha:
                lab[j] = k
        k += 1
    return lab, k


@pytest.mark.parametrize("seed,alpha", [(1, 0.1), (2, 0.25), (3, 0.05)])
def test_one_block_is_the_serial_greedy(seed, alpha):
    x, y = _blobs(seed, 400)
    a = O.aggregate_points(x, y, alpha)
    lab, k = _greedy_no_pruning(x, y, alpha)
    assert a.k == k and a.n_blocks == 1
    np.testing.assert_array_equal(a.labels, lab)


def test_centers_counts_and_sse():
    x, y = _blobs(4, 3000)
    alpha = 0.1
    for B in (1 << 40, 375):
        a = O.aggregate_points(x, y, alpha, B)
        cnt = np.bincount(a.labels, minlength=a.k)
        np.testing.assert_array_equal(a.count, cnt)
        np.testing.assert_allclose(a.cx, np.bincount(a.labels, weights=x) / cnt, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(a.cy, np.bincount(a.labels, weights=y) / cnt, rtol=1e-12, atol=1e-14)
        sse = np.sum((x - a.cx[a.labels]) ** 2 + (y - a.cy[a.labels]) ** 2)
        np.testing.assert_allclose(a.sse, sse, rtol=1e-12)
    serial = O.aggregate_points(x, y, alpha)
    assert serial.sse <= alpha ** 2 * (x.size - serial.k)


def test_unit_blocks_with_distinct_keys_equal_serial():
    x, y = _blobs(5, 500)
    a1 = O.aggregate_points(x, y, 0.2, 1)
    a = O.aggregate_points(x, y, 0.2)
    assert a1.n_blocks == 500
    np.testing.assert_array_equal(a1.labels, a.labels)


def test_two_stage_members_within_two_alpha_of_their_symbol_start():
    # a member joins a Stage I start within alpha, which joins its global
    # start within alpha; every cluster's diameter is therefore at most 4 alpha
    x, y = _blobs(6, 4000)
    alpha = 0.1
    a = O.aggregate_points(x, y, alpha, 500)
    for c in range(a.k):
        m = a.labels == c
        px, py = x[m], y[m]
        d2 = (px[:, None] - px[None, :]) ** 2 + (py[:, None] - py[None, :]) ** 2
        assert d2.max() <= (4 * alpha) ** 2 * (1 + 1e-12)


def test_degenerate_inputs():
    a = O.aggregate_points(np.zeros(0), np.zeros(0), 0.1)
    assert a.k == 0 and a.sse == 0.0
    a = O.aggregate_points(np.array([0.3]), np.array([-2.0]), 0.1)
    assert a.k == 1 and a.cx.tolist() == [0.3] and a.cy.tolist() == [-2.0] and a.sse == 0.0
    a = O.aggregate_points(np.full(50, 1.5), np.full(50, -0.5), 0.0, 7)
    assert a.k == 1 and a.count.tolist() == [50] and a.sse == 0.0
    with pytest.raises(O.OracleError):
        O.aggregate_points(np.array([np.nan]), np.array([0.0]), 0.1)
