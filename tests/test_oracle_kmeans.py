"""Pins for the oracle's k-means digitization (Sec. 3.2, Lloyd's algorithm).

Checked against a hand-worked case, against scikit-learn's Lloyd iterations
on well separated clusters (no empty cluster, so no relocation rule
differs), and against the fixed-point properties a converged result must
have: every piece is nearest to its own center (brute force in numpy) and
every center is its members' mean.
"""
import numpy as np
import pytest

import oracle as O


def test_hand_worked_two_clusters():
    # sigma = scl = 1: x = len, y = inc.  Two groups; initial centers on one
    # member of each; one update moves each center to its group's mean.
    ln = np.array([1, 1, 2, 9, 10, 10], np.int32)
    inc = np.array([0.0, 1.0, 0.5, 4.0, 5.0, 6.0])
    r = O.kmeans(ln, inc, 1.0, 1.0, 1.0, [1.0, 10.0], [0.0, 5.0], 10)
    np.testing.assert_array_equal(r.symbols, [0, 0, 0, 1, 1, 1])
    np.testing.assert_array_equal(r.count, [3, 3])
    assert r.center_len.tolist() == [4 / 3, 29 / 3]
    assert r.center_inc.tolist() == [0.5, 5.0]
    assert r.cx.tolist() == [4 / 3, 29 / 3] and r.cy.tolist() == [0.5, 5.0]
    assert r.iterations == 2  # the second assignment repeats the first


def _blobs(seed, k, per, spread):
    rng = np.random.default_rng(seed)
    lens, incs = [], []
    for c in range(k):
        L0 = 2 + 6 * c
        I0 = rng.uniform(-3, 3)
        lens.append(np.clip(np.round(L0 + rng.normal(0, spread, per)), 1, None).astype(np.int32))
        incs.append(I0 + rng.normal(0, 0.05, per))
    return np.concatenate(lens), np.concatenate(incs)


def test_matches_scikit_learn_lloyd():
    sklearn = pytest.importorskip("sklearn.cluster")
    ln, inc = _blobs(3, 6, 300, 0.8)
    sl, si, scl = 1.7, 0.9, 1.0
    X = np.stack([scl * (ln / sl), inc / si], axis=1)
    init = X[[0, 300, 600, 900, 1200, 1500]]
    r = O.kmeans(ln, inc, sl, si, scl, init[:, 0], init[:, 1], 100)
    km = sklearn.KMeans(n_clusters=6, init=init, n_init=1, max_iter=100, tol=0.0, algorithm="lloyd").fit(X)
    np.testing.assert_array_equal(r.symbols, km.labels_)
    np.testing.assert_allclose(r.cx, km.cluster_centers_[:, 0], rtol=1e-12)
    np.testing.assert_allclose(r.cy, km.cluster_centers_[:, 1], rtol=1e-12)


def test_converged_fixed_point():
    rng = np.random.default_rng(7)
    ln = rng.integers(1, 20, 2000).astype(np.int32)
    inc = rng.normal(0, 1, 2000)
    sl, si, scl = 5.0, 1.1, 2.0
    x, y = scl * (ln / sl), inc / si
    pick = rng.choice(2000, 25, replace=False)
    r = O.kmeans(ln, inc, sl, si, scl, x[pick], y[pick], 500)
    assert r.iterations < 500
    # nearest center by brute force (ties to the lowest index)
    d2 = (x[:, None] - r.cx[None, :]) ** 2 + (y[:, None] - r.cy[None, :]) ** 2
    np.testing.assert_array_equal(r.symbols, np.argmin(d2, axis=1))
    for c in range(25):
        m = r.symbols == c
        if m.any():
            assert r.count[c] == m.sum()
            assert r.center_len[c] == ln[m].sum() / m.sum()
            np.testing.assert_allclose(r.center_inc[c], inc[m].mean(), rtol=1e-13)


def test_sse_never_increases():
    rng = np.random.default_rng(11)
    ln = rng.integers(1, 10, 500).astype(np.int32)
    inc = rng.normal(0, 1, 500)
    x, y = ln / 3.0, inc
    cx0, cy0 = x[:8].copy(), y[:8].copy()
    prev = None
    for it in range(1, 8):
        r = O.kmeans(ln, inc, 3.0, 1.0, 1.0, cx0, cy0, it)
        sse = float(np.sum((x - r.cx[r.symbols]) ** 2 + (y - r.cy[r.symbols]) ** 2))
        if prev is not None:
            assert sse <= prev * (1 + 1e-12)
        prev = sse


def test_lloyd_from_the_aggregation_codebook_lowers_its_sse():
    # Lloyd seeded with the greedy aggregation's centers ends at or below the
    # aggregation's SSE (Sec. 5: aggregation is a suboptimal k-means solution),
    # which itself stays under alpha^2 (N - k).
    rng = np.random.default_rng(5)
    ln = rng.integers(1, 6, 3000).astype(np.int32)
    inc = rng.normal(0, 1, 3000)
    alpha = 0.2
    d = O.digitize(ln, inc, alpha, 1.0, 1 << 30)
    agg = O.quality(ln, inc, d.symbols, d.sigma_len, d.sigma_inc, 1.0, d.cx, d.cy).sse
    assert agg <= alpha ** 2 * (ln.size - d.k) * (1 + 1e-12)
    r = O.kmeans(ln, inc, d.sigma_len, d.sigma_inc, 1.0, d.cx.copy(), d.cy.copy(), 50)
    km = O.quality(ln, inc, r.symbols, d.sigma_len, d.sigma_inc, 1.0, r.cx, r.cy).sse
    assert km <= agg * (1 + 1e-12)
    assert km < agg  # the aggregation's assignment is not nearest-center here, so Lloyd moves it
