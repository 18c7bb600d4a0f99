"""Pins for the oracle's inverse symbolization (Sec. 3.3, Eq. repolygon).

  * quantization: sum of len^ over the first j pieces equals round(sum of len~)
    (halves away from zero), checked with exact rationals; every len^ >= 1;
  * alpha = 0 with distinct pieces: the dictionary is the pieces themselves and
    the reconstruction is the compression polyline;
  * inverse compression of exact integer piecewise-linear data is exact;
  * the reported MSE equals the mean squared difference recomputed by numpy.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle as O


def round_half_away(q: F) -> int:
    return int(math.floor(q + F(1, 2))) if q >= 0 else -int(math.floor(-q + F(1, 2)))


def _workload(seed, n_series=6, n=700):
    rng = np.random.default_rng(seed)
    ser = []
    for _ in range(n_series):
        v = np.cumsum(rng.standard_normal(n))
        ser.append((v - v.mean()) / v.std())
    off = np.arange(n_series + 1, dtype=np.int64) * n
    return np.concatenate(ser), off


@pytest.mark.parametrize("alpha", [0.05, 0.1, 0.4])
def test_quantization_closed_form(alpha):
    vals, off = _workload(1)
    ln, inc, po = O.compress(vals, off, D=200, tol=0.1)
    d = O.digitize(ln, inc, alpha=alpha, B=256)
    t0 = vals[off[:-1]]
    out, oo, lhat, sse, cnt = O.reconstruct(d.symbols, po, off, t0, d.center_len, d.center_inc, orig=vals)
    for s in range(off.size - 1):
        a, b = po[s], po[s + 1]
        acc = F(0)
        tot = 0
        for j in range(a, b):
            lt = F(float(d.center_len[d.symbols[j]]))
            acc += lt
            tot += int(lhat[j])
            assert tot == round_half_away(acc)
            assert abs(acc - tot) <= F(1, 2)
            assert lhat[j] >= 1
        assert oo[s + 1] - oo[s] == 1 + tot
    # MSE over min(n, n^) points, recomputed with numpy
    for s in range(off.size - 1):
        n = off[s + 1] - off[s]
        m = min(n, oo[s + 1] - oo[s])
        ref = float(np.sum((vals[off[s]:off[s] + m] - out[oo[s]:oo[s] + m]) ** 2))
        assert cnt[s] == m
        assert abs(sse[s] - ref) <= 1e-12 * max(ref, 1.0)


def test_alpha_zero_reproduces_compression_polyline():
    vals, off = _workload(2)
    ln, inc, po = O.compress(vals, off, D=300, tol=0.05)
    pairs = list(zip(ln.tolist(), inc.tolist()))
    assert len(set(pairs)) == len(pairs)
    d = O.digitize(ln, inc, alpha=0.0, B=4096)
    assert d.k == ln.size
    t0 = vals[off[:-1]]
    out, oo, lhat, _, _ = O.reconstruct(d.symbols, po, off, t0, d.center_len, d.center_inc)
    np.testing.assert_array_equal(lhat, ln)
    np.testing.assert_array_equal(oo, off)
    out2, oo2 = O.reconstruct_pieces(ln, inc, po, t0)
    np.testing.assert_array_equal(oo2, off)
    np.testing.assert_array_equal(out, out2)
    # break points sit on the series up to the rounding of the running sum
    ends = off[:-1].repeat(np.diff(po)) + np.concatenate([np.cumsum(ln[po[s]:po[s + 1]]) for s in range(off.size - 1)])
    np.testing.assert_allclose(out[ends], vals[ends], rtol=0, atol=1e-12)


def test_inverse_compression_exact_on_integer_pwl():
    rng = np.random.default_rng(4)
    n = 400
    knots = np.sort(rng.choice(np.arange(1, n - 1), 9, replace=False))
    bps = np.concatenate(([0], knots, [n - 1]))
    vals = np.zeros(n)
    for i in range(bps.size - 1):
        a, b = bps[i], bps[i + 1]
        vals[a + 1:b + 1] = vals[a] + (2 * (i % 2) - 1) * (i + 1) * np.arange(1, b - a + 1)
    ln, inc, po = O.compress(vals, np.array([0, n]), D=1000, tol=0.0)
    out, oo = O.reconstruct_pieces(ln, inc, po, vals[:1])
    # slopes are integers, so every interpolated value is exact
    np.testing.assert_array_equal(out, vals)


def test_reconstruct_degenerate_series():
    vals = np.array([5.0, 1.0, 2.0, 4.0])
    off = np.array([0, 0, 1, 4], np.int64)  # empty, single point, 3 points
    ln, inc, po = O.compress(vals, off, D=10, tol=0.0)
    assert po.tolist() == [0, 0, 0, 2]
    d = O.digitize(ln, inc, alpha=0.0)
    t0 = np.array([0.0, 5.0, 1.0])
    out, oo, lhat, _, _ = O.reconstruct(d.symbols, po, off, t0, d.center_len, d.center_inc)
    assert oo.tolist() == [0, 0, 1, 4]
    assert out.tolist() == [5.0, 1.0, 2.0, 4.0]


def test_half_lengths_round_away_from_zero():
    # two symbols with center lengths 1.5 and 2.5: cumulative 1.5 -> 2, 4.0 -> 4
    sym = np.array([0, 1, 0], np.int32)
    po = np.array([0, 3], np.int64)
    off = np.array([0, 9], np.int64)
    out, oo, lhat, _, _ = O.reconstruct(sym, po, off, np.array([0.0]), np.array([1.5, 2.5]),
                                        np.array([1.0, -1.0]))
    assert lhat.tolist() == [2, 2, 2]   # 1.5->2, 4.0->4, 5.5->6
    assert oo.tolist() == [0, 7]
    assert out.tolist() == [0.0, 0.5, 1.0, 0.5, 0.0, 0.5, 1.0]
