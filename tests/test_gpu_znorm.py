"""Compression of z-normalised series on the device (the normalisation fused
into the compression's loads) against the oracle's normalise-then-compress:
per-series mean and deviation and the pieces bit-exact."""
import numpy as np
import pytest

import oracle as O
from gpu_util import gpu_compress, say
from paper_2401_00109_amd.inputs import make_workload

pytestmark = pytest.mark.gpu


def _raw(seed, lengths, scale=5.0, offset=3.0):
    rng = np.random.default_rng(seed)
    series = [offset + scale * np.cumsum(rng.standard_normal(n)) for n in lengths]
    so = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    v = np.concatenate(series) if series else np.zeros(0)
    return v, so


def _check(v, so, D, tol, tuning=None):
    ln, inc, po, st, m, sd = gpu_compress(v, so, D, tol, tuning=tuning, znorm=True)
    assert st == 0
    z, om, osd = O.znorm(v, so)
    np.testing.assert_array_equal(m.view(np.uint64), om.view(np.uint64))
    np.testing.assert_array_equal(sd.view(np.uint64), osd.view(np.uint64))
    ol, oi, opo = O.compress(z, so, D, tol)
    np.testing.assert_array_equal(ln, ol)
    np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))
    np.testing.assert_array_equal(po, opo)
    return ln.size


@pytest.mark.parametrize("lengths,D", [([1000] * 16, 999), ([10_000] * 40, 1000), ([1, 2, 3, 1025, 0, 70_001, 5], 500),
                                       ([1_100_000], 4096)])
def test_znorm_compress_parity(lengths, D):
    v, so = _raw(len(lengths), lengths)
    say(f"znorm compress {len(lengths)} series, {v.size} points, D={D}")
    n = _check(v, so, D, 0.05)
    say(f"  pieces {n}")


@pytest.mark.parametrize("W", [1, 4, 64])
def test_znorm_lane_width_never_changes_results(W):
    v, so = _raw(9, [3000] * 8)
    say(f"znorm compress, {W} lanes per domain")
    _check(v, so, 400, 0.1, tuning={"lanes_per_domain": W})


@pytest.mark.parametrize("G", [-1, 32, 77])
def test_znorm_segments_never_change_results(G):
    v, so = _raw(10, [5000] * 6 + [123])
    say(f"znorm compress, segments of {G} intervals")
    _check(v, so, 2000, 0.05, tuning={"segment_intervals": G})


def test_znorm_degenerate_series():
    v = np.concatenate([np.full(500, 7.0), [3.0], 2.0 + 0.25 * np.arange(800)])
    so = np.array([0, 500, 501, 501, 1301], np.int64)
    say("znorm compress: constant, one-point, empty and straight series")
    _check(v, so, 100, 0.01)


def test_znorm_of_normalised_workload_is_near_identity():
    # the workloads are already z-normalised on the host: the device statistics are (0, 1) up to rounding
    w = make_workload(1, seed=0, scale=1.0)
    ln, inc, po, st, m, sd = gpu_compress(w.values, w.series_off, w.D, w.tol, znorm=True)
    assert st == 0
    assert np.all(np.abs(m) < 1e-12) and np.all(np.abs(sd - 1.0) < 1e-12)
