"""Pins for the oracle's series z-normalisation (the preprocessing ahead of
compression): closed forms on small integer series (every sum exact), numpy's
mean and population deviation on random series, the degenerate series, and
compression of a normalised straight line (one piece per domain)."""
import numpy as np
import pytest

import oracle as O


def test_closed_form_small_series():
    v = np.array([1.0, 2.0, 3.0, 4.0, 10.0, 10.0, 10.0, 7.0])
    so = np.array([0, 4, 7, 8])
    z, m, sd = O.znorm(v, so)
    assert m.tolist() == [2.5, 10.0, 7.0]
    assert sd.tolist() == [np.sqrt(1.25), 1.0, 1.0]       # constant and one-point series: only centred
    np.testing.assert_array_equal(z[:4], np.array([-1.5, -0.5, 0.5, 1.5]) / np.sqrt(1.25))
    np.testing.assert_array_equal(z[4:], [0.0, 0.0, 0.0, 0.0])


@pytest.mark.parametrize("n", [2, 1000, 1025, 5000, 70000])
def test_matches_numpy(n):
    rng = np.random.default_rng(n)
    v = 3.0 + 2.0 * rng.standard_normal(n)
    z, m, sd = O.znorm(v, np.array([0, n]))
    np.testing.assert_allclose(m[0], v.mean(), rtol=1e-14)
    np.testing.assert_allclose(sd[0], v.std(), rtol=1e-13)
    np.testing.assert_allclose(z, (v - v.mean()) / v.std(), rtol=1e-12, atol=1e-13)
    assert abs(z.mean()) < 1e-12 and abs(z.std() - 1.0) < 1e-12


def test_series_are_independent_and_empty_series():
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(300), 5 + rng.standard_normal(700)
    z, m, sd = O.znorm(np.concatenate([a, b]), np.array([0, 300, 300, 1000]))
    za, ma, sa = O.znorm(a, np.array([0, 300]))
    zb, mb, sb = O.znorm(b, np.array([0, 700]))
    np.testing.assert_array_equal(z, np.concatenate([za, zb]))
    assert m.tolist() == [ma[0], 0.0, mb[0]] and sd.tolist() == [sa[0], 1.0, sb[0]]


def test_normalised_line_compresses_to_one_piece_per_domain():
    n, D = 5001, 700
    v = 4.0 + 0.5 * np.arange(n)
    z, _, _ = O.znorm(v, np.array([0, n]))
    ln, inc, po = O.compress(z, np.array([0, n]), D, 1e-6)
    assert ln.size == -(-(n - 1) // D)
