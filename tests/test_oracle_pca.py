"""Pins for the oracle's PCA sort key (Sec. 5: the sort key may be a PCA
projection instead of the norm).

The axis is checked against numpy's symmetric eigensolver on the plain
population covariance of the scaled points, against closed forms (scl = 1
standardises both coordinates, so the axis is a diagonal; scl = 0 leaves
only y), and against degenerate inputs.  The keyed digitization is checked
against its sort order recomputed in numpy and, for scl = 0, against a
brute-force one-dimensional run segmentation.
"""
import numpy as np
import pytest

import oracle as O


def _pieces(seed, n=4000, slope=0.3):
    rng = np.random.default_rng(seed)
    ln = rng.integers(1, 25, n).astype(np.int32)
    inc = slope * ln + rng.normal(0, 1, n)
    return ln, inc


@pytest.mark.parametrize("scl,slope", [(0.3, 0.3), (1.0, 0.3), (2.5, -0.2), (4.0, 0.05), (0.7, -1.0)])
def test_axis_is_numpy_principal_eigenvector(scl, slope):
    ln, inc = _pieces(1, slope=slope)
    sl, si = O.scaling(ln, inc, scl)[:2]
    x, y = scl * (ln / sl), inc / si
    w, v = np.linalg.eigh(np.cov(np.stack([x, y]), bias=True))
    ref = v[:, np.argmax(w)]
    ref = ref if ref[0] > 0 or (ref[0] == 0 and ref[1] > 0) else -ref
    u = O.pca_axis(ln, inc, scl)
    np.testing.assert_allclose(u, ref, atol=1e-9)
    assert abs(np.hypot(u[0], u[1]) - 1.0) < 1e-15


def test_standardised_axis_is_a_diagonal():
    # with scl = 1 both coordinates have unit variance: eigenvectors (1, +-1)/sqrt(2)
    for slope, sign in [(0.4, 1.0), (-0.4, -1.0)]:
        ln, inc = _pieces(2, slope=slope)
        u = O.pca_axis(ln, inc, 1.0)
        assert abs(u[0] - 2 ** -0.5) <= 4e-16          # within two ulps of the closed form
        assert abs(u[1] - sign * 2 ** -0.5) <= 4e-16


def test_degenerate_axes():
    ln, inc = _pieces(3)
    np.testing.assert_array_equal(O.pca_axis(ln, inc, 0.0), [0.0, 1.0])      # scl = 0: only y varies
    same_len = np.full(500, 4, np.int32)
    np.testing.assert_array_equal(O.pca_axis(same_len, inc[:500], 1.0), [0.0, 1.0])
    same_inc = np.full(500, 0.5)
    np.testing.assert_array_equal(O.pca_axis(ln[:500], same_inc, 1.0), [1.0, 0.0])
    np.testing.assert_array_equal(O.pca_axis(np.zeros(0, np.int32), np.zeros(0), 1.0), [1.0, 0.0])
    # uncorrelated by construction: len and inc from disjoint halves, mirrored so cov = 0 exactly
    l2 = np.array([1, 3, 1, 3], np.int32)
    i2 = np.array([-1.0, -1.0, 1.0, 1.0])
    np.testing.assert_array_equal(O.pca_axis(l2, i2, 2.0), [1.0, 0.0])     # var(x) = 4 > var(y) = 1
    np.testing.assert_array_equal(O.pca_axis(l2, i2, 0.5), [0.0, 1.0])     # var(x) = 1/4 < 1


@pytest.mark.parametrize("scl", [0.5, 1.0, 3.0])
def test_sort_order_is_the_projection(scl):
    ln, inc = _pieces(4, n=3000, slope=-0.25)
    d = O.digitize(ln, inc, 0.1, scl, 1 << 30, key="pca")
    x, y = scl * (ln / d.sigma_len), inc / d.sigma_inc
    key = d.axis[0] * x + d.axis[1] * y
    np.testing.assert_array_equal(d.perm, np.lexsort((np.arange(ln.size), key)))
    np.testing.assert_array_equal(d.axis, O.pca_axis(ln, inc, scl))


def test_members_stay_within_alpha_of_their_start():
    ln, inc = _pieces(5, n=3000)
    alpha = 0.15
    d = O.digitize(ln, inc, alpha, 1.5, 1 << 30, key="pca")
    x, y = 1.5 * (ln / d.sigma_len), inc / d.sigma_inc
    key = d.axis[0] * x + d.axis[1] * y
    st = d.perm[d.local_start]   # canonical index of each sorted position's start
    mem = d.perm
    assert np.all(key[mem] >= key[st])
    assert np.all(key[mem] - key[st] <= alpha)
    assert np.all((x[mem] - x[st]) ** 2 + (y[mem] - y[st]) ** 2 <= alpha * alpha)


def test_scl_zero_is_one_dimensional_run_segmentation():
    # scl = 0: x = 0 and the axis is (0, 1), so the key is y and one block is
    # the greedy run segmentation of the sorted increments
    rng = np.random.default_rng(6)
    ln = rng.integers(1, 9, 2500).astype(np.int32)
    inc = rng.normal(0, 1, 2500)
    alpha = 0.05
    d = O.digitize(ln, inc, alpha, 0.0, 1 << 30, key="pca")
    y = inc / d.sigma_inc
    order = sorted(range(ln.size), key=lambda i: (y[i], i))
    sym = np.empty(ln.size, np.int64)
    g, start = -1, None
    for i in order:
        if start is None or not (y[i] - start <= alpha):
            g += 1
            start = y[i]
        sym[i] = g
    np.testing.assert_array_equal(d.symbols, sym)
    assert d.k == g + 1


def test_norm_key_unchanged_by_the_key_option():
    ln, inc = _pieces(7)
    a = O.digitize(ln, inc, 0.1, 1.0, 512)
    b = O.digitize(ln, inc, 0.1, 1.0, 512, key="norm")
    np.testing.assert_array_equal(a.symbols, b.symbols)
    assert a.axis is None and b.axis is None
    with pytest.raises(ValueError):
        O.digitize(ln, inc, 0.1, 1.0, 512, key="sum")
