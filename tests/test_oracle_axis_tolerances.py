"""Pins for separate length and increment tolerances (Sec. 3.2, Eq. Var1).

The variant's test is ((x - x_s)/alpha_len)^2 + ((y - y_s)/alpha_inc)^2 <= 1.
Checked: equal tolerances give the plain aggregation; with one block every
member passes that test against its start when evaluated directly in the
unrescaled space, and every symbol meets Var_len <= alpha_len^2 and
Var_inc <= alpha_inc^2 (Eq. Var1) computed by brute force; a tolerance that
widens one axis lets pieces join that the disc keeps apart.  The library's
host helper returns the same parameters.
"""
import ctypes as C

import numpy as np
import pytest

import oracle as O


def _pieces(seed, n=3000):
    rng = np.random.default_rng(seed)
    ln = rng.integers(1, 30, n).astype(np.int32)
    inc = 0.2 * ln + rng.normal(0, 1.5, n)
    return ln, inc


def test_equal_tolerances_are_the_aggregation():
    ln, inc = _pieces(1)
    for a in (0.05, 0.2):
        al, s = O.axis_tolerances(a, a, 1.7)
        assert al == a and s == 1.7
        d0 = O.digitize(ln, inc, a, 1.7, 256)
        d1 = O.digitize(ln, inc, al, s, 256)
        np.testing.assert_array_equal(d0.symbols, d1.symbols)


@pytest.mark.parametrize("alen,ainc", [(0.4, 0.05), (0.05, 0.3), (0.2, 0.2), (1.0, 0.01)])
def test_members_inside_the_ellipse_and_var_bounds(alen, ainc):
    ln, inc = _pieces(2)
    scl = 1.0
    alpha, s = O.axis_tolerances(alen, ainc, scl)
    d = O.digitize(ln, inc, alpha, s, 1 << 30)            # one block: the serial greedy
    x = scl * (ln / d.sigma_len)                           # unrescaled space
    y = inc / d.sigma_inc
    st = d.perm[d.local_start]
    mem = d.perm
    q = ((x[mem] - x[st]) / alen) ** 2 + ((y[mem] - y[st]) / ainc) ** 2
    assert np.all(q <= 1.0 + 1e-12)
    for c in range(d.k):
        m = d.symbols == c
        assert np.var(x[m]) <= alen ** 2 * (1 + 1e-12)
        assert np.var(y[m]) <= ainc ** 2 * (1 + 1e-12)
    assert max(np.var(x[d.symbols == c]) for c in range(d.k)) <= max(alen, ainc) ** 2 * (1 + 1e-12)


def test_wider_length_tolerance_merges_what_the_disc_separates():
    # two pieces per increment level whose scaled lengths differ by more than
    # alpha: the disc keeps them apart, alpha_len = 4 alpha joins them
    ln = np.array([1, 2] * 50, np.int32)
    inc = np.repeat(np.linspace(-1, 1, 50), 2)
    a = 0.02
    d_disc = O.digitize(ln, inc, a, 1.0, 1 << 30)
    alpha, s = O.axis_tolerances(4.0, a, 1.0)
    d_ell = O.digitize(ln, inc, alpha, s, 1 << 30)
    assert d_disc.k == 100            # every piece alone: lengths 1 and 2 are 2 scaled units apart
    assert d_ell.k == 50              # each increment level becomes one symbol
    for c in range(d_ell.k):
        assert sorted(ln[d_ell.symbols == c].tolist()) == [1, 2]


def test_bad_tolerances_rejected():
    for bad in [(0.0, 0.1), (0.1, 0.0), (-1.0, 0.1), (np.nan, 0.1), (0.1, np.inf)]:
        with pytest.raises(ValueError):
            O.axis_tolerances(*bad)


def test_library_helper_agrees():
    from paper_2401_00109_amd import _lib
    L = _lib.lib()
    a, s = C.c_double(), C.c_double()
    for alen, ainc, scl in [(0.4, 0.05, 1.0), (0.05, 0.3, 2.5), (0.1, 0.1, 0.0), (3.0, 1e-3, 0.7)]:
        assert L.jabba_axis_tolerances(alen, ainc, scl, C.byref(a), C.byref(s)) == 0
        assert (a.value, s.value) == O.axis_tolerances(alen, ainc, scl)
    for bad in [(0.0, 0.1, 1.0), (0.1, -0.1, 1.0), (0.1, 0.1, -1.0), (float("nan"), 0.1, 1.0)]:
        assert L.jabba_axis_tolerances(*bad, C.byref(a), C.byref(s)) == _lib.JABBA_EINVAL
