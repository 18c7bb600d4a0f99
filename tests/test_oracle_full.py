"""The full-size oracle harness (tests/oracle_full.py) equals the oracle's own
one-call results bit for bit: chunked compression against oracle.compress,
and the step-by-step digitization against oracle.digitize (symbols, k,
starting points, counts, center lengths and increments, scaled centers), on
a workload with every generator, on tie-heavy integer data and with block
sizes from 1 to beyond N."""
import numpy as np
import pytest

import oracle as O
from paper_2401_00109_amd.inputs import make_workload

import oracle_full as F


def _check(ln, inc, alpha, scl, B, nt):
    ref = O.digitize(ln, inc, alpha, scl, B)
    st = F.Digitization(ln, inc, alpha, scl, B, n_threads=nt)
    st.scaling()
    assert st.sigma_len == ref.sigma_len and st.sigma_inc == ref.sigma_inc
    st.sort()
    np.testing.assert_array_equal(st.perm, ref.perm)
    st.stage1()
    assert st.G == ref.n_starts
    np.testing.assert_array_equal(st.lab, ref.local_start)
    st.stage2()
    assert st.k == ref.k
    np.testing.assert_array_equal(st.gmap[: st.G], ref.gmap)
    np.testing.assert_array_equal(st.symbols, ref.symbols)
    st.centers()
    np.testing.assert_array_equal(st.count, ref.count)
    np.testing.assert_array_equal(st.center_len.view(np.uint64), ref.center_len.view(np.uint64))
    np.testing.assert_array_equal(st.cx.view(np.uint64), ref.cx.view(np.uint64))
    np.testing.assert_array_equal(st.center_inc.view(np.uint64), ref.center_inc.view(np.uint64))
    np.testing.assert_array_equal(st.cy.view(np.uint64), ref.cy.view(np.uint64))


def test_chunked_compress_equals_one_call():
    w = make_workload(3, seed=0, scale=0.01)
    ref = O.compress(w.values, w.series_off, w.D, w.tol)
    for nt in (1, 3, 8):
        got = F.compress(w.values, w.series_off, w.D, w.tol, n_threads=nt)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))


@pytest.mark.parametrize("nt", [1, 5])
def test_stepwise_digitize_equals_one_call(nt):
    w = make_workload(2, seed=0, scale=0.1)
    ln, inc, _ = O.compress(w.values, w.series_off, w.D, w.tol)
    assert ln.size > (1 << 20)  # the chunked sort path runs
    _check(ln, inc, w.alpha, w.scl, w.B, nt)


@pytest.mark.parametrize("B", [1, 7, 4096, 10 ** 9])
def test_stepwise_digitize_with_ties_and_block_sizes(B):
    rng = np.random.default_rng(B)
    n = 60_000 if B == 1 else 1_300_000  # B = 1 is one block (one call) per piece
    ln = rng.integers(1, 6, n).astype(np.int32)
    inc = rng.integers(-4, 5, n) * 0.25  # many exactly equal pieces and keys
    _check(ln, inc, 0.3, 1.0, B, 4)


def test_sort_order_is_the_key_index_order():
    rng = np.random.default_rng(3)
    key = np.round(rng.standard_normal(3_000_000), 3)  # long runs of equal keys across chunks
    p = F.sort_order(key, 7)
    np.testing.assert_array_equal(p, np.lexsort((np.arange(key.size), key)))


def test_sort_order_with_one_dominant_key():
    rng = np.random.default_rng(4)
    key = np.where(rng.random(2_500_000) < 0.6, 1.5, rng.standard_normal(2_500_000))
    p = F.sort_order(key, 6)
    np.testing.assert_array_equal(p, np.lexsort((np.arange(key.size), key)))


def test_chunked_reconstruct_equals_one_call():
    w = make_workload(3, seed=0, scale=0.004)
    ln, inc, po = O.compress(w.values, w.series_off, w.D, w.tol)
    d = O.digitize(ln, inc, w.alpha, w.scl, w.B)
    t0 = np.where(np.diff(w.series_off) > 0, w.values[np.minimum(w.series_off[:-1], w.n_points - 1)], 0.0)
    ref = O.reconstruct(d.symbols, po, w.series_off, t0, d.center_len, d.center_inc, orig=w.values)
    got = F.reconstruct(d.symbols, po, w.series_off, t0, d.center_len, d.center_inc, w.values, n_threads=5)
    np.testing.assert_array_equal(got[0].view(np.uint64), ref[0].view(np.uint64))
    np.testing.assert_array_equal(got[1], ref[1])
    np.testing.assert_array_equal(got[2].view(np.uint64), ref[3].view(np.uint64))
    np.testing.assert_array_equal(got[3], ref[4])
