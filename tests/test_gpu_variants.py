"""Digitizer variants on the device against the oracle: the PCA-projection
sort key (Sec. 5), separate length and increment tolerances (Sec. 3.2,
Eq. Var1) and the length weight scl (Sec. 3.2), through the C ABI."""
import numpy as np
import pytest

import oracle as O
from gpu_util import assert_centers_close, gpu_digitize, say
from paper_2401_00109_amd.inputs import make_workload

pytestmark = pytest.mark.gpu

SMALL = {1: 1.0, 2: 0.01, 3: 0.002, 4: 1.0 / 256}


def _pieces(wid):
    w = make_workload(wid, seed=0, scale=SMALL[wid])
    ln, inc, _ = O.compress(w.values, w.series_off, w.D, w.tol, w.max_len)
    return w, ln, inc


def _same(sym, d, od, inc):
    assert d["k"] == od.k
    np.testing.assert_array_equal(sym, od.symbols)
    np.testing.assert_array_equal(d["count"], od.count)
    np.testing.assert_array_equal(d["center_len"].view(np.uint64), od.center_len.view(np.uint64))
    np.testing.assert_array_equal(d["cx"].view(np.uint64), od.cx.view(np.uint64))
    assert_centers_close(d, od, inc, od.symbols)


@pytest.mark.parametrize("wid", [1, 2, 4])
@pytest.mark.parametrize("B", [7, 256, 10**9])
def test_pca_key_parity(wid, B):
    w, ln, inc = _pieces(wid)
    say(f"pca digitize workload {wid} N={ln.size} B={B}")
    sym, d, st = gpu_digitize(ln, inc, w.alpha, w.scl, B, key="pca")
    assert st == 0
    od = O.digitize(ln, inc, w.alpha, w.scl, B, key="pca")
    np.testing.assert_array_equal(d["axis"].view(np.uint64), od.axis.view(np.uint64))
    assert d["stats"]["G"] == od.n_starts
    _same(sym, d, od, inc)


@pytest.mark.parametrize("case", ["empty", "one_piece", "identical", "same_length", "scl0", "anticorrelated",
                                  "scl3"])
def test_pca_key_edge_cases(case):
    rng = np.random.default_rng(21)
    alpha, scl, B = 0.1, 1.0, 64
    if case == "empty":
        ln, inc = np.zeros(0, np.int32), np.zeros(0)
    elif case == "one_piece":
        ln, inc = np.array([5], np.int32), np.array([-0.5])
    elif case == "identical":
        ln, inc = np.full(700, 3, np.int32), np.full(700, 0.25)
    elif case == "same_length":
        ln, inc = np.full(3000, 2, np.int32), rng.standard_normal(3000)
    elif case == "scl0":
        ln, inc = rng.integers(1, 9, 3000).astype(np.int32), rng.standard_normal(3000)
        scl = 0.0
    elif case == "anticorrelated":   # negative keys and a (1, -1) axis
        ln = rng.integers(1, 40, 5000).astype(np.int32)
        inc = -0.3 * ln + rng.normal(0, 1, 5000)
    else:
        ln = rng.integers(1, 40, 5000).astype(np.int32)
        inc = 0.1 * ln + rng.normal(0, 1, 5000)
        scl = 3.0
    say(f"pca digitize edge case {case} N={ln.size}")
    sym, d, st = gpu_digitize(ln, inc, alpha, scl, B, key="pca")
    assert st == 0
    od = O.digitize(ln, inc, alpha, scl, B, key="pca")
    np.testing.assert_array_equal(d["axis"].view(np.uint64), od.axis.view(np.uint64))
    _same(sym, d, od, inc)


@pytest.mark.parametrize("alen,ainc", [(0.4, 0.05), (0.05, 0.3), (1.0, 0.01)])
def test_axis_tolerances_parity(alen, ainc):
    import paper_2401_00109_amd as J
    w, ln, inc = _pieces(2)
    alpha, scl = J.axis_tolerances(alen, ainc, w.scl)
    assert (alpha, scl) == O.axis_tolerances(alen, ainc, w.scl)
    say(f"axis tolerances alpha_len={alen} alpha_inc={ainc} N={ln.size}")
    for key in ("norm", "pca"):
        sym, d, st = gpu_digitize(ln, inc, alpha, scl, 512, key=key)
        assert st == 0
        od = O.digitize(ln, inc, alpha, scl, 512, key=key)
        _same(sym, d, od, inc)


def test_digitizer_sweep_matches_oracle():
    from paper_2401_00109_amd import experiments as E
    settings = [{"scl": 0.0}, {"scl": 0.5}, {"scl": 2.0}, {"key": "pca"}, {"alpha_len": 0.3, "alpha_inc": 0.05}]
    say("digitizer sweep on workload 1")
    rows = E.digitizer_sweep(settings, workload_id=1, scale=1.0)
    w = make_workload(1, seed=0, scale=1.0)
    ln, inc, po = O.compress(w.values, w.series_off, w.D, w.tol, w.max_len)
    t0 = w.values[w.series_off[:-1]]
    for st, row in zip(settings, rows):
        scl, alpha = st.get("scl", w.scl), w.alpha
        if "alpha_len" in st:
            alpha, scl = O.axis_tolerances(st["alpha_len"], st["alpha_inc"], scl)
        od = O.digitize(ln, inc, alpha, scl, w.B, key=st.get("key", "norm"))
        assert row["pieces"] == ln.size and row["symbols"] == od.k and row["starts"] == od.n_starts
        q = O.quality(ln, inc, od.symbols, od.sigma_len, od.sigma_inc, scl, od.cx, od.cy)
        np.testing.assert_allclose(row["sse"], q.sse, rtol=1e-12)
        _, _, _, sse, cnt = O.reconstruct(od.symbols, po, w.series_off, t0, od.center_len, od.center_inc,
                                          orig=w.values)
        # centers' increments within 1e-12 accumulate along a series (see test_gpu_experiments)
        np.testing.assert_allclose(row["mse"], sse.sum() / cnt.sum(), rtol=1e-9)
