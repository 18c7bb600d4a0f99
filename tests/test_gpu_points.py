"""Two-stage aggregation of raw 2-D points on the device (Sec. 5, Sec. 7.1)
against the oracle, through the C ABI: labels, counts and centers bit-exact,
the SSE within the rounding of its pairwise sum; edge cases and the
Gaussian-blob table."""
import numpy as np
import pytest

import oracle as O
from gpu_util import say, to_dev
from paper_2401_00109_amd.inputs import gaussian_blobs

pytestmark = pytest.mark.gpu


def _run(x, y, alpha, B, capacity=None, max_points=None):
    import torch
    import paper_2401_00109_amd as J
    n = x.size
    mp = max(n, 1) if max_points is None else max_points
    X = torch.zeros(mp, dtype=torch.float64, device="cuda:0")
    Y = torch.zeros(mp, dtype=torch.float64, device="cuda:0")
    if n:
        X[:n] = to_dev(x)
        Y[:n] = to_dev(y)
    npt = torch.tensor([n], dtype=torch.int64, device="cuda:0")
    r = J.aggregate_points(X, Y, alpha, B, n_points=npt, capacity=capacity)
    torch.cuda.synchronize()
    st = J.workspace_status(r["workspace"])
    k = int(r["k"].item())
    kc = min(k, r["cx"].numel())
    return {"labels": r["labels"][:n].cpu().numpy(), "k": k, "cx": r["cx"][:kc].cpu().numpy(),
            "cy": r["cy"][:kc].cpu().numpy(), "count": r["count"][:kc].cpu().numpy(),
            "sse": float(r["sse"].item()), "status": st}


def _same(g, o):
    assert g["status"] == 0
    assert g["k"] == o.k
    np.testing.assert_array_equal(g["labels"], o.labels)
    np.testing.assert_array_equal(g["count"], o.count)
    np.testing.assert_array_equal(g["cx"].view(np.uint64), o.cx.view(np.uint64))
    np.testing.assert_array_equal(g["cy"].view(np.uint64), o.cy.view(np.uint64))
    # the device's pairwise sum of the same rounded terms: relative error <= (log2 N + 2) eps
    np.testing.assert_allclose(g["sse"], o.sse, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("n", [5000, 10000, 70001])
@pytest.mark.parametrize("alpha", [0.1, 0.05])
@pytest.mark.parametrize("M", [1, 4, 8, 97])
def test_points_parity(n, alpha, M):
    x, y = gaussian_blobs(0, n)
    B = -(-n // M)
    say(f"aggregate points n={n} alpha={alpha} M={M} B={B}")
    g = _run(x, y, alpha, B)
    o = O.aggregate_points(x, y, alpha, B)
    _same(g, o)


@pytest.mark.parametrize("centers", [3, 10])
def test_points_parity_several_blobs(centers):
    x, y = gaussian_blobs(4, 20000, centers=centers, std=0.5)
    say(f"aggregate points, {centers} blobs")
    for B in (20000, 777):
        _same(_run(x, y, 0.05, B), O.aggregate_points(x, y, 0.05, B))


@pytest.mark.parametrize("case", ["empty", "one", "identical", "ties", "alpha0", "spare_capacity"])
def test_points_edge_cases(case):
    rng = np.random.default_rng(3)
    alpha, B, mp = 0.1, 64, None
    if case == "empty":
        x, y = np.zeros(0), np.zeros(0)
    elif case == "one":
        x, y = np.array([0.5]), np.array([-1.25])
    elif case == "identical":
        x, y = np.full(900, 0.75), np.full(900, -0.25)
    elif case == "ties":             # many equal keys across block cuts
        x = rng.integers(-3, 4, 5000) * 0.5
        y = rng.integers(-3, 4, 5000) * 0.5
    elif case == "alpha0":
        x = np.round(rng.standard_normal(3000), 1)
        y = np.round(rng.standard_normal(3000), 1)
        alpha = 0.0
    else:                            # fewer live points than the buffers hold
        x, y = gaussian_blobs(2, 3000)
        mp = 5000
    say(f"aggregate points edge case {case}")
    g = _run(x, y, alpha, B, max_points=mp)
    _same(g, O.aggregate_points(x, y, alpha, B))


def test_points_capacity_and_nonfinite_status():
    from paper_2401_00109_amd import _lib
    x, y = gaussian_blobs(1, 4000)
    say("aggregate points with a too-small capacity")
    g = _run(x, y, 0.1, 4000, capacity=10)
    o = O.aggregate_points(x, y, 0.1, 4000)
    assert g["status"] == _lib.JABBA_ECAPACITY and g["k"] == o.k
    np.testing.assert_array_equal(g["labels"], o.labels)
    np.testing.assert_array_equal(g["cx"].view(np.uint64), o.cx[:10].view(np.uint64))
    x2 = x.copy()
    x2[17] = np.nan
    say("aggregate points with a NaN")
    g = _run(x2, y, 0.1, 512)
    assert g["status"] == _lib.JABBA_ENONFINITE


def test_blob_table_matches_oracle():
    from paper_2401_00109_amd import experiments as E
    say("Gaussian-blob table (small repeats)")
    rows = E.gaussian_blobs(sizes=(5000,), alphas=(0.1,), blocks=(1, 4, 8), repeats=2)
    x, y = gaussian_blobs(0, 5000)
    s = O.aggregate_points(x, y, 0.1)
    for r in rows:
        o = O.aggregate_points(x, y, 0.1, r["B"])
        assert r["clusters"] == o.k and r["clusters_serial"] == s.k
        np.testing.assert_allclose(r["sse_ratio"], o.sse / s.sse, rtol=1e-12)
