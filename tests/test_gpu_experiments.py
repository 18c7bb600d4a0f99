"""The Sec. 7.3 noise experiment on the device against the oracle (small n).

Per partition count M the device's piece count, aggregation symbols and
k-means symbols (element by element), symbol counts and iteration counts
equal the oracle's.  The VQ objective agrees to 1e-12 relative: each side
measures against its own centers, which differ by at most 1e-12 of their
scale, and the squared deviations from a member mean change only to second
order in that difference.  The reconstruction MSE agrees to 1e-9 relative:
the reconstruction adds the centers' increments along each partition
(Sec. 3.3), so the two sides' values drift apart by up to the number of
pieces in a partition (~10^3 here) times the 1e-12 center difference."""
import numpy as np
import pytest

import oracle as O
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,init", [(1, "aggregation"), (4, "spread"), (9, "aggregation")])
def test_noise_partitions_match_oracle(M, init):
    from paper_2401_00109_amd import experiments as E
    n, tol, alpha = 20_000, 0.01, 0.05
    say(f"noise experiment n={n} M={M} kmeans_init={init}")
    row = E.noise_partitions([M], n=n, tol=tol, alpha=alpha, kmeans_iter=40, kmeans_init=init, keep_symbols=True)[0]
    x = E.noise_series(n)
    D = max(1, -(-(n - 1) // M))
    so = np.array([0, n], np.int64)
    ln, ic, po = O.compress(x, so, D, tol)
    assert row["pieces"] == ln.size
    od = O.digitize(ln, ic, alpha, 1.0, 1 << 30)
    assert row["symbols"] == od.k
    np.testing.assert_array_equal(row["symbols_aggregation"], od.symbols)
    values, dso, dpo, t0 = E._domains(x, ln, D)
    _, _, _, sse, cnt = O.reconstruct(od.symbols, dpo, dso, t0, od.center_len, od.center_inc, orig=values)
    np.testing.assert_allclose(row["mse_aggregation"], sse.sum() / cnt.sum(), rtol=1e-9)
    if init == "aggregation":
        cx0, cy0 = od.cx.copy(), od.cy.copy()
    else:
        pick = np.linspace(0, ln.size - 1, od.k).astype(np.int64)
        cx0 = ln[pick] / od.sigma_len
        cy0 = ic[pick] / od.sigma_inc
    km = O.kmeans(ln, ic, od.sigma_len, od.sigma_inc, 1.0, cx0, cy0, 40)
    assert row["kmeans_iterations"] == km.iterations
    np.testing.assert_array_equal(row["symbols_kmeans"], km.symbols)
    _, _, _, sse2, cnt2 = O.reconstruct(km.symbols, dpo, dso, t0, km.center_len, km.center_inc, orig=values)
    np.testing.assert_allclose(row["mse_kmeans"], sse2.sum() / cnt2.sum(), rtol=1e-9)
    q = O.quality(ln, ic, od.symbols, od.sigma_len, od.sigma_inc, 1.0, od.cx, od.cy)
    np.testing.assert_allclose(row["sse_aggregation"], q.sse, rtol=1e-12)
    qk = O.quality(ln, ic, km.symbols, od.sigma_len, od.sigma_inc, 1.0, km.cx, km.cy)
    np.testing.assert_allclose(row["sse_kmeans"], qk.sse, rtol=1e-12)
    if init == "aggregation":
        # Lloyd seeded with the aggregation's codebook never ends above it (Sec. 5: Lloyd lowers SSE)
        assert row["sse_kmeans"] <= row["sse_aggregation"] * (1 + 1e-12)

