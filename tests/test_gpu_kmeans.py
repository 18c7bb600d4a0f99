"""k-means digitization on the GPU (Sec. 3.2, Lloyd's algorithm) against the oracle.

Both sides assign by exact rounded distances (ties to the lowest symbol) and
form the means in the same documented order (exact integer length sums,
increments added in canonical order), so symbols, centers and iteration
counts are bit-identical across all iterations.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import DEV, say, to_dev, torch
from paper_2401_00109_amd.inputs import make_workload

pytestmark = pytest.mark.gpu


def _case(wid, scale, k, seed, max_iter):
    import paper_2401_00109_amd as J
    T = torch()
    w = make_workload(wid, 0, scale)
    ln, ic, _ = O.compress(w.values, w.series_off, w.D, w.tol)
    sl, si = O.scaling(ln, ic, w.scl)[:2]
    x, y = w.scl * (ln / sl), ic / si
    rng = np.random.default_rng(seed)
    pick = rng.choice(ln.size, k, replace=False)
    ref = O.kmeans(ln, ic, sl, si, w.scl, x[pick], y[pick], max_iter)
    n = ln.size
    d = J.Dictionary.from_host(sl, si, w.scl, 0.0, np.zeros(k), np.zeros(k), x[pick], y[pick], device=DEV)
    L, I = to_dev(ln.astype(np.int32)), to_dev(ic)
    npc = T.tensor([n], dtype=T.int64, device=DEV)
    sym, iters = J.kmeans(L, I, npc, n, d, max_iter=max_iter)
    T.cuda.synchronize()
    h = d.host()
    return ref, sym[:n].cpu().numpy(), int(iters.item()), h


@pytest.mark.parametrize("wid,scale,k,max_iter", [(1, 1.0, 40, 100), (2, 0.01, 358, 12), (4, 0.01, 64, 30),
                                                  (2, 0.005, 1, 5)])
def test_kmeans_matches_oracle(wid, scale, k, max_iter):
    say(f"kmeans workload {wid} scale {scale} k {k} max_iter {max_iter}")
    ref, sym, iters, h = _case(wid, scale, k, 5, max_iter)
    assert iters == ref.iterations
    np.testing.assert_array_equal(sym, ref.symbols)
    np.testing.assert_array_equal(h["count"], ref.count)
    for key, val in (("cx", ref.cx), ("cy", ref.cy), ("center_len", ref.center_len), ("center_inc", ref.center_inc)):
        np.testing.assert_array_equal(h[key].view(np.uint64), val.view(np.uint64), err_msg=key)
