"""Digitization quality on the GPU (Sec. 3.2: Eq. sse, Eq. Var) against the oracle.

The GPU sums the squared deviations in the fixed order of the center sums;
the oracle sums them exactly.  Both use their own centers, which differ by at
most d = 1e-12 of their scale, and a variance about a point c that is off the
members' mean by d changes by d^2 only (the first-order term cancels).  The
summation order adds at most (6 + m/64) u relative for a symbol of m members
(under 1e-13 at these sizes).  So per-symbol variances, their maxima and the
SSE agree to 1e-12 relative, with an absolute floor for symbols whose
variance is zero.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import DEV, say, to_dev, torch
from paper_2401_00109_amd.inputs import make_workload

pytestmark = pytest.mark.gpu


def _run(wid, scale, B):
    import paper_2401_00109_amd as J
    T = torch()
    w = make_workload(wid, 0, scale)
    ln, ic, _ = O.compress(w.values, w.series_off, w.D, w.tol)
    od = O.digitize(ln, ic, w.alpha, w.scl, B)
    oq = O.quality(ln, ic, od.symbols, od.sigma_len, od.sigma_inc, od.scl, od.cx, od.cy)
    n = ln.size
    L, I = to_dev(ln.astype(np.int32)), to_dev(ic)
    npc = T.tensor([n], dtype=T.int64, device=DEV)
    sym, d, ws = J.digitize(L, I, npc, n, w.alpha, w.scl, B)
    q = J.digitize_quality(L, I, npc, n, w.alpha, B, d, ws)
    T.cuda.synchronize()
    assert J.workspace_status(ws) == 0
    np.testing.assert_array_equal(sym[:n].cpu().numpy(), od.symbols)
    k = od.k
    return w, oq, {key: v.cpu().numpy() for key, v in q.items()}, k


@pytest.mark.parametrize("wid,scale,B", [(1, 1.0, 4096), (1, 1.0, 7), (2, 0.01, 256), (2, 0.01, 10 ** 9),
                                         (4, 0.02, 4096), (3, 0.002, 1)])
def test_quality_matches_oracle(wid, scale, B):
    say(f"quality workload {wid} scale {scale} B {B}")
    w, oq, q, k = _run(wid, scale, B)
    floor = 1e-15 * max(1.0, float(np.max(oq.var_len + oq.var_inc)))
    np.testing.assert_allclose(q["var_len"][:k], oq.var_len, rtol=1e-12, atol=floor)
    np.testing.assert_allclose(q["var_inc"][:k], oq.var_inc, rtol=1e-12, atol=floor)
    np.testing.assert_allclose(q["totals"][0], oq.sse, rtol=1e-12, atol=floor)
    np.testing.assert_allclose(q["totals"][1], np.max(oq.var_len), rtol=1e-12, atol=floor)
    np.testing.assert_allclose(q["totals"][2], np.max(oq.var_inc), rtol=1e-12, atol=floor)
    # the two-stage bound (members within 2 alpha of their global start)
    assert q["totals"][0] <= 4 * w.alpha ** 2 * (oq.count.sum() - k) * (1 + 1e-9)


def test_quality_is_deterministic():
    import paper_2401_00109_amd as J
    T = torch()
    w = make_workload(2, 0, 0.01)
    ln, ic, _ = O.compress(w.values, w.series_off, w.D, w.tol)
    n = ln.size
    L, I = to_dev(ln.astype(np.int32)), to_dev(ic)
    npc = T.tensor([n], dtype=T.int64, device=DEV)
    outs = []
    for _ in range(2):
        sym, d, ws = J.digitize(L, I, npc, n, w.alpha, w.scl, 512)
        q = J.digitize_quality(L, I, npc, n, w.alpha, 512, d, ws)
        T.cuda.synchronize()
        outs.append({key: v.cpu().numpy().view(np.uint64) for key, v in q.items()})
    for key in outs[0]:
        np.testing.assert_array_equal(outs[0][key], outs[1][key])
