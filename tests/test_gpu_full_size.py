"""Full-size parity for the uneven workload (50,000 series of log-uniform
length, 7.2e8 points) and the multivariate one (1,024 samples x 64 channels
of 5,000 points, 3.3e8 points), in the launch configuration the benchmark
uses at these sizes: one Symbolizer on the default stream.

The oracle's global digitization of 1.5e8-3e8 pieces would take minutes, so
the digitization is checked through what holds at any size, each against an
independent host computation:
  * sigma_len and sigma_inc equal the oracle's scaling of the same pieces;
  * counts are the symbol histogram and center_len the exact member mean
    (an integer sum divided once), bit for bit;
  * every symbol's scaled members lie within 2 alpha of one point (a member
    is within alpha of its Stage I start, which is within alpha of its
    global start), so the mean squared distance to the center is at most
    4 alpha^2 per symbol.
Compression and reconstruction are per series: sampled series are compared
with the oracle bit for bit (pieces, reconstructed points, offsets), the
squared error within rtol 1e-12.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import say, to_dev, torch
from paper_2401_00109_amd.inputs import make_workload, pack

pytestmark = pytest.mark.gpu


def _sample(n_series, k=64):
    rng = np.random.default_rng(11)
    idx = np.concatenate([np.arange(16), np.arange(n_series - 16, n_series),
                          rng.choice(n_series, k - 32, replace=False)])
    return np.unique(idx[(idx >= 0) & (idx < n_series)])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("wid", [3, 4])
def test_full_size_workload(wid):
    import paper_2401_00109_amd as J
    T = torch()
    w = make_workload(wid, seed=0)
    say(f"full-size workload {w.name}: {w.n_series} series, {w.n_points} points")
    v, so = to_dev(w.values), to_dev(w.series_off)
    sz = J.Symbolizer(w.n_series, w.n_points, w.D, w.tol, w.alpha, w.scl, w.B, max_len=w.max_len)
    sz.run(v, so)
    T.cuda.synchronize()
    assert sz.status() == (0, 0)
    ln, inc, po = sz.pieces.host()
    N = ln.size
    sym = sz.symbols[:N].cpu().numpy()
    d = sz.dictionary.host()
    k = d["k"]
    say(f"  N={N} pieces, k={k} symbols")

    # compression, sampled series against the oracle
    idx = _sample(w.n_series)
    sub = [w.values[w.series_off[s]:w.series_off[s + 1]] for s in idx]
    sv, soff = pack(sub)
    ol, oi, opo = O.compress(sv, soff, w.D, w.tol, w.max_len)
    gl = np.concatenate([ln[po[s]:po[s + 1]] for s in idx])
    gi = np.concatenate([inc[po[s]:po[s + 1]] for s in idx])
    np.testing.assert_array_equal(np.diff(opo), po[idx + 1] - po[idx])
    np.testing.assert_array_equal(gl, ol)
    np.testing.assert_array_equal(gi.view(np.uint64), oi.view(np.uint64))
    say(f"  compress: {idx.size} sampled series ({ol.size} pieces) equal the oracle's")

    # digitization, properties at full size
    sl, si, x, y, _ = O.scaling(ln, inc, w.scl)
    assert (d["sigma_len"], d["sigma_inc"]) == (sl, si)
    assert sym.min() >= 0 and sym.max() < k
    cnt = np.bincount(sym, minlength=k)
    np.testing.assert_array_equal(d["count"], cnt)
    assert cnt.min() >= 1
    mean_len = np.bincount(sym, weights=ln.astype(np.float64), minlength=k) / cnt
    np.testing.assert_array_equal(d["center_len"].view(np.uint64), mean_len.view(np.uint64))
    cx = w.scl * (mean_len / sl)
    cy = d["center_inc"] / si
    dev2 = (x - cx[sym]) ** 2 + (y - cy[sym]) ** 2
    del x, y
    per = np.bincount(sym, weights=dev2, minlength=k) / cnt
    del dev2
    assert per.max() <= 4.0 * w.alpha ** 2 * (1 + 1e-9), per.max()
    say(f"  digitize: scaling, counts, center lengths exact; worst symbol mean squared spread "
        f"{per.max():.3e} <= 4 alpha^2 = {4 * w.alpha ** 2:.3e}")

    # reconstruction, sampled series against the oracle (same dictionary)
    t0 = np.where(np.diff(w.series_off) > 0, w.values[np.minimum(w.series_off[:-1], max(w.n_points - 1, 0))], 0.0)
    r = J.reconstruct(sz.symbols, sz.pieces.piece_off, so, to_dev(t0), sz.dictionary, values=v)
    T.cuda.synchronize()
    assert r["status"] == 0
    out_off = r["out_off"].cpu().numpy()
    ssym = np.concatenate([sym[po[s]:po[s + 1]] for s in idx])
    spo = np.concatenate([[0], np.cumsum(po[idx + 1] - po[idx])])
    out, oo, _, sse, cnt_e = O.reconstruct(ssym, spo, soff, t0[idx], d["center_len"], d["center_inc"], orig=sv)
    gout = np.concatenate([r["out"][out_off[s]:out_off[s + 1]].cpu().numpy() for s in idx])
    np.testing.assert_array_equal(np.diff(oo), out_off[idx + 1] - out_off[idx])
    np.testing.assert_array_equal(gout.view(np.uint64), out.view(np.uint64))
    np.testing.assert_array_equal(r["cnt"].cpu().numpy()[idx], cnt_e)
    np.testing.assert_allclose(r["sse"].cpu().numpy()[idx], sse, rtol=1e-12, atol=1e-300)
    say(f"  reconstruct: {idx.size} sampled series ({out.size} points) equal the oracle's")
