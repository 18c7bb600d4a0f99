"""Serving loop and autotuner on the GPU.

* Requests that overlap on the device (continuous batching over several
  streams) give exactly the symbols they give alone, and exactly the oracle's
  compress + nearest-center encode with the same (oracle-built) dictionary.
* Memory-based admission: a small arena forces queueing, not failure.
* The autotuner only returns launch shapes whose outputs equal the default's.
"""
import numpy as np
import pytest

import oracle as O
from paper_2401_00109_amd.inputs import make_workload, request_stream

from gpu_util import DEV, say, to_dev, torch

pytestmark = pytest.mark.gpu


def _oracle_dictionary():
    import paper_2401_00109_amd as J
    w1 = make_workload(1)
    l1, i1, _ = O.compress(w1.values, w1.series_off, w1.D, w1.tol)
    od = O.digitize(l1, i1, w1.alpha, 1.0, 4096)
    d = J.Dictionary.from_host(od.sigma_len, od.sigma_inc, od.scl, od.alpha, od.center_len, od.center_inc, od.cx,
                               od.cy, od.count, DEV)
    return od, d


@pytest.mark.parametrize("arena_points", [None, 60_000])
def test_mix_equals_alone_and_oracle(arena_points):
    from paper_2401_00109_amd.serve import Server
    od, d = _oracle_dictionary()
    reqs = request_stream(7, 12, rate_hz=2000.0, max_series=8, min_len=500, max_len=6000)
    arena = None if arena_points is None else Server.need(arena_points)
    srv = Server(d, D=2000, tol=0.05, slots=3, max_series=8, max_points=8 * 6000, arena_bytes=arena, device=DEV)
    say(f"serving 12 requests, 3 slots, arena={arena}")
    mixed = {r.rid: r for r in srv.run(reqs, realtime=True)}
    assert len(mixed) == 12
    say(f"  at most {srv.peak_in_flight} requests in flight")
    if arena is None:
        assert srv.peak_in_flight > 1  # the requests did overlap on the device
    for r in reqs:
        alone = srv.run([r], realtime=False)[0]
        m = mixed[r.rid]
        np.testing.assert_array_equal(alone.symbols, m.symbols)
        np.testing.assert_array_equal(alone.piece_off, m.piece_off)
        ln, inc, po = O.compress(r.values, r.series_off, 2000, 0.05)
        exp = O.encode(ln, inc, od.sigma_len, od.sigma_inc, od.scl, od.cx, od.cy)
        np.testing.assert_array_equal(m.symbols, exp)
        np.testing.assert_array_equal(m.piece_off, po)


def test_full_size_requests_mix_equals_alone_and_oracle():
    # requests of the serving workload's full shape: 1-256 random walks of
    # 500-50,000 points each, four slots, arrivals faster than service
    from paper_2401_00109_amd.serve import Server
    od, d = _oracle_dictionary()
    reqs = request_stream(11, 8, rate_hz=5000.0)
    pts = [r.values.size for r in reqs]
    say(f"serving 8 full-size requests ({min(pts)}-{max(pts)} points, "
        f"{max(r.series_off.size - 1 for r in reqs)} series at most), 4 slots")
    srv = Server(d, D=2000, tol=0.05, slots=4, device=DEV)
    mixed = {r.rid: r for r in srv.run(reqs, realtime=True)}
    assert len(mixed) == 8
    say(f"  at most {srv.peak_in_flight} requests in flight")
    assert srv.peak_in_flight > 1
    for r in reqs:
        alone = srv.run([r], realtime=False)[0]
        m = mixed[r.rid]
        np.testing.assert_array_equal(alone.symbols, m.symbols)
        np.testing.assert_array_equal(alone.piece_off, m.piece_off)
        ln, inc, po = O.compress(r.values, r.series_off, 2000, 0.05)
        exp = O.encode(ln, inc, od.sigma_len, od.sigma_inc, od.scl, od.cx, od.cy)
        np.testing.assert_array_equal(m.symbols, exp)
        np.testing.assert_array_equal(m.piece_off, po)


def test_autotuner_only_keeps_identical_outputs(tmp_path):
    from paper_2401_00109_amd import tune
    w = make_workload(3, 0, 0.002)
    v, so = to_dev(w.values), to_dev(w.series_off)
    space = [{"lanes_per_domain": W, "waves_per_block": 2, "blocks_per_cu": 4} for W in (1, 4, 16)]
    say("autotune (small search space)")
    best = tune.tune(v, so, w.D, w.tol, w.alpha, w.scl, w.B, reps=1, compress_space=space, stage1_space=[1, 4],
                     cache_path=str(tmp_path / "t.json"), log=lambda *a: None)
    assert best["lanes_per_domain"] in (1, 4, 16) and best["stage1_waves"] in (1, 4)
    assert tune.lookup(torch().device(DEV), w.n_series, w.n_points, w.D, str(tmp_path / "t.json")) == best
    import paper_2401_00109_amd as J
    a = J.compress(v, so, w.D, w.tol, tuning=best)
    b = J.compress(v, so, w.D, w.tol)
    torch().cuda.synchronize()
    la, ia, pa = a.host()
    lb, ib, pb = b.host()
    np.testing.assert_array_equal(la, lb)
    np.testing.assert_array_equal(ia.view(np.uint64), ib.view(np.uint64))
