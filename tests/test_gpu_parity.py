"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by
element on the same seeded inputs.

Bar: bit-exact for piece lengths, increments, piece offsets, sigma, sort
blocks, starting points, symbols, k, counts, center lengths, quantized
lengths and reconstructions given the same dictionary; center increments
(a sum over up to ~1e5 members in a different fixed order) within 1e-12 of
max(|mean|, mean |inc|) of the group.
"""
import numpy as np
import pytest

import oracle as O
from paper_2401_00109_amd.inputs import make_workload, pack, random_walk, series_rng, znorm

from gpu_util import DEV, assert_centers_close, gpu_compress, gpu_digitize, say, to_dev, torch

pytestmark = pytest.mark.gpu

SMALL = {1: 1.0, 2: 0.01, 3: 0.002, 4: 1.0 / 256}


def _workload(wid):
    return make_workload(wid, seed=0, scale=SMALL[wid])


# ------------------------------------------------------------------ numerics
def test_fp64_division_and_sqrt_are_correctly_rounded():
    import ctypes as C
    import paper_2401_00109_amd as J
    T = torch()
    rng = np.random.default_rng(0)
    n = 1 << 21
    a = np.abs(rng.standard_normal(n)) * np.exp2(rng.integers(-200, 200, n))
    b = rng.standard_normal(n) * np.exp2(rng.integers(-200, 200, n))
    edge = np.array([1.0, 2.0, 4.0, 0.0, 1e-310, 2.0 ** -1074, 1.7976931348623157e308, 0.5, 3.0, 1e16, 1e-16, 9.0])
    a = np.concatenate([a, edge, np.arange(1, 5000, dtype=np.float64)])
    b = np.concatenate([b, np.resize(np.array([3.0, 7.0, -1.0, 1e-300, 5.0]), edge.size + 4999)])
    da, db = to_dev(a), to_dev(b)
    q = T.empty_like(da)
    r = T.empty_like(da)
    say(f"fp64 selftest n={a.size}")
    rc = J.lib().jabba_fp64_selftest(C.c_void_p(da.data_ptr()), C.c_void_p(db.data_ptr()), C.c_void_p(q.data_ptr()),
                                     C.c_void_p(r.data_ptr()), a.size, C.c_void_p(T.cuda.current_stream().cuda_stream))
    assert rc == 0
    T.cuda.synchronize()
    np.testing.assert_array_equal(q.cpu().numpy().view(np.uint64), (a / b).view(np.uint64))
    np.testing.assert_array_equal(r.cpu().numpy().view(np.uint64), np.sqrt(a).view(np.uint64))


# ------------------------------------------------------------------ compress
@pytest.mark.parametrize("wid", [1, 2, 3, 4])
def test_compress_parity(wid):
    w = _workload(wid)
    say(f"compress workload {wid}: {w.n_series} series {w.n_points} points D={w.D} tol={w.tol}")
    ln, inc, po, st = gpu_compress(w.values, w.series_off, w.D, w.tol)
    assert st == 0
    ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
    np.testing.assert_array_equal(po, opo)
    np.testing.assert_array_equal(ln, ol)
    np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))


@pytest.mark.parametrize("W", [1, 2, 4, 8, 16, 32, 64])
def test_compress_lane_width_never_changes_results(W):
    w = _workload(2)
    ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
    for wpb, bpc in [(1, 1), (4, 8), (16, 2)]:
        say(f"compress W={W} waves_per_block={wpb} blocks_per_cu={bpc}")
        ln, inc, po, st = gpu_compress(w.values, w.series_off, w.D, w.tol,
                                       tuning={"lanes_per_domain": W, "waves_per_block": wpb, "blocks_per_cu": bpc})
        assert st == 0
        np.testing.assert_array_equal(ln, ol)
        np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))
        np.testing.assert_array_equal(po, opo)


@pytest.mark.parametrize("G", [-1, 32, 57, 128, 999, 5000])
def test_compress_segment_length_never_changes_results(G):
    # domains compressed as segments of G intervals and repaired (G = -1: whole domains)
    for wid in (2, 3):
        w = _workload(wid)
        ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
        for W in (1, 4):
            say(f"compress workload {wid} segments of {G} intervals, W={W}")
            ln, inc, po, st = gpu_compress(w.values, w.series_off, w.D, w.tol,
                                           tuning={"segment_intervals": G, "lanes_per_domain": W})
            assert st == 0
            np.testing.assert_array_equal(ln, ol)
            np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))
            np.testing.assert_array_equal(po, opo)


def test_compress_segments_with_limits_and_ties():
    # tol = 0, max_len, constant and straight stretches: pieces longer than the segments
    rng = np.random.default_rng(5)
    vals = np.concatenate([np.cumsum(rng.standard_normal(6000)), 0.25 * np.arange(3000.0), np.full(2000, 1.5),
                           np.repeat(rng.integers(-3, 4, 150).astype(np.float64), 20)])
    off = np.array([0, 6000, 9000, 11000, 14000], np.int64)
    for tol, max_len in [(0.0, 0), (0.5, 5), (5.0, 0), (5.0, 40)]:
        ol, oi, opo = O.compress(vals, off, 2500, tol, max_len)
        for G in (32, 100):
            say(f"compress segments of {G}, tol={tol} max_len={max_len}")
            ln, inc, po, st = gpu_compress(vals, off, 2500, tol, max_len, tuning={"segment_intervals": G})
            assert st == 0
            np.testing.assert_array_equal(ln, ol)
            np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))


def test_compress_plain_launches_equal_batched():
    w = _workload(3)
    say("compress plain per-series launches")
    ln, inc, po, st = gpu_compress(w.values, w.series_off, w.D, w.tol, plain=True)
    assert st == 0
    ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
    np.testing.assert_array_equal(ln, ol)
    np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))
    np.testing.assert_array_equal(po, opo)


@pytest.mark.parametrize("case", ["degenerate_lengths", "straight", "tol0_pwl", "max_len", "D1", "constant",
                                  "long_domains"])
def test_compress_edge_cases(case):
    rng = np.random.default_rng(5)
    D, tol, max_len = 7, 0.1, 0
    if case == "degenerate_lengths":
        lens = [0, 1, 2, 3, 0, 8, 1, 65, 64, 63, 129]
        vals, off = pack([rng.standard_normal(n) for n in lens])
    elif case == "straight":
        vals, off = pack([3.0 + 0.25 * np.arange(n) for n in (5, 100, 1001, 2)])
        D, tol = 100, 0.0
    elif case == "tol0_pwl":
        v = np.concatenate([np.arange(0, 50) * 2.0, 98.0 - np.arange(1, 70) * 3.0])
        vals, off = pack([v, v[::-1].copy()])
        D, tol = 1000, 0.0
    elif case == "max_len":
        vals, off = pack([np.cumsum(rng.standard_normal(500)) * 0.01])
        D, tol, max_len = 1000, 10.0, 5
    elif case == "D1":
        vals, off = pack([rng.standard_normal(50)])
        D = 1
    elif case == "constant":
        vals, off = pack([np.full(300, 2.5), np.zeros(70)])
        D, tol = 64, 0.0
    else:  # domains far longer than a wavefront's 64 candidates
        vals, off = pack([np.linspace(0, 1, 3000) + 1e-9 * rng.standard_normal(3000)])
        D, tol = 2999, 0.01
    say(f"compress edge case {case}")
    for W in (1, 4, 64):
        ln, inc, po, st = gpu_compress(vals, off, D, tol, max_len, tuning={"lanes_per_domain": W})
        assert st == 0
        ol, oi, opo = O.compress(vals, off, D, tol, max_len)
        np.testing.assert_array_equal(po, opo)
        np.testing.assert_array_equal(ln, ol)
        np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))


def test_compress_exact_path_in_later_domains():
    # tol = 0 on straight lines leaves the certified filter undecided at every
    # candidate, so each round evaluates the definition itself, reading the
    # piece's points back (from the lane's ring where they lie in its
    # window).  With many more domains than lanes, lanes take new domains
    # from the queue between refills; their first rounds must read the new
    # domain's points, not what the ring held for the domain before.
    vals, off = pack([3.0 + 0.25 * np.arange(100_000) for _ in range(40)])
    D, tol = 8, 0.0
    say(f"compress, exact path in {40 * 100_000 // D} short domains")
    ln, inc, po, st = gpu_compress(vals, off, D, tol)
    assert st == 0
    ol, oi, opo = O.compress(vals, off, D, tol)
    np.testing.assert_array_equal(po, opo)
    np.testing.assert_array_equal(ln, ol)
    np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))
    # every domain is one piece: 12,499 of 8 intervals and one of 7 per series
    assert ol.size == 40 * 12_500 and np.count_nonzero(ol == 7) == 40 and np.count_nonzero(ol == 8) == 40 * 12_499


@pytest.mark.parametrize("znorm", [False, True])
def test_compress_grouped_and_single_piece_stores(znorm):
    """Tens of thousands of short domains: with one wavefront per compute
    unit they outnumber the lanes, and the one-lane kernel keeps the pieces
    in groups of four staging slots (partial groups at both ends of every
    domain); with the widest launch the lanes outnumber them and each piece
    is stored at once.  Domains of 7 intervals over series of 1 to 400
    points give every alignment of a domain's first slot and every piece
    count modulo 4.  Both launches equal the oracle, z-normalised too."""
    rng = np.random.default_rng(11)
    lengths = rng.integers(1, 400, size=2000)
    vals, off = pack([3.0 + np.cumsum(rng.standard_normal(int(n))) for n in lengths])
    D = 7
    src = vals
    if znorm:
        src, om, osd = O.znorm(vals, off)
    for tol in (0.0, 0.5):
        ol, oi, opo = O.compress(src, off, D, tol)
        for tuning in ({"lanes_per_domain": 1, "waves_per_block": 1, "blocks_per_cu": 1},
                       {"lanes_per_domain": 1, "waves_per_block": 4, "blocks_per_cu": 32}):
            say(f"compress {off[-1]} points in {off[-1] // D + len(lengths)} domains or fewer, tol={tol}, "
                f"znorm={znorm}, {tuning}")
            r = gpu_compress(vals, off, D, tol, tuning=tuning, znorm=znorm)
            ln, inc, po, st = r[:4]
            assert st == 0
            if znorm:
                np.testing.assert_array_equal(r[4].view(np.uint64), om.view(np.uint64))
                np.testing.assert_array_equal(r[5].view(np.uint64), osd.view(np.uint64))
            np.testing.assert_array_equal(po, opo)
            np.testing.assert_array_equal(ln, ol)
            np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))


def test_compress_empty_input():
    say("compress empty input")
    ln, inc, po, st = gpu_compress(np.zeros(0), np.zeros(1, np.int64), 10, 0.1)
    assert ln.size == 0 and po.tolist() == [0] and st == 0


def test_compress_nonfinite_sets_device_status():
    from paper_2401_00109_amd import _lib
    v = np.cumsum(np.random.default_rng(1).standard_normal(2000))
    v[777] = np.nan
    say("compress with a NaN value")
    _, _, _, st = gpu_compress(v, np.array([0, 2000]), 100, 0.1)
    assert st == _lib.JABBA_ENONFINITE
    v[777] = np.inf
    _, _, _, st = gpu_compress(v, np.array([0, 2000]), 100, 0.1)
    assert st == _lib.JABBA_ENONFINITE


# ------------------------------------------------------------------ digitize
def _pieces(wid):
    w = _workload(wid)
    ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
    return w, ol, oi, opo


@pytest.mark.parametrize("wid", [1, 2, 3, 4])
@pytest.mark.parametrize("B", [1, 7, 256, 4096, 10**9])
def test_digitize_parity(wid, B):
    w, ol, oi, _ = _pieces(wid)
    say(f"digitize workload {wid} N={ol.size} B={B} alpha={w.alpha}")
    sym, d, st = gpu_digitize(ol, oi, w.alpha, w.scl, B)
    assert st == 0
    od = O.digitize(ol, oi, w.alpha, w.scl, B)
    assert d["sigma_len"] == od.sigma_len and d["sigma_inc"] == od.sigma_inc
    assert d["k"] == od.k
    assert d["stats"]["G"] == od.n_starts and d["stats"]["N"] == ol.size and d["stats"]["k"] == od.k
    np.testing.assert_array_equal(sym, od.symbols)
    np.testing.assert_array_equal(d["count"], od.count)
    np.testing.assert_array_equal(d["center_len"].view(np.uint64), od.center_len.view(np.uint64))
    np.testing.assert_array_equal(d["cx"].view(np.uint64), od.cx.view(np.uint64))
    worst = assert_centers_close(d, od, oi, od.symbols)
    say(f"  k={od.k} G={od.n_starts} center_inc worst rel err {worst:.3e}")


@pytest.mark.parametrize("case", ["one_piece", "identical", "alpha0", "ties_across_blocks", "scl0", "big_tie_block"])
def test_digitize_edge_cases(case):
    rng = np.random.default_rng(11)
    alpha, scl, B = 0.1, 1.0, 16
    if case == "one_piece":
        ln, inc = np.array([3], np.int32), np.array([0.25])
    elif case == "identical":
        ln, inc = np.full(500, 2, np.int32), np.full(500, -0.5)
    elif case == "alpha0":
        ln = rng.integers(1, 5, 3000).astype(np.int32)
        inc = np.round(rng.standard_normal(3000), 1)
        alpha = 0.0
    elif case == "ties_across_blocks":
        ln = rng.integers(1, 3, 4000).astype(np.int32)
        inc = rng.integers(-2, 3, 4000) * 0.5
        B = 64
    elif case == "scl0":
        ln = rng.integers(1, 9, 2000).astype(np.int32)
        inc = rng.standard_normal(2000)
        scl = 0.0
    else:  # more equal keys than one LDS bitmap holds
        ln = np.ones(80_000, np.int32)
        inc = np.where(rng.random(80_000) < 0.9, 0.25, -0.75)
        B, alpha = 1024, 0.05
    say(f"digitize edge case {case}")
    sym, d, st = gpu_digitize(ln, inc, alpha, scl, B)
    assert st == 0
    od = O.digitize(ln, inc, alpha, scl, B)
    assert d["k"] == od.k
    np.testing.assert_array_equal(sym, od.symbols)
    np.testing.assert_array_equal(d["center_len"].view(np.uint64), od.center_len.view(np.uint64))
    assert_centers_close(d, od, inc, od.symbols)


@pytest.mark.parametrize("cluster", [0, 900, 1024, 1025, 5000, 60_000])
def test_digitize_prefix_groups_and_fallback(cluster):
    """The main sort orders the highest four varying key digits by radix
    passes and finishes each prefix group locally; a group that crosses a
    tile's end (1,024 positions) and reaches more than 256 positions past its
    start goes to the fallback sort.  A cluster of distinct keys within 1e-11
    relative of each other shares one prefix group, of the cluster's size,
    among spread pieces."""
    rng = np.random.default_rng(1000 + cluster)
    m = 150_000
    ln = rng.integers(1, 9, m).astype(np.int32)
    inc = rng.standard_normal(m)
    if cluster:
        ln = np.concatenate([ln, np.full(cluster, 3, np.int32)])
        inc = np.concatenate([inc, 0.5 + 1e-15 * rng.permutation(cluster)])
        order = rng.permutation(ln.size)
        ln, inc = ln[order], inc[order]
    say(f"digitize with a cluster of {cluster} nearly equal keys among {m} pieces")
    for B in (4096, 97):
        sym, d, st = gpu_digitize(ln, inc, 0.05, 1.0, B)
        assert st == 0
        od = O.digitize(ln, inc, 0.05, 1.0, B)
        say(f"  B={B}: {d['stats']['sort_passes']} radix passes, {d['stats']['sort_large']} pieces by the fallback")
        if cluster > 1024:
            assert d["stats"]["sort_large"] >= cluster
        assert d["k"] == od.k and d["stats"]["G"] == od.n_starts
        np.testing.assert_array_equal(sym, od.symbols)
        np.testing.assert_array_equal(d["center_len"].view(np.uint64), od.center_len.view(np.uint64))
        assert_centers_close(d, od, inc, od.symbols)


@pytest.mark.parametrize("n", [200, 300, 700])
def test_digitize_long_active_lists(n):
    """Many live Stage I starts at once with separated length columns.  A
    large scl makes x dominate the key, so the pieces of one length share a
    key window while their y lie about alpha or more apart: most start their
    own group and stay active, more than the 256 mirrored per wavefront (the
    per-bucket chains are dropped and rebuilt).  Bit for bit against the
    oracle, in one block and in blocks of 257."""
    rng = np.random.default_rng(21)
    ln = np.concatenate([np.full(n, 5), np.full(n, 6), np.full(n // 3, 7)]).astype(np.int32)
    inc = np.concatenate([np.linspace(-1, 1, n), np.linspace(-1, 1, n) + 0.003, np.linspace(-1, 1, n // 3)])
    order = rng.permutation(ln.size)
    ln, inc = ln[order], inc[order]
    alpha, scl = 0.005, 1000.0
    for B in (1 << 20, 257):
        say(f"digitize, long active lists: n={n} B={B}")
        sym, d, st = gpu_digitize(ln, inc, alpha, scl, B)
        assert st == 0
        od = O.digitize(ln, inc, alpha, scl, B)
        if B > ln.size:
            assert od.n_starts > 256  # the premise: more live starts than the mirror holds
        assert d["k"] == od.k
        np.testing.assert_array_equal(sym, od.symbols)
        np.testing.assert_array_equal(d["center_len"].view(np.uint64), od.center_len.view(np.uint64))


def test_digitize_nonfinite_status():
    from paper_2401_00109_amd import _lib
    w, ol, oi, _ = _pieces(1)
    bad = oi.copy()
    bad[5] = np.inf
    say("digitize with an infinite increment")
    _, _, st = gpu_digitize(ol, bad, w.alpha, 1.0, 256)
    assert st == _lib.JABBA_ENONFINITE


def test_digitize_capacity_status():
    from paper_2401_00109_amd import _lib
    w, ol, oi, _ = _pieces(1)
    say("digitize with a too-small dictionary")
    sym, d, st = gpu_digitize(ol, oi, w.alpha, 1.0, 4096, capacity=10)
    assert st == _lib.JABBA_ECAPACITY
    od = O.digitize(ol, oi, w.alpha, 1.0, 4096)
    assert d["k"] == od.k
    np.testing.assert_array_equal(sym, od.symbols)


def test_digitize_stage1_waves_never_change_results():
    w, ol, oi, _ = _pieces(2)
    od = O.digitize(ol, oi, w.alpha, w.scl, 512)
    for s1 in (1, 2, 8, 16):
        say(f"digitize stage1_waves={s1}")
        sym, d, st = gpu_digitize(ol, oi, w.alpha, w.scl, 512, tuning={"stage1_waves": s1})
        np.testing.assert_array_equal(sym, od.symbols)


# ------------------------------------------------------------------ encode
@pytest.mark.parametrize("wid", [1, 2])
def test_encode_parity(wid):
    import paper_2401_00109_amd as J
    T = torch()
    w1 = _workload(1)
    l1, i1, _ = O.compress(w1.values, w1.series_off, w1.D, w1.tol)
    od = O.digitize(l1, i1, w1.alpha, 1.0, 4096)
    w, ol, oi, _ = _pieces(wid)
    say(f"encode workload {wid} ({ol.size} pieces) against k={od.k}")
    d = J.Dictionary.from_host(od.sigma_len, od.sigma_inc, od.scl, od.alpha, od.center_len, od.center_inc, od.cx,
                               od.cy, od.count, DEV)
    L, I = to_dev(ol), to_dev(oi)
    npc = T.tensor([ol.size], dtype=T.int64, device=DEV)
    sym = J.encode(L, I, npc, ol.size, d)
    T.cuda.synchronize()
    exp = O.encode(ol, oi, od.sigma_len, od.sigma_inc, od.scl, od.cx, od.cy)
    np.testing.assert_array_equal(sym[: ol.size].cpu().numpy(), exp)


# ------------------------------------------------------------------ reconstruct
@pytest.mark.parametrize("wid", [1, 3])
def test_reconstruct_parity(wid):
    import paper_2401_00109_amd as J
    w, ol, oi, opo = _pieces(wid)
    od = O.digitize(ol, oi, w.alpha, 1.0, 4096)
    t0 = w.values[w.series_off[:-1]] if w.n_series else np.zeros(0)
    t0 = np.where(np.diff(w.series_off) > 0, t0, 0.0)
    out, oo, lhat, sse, cnt = O.reconstruct(od.symbols, opo, w.series_off, t0, od.center_len, od.center_inc,
                                            orig=w.values)
    say(f"reconstruct workload {wid}: {out.size} points")
    d = J.Dictionary.from_host(od.sigma_len, od.sigma_inc, od.scl, od.alpha, od.center_len, od.center_inc, od.cx,
                               od.cy, od.count, DEV)
    r = J.reconstruct(to_dev(od.symbols), to_dev(opo), to_dev(w.series_off), to_dev(t0), d, values=to_dev(w.values),
                      want_lhat=True)
    assert r["status"] == 0
    np.testing.assert_array_equal(r["out_off"].cpu().numpy(), oo)
    np.testing.assert_array_equal(r["lhat"][: ol.size].cpu().numpy(), lhat)
    np.testing.assert_array_equal(r["out"].cpu().numpy().view(np.uint64), out.view(np.uint64))
    np.testing.assert_array_equal(r["cnt"].cpu().numpy()[: w.n_series], cnt)
    np.testing.assert_allclose(r["sse"].cpu().numpy()[: w.n_series], sse, rtol=1e-12, atol=1e-300)


def test_reconstruct_pieces_parity():
    import paper_2401_00109_amd as J
    w, ol, oi, opo = _pieces(2)
    t0 = w.values[w.series_off[:-1]]
    out, oo = O.reconstruct_pieces(ol, oi, opo, t0)
    say("reconstruct from raw pieces")
    g, go = J.reconstruct_pieces(to_dev(ol), to_dev(oi), to_dev(opo), to_dev(w.series_off), to_dev(t0))
    np.testing.assert_array_equal(go.cpu().numpy(), oo)
    np.testing.assert_array_equal(g[: out.size].cpu().numpy().view(np.uint64), out.view(np.uint64))


def test_reconstruct_half_lengths():
    import paper_2401_00109_amd as J
    sym = np.array([0, 1, 0], np.int32)
    po = np.array([0, 3], np.int64)
    off = np.array([0, 9], np.int64)
    cl, ci = np.array([1.5, 2.5]), np.array([1.0, -1.0])
    d = J.Dictionary.from_host(1.0, 1.0, 1.0, 0.1, cl, ci, cl, ci, device=DEV)
    say("reconstruct halves")
    r = J.reconstruct(to_dev(sym), to_dev(po), to_dev(off), to_dev(np.array([0.0])), d, want_lhat=True)
    assert r["lhat"][:3].cpu().tolist() == [2, 2, 2]
    assert r["out"].cpu().tolist() == [0.0, 0.5, 1.0, 0.5, 0.0, 0.5, 1.0]


def test_reconstruct_every_chunk_count():
    """Series of 0 to 385 pieces: every count of 64-piece chunks from 0 to 7
    (the symbols are loaded three chunks ahead through four rotating
    registers, so each count ends the rotation at a different register),
    with counts just below, at and above each multiple of 64."""
    import paper_2401_00109_amd as J
    rng = np.random.default_rng(12)
    counts = [0, 1, 2, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256, 257, 319, 320, 321, 383, 384, 385]
    k = 37
    cl = 1.0 + rng.integers(0, 16, size=k) / 4.0
    ci = rng.standard_normal(k)
    sym = rng.integers(0, k, size=sum(counts)).astype(np.int32)
    po = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = [int(c * 3 + 1) for c in counts]
    off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    values = rng.standard_normal(int(off[-1]))
    t0 = values[np.minimum(off[:-1], off[-1] - 1)]
    out, oo, lhat, sse, cnt = O.reconstruct(sym, po, off, t0, cl, ci, orig=values)
    say(f"reconstruct {len(counts)} series of 0 to {max(counts)} pieces")
    d = J.Dictionary.from_host(1.0, 1.0, 1.0, 0.1, cl, ci, cl, ci, device=DEV)
    r = J.reconstruct(to_dev(sym), to_dev(po), to_dev(off), to_dev(t0), d, values=to_dev(values), want_lhat=True)
    assert r["status"] == 0
    np.testing.assert_array_equal(r["out_off"].cpu().numpy(), oo)
    np.testing.assert_array_equal(r["lhat"][: sym.size].cpu().numpy(), lhat)
    np.testing.assert_array_equal(r["out"][: out.size].cpu().numpy().view(np.uint64), out.view(np.uint64))
    np.testing.assert_array_equal(r["cnt"].cpu().numpy()[: len(counts)], cnt)
    np.testing.assert_allclose(r["sse"].cpu().numpy()[: len(counts)], sse, rtol=1e-12, atol=1e-300)


def test_reconstruct_long_center_lengths():
    """A center length of 2^25 + 3/4 among short ones: the 64-piece chunks
    that hold it scan the fixed-point lengths in 128 bits, the others in
    32-bit limbs, and the carry passes between the two forms (series 0:
    chunks 0, 2 and 3 short, chunk 1 long; series 1: its first chunk long)."""
    import paper_2401_00109_amd as J
    rng = np.random.default_rng(7)
    cl = np.array([1.5, 2.25, 3.0, 2.0 ** 25 + 0.75])
    ci = np.array([1.0, -0.5, 0.25, 3.0])
    sym = rng.integers(0, 3, size=330).astype(np.int32)
    sym[100] = 3
    sym[250] = 3
    po = np.array([0, 200, 330], np.int64)
    off = np.array([0, 1000, 2000], np.int64)
    t0 = np.array([0.5, -2.0])
    values = rng.normal(size=2000)
    out, oo, lhat, sse, cnt = O.reconstruct(sym, po, off, t0, cl, ci, orig=values)
    say(f"reconstruct with two pieces of 2^25 points: {out.size} points")
    d = J.Dictionary.from_host(1.0, 1.0, 1.0, 0.1, cl, ci, cl, ci, device=DEV)
    r = J.reconstruct(to_dev(sym), to_dev(po), to_dev(off), to_dev(t0), d, values=to_dev(values), want_lhat=True)
    assert r["status"] == 0
    np.testing.assert_array_equal(r["out_off"].cpu().numpy(), oo)
    np.testing.assert_array_equal(r["lhat"][: sym.size].cpu().numpy(), lhat)
    assert lhat[100] >= 2 ** 25 and lhat[250] >= 2 ** 25
    np.testing.assert_array_equal(r["out"][: out.size].cpu().numpy().view(np.uint64), out.view(np.uint64))
    np.testing.assert_array_equal(r["cnt"].cpu().numpy()[:2], cnt)
    np.testing.assert_allclose(r["sse"].cpu().numpy()[:2], sse, rtol=1e-12, atol=1e-300)


# ------------------------------------------------------------------ graph plan
def test_plan_graph_replays_match_eager():
    import paper_2401_00109_amd as J
    T = torch()
    w = _workload(3)
    v, so = to_dev(w.values), to_dev(w.series_off)
    say(f"plan capture: {w.n_series} series")
    plan = J.Plan(v, so, w.D, w.tol, w.alpha, w.scl, w.B, tuning={"lanes_per_domain": 4})
    ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
    od = O.digitize(ol, oi, w.alpha, w.scl, w.B)
    for rep in range(3):
        plan.pieces.len.fill_(-1)
        plan.symbols.fill_(-1)
        T.cuda.synchronize()
        plan.run()
        T.cuda.synchronize()
        say(f"  replay {rep}")
        ln, inc, po = plan.pieces.host()
        np.testing.assert_array_equal(ln, ol)
        np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))
        np.testing.assert_array_equal(plan.symbols[: ol.size].cpu().numpy(), od.symbols)
        assert plan.dictionary.size() == od.k
        # eager work between replays
        J.compress(v, so, w.D, w.tol)
        T.cuda.synchronize()
    assert plan.status() == (0, 0)
    plan.close()


def test_autotuned_plan_on_symbolizer_buffers():
    # no tuning: jabba_plan_create picks the launch shapes (output-checked on the
    # device); the plan shares the eager Symbolizer's buffers, sized for the
    # live piece count, and its replays equal the oracle
    import paper_2401_00109_amd as J
    T = torch()
    w = _workload(3)
    v, so = to_dev(w.values), to_dev(w.series_off)
    ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
    od = O.digitize(ol, oi, w.alpha, w.scl, w.B)
    sz = J.Symbolizer(w.n_series, w.n_points, w.D, w.tol, w.alpha, w.scl, w.B, max_pieces=ol.size)
    say(f"autotuned plan: {w.n_series} series, {ol.size} pieces")
    plan = J.Plan.from_symbolizer(sz, v, so)
    t = plan.tuning()
    say(f"  chosen {t}")
    assert t["lanes_per_domain"] in (1, 2, 4) and t["waves_per_block"] in (1, 2, 4)
    assert t["blocks_per_cu"] in (2, 4, 8) and t["stage1_waves"] in (1, 2, 4)
    for rep in range(3):
        sz.symbols.fill_(-1)
        sz.pieces.len.fill_(-1)
        T.cuda.synchronize()
        plan.run()
        T.cuda.synchronize()
        ln, inc, po = sz.pieces.host()
        np.testing.assert_array_equal(ln, ol)
        np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))
        np.testing.assert_array_equal(po, opo)
        np.testing.assert_array_equal(sz.symbols[: ol.size].cpu().numpy(), od.symbols)
        assert sz.dictionary.size() == od.k
        sz.run(v, so)  # eager work on the same buffers between replays
        T.cuda.synchronize()
        np.testing.assert_array_equal(sz.symbols[: ol.size].cpu().numpy(), od.symbols)
    assert plan.status() == (0, 0)
    plan.close()


# ------------------------------------------------------------------ full size
@pytest.fixture(scope="module")
def full_scale():
    """The 4,096 x 10,000-point workload and the oracle's pieces and digitization."""
    w = make_workload(2, seed=0)
    say(f"full-size workload 2: {w.n_series} series, {w.n_points} points; oracle compress + digitize")
    ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
    od = O.digitize(ol, oi, w.alpha, w.scl, w.B)
    return w, ol, oi, opo, od


def test_full_size_scale_workload(full_scale):
    """4,096 x 10,000 points through one Symbolizer on the default stream."""
    import paper_2401_00109_amd as J
    T = torch()
    w, ol, oi, opo, od = full_scale
    v, so = to_dev(w.values), to_dev(w.series_off)
    sz = J.Symbolizer(w.n_series, w.n_points, w.D, w.tol, w.alpha, w.scl, w.B)
    sz.run(v, so)
    T.cuda.synchronize()
    assert sz.status() == (0, 0)
    ln, inc, po = sz.pieces.host()
    np.testing.assert_array_equal(po, opo)
    np.testing.assert_array_equal(ln, ol)
    np.testing.assert_array_equal(inc.view(np.uint64), oi.view(np.uint64))
    say(f"  compress parity ok: N={ol.size}")
    d = sz.dictionary.host()
    assert d["k"] == od.k
    np.testing.assert_array_equal(sz.symbols[: ol.size].cpu().numpy(), od.symbols)
    np.testing.assert_array_equal(d["center_len"].view(np.uint64), od.center_len.view(np.uint64))
    worst = assert_centers_close(d, od, oi, od.symbols)
    say(f"  digitize parity ok: k={od.k} G={od.n_starts} center_inc worst rel {worst:.3e}")


@pytest.mark.parametrize("n_sets", [1, 2])
def test_pipeline_small(n_sets):
    """Batches in flight on a small scale workload (41 series): one and two
    buffer sets, round robin and one batch at a time; every set's symbols,
    encodings and reconstruction equal a plain single-stream run's, and the
    symbols the oracle's."""
    import paper_2401_00109_amd as J
    from paper_2401_00109_amd.pipeline import Pipeline
    from paper_2401_00109_amd.serve import build_resident_dictionary
    T = torch()
    w = _workload(2)
    ol, oi, opo = O.compress(w.values, w.series_off, w.D, w.tol)
    od = O.digitize(ol, oi, w.alpha, w.scl, w.B)
    N = ol.size
    v, so = to_dev(w.values), to_dev(w.series_off)
    t0h = np.where(np.diff(w.series_off) > 0, w.values[np.minimum(w.series_off[:-1], max(w.n_points - 1, 0))], 0.0)
    resident = build_resident_dictionary(DEV)
    say(f"pipeline, {n_sets} set(s), {N} pieces")
    pipe = Pipeline(v, so, to_dev(t0h), w.D, w.tol, w.alpha, w.scl, w.B, N, resident, n_sets=n_sets)
    ref = None
    for pipelined in (True, False):
        pipe.run(3 * n_sets, pipelined=pipelined)
        T.cuda.synchronize()
        for S in pipe.sets:
            assert S.sz.status() == (0, 0)
            np.testing.assert_array_equal(S.sz.symbols[:N].cpu().numpy(), od.symbols)
            got = (S.enc[:N].cpu().numpy(), S.rec.out_off.cpu().numpy(),
                   S.rec.out[: int(S.rec.out_off[-1].item())].cpu().numpy())
            if ref is None:
                enc = J.encode(S.pieces.len, S.pieces.inc, S.pieces.n_pieces, N, resident)
                r = J.reconstruct(S.sz.symbols, S.pieces.piece_off, so, to_dev(t0h), S.sz.dictionary)
                T.cuda.synchronize()
                ref = (enc[:N].cpu().numpy(), r["out_off"].cpu().numpy(), r["out"].cpu().numpy())
            np.testing.assert_array_equal(got[0], ref[0])
            np.testing.assert_array_equal(got[1], ref[1])
            np.testing.assert_array_equal(got[2].view(np.uint64), ref[2].view(np.uint64))


def test_full_size_pipelined_step(full_scale):
    """The benchmark's timed configuration: three buffer sets on three
    streams, each step compress, encode against the resident dictionary,
    digitize and reconstruct (with the squared error).  After two steps per
    set, every set's symbols equal the oracle's; its encodings equal the
    oracle's nearest centers on a sample of pieces (every 16th, and both
    ends); its reconstruction equals, bit for bit, the oracle's
    reconstruction from the set's own dictionary, whose lengths are the
    oracle's bit for bit and whose increments are within the centers'
    tolerance."""
    from paper_2401_00109_amd.pipeline import Pipeline
    from paper_2401_00109_amd.serve import build_resident_dictionary
    T = torch()
    w, ol, oi, opo, od = full_scale
    N = ol.size
    v, so = to_dev(w.values), to_dev(w.series_off)
    t0h = np.where(np.diff(w.series_off) > 0, w.values[np.minimum(w.series_off[:-1], max(w.n_points - 1, 0))], 0.0)
    resident = build_resident_dictionary(DEV)
    say(f"pipelined full step, 3 sets, resident k={resident.size()}")
    pipe = Pipeline(v, so, to_dev(t0h), w.D, w.tol, w.alpha, w.scl, w.B, N, resident, n_sets=3)
    pipe.run(6)
    T.cuda.synchronize()
    rd = resident.host()
    idx = np.unique(np.concatenate([np.arange(0, N, 16), np.arange(min(1000, N)), np.arange(max(N - 1000, 0), N)]))
    enc_exp = O.encode(ol[idx], oi[idx], rd["sigma_len"], rd["sigma_inc"], rd["scl"], rd["cx"], rd["cy"])
    for i, S in enumerate(pipe.sets):
        assert S.steps == 2 and S.sz.status() == (0, 0)
        np.testing.assert_array_equal(S.sz.symbols[:N].cpu().numpy(), od.symbols)
        np.testing.assert_array_equal(S.enc[:N].cpu().numpy()[idx], enc_exp)
        d = S.sz.dictionary.host()
        np.testing.assert_array_equal(d["center_len"].view(np.uint64), od.center_len.view(np.uint64))
        out, oo, _, sse, cnt = O.reconstruct(od.symbols, opo, w.series_off, t0h, d["center_len"], d["center_inc"],
                                             orig=w.values)
        np.testing.assert_array_equal(S.rec.out_off.cpu().numpy(), oo)
        np.testing.assert_array_equal(S.rec.out[: out.size].cpu().numpy().view(np.uint64), out.view(np.uint64))
        np.testing.assert_array_equal(S.rec.cnt[: w.n_series].cpu().numpy(), cnt)
        np.testing.assert_allclose(S.rec.sse[: w.n_series].cpu().numpy(), sse, rtol=1e-12, atol=1e-300)
        say(f"  set {i}: symbols, {idx.size} sampled encodings and {out.size} reconstructed points ok")


def _gpu_encode(ln, inc, sl, si, scl, cx, cy):
    import paper_2401_00109_amd as J
    T = torch()
    k = len(cx)
    d = J.Dictionary.from_host(sl, si, scl, 0.1, np.ones(k), np.zeros(k), cx, cy, device=DEV)
    npc = T.tensor([len(ln)], dtype=T.int64, device=DEV)
    sym = J.encode(to_dev(np.asarray(ln, np.int32)), to_dev(np.asarray(inc, np.float64)), npc, len(ln), d)
    T.cuda.synchronize()
    return sym[: len(ln)].cpu().numpy()


@pytest.mark.parametrize("k", [1, 2, 37, 4096, 4097, 20000])
def test_encode_large_and_tied_dictionaries(k):
    rng = np.random.default_rng(k)
    # centers on discrete length columns with duplicated and mirrored points
    cx = rng.integers(1, 30, k) * 0.37
    cy = np.round(rng.standard_normal(k), 2)
    if k > 10:
        cx[k // 2:k // 2 + 5] = cx[0]
        cy[k // 2:k // 2 + 5] = cy[0]  # exact duplicates: lowest id must win
    ln = rng.integers(1, 30, 20000).astype(np.int32)
    inc = np.round(rng.standard_normal(20000), 2) * 0.9
    sl, si = 2.7027027027027026, 0.9
    say(f"encode k={k}")
    got = _gpu_encode(ln, inc, sl, si, 1.0, cx, cy)
    exp = O.encode(ln, inc, sl, si, 1.0, cx, cy)
    np.testing.assert_array_equal(got, exp)


@pytest.mark.parametrize("k", [3, 300, 3000])
def test_encode_one_column_with_signed_zeros(k):
    # scl = 0 puts every piece at x = 0; the centers' cx mixes +0.0 and -0.0
    # (one column), with repeated cy values and exact duplicates
    rng = np.random.default_rng(100 + k)
    cx = np.where(rng.random(k) < 0.5, 0.0, -0.0)
    cy = np.round(rng.standard_normal(k), 1)
    ln = rng.integers(1, 9, 5000).astype(np.int32)
    inc = np.round(rng.standard_normal(5000), 2)
    say(f"encode one column k={k}")
    got = _gpu_encode(ln, inc, 1.0, 1.0, 0.0, cx, cy)
    exp = O.encode(ln, inc, 1.0, 1.0, 0.0, cx, cy)
    np.testing.assert_array_equal(got, exp)


def test_encode_equidistant_ties():
    # queries exactly halfway between two centers (dyadic values: exact distances)
    cx = np.array([1.0, 1.0, 2.0, 0.0, 1.5])
    cy = np.array([0.5, -0.5, 0.0, 0.0, 0.0])
    ln = np.array([1, 1, 1, 1], np.int32)
    inc = np.array([0.0, 0.25, -0.25, 0.5])
    got = _gpu_encode(ln, inc, 1.0, 1.0, 1.0, cx, cy)
    exp = O.encode(ln, inc, 1.0, 1.0, 1.0, cx, cy)
    np.testing.assert_array_equal(got, exp)
