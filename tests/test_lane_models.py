"""Host models of cross-lane steps the kernels take on a 64-lane wavefront.

* The lane moves of lane_ops.h, written from the documented semantics of
  each DPP control and permlane swap, give lane ^ M for every M used.
* The Stage I sums' segmented scan (row shifts by 1, 2, 4, 8 inside rows of
  16 lanes, then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31
  into rows 2 and 3; a lane adds its source only when the source's segment
  equals its own) equals the plain segmented inclusive sum whenever the
  segments are sorted across the lanes, as the bitonic network leaves them.
* The reconstruction's series order (a counting sort by descending
  power-of-two class of the chunk count, each workgroup reserving a range
  per class) is a permutation that never puts a series before one of a
  higher class.
"""
import numpy as np
import pytest

LANES = np.arange(64)


def dpp_quad_perm(v, sel):
    return np.array([v[(l & ~3) + sel[l & 3]] for l in LANES])


def dpp_row(v, src_of, old, bound=lambda s, l: (s // 16) == (l // 16)):
    out = np.array(old, copy=True)
    for l in LANES:
        s = src_of(l)
        if 0 <= s < 64 and bound(s, l):
            out[l] = v[s]
    return out


def row_shl(v, n, old):   # lane l reads lane l + n of its row
    return dpp_row(v, lambda l: l + n, old)


def row_shr(v, n, old):   # lane l reads lane l - n of its row
    return dpp_row(v, lambda l: l - n, old)


def row_ror(v, n):        # lane l reads lane (l + n) mod 16 of its row
    return np.array([v[(l & ~15) + ((l + n) & 15)] for l in LANES])


def permlane16_swap(a, b):
    # odd rows of the first operand swap with even rows of the second
    a2, b2 = a.copy(), b.copy()
    for r in (0, 2):
        a2[(r + 1) * 16:(r + 2) * 16], b2[r * 16:(r + 1) * 16] = b[r * 16:(r + 1) * 16], a[(r + 1) * 16:(r + 2) * 16]
    return a2, b2


def permlane32_swap(a, b):
    # the upper half of the first operand swaps with the lower half of the second
    a2, b2 = a.copy(), b.copy()
    a2[32:], b2[:32] = b[:32], a[32:]
    return a2, b2


def xor_lane(v, m):
    if m == 1:
        return dpp_quad_perm(v, [1, 0, 3, 2])
    if m == 2:
        return dpp_quad_perm(v, [2, 3, 0, 1])
    if m == 4:
        up, dn = row_shl(v, 4, np.zeros(64, v.dtype)), row_shr(v, 4, np.zeros(64, v.dtype))
        return np.where(LANES & 4, dn, up)
    if m == 8:
        return row_ror(v, 8)
    if m == 16:
        r0, r1 = permlane16_swap(v, v)
        return np.where(LANES & 16, r0, r1)
    r0, r1 = permlane32_swap(v, v)
    return np.where(LANES & 32, r0, r1)


@pytest.mark.parametrize("m", [1, 2, 4, 8, 16, 32])
def test_xor_lane_moves(m):
    v = np.arange(64) * 3 + 1000
    np.testing.assert_array_equal(xor_lane(v, m), v[LANES ^ m])


def test_bitonic_network_with_xor_partners_sorts():
    rng = np.random.default_rng(1)
    for _ in range(200):
        k = rng.integers(0, 1 << 20, size=64)
        size = 2
        while size <= 64:
            stride = size // 2
            while stride:
                o = xor_lane(k, stride)
                up = ((LANES & size) == 0) | (size == 64)
                low = (LANES & stride) == 0
                k = np.where(low == up, np.minimum(k, o), np.maximum(k, o))
                stride //= 2
            size *= 2
        assert np.all(np.diff(k) >= 0)


NOSRC = -1


def seg_step(seg, v, src_of, rows):
    ys = np.full(64, NOSRC)
    yv = np.zeros(64, v.dtype)
    for l in LANES:
        if (l // 16) not in rows:
            continue
        s = src_of(l)
        if s is not None and 0 <= s < 64:
            ys[l], yv[l] = seg[s], v[s]
    return np.where(ys == seg, v + yv, v)


def dpp_segmented_scan(seg, v):
    for d in (1, 2, 4, 8):
        v = seg_step(seg, v, lambda l, d=d: l - d if (l - d) // 16 == l // 16 else None, {0, 1, 2, 3})
    v = seg_step(seg, v, lambda l: (l // 16) * 16 - 1, {1, 3})   # lane 15 of the row before
    v = seg_step(seg, v, lambda l: 31, {2, 3})
    return v


@pytest.mark.parametrize("n_segments", [1, 2, 5, 17, 40, 64])
def test_row_broadcast_segmented_scan_equals_plain(n_segments):
    rng = np.random.default_rng(n_segments)
    for _ in range(200):
        seg = np.sort(rng.integers(0, n_segments, size=64))
        v = rng.integers(-1000, 1000, size=64)
        want = np.array([v[(seg == seg[l]) & (LANES <= l)].sum() for l in LANES])
        np.testing.assert_array_equal(dpp_segmented_scan(seg, v), want)


def order_class(pieces):
    nch = (pieces + 63) // 64
    if nch <= 0:
        return 33
    lg = int(nch).bit_length() - 1
    return 32 - lg if lg < 32 else 0


def series_order(piece_counts, threads=256):
    cls = [order_class(p) for p in piece_counts]
    hist = np.bincount(cls, minlength=34)
    base = np.concatenate([[0], np.cumsum(hist)[:-1]])
    cursor = np.zeros(34, np.int64)
    order = np.full(len(piece_counts), -1)
    # workgroups in an arbitrary order, as the dispatcher may run them
    chunks = [list(range(s0, min(s0 + threads, len(piece_counts)))) for s0 in range(0, len(piece_counts), threads)]
    rng = np.random.default_rng(len(piece_counts))
    for ci in rng.permutation(len(chunks)):
        ids = chunks[ci]
        h = np.zeros(34, np.int64)
        rank = {}
        for s in rng.permutation(ids):   # LDS atomics in any lane order
            rank[s] = h[cls[s]]
            h[cls[s]] += 1
        at = {c: base[c] + cursor[c] for c in range(34) if h[c]}
        for c in at:
            cursor[c] += h[c]
        for s in ids:
            order[at[cls[s]] + rank[s]] = s
    return order, cls


@pytest.mark.parametrize("n", [1, 255, 256, 257, 5000])
def test_series_order_is_a_longest_class_first_permutation(n):
    rng = np.random.default_rng(n)
    pieces = np.floor(np.exp(rng.uniform(0, np.log(50_000), size=n))).astype(np.int64)
    pieces[rng.random(n) < 0.05] = 0
    order, cls = series_order(pieces)
    assert sorted(order.tolist()) == list(range(n))
    c = np.array(cls)[order]
    assert np.all(np.diff(c) >= 0)
    # power-of-two classes: no later series has twice the chunks of an earlier one
    nch = (pieces[order] + 63) // 64
    later_max = np.maximum.accumulate(nch[::-1])[::-1]
    for i in range(n - 1):
        if nch[i] > 0:
            assert later_max[i + 1] < 2 * nch[i]
