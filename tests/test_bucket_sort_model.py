"""Host model of the digitizer's bucket sort (the main sort's finish after the
prefix radix passes): tiles take the prefix groups that start in them,
groups up to the cap are ranked locally, larger groups go to the fallback,
which sorts them together and places them in order into their positions.
The model follows the kernels' index arithmetic (tile bounds, the search for
the last group's end, the fallback plan and offsets) and is checked against
a plain lexicographic sort on inputs built to stress it: groups crossing tile
ends, tail groups exactly at the cap, groups larger than the cap inside one
tile, one group spanning many tiles, every key equal, a tiny array."""
import numpy as np
import pytest

TILE, CAP = 1024, 256


def bucket_sort_model(keys, prefix_shift, tile=TILE, cap=CAP):
    """keys: uint64 already grouped by prefix (stable); returns the permutation."""
    n = keys.size
    pre = (keys >> np.uint64(prefix_shift)) if prefix_shift < 64 else np.zeros(n, np.uint64)
    head = np.ones(n, bool)
    head[1:] = pre[1:] != pre[:-1]
    out = np.full(n, -1, np.int64)
    ntiles = -(-n // tile)
    thead = np.full(ntiles, -1, np.int64)
    tlarge = np.full(ntiles, -1, np.int64)
    for t in range(ntiles):
        b0 = t * tile
        b1 = min(b0 + tile, n)
        hs = np.flatnonzero(head[b0:b1]) + b0
        if hs.size == 0:
            continue
        lo, s_last = int(hs[0]), int(hs[-1])
        e_lim = min(b1 + cap, n)
        nxt = np.flatnonzero(head[b1:e_lim]) + b1
        e = int(nxt[0]) if nxt.size else (n if e_lim == n else None)
        large = e is None or e - s_last > cap
        hi = s_last if large else e
        assert hi - lo <= tile + cap
        thead[t] = lo
        tlarge[t] = s_last if large else -1
        # local ranks by (key, position) inside each group of [lo, hi)
        seg_h = np.flatnonzero(head[lo:hi]) + lo
        ends = np.append(seg_h[1:], hi)
        for a, b in zip(seg_h, ends):
            idx = np.arange(a, b)
            order = idx[np.lexsort((idx, keys[a:b]))]
            out[a:b] = order
    # fallback: large groups end at the next tile's first group start
    lsize = np.zeros(ntiles, np.int64)
    for t in range(ntiles):
        if tlarge[t] >= 0:
            later = thead[t + 1:]
            later = later[later >= 0]
            e = int(later[0]) if later.size else n
            lsize[t] = e - tlarge[t]
    loff = np.concatenate([[0], np.cumsum(lsize)])
    total = int(loff[-1])
    pos = np.empty(total, np.int64)
    for j in range(total):
        a = int(np.searchsorted(loff[:ntiles], j, side="right") - 1)
        pos[j] = tlarge[a] + (j - loff[a])
    assert np.all(np.diff(pos) > 0)
    srt = pos[np.lexsort((pos, keys[pos]))]
    out[pos] = srt
    assert np.all(out >= 0)
    return out, total


def _grouped(keys, shift):
    pre = keys >> np.uint64(shift) if shift < 64 else np.zeros(keys.size, np.uint64)
    return keys[np.argsort(pre, kind="stable")]


@pytest.mark.parametrize("case", ["random", "crossing", "at_cap", "spanning", "all_equal", "tiny", "cap_plus_one"])
def test_bucket_sort_model_matches_lexsort(case):
    rng = np.random.default_rng(hash(case) % 1000)
    shift = 20
    if case == "random":
        keys = rng.integers(0, 1 << 40, 200_000, dtype=np.uint64)
    elif case == "crossing":  # many groups of 300-700 members crossing tile ends
        g = np.repeat(np.arange(300, dtype=np.uint64), rng.integers(300, 700, 300))
        keys = (g << np.uint64(shift)) | rng.integers(0, 1 << 18, g.size, dtype=np.uint64)
    elif case == "at_cap":  # tail groups exactly at the cap, and groups of a whole tile
        g = np.repeat(np.arange(50, dtype=np.uint64), np.where(np.arange(50) % 2 == 0, CAP, TILE))
        keys = (g << np.uint64(shift)) | rng.integers(0, 8, g.size, dtype=np.uint64)
    elif case == "cap_plus_one":  # groups just above the cap, and large groups inside one tile
        g = np.repeat(np.arange(40, dtype=np.uint64), np.where(np.arange(40) % 3 == 0, CAP + 1, 700))
        keys = (g << np.uint64(shift)) | rng.integers(0, 1 << 10, g.size, dtype=np.uint64)
    elif case == "spanning":  # one group over many tiles among small ones
        g = np.concatenate([np.zeros(500), np.ones(20_000), np.arange(2, 3000).repeat(3)]).astype(np.uint64)
        keys = (g << np.uint64(shift)) | rng.integers(0, 1 << 12, g.size, dtype=np.uint64)
    elif case == "all_equal":
        keys = np.full(50_000, 12345, np.uint64)
        shift = 64
    else:
        keys = np.array([5, 3, 9], np.uint64)
    keys = _grouped(keys, shift)
    perm, large = bucket_sort_model(keys, shift)
    exp = np.lexsort((np.arange(keys.size), keys))
    np.testing.assert_array_equal(perm, exp)
    if case in ("spanning", "all_equal", "cap_plus_one"):
        assert large > 0
    if case == "tiny":
        assert large == 0
