"""The oracle at full workload size, step by step.

Test infrastructure only.  ``oracle.digitize`` runs the whole two-stage
digitization in one sequential call, which takes minutes for the 3e8 pieces
of the uneven workload; a test must report back well within that.  This
module runs the same steps (Sec. 5: scaling, one global sorting index,
contiguous blocks, Stage I per block, Stage II over the starting points,
label propagation, group means) as separate calls to the oracle's own step
functions (``scaling``, ``blocks``, ``aggregate_sorted``), so that each can
be a test of its own, and spreads the independent parts over threads (the
oracle releases the interpreter lock while it runs):

* compression: series are independent (Sec. 4.1.2), so chunks of series are
  compressed in parallel and concatenated;
* the sort: the order is the one total order by (key, canonical index).  It
  is computed with numpy's stable argsort (a library sort) as a sample sort:
  key ranges from a sample, indices moved to their range in index order,
  each range sorted in parallel; equal keys share a range, so ties stay in
  index order;
* Stage I: blocks are independent; each block is one ``aggregate_sorted``
  call on its slice.

Nothing here adds arithmetic of its own: group means use the exact length
sum and, for the increments, the oracle's own exact sum (correctly rounded),
as the oracle's dictionary step does.  ``tests/test_oracle_full.py`` checks that
these steps give ``oracle.digitize``'s result bit for bit.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O


def threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def compress(values, series_off, D, tol, max_len=0, n_threads=None):
    """oracle.compress over chunks of whole series in parallel, concatenated."""
    so = np.asarray(series_off, np.int64)
    ns = so.size - 1
    nt = n_threads or threads()
    cuts = np.unique(np.linspace(0, ns, min(ns, 4 * nt) + 1).astype(np.int64)) if ns else np.array([0])

    def run(i):
        a, b = int(cuts[i]), int(cuts[i + 1])
        return O.compress(values[so[a]:so[b]], so[a:b + 1] - so[a], D, tol, max_len)

    with ThreadPoolExecutor(nt) as ex:
        parts = list(ex.map(run, range(cuts.size - 1)))
    ln = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.int32)
    inc = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0)
    po = np.zeros(ns + 1, np.int64)
    base = 0
    for i, p in enumerate(parts):
        a, b = int(cuts[i]), int(cuts[i + 1])
        po[a:b + 1] = p[2] + base
        base += int(p[2][-1])
    return ln, inc, po


def reconstruct(symbols, piece_off, series_off, t0, center_len, center_inc, orig, n_threads=None):
    """oracle.reconstruct over chunks of whole series in parallel, concatenated.

    Returns (out, out_off, sse, cnt) as oracle.reconstruct does (without the
    quantized lengths)."""
    po, so = np.asarray(piece_off, np.int64), np.asarray(series_off, np.int64)
    ns = so.size - 1
    nt = n_threads or threads()
    cuts = np.unique(np.linspace(0, ns, min(ns, 4 * nt) + 1).astype(np.int64)) if ns else np.array([0])

    def run(i):
        a, b = int(cuts[i]), int(cuts[i + 1])
        out, oo, _, sse, cnt = O.reconstruct(symbols[po[a]:po[b]], po[a:b + 1] - po[a], so[a:b + 1] - so[a],
                                             t0[a:b], center_len, center_inc, orig=orig[so[a]:so[b]])
        return out, oo, sse, cnt

    with ThreadPoolExecutor(nt) as ex:
        parts = list(ex.map(run, range(cuts.size - 1)))
    out = np.concatenate([p[0] for p in parts])
    oo = np.zeros(ns + 1, np.int64)
    base = 0
    for i, p in enumerate(parts):
        a, b = int(cuts[i]), int(cuts[i + 1])
        oo[a:b + 1] = p[1] + base
        base += int(p[1][-1])
    return out, oo, np.concatenate([p[2] for p in parts]), np.concatenate([p[3] for p in parts])


def _stable_bucket_order(b, nb):
    """Indices ordered by bucket, index order inside a bucket (a counting sort)."""
    if nb <= 1 << 16:
        return np.argsort(b.astype(np.uint16), kind="stable")  # numpy's radix sort
    return np.argsort(b, kind="stable")


def sort_order(key, n_threads=None):
    """Permutation sorting (key, index) ascending.

    Sample sort: bucket bounds from a regular sample of the keys, every index
    moved to its key's bucket in index order, each bucket sorted (stable) in
    parallel.  Equal keys fall in one bucket, so ties keep index order."""
    n = key.size
    nt = n_threads or threads()
    if n < (1 << 20) or nt == 1:
        return np.argsort(key, kind="stable")
    nb = 8 * nt
    bounds = np.unique(np.sort(key[:: max(1, n // (64 * nb))])[:: 64][1:])
    cuts = np.linspace(0, n, nt + 1).astype(np.int64)
    bucket = np.empty(n, np.int32)

    def locate(i):
        a, b = int(cuts[i]), int(cuts[i + 1])
        bucket[a:b] = np.searchsorted(bounds, key[a:b], side="right")

    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(locate, range(nt)))
    order = _stable_bucket_order(bucket, bounds.size + 1)
    edges = np.concatenate(([0], np.cumsum(np.bincount(bucket, minlength=bounds.size + 1))))
    del bucket

    def run(j):
        a, b = int(edges[j]), int(edges[j + 1])
        seg = order[a:b]
        order[a:b] = seg[np.argsort(key[seg], kind="stable")]

    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(run, range(edges.size - 1)))
    return order


class Digitization:
    """The oracle's two-stage digitization, one step per method (call in order)."""

    def __init__(self, length, inc, alpha, scl=1.0, B=4096, n_threads=None):
        self.len = np.ascontiguousarray(length, np.int32)
        self.inc = np.ascontiguousarray(inc, np.float64)
        self.alpha, self.scl, self.B = float(alpha), float(scl), int(B)
        self.nt = n_threads or threads()
        self.N = self.len.size

    def scaling(self):
        self.sigma_len, self.sigma_inc, self.x, self.y, self.key = O.scaling(self.len, self.inc, self.scl)

    def sort(self):
        self.perm = sort_order(self.key, self.nt)
        self.sk = self.key[self.perm]
        del self.key
        self.sx = self.x[self.perm]
        del self.x
        self.sy = self.y[self.perm]
        del self.y

    def stage1(self):
        self.bstart = O.blocks(self.sk, self.B)
        M = self.bstart.size - 1
        lab = np.empty(self.N, np.int64)
        bs = self.bstart

        def run(r):
            for b in range(r[0], r[1]):
                lo, hi = int(bs[b]), int(bs[b + 1])
                lab[lo:hi] = O.aggregate_sorted(self.sx[lo:hi], self.sy[lo:hi], self.sk[lo:hi], self.alpha) + lo

        step = max(1, -(-M // (8 * self.nt)))
        with ThreadPoolExecutor(self.nt) as ex:
            list(ex.map(run, [(a, min(a + step, M)) for a in range(0, M, step)]))
        self.lab = lab
        self.starts = np.flatnonzero(lab == np.arange(self.N, dtype=np.int64))
        self.G = int(self.starts.size)

    def stage2(self):
        s = self.starts
        glab = O.aggregate_sorted(self.sx[s], self.sy[s], self.sk[s], self.alpha)
        del self.sx, self.sy, self.sk
        own = glab == np.arange(self.G, dtype=np.int64)
        sym_of_start = np.cumsum(own) - 1          # global symbols numbered by sorted position of their start
        self.k = int(own.sum())
        self.gmap = sym_of_start[glab]
        sidx = np.full(self.N, -1, np.int64)
        sidx[s] = np.arange(self.G, dtype=np.int64)
        symbols = np.empty(self.N, np.int32)
        symbols[self.perm] = self.gmap[sidx[self.lab]].astype(np.int32)
        del sidx
        self.symbols = symbols

    def centers(self):
        """count, center_len (exact length sum), center_inc (exact increment sum, correctly rounded), cx, cy."""
        k = self.k
        self.count = np.bincount(self.symbols, minlength=k).astype(np.int64)
        slen = np.bincount(self.symbols, weights=self.len.astype(np.float64), minlength=k)  # exact below 2^53
        assert float(np.max(slen, initial=0.0)) < 2.0 ** 53
        cnt = self.count.astype(np.float64)
        self.center_len = slen / cnt
        self.cx = self.scl * (self.center_len / self.sigma_len)
        order = _stable_bucket_order(self.symbols, k)
        vals = self.inc[order]
        del order
        edges = np.concatenate(([0], np.cumsum(self.count)))
        sums = np.zeros(k)

        def run(r):
            for c in range(r[0], r[1]):
                sums[c] = O.exact_sum(vals[edges[c]:edges[c + 1]])

        step = max(1, -(-k // (8 * self.nt)))
        with ThreadPoolExecutor(self.nt) as ex:
            list(ex.map(run, [(a, min(a + step, k)) for a in range(0, k, step)]))
        self.center_inc = sums / cnt
        self.cy = self.center_inc / self.sigma_inc
