"""The paper's own synthetic experiment on the device (Sec. 7.3).

One series of N(0, 1) noise, n = 100,000 points, tol = 0.01, alpha = 0.05,
cut into M equal partitions (the domains of Alg. 1 Phase I: D = ceil((n-1)/M)
intervals each).  Per M the device compresses (boundary artifacts add
pieces as M grows, Sec. 4.1.3), digitizes with the aggregation over a single
block (the paper keeps digitization sequential here), and reconstructs every
partition from its own first value (partition points restart the
reconstruction); it also digitizes with Lloyd's k-means for the aggregation's
symbol count (the paper feeds that count to ABBA's k-means), seeded by
default with the aggregation's own centers so Lloyd refines that codebook
(its SSE can only fall from the nearest-center assignment of those centers);
``kmeans_init="spread"`` seeds from k evenly spaced pieces instead.  Reported per M:
pieces, pieces added by the partition boundaries, symbols, and for both
digitizations the reconstruction MSE and the VQ objective (Eq. sse).

    python -m paper_2401_00109_amd.experiments --partitions 1,2,4,8,16,32,64
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import api
from .inputs import series_rng

NOISE_ID = 7  # generator stream id of this experiment


def noise_series(n: int = 100_000, seed: int = 0) -> np.ndarray:
    """N(0, 1) noise (already zero mean, unit deviation in law; not re-normalised)."""
    return series_rng(seed, NOISE_ID, 0).standard_normal(n)


def _pieces(v, so, D, tol, dev):
    p = api.compress(v, so, D, tol)
    torch.cuda.synchronize()
    return p


def _domains(x: np.ndarray, ln: np.ndarray, D: int):
    """Each partition as its own series: point ranges [dD, min((d+1)D, n-1)], its pieces and its first value."""
    n = x.size
    starts = np.arange(0, max(n - 1, 1), D, dtype=np.int64)
    ends = np.minimum(starts + D, n - 1)
    # pieces never cross a partition boundary: partition d's pieces end where the length sum reaches ends[d]
    cum = np.concatenate([[0], np.cumsum(ln.astype(np.int64))])
    piece_off = np.searchsorted(cum, ends - starts[0], side="left")
    piece_off = np.concatenate([[0], piece_off]).astype(np.int64)
    seg = [x[a:e + 1] for a, e in zip(starts, ends)]
    series_off = np.concatenate([[0], np.cumsum([s.size for s in seg])]).astype(np.int64)
    return np.concatenate(seg), series_off, piece_off, x[starts].copy()


def _mse(sym, dictionary, dom, dev):
    """Reconstruction error with every partition restarted from its true first value."""
    values, series_off, piece_off, t0 = dom
    r = api.reconstruct(sym, torch.from_numpy(piece_off).to(dev), torch.from_numpy(series_off).to(dev),
                        torch.from_numpy(t0).to(dev), dictionary, values=torch.from_numpy(values).to(dev))
    sse = float(r["sse"].sum().item())
    cnt = int(r["cnt"].sum().item())
    return sse / max(cnt, 1)


def _sse(ln, ic, sym, h):
    """VQ objective in the scaled space (Eq. sse) from host copies."""
    x = h["scl"] * (ln / h["sigma_len"])
    y = ic / h["sigma_inc"]
    return float(np.sum((x - h["cx"][sym]) ** 2 + (y - h["cy"][sym]) ** 2))


def noise_partitions(partitions, n: int = 100_000, tol: float = 0.01, alpha: float = 0.05, seed: int = 0,
                     kmeans_iter: int = 100, kmeans_init: str = "aggregation", device=None) -> list[dict]:
    if kmeans_init not in ("aggregation", "spread"):
        raise ValueError(f"kmeans_init must be 'aggregation' or 'spread', not {kmeans_init!r}")
    dev = torch.device("cuda", 0) if device is None else torch.device(device)
    x = noise_series(n, seed)
    v = torch.from_numpy(x).to(dev)
    so = torch.tensor([0, n], dtype=torch.int64, device=dev)
    t0 = v[:1].clone()
    rows = []
    base_pieces = None
    for M in partitions:
        D = max(1, -(-(n - 1) // M))
        p = _pieces(v, so, D, tol, dev)
        N = p.count()
        if base_pieces is None and M == 1:
            base_pieces = N
        ln = p.len[:N].cpu().numpy()
        ic = p.inc[:N].cpu().numpy()
        dom = _domains(x, ln, D)
        sym, d, ws = api.digitize(p.len, p.inc, p.n_pieces, N, alpha, 1.0, 1 << 30)
        torch.cuda.synchronize()
        k = d.size()
        h = d.host()
        mse_agg = _mse(sym, d, dom, dev)
        sse_agg = _sse(ln, ic, sym[:N].cpu().numpy(), h)
        # k-means with the aggregation's symbol count
        if kmeans_init == "aggregation":
            cx0, cy0 = h["cx"].copy(), h["cy"].copy()
        else:
            pick = np.linspace(0, N - 1, k).astype(np.int64)
            cx0 = h["scl"] * (ln[pick] / h["sigma_len"])
            cy0 = ic[pick] / h["sigma_inc"]
        dk = api.Dictionary.from_host(h["sigma_len"], h["sigma_inc"], h["scl"], alpha, np.zeros(k), np.zeros(k), cx0,
                                      cy0, device=dev)
        symk, iters = api.kmeans(p.len, p.inc, p.n_pieces, N, dk, max_iter=kmeans_iter)
        torch.cuda.synchronize()
        mse_km = _mse(symk, dk, dom, dev)
        sse_km = _sse(ln, ic, symk[:N].cpu().numpy(), dk.host())
        rows.append({"M": M, "D": D, "pieces": N, "boundary_pieces": None if base_pieces is None else N - base_pieces,
                     "symbols": k, "mse_aggregation": mse_agg, "mse_kmeans": mse_km, "sse_aggregation": sse_agg,
                     "sse_kmeans": sse_km, "kmeans_iterations": int(iters.item())})
    return rows


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--partitions", default="1,2,4,8,16,32,64,128")
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--kmeans-init", default="aggregation", choices=["aggregation", "spread"])
    ap.add_argument("--kmeans-iter", type=int, default=100)
    a = ap.parse_args()
    rows = noise_partitions([int(m) for m in a.partitions.split(",")], n=a.n, kmeans_iter=a.kmeans_iter,
                            kmeans_init=a.kmeans_init)
    for r in rows:
        print(json.dumps(r))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
