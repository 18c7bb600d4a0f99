"""The paper's own synthetic experiment on the device (Sec. 7.3).

One series of N(0, 1) noise, n = 100,000 points, tol = 0.01, alpha = 0.05,
cut into M equal partitions (the domains of Alg. 1 Phase I: D = ceil((n-1)/M)
intervals each).  Per M the device compresses (boundary artifacts add
pieces as M grows, Sec. 4.1.3), digitizes with the aggregation over a single
block (the paper keeps digitization sequential here), and reconstructs; it
also digitizes with k-means for the aggregation's symbol count (the paper
feeds that count to ABBA's k-means).  Reported per M: pieces, pieces added
by the partition boundaries, symbols, and the reconstruction MSE of both
digitizations.

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


def _mse(p, sym, dictionary, values, so, t0):
    r = api.reconstruct(sym, p.piece_off, so, t0, dictionary, values=values)
    sse = float(r["sse"].sum().item())
    cnt = int(r["cnt"].sum().item())
    return sse / max(cnt, 1)


def noise_partitions(partitions, n: int = 100_000, tol: float = 0.01, alpha: float = 0.05, seed: int = 0,
                     kmeans_iter: int = 100, device=None) -> list[dict]:
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
        sym, d, ws = api.digitize(p.len, p.inc, p.n_pieces, N, alpha, 1.0, 1 << 30)
        torch.cuda.synchronize()
        k = d.size()
        mse_agg = _mse(p, sym, d, v, so, t0)
        # k-means with the aggregation's symbol count, from k evenly spaced pieces
        h = d.host()
        pick = np.linspace(0, N - 1, k).astype(np.int64)
        ln = p.len[:N].cpu().numpy()
        ic = p.inc[:N].cpu().numpy()
        cx0 = h["scl"] * (ln[pick] / h["sigma_len"])
        cy0 = ic[pick] / h["sigma_inc"]
        dk = api.Dictionary.from_host(h["sigma_len"], h["sigma_inc"], h["scl"], alpha, np.zeros(k), np.zeros(k), cx0,
                                      cy0, device=dev)
        symk, iters = api.kmeans(p.len, p.inc, p.n_pieces, N, dk, max_iter=kmeans_iter)
        torch.cuda.synchronize()
        mse_km = _mse(p, symk, dk, v, so, t0)
        rows.append({"M": M, "D": D, "pieces": N, "boundary_pieces": None if base_pieces is None else N - base_pieces,
                     "symbols": k, "mse_aggregation": mse_agg, "mse_kmeans": mse_km,
                     "kmeans_iterations": int(iters.item())})
    return rows


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--partitions", default="1,2,4,8,16,32,64,128")
    ap.add_argument("--n", type=int, default=100_000)
    a = ap.parse_args()
    rows = noise_partitions([int(m) for m in a.partitions.split(",")], n=a.n)
    for r in rows:
        print(json.dumps(r))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
