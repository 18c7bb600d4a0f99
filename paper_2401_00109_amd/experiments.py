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

The Gaussian-blob table (Sec. 7.1, Table 2) runs the two-stage aggregation
on raw 2-D points:

    python -m paper_2401_00109_amd.experiments --blobs

The digitizer sweep (scl, separate tolerances, PCA key) runs on a compressed
workload of the input recipe:

    python -m paper_2401_00109_amd.experiments --sweep '[{"scl": 0}, {"scl": 1}, {"key": "pca"}]'
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
    return api.reconstruction_mse(r["sse"], r["cnt"], series_off.size - 1)


def _sse(ln, ic, sym, h):
    """VQ objective in the scaled space (Eq. sse) from host copies."""
    x = h["scl"] * (ln / h["sigma_len"])
    y = ic / h["sigma_inc"]
    return float(np.sum((x - h["cx"][sym]) ** 2 + (y - h["cy"][sym]) ** 2))


def noise_partitions(partitions, n: int = 100_000, tol: float = 0.01, alpha: float = 0.05, seed: int = 0,
                     kmeans_iter: int = 100, kmeans_init: str = "aggregation", device=None,
                     keep_symbols: bool = False) -> list[dict]:
    """One row per partition count M; keep_symbols adds both digitizations' symbols (host arrays)."""
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
        if keep_symbols:
            rows[-1]["symbols_aggregation"] = sym[:N].cpu().numpy()
            rows[-1]["symbols_kmeans"] = symk[:N].cpu().numpy()
    return rows


def digitizer_sweep(settings, workload_id: int = 2, scale: float = 1.0, seed: int = 0, B: int | None = None,
                    device=None) -> list[dict]:
    """The digitizer variants of Sec. 3.2 and Sec. 5 on one compressed workload.

    Each setting is a dict with optional keys scl (length weight, Sec. 3.2: 0 clusters increments only, 1
    weighs both alike), alpha, alpha_len / alpha_inc (separate tolerances, Eq. Var1; they replace alpha and
    scale scl) and key ("norm" or "pca", Sec. 5).  The series are compressed once on the device; per setting
    the device digitizes, reports k, the Stage I starting points, the VQ objective and largest per-symbol
    variances in the digitizer's own scaled space (Eq. sse, Eq. Var), and the reconstruction MSE."""
    from .inputs import make_workload
    dev = torch.device("cuda", 0) if device is None else torch.device(device)
    w = make_workload(workload_id, seed, scale)
    v = torch.from_numpy(w.values).to(dev)
    so = torch.from_numpy(w.series_off).to(dev)
    t0 = torch.from_numpy(w.values[w.series_off[:-1]].copy()).to(dev)
    B = w.B if B is None else int(B)
    p = api.compress(v, so, w.D, w.tol, w.max_len)
    torch.cuda.synchronize()
    N = p.count()
    rows = []
    for st in settings:
        scl = float(st.get("scl", w.scl))
        alpha = float(st.get("alpha", w.alpha))
        if "alpha_len" in st:
            alpha, scl = api.axis_tolerances(st["alpha_len"], st["alpha_inc"], scl)
        key = st.get("key", "norm")
        sym, d, ws = api.digitize(p.len, p.inc, p.n_pieces, p.max_pieces, alpha, scl, B, key=key)
        q = api.digitize_quality(p.len, p.inc, p.n_pieces, p.max_pieces, alpha, B, d, ws)
        r = api.reconstruct(sym, p.piece_off, so, t0, d, values=v)
        torch.cuda.synchronize()
        stats = api.digitize_stats(ws, p.max_pieces, B)
        tot = q["totals"].cpu().numpy()
        row = dict(st)
        row.update({"workload": workload_id, "pieces": N, "alpha_used": alpha, "scl_used": scl, "symbols": d.size(),
                    "starts": stats["G"], "sse": float(tot[0]), "max_var_len": float(tot[1]),
                    "max_var_inc": float(tot[2]),
                    "mse": api.reconstruction_mse(r["sse"], r["cnt"], so.numel() - 1)})
        if key == "pca":
            row["axis"] = d.axis.cpu().numpy().tolist()
        rows.append(row)
    return rows


def gaussian_blobs(sizes=(5000, 10000), alphas=(0.1, 0.05), blocks=(1, 4, 8), seed: int = 0, repeats: int = 20,
                   device=None) -> list[dict]:
    """Table 2 of Sec. 7.1 on the device: the two-stage aggregation of 2-D Gaussian-blob points with M blocks
    of ceil(N/M) points (M = 1 is the serial greedy aggregation).  Per (alpha, N, M): clusters, SSE (Eq. sse),
    SSE ratio against M = 1, and the device time of one aggregation (median of `repeats`, HIP events)."""
    from .inputs import gaussian_blobs as blobs
    dev = torch.device("cuda", 0) if device is None else torch.device(device)
    rows = []
    for alpha in alphas:
        for n in sizes:
            x, y = blobs(seed, n)
            X = torch.from_numpy(x).to(dev)
            Y = torch.from_numpy(y).to(dev)
            serial = None
            for M in blocks:
                B = -(-n // M)
                r = api.aggregate_points(X, Y, alpha, B)
                ws = r["workspace"]
                times = []
                for _ in range(repeats):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    api.aggregate_points(X, Y, alpha, B, workspace=ws)
                    b.record()
                    torch.cuda.synchronize()
                    times.append(a.elapsed_time(b))
                k = int(r["k"].item())
                sse = float(r["sse"].item())
                if M == 1:
                    serial = (k, sse)
                rows.append({"alpha": alpha, "N": n, "M": M, "B": B, "clusters": k, "sse": sse,
                             "sse_ratio": sse / serial[1] if serial and serial[1] > 0 else None,
                             "clusters_serial": serial[0] if serial else None,
                             "device_ms": float(np.median(times))})
    return rows


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--partitions", default="1,2,4,8,16,32,64,128")
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--kmeans-init", default="aggregation", choices=["aggregation", "spread"])
    ap.add_argument("--kmeans-iter", type=int, default=100)
    ap.add_argument("--sweep", default="", help="digitizer settings as JSON list (runs the sweep instead)")
    ap.add_argument("--blobs", action="store_true", help="run the Gaussian-blob table (Sec. 7.1) instead")
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0)
    a = ap.parse_args()
    if a.blobs:
        rows = gaussian_blobs()
    elif a.sweep:
        rows = digitizer_sweep(json.loads(a.sweep), workload_id=a.workload, scale=a.scale)
    else:
        rows = noise_partitions([int(m) for m in a.partitions.split(",")], n=a.n, kmeans_iter=a.kmeans_iter,
                                kmeans_init=a.kmeans_init)
    for r in rows:
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
