"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
bring the results to the host.  Nothing here computes the method."""
from __future__ import annotations

import sys

import numpy as np

DEV = "cuda:0"


def say(msg: str) -> None:
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def torch():
    import torch as T
    return T


def to_dev(a, dtype=None):
    T = torch()
    t = T.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def gpu_compress(values, series_off, D, tol, max_len=0, tuning=None, plain=False, znorm=False):
    import paper_2401_00109_amd as J
    T = torch()
    v = to_dev(np.asarray(values, np.float64))
    so = to_dev(np.asarray(series_off, np.int64))
    if plain:
        p = J.compress_plain(v, so, np.asarray(series_off, np.int64), D, tol, max_len)
    else:
        p = J.compress(v, so, D, tol, max_len, tuning=tuning, znorm=znorm)
    T.cuda.synchronize()
    st = J.workspace_status(p.workspace)
    ln, inc, po = p.host()
    if znorm:
        ns = len(series_off) - 1
        return ln, inc, po, st, p.mean[:ns].cpu().numpy(), p.std[:ns].cpu().numpy()
    return ln, inc, po, st


def gpu_digitize(ln, inc, alpha, scl=1.0, B=4096, capacity=None, tuning=None, max_pieces=None, key="norm"):
    import paper_2401_00109_amd as J
    T = torch()
    n = int(np.asarray(ln).size)
    mp = max(n, 1) if max_pieces is None else max_pieces
    L = T.zeros(mp, dtype=T.int32, device=DEV)
    I = T.zeros(mp, dtype=T.float64, device=DEV)
    if n:
        L[:n] = to_dev(np.asarray(ln, np.int32))
        I[:n] = to_dev(np.asarray(inc, np.float64))
    npc = T.tensor([n], dtype=T.int64, device=DEV)
    sym, d, ws = J.digitize(L, I, npc, mp, alpha, scl, B, capacity=capacity, tuning=tuning, key=key)
    T.cuda.synchronize()
    st = J.workspace_status(ws)
    h = d.host()
    if key == "pca":
        h["axis"] = d.axis.cpu().numpy()
    h["stats"] = J.api.digitize_stats(ws, mp, B)
    return sym[:n].cpu().numpy(), h, st


def assert_centers_close(got, ora, inc, symbols, rel=1e-12):
    """center_inc / cy: within rel of max(|exact mean|, mean |inc| of the members)."""
    k = ora.k
    cnt = np.bincount(symbols, minlength=k).astype(np.float64)
    absmean = np.bincount(symbols, weights=np.abs(inc), minlength=k) / np.maximum(cnt, 1)
    scale = np.maximum(np.abs(ora.center_inc), absmean)
    err = np.abs(got["center_inc"] - ora.center_inc)
    assert np.all(err <= rel * scale), f"center_inc max rel err {np.max(err / np.maximum(scale, 1e-300))}"
    scale_y = scale / ora.sigma_inc
    erry = np.abs(got["cy"] - ora.cy)
    assert np.all(erry <= rel * scale_y * (1 + 1e-15) + 1e-300)
    return float(np.max(err / np.maximum(scale, 1e-300))) if k else 0.0
