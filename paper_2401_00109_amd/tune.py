"""Autotuner for the launch shapes of the batched path.

Searches lanes per domain, wavefronts per workgroup and persistent
workgroups per compute unit for the compression kernel, and wavefronts per
workgroup for Stage I of digitization.  A variant counts only if its output
is bit-identical to the default launch's (lengths, increments, offsets,
symbols); the knobs never change results, and the tuner checks that they did
not.  The winner is cached per device and workload shape in a JSON file.

    python -m paper_2401_00109_amd.tune --workload uneven --scale 0.1
"""
from __future__ import annotations

import argparse
import json
import os
import time

import torch

from . import api

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "jabba", "tuning.json")

COMPRESS_SPACE = [
    {"lanes_per_domain": w, "waves_per_block": wpb, "blocks_per_cu": bpc, "segment_intervals": g}
    for w in (1, 2, 4, 8, 16)
    for wpb in (1, 2, 4)
    for bpc in (2, 4, 8, 16)
    for g in (-1, 64, 128, 256)
]
STAGE1_SPACE = [1, 2, 4]  # larger values are clamped to 4 by the library


def shape_key(device, n_series: int, total_points: int, D: int) -> str:
    name = torch.cuda.get_device_name(device)
    bucket = 1 << max(int(total_points).bit_length() - 1, 0)
    return f"{name}|series~{1 << max(n_series.bit_length() - 1, 0)}|points~{bucket}|D={D}"


def _time(fn, reps: int) -> float:
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        ts.append(s.elapsed_time(e))
    ts.sort()
    return ts[len(ts) // 2]


def tune(values: torch.Tensor, series_off: torch.Tensor, D: int, tol: float, alpha: float, scl: float = 1.0,
         B: int = 4096, max_len: int = 0, reps: int = 3, compress_space=None, stage1_space=None,
         cache_path: str | None = CACHE, log=print) -> dict:
    """Returns the fastest output-preserving tuning (a jabba_tuning field dict)."""
    dev = values.device
    ns, total = series_off.numel() - 1, values.numel()
    key = shape_key(dev, ns, total, D)
    ws = api._ws(api.compress_workspace_bytes(ns, total, D), dev)

    def new_pieces():
        return api.Pieces(torch.empty(max(total, 1), dtype=torch.int32, device=dev),
                          torch.empty(max(total, 1), dtype=torch.float64, device=dev),
                          torch.empty(ns + 1, dtype=torch.int64, device=dev),
                          torch.empty(1, dtype=torch.int64, device=dev), max(total, 1))

    ref = api.compress(values, series_off, D, tol, max_len, out=new_pieces(), workspace=ws)
    torch.cuda.synchronize()
    N = ref.count()
    results = []
    trial = new_pieces()
    for t in (compress_space or COMPRESS_SPACE):
        def run(t=t):
            api.compress(values, series_off, D, tol, max_len, tuning=t, out=trial, workspace=ws)
        ms = _time(run, reps)
        same = (torch.equal(trial.n_pieces, ref.n_pieces) and torch.equal(trial.len[:N], ref.len[:N])
                and torch.equal(trial.inc[:N].view(torch.int64), ref.inc[:N].view(torch.int64))
                and torch.equal(trial.piece_off, ref.piece_off))
        results.append((ms, same, t))
        log(f"[tune] compress {t} {ms:.3f} ms {'ok' if same else 'DIFFERENT OUTPUT - rejected'}")
    ok = [r for r in results if r[1]]
    best_c = min(ok, key=lambda r: r[0])[2]

    # Stage I wavefronts per workgroup, digitize outputs compared bit for bit
    dws = api._ws(api.digitize_workspace_bytes(max(N, 1), B), dev)
    sym_ref, d_ref, _ = api.digitize(ref.len, ref.inc, ref.n_pieces, max(N, 1), alpha, scl, B, workspace=dws)
    torch.cuda.synchronize()
    sym_ref = sym_ref[:N].clone()
    best_s, best_ms = None, float("inf")
    sym = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
    d = api.Dictionary(max(N, 1), dev)
    for s1 in (stage1_space or STAGE1_SPACE):
        def run(s1=s1):
            api.digitize(ref.len, ref.inc, ref.n_pieces, max(N, 1), alpha, scl, B, tuning={"stage1_waves": s1},
                         symbols=sym, dictionary=d, workspace=dws)
        ms = _time(run, reps)
        same = torch.equal(sym[:N], sym_ref)
        log(f"[tune] stage1_waves={s1} {ms:.3f} ms {'ok' if same else 'DIFFERENT OUTPUT - rejected'}")
        if same and ms < best_ms:
            best_s, best_ms = s1, ms
    best = dict(best_c)
    if best_s is not None:
        best["stage1_waves"] = best_s
    if cache_path:
        save(cache_path, key, best)
    return best


def save(path: str, key: str, tuning: dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    data = {}
    if os.path.exists(path):
        try:
            data = json.load(open(path))
        except (OSError, ValueError):
            data = {}
    data[key] = {"tuning": tuning, "time": time.time()}
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(device, n_series: int, total_points: int, D: int, path: str = CACHE) -> dict | None:
    """Cached tuning for this device and shape, or None."""
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = data.get(shape_key(device, n_series, total_points, D))
    return None if e is None else e.get("tuning")


def main() -> int:
    from .inputs import make_workload
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--scale", type=float, default=0.1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=CACHE)
    a = ap.parse_args()
    w = make_workload(a.workload, 0, a.scale)
    dev = torch.device("cuda", 0)
    v = torch.from_numpy(w.values).to(dev)
    so = torch.from_numpy(w.series_off).to(dev)
    best = tune(v, so, w.D, w.tol, w.alpha, w.scl, w.B, reps=a.reps, cache_path=a.cache)
    print(json.dumps({"workload": w.name, "points": w.n_points, "best": best}))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
