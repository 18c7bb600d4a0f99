"""Serving loop: continuous batching of symbolization requests against a
dictionary kept resident on the device.

A request is a batch of series.  The loop admits a request as soon as it has
arrived, a slot is free and the slot arena can hold it.  Each admitted request
gets its own HIP stream (default priority) and runs the pinned host-to-device
copy, compression (Phase II), nearest-center encoding against the resident
dictionary, and the device-to-host copy of its symbols.  Requests that arrive
while others are on the GPU therefore overlap on the device.  Latency is
arrival time -> symbols on the host; points/s counts the input points served.

    python -m paper_2401_00109_amd.serve --requests 300 --rates 0.25,0.5,0.9
"""
from __future__ import annotations

import argparse
import json
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    points: int
    pieces: int
    symbols: np.ndarray = field(repr=False)
    piece_off: np.ndarray = field(repr=False)


class Slot:
    """Device buffers, pinned staging and a stream for one in-flight request."""

    def __init__(self, dictionary: api.Dictionary, max_series: int, max_points: int, D: int, device):
        self.max_series, self.max_points = max_series, max_points
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.h_values = torch.empty(max_points, dtype=torch.float64, pin_memory=True)
        self.h_off = torch.empty(max_series + 1, dtype=torch.int64, pin_memory=True)
        self.h_sym = torch.empty(max_points, dtype=torch.int32, pin_memory=True)
        self.h_npc = torch.empty(1, dtype=torch.int64, pin_memory=True)
        self.h_poff = torch.empty(max_series + 1, dtype=torch.int64, pin_memory=True)
        self.values = torch.empty(max_points, dtype=torch.float64, device=device)
        self.series_off = torch.empty(max_series + 1, dtype=torch.int64, device=device)
        self.pieces = api.Pieces(torch.empty(max_points, dtype=torch.int32, device=device),
                                 torch.empty(max_points, dtype=torch.float64, device=device),
                                 torch.empty(max_series + 1, dtype=torch.int64, device=device),
                                 torch.empty(1, dtype=torch.int64, device=device), max_points)
        self.symbols = torch.empty(max_points, dtype=torch.int32, device=device)
        self.enc_ws = api._ws(api.encode_workspace_bytes(dictionary.capacity), device)
        self.cws = {}
        self.done_ev = torch.cuda.Event()
        self.req = None

    def bytes(self) -> int:
        return int(self.values.numel() * 8 + self.pieces.len.numel() * 12 + self.symbols.numel() * 4)


class Server:
    def __init__(self, dictionary: api.Dictionary, D: int = 2000, tol: float = 0.05, max_len: int = 0,
                 slots: int = 4, max_series: int = 256, max_points: int = 256 * 50_000,
                 arena_bytes: int | None = None, tuning: dict | None = None, device=None):
        self.dev = torch.device("cuda", 0) if device is None else torch.device(device)
        self.dict, self.D, self.tol, self.max_len, self.tuning = dictionary, D, tol, max_len, tuning
        self.slots = [Slot(dictionary, max_series, max_points, D, self.dev) for _ in range(slots)]
        # arena: memory the in-flight requests may hold; a request needs ~ its points x 24 B
        self.arena = arena_bytes if arena_bytes is not None else slots * max_points * 24
        self.in_use = 0
        self.peak_in_flight = 0  # most requests on the device at once during the last run()

    @staticmethod
    def need(points: int) -> int:
        return int(points) * 24

    def _workspace(self, slot: Slot, n_series: int, total: int) -> torch.Tensor:
        nb = api.compress_workspace_bytes(n_series, total, self.D)
        ws = slot.cws.get("ws")
        if ws is None or ws.numel() < nb:
            ws = api._ws(max(nb, 1 << 20), self.dev)
            slot.cws["ws"] = ws
        return ws

    def _launch(self, slot: Slot, req) -> None:
        n = req.values.size
        ns = req.series_off.size - 1
        slot.h_values[:n].numpy()[:] = req.values
        slot.h_off[: ns + 1].numpy()[:] = req.series_off
        ws = self._workspace(slot, ns, n)
        with torch.cuda.stream(slot.stream):
            v = slot.values[:n]
            so = slot.series_off[: ns + 1]
            v.copy_(slot.h_values[:n], non_blocking=True)
            so.copy_(slot.h_off[: ns + 1], non_blocking=True)
            p = slot.pieces
            po = p.piece_off[: ns + 1]
            view = api.Pieces(p.len, p.inc, po, p.n_pieces, p.max_pieces)
            api.compress(v, so, self.D, self.tol, self.max_len, self.tuning, out=view, workspace=ws,
                         stream=slot.stream)
            api.encode(p.len, p.inc, p.n_pieces, n, self.dict, symbols=slot.symbols, workspace=slot.enc_ws,
                       stream=slot.stream)
            slot.h_npc.copy_(p.n_pieces, non_blocking=True)
            slot.h_poff[: ns + 1].copy_(po, non_blocking=True)
            slot.h_sym[:n].copy_(slot.symbols[:n], non_blocking=True)
            slot.done_ev.record(slot.stream)

    def run(self, requests, realtime: bool = True) -> list[Result]:
        """Serve `requests` (inputs.Request, arrival offsets in seconds from now)."""
        pending = sorted(requests, key=lambda r: r.arrival_s)
        waiting, out = [], []
        self.peak_in_flight = 0
        t0 = time.perf_counter()
        i = 0
        while i < len(pending) or waiting or any(s.req is not None for s in self.slots):
            now = time.perf_counter() - t0
            while i < len(pending) and (not realtime or pending[i].arrival_s <= now):
                waiting.append(pending[i])
                i += 1
            # completions
            for s in self.slots:
                if s.req is not None and s.done_ev.query():
                    r, adm = s.req
                    n = r.values.size
                    ns = r.series_off.size - 1
                    npc = int(s.h_npc[0])
                    out.append(Result(r.rid, r.arrival_s, adm, time.perf_counter() - t0, n, npc,
                                      s.h_sym[:npc].numpy().copy(), s.h_poff[: ns + 1].numpy().copy()))
                    self.in_use -= self.need(n)
                    s.req = None
            # admissions: first come first served while a slot and arena memory are free
            while waiting:
                r = waiting[0]
                free = [s for s in self.slots if s.req is None]
                if not free or self.in_use + self.need(r.values.size) > self.arena:
                    break
                if r.values.size > free[0].max_points or r.series_off.size - 1 > free[0].max_series:
                    raise ValueError(f"request {r.rid} exceeds the slot size")
                waiting.pop(0)
                s = free[0]
                self.in_use += self.need(r.values.size)
                s.req = (r, time.perf_counter() - t0)
                self._launch(s, r)
                self.peak_in_flight = max(self.peak_in_flight, sum(1 for q in self.slots if q.req is not None))
            if i < len(pending) and not waiting and all(s.req is None for s in self.slots):
                # idle until the next arrival
                dt = pending[i].arrival_s - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(min(dt, 0.001))
        return sorted(out, key=lambda r: r.rid)


def summarize(res: list[Result], wall: float) -> dict:
    lat = np.array([r.done - r.arrival for r in res]) * 1e3
    pts = sum(r.points for r in res)
    return {"requests": len(res), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "points_per_s": pts / wall if wall > 0 else 0.0, "points": pts}


def build_resident_dictionary(device) -> api.Dictionary:
    """The 16 x 1,000 random-walk workload's dictionary (tol = alpha = 0.1)."""
    from .inputs import make_workload
    w = make_workload(1, 0)
    sz = api.Symbolizer(w.n_series, w.n_points, w.D, w.tol, w.alpha, w.scl, w.B, device=device)
    sz.run(torch.from_numpy(w.values).to(device), torch.from_numpy(w.series_off).to(device))
    torch.cuda.synchronize()
    k = sz.dictionary.size()
    h = sz.dictionary.host()
    return api.Dictionary.from_host(h["sigma_len"], h["sigma_inc"], h["scl"], h["alpha"], h["center_len"],
                                    h["center_inc"], h["cx"], h["cy"], h["count"], device) if k else sz.dictionary


def main() -> int:
    from .inputs import request_stream
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--rates", default="0.25,0.5,0.9", help="fractions of the closed-loop saturation rate")
    ap.add_argument("--max-series", type=int, default=256)
    ap.add_argument("--tuning", default=None, help="JSON dict of jabba_tuning fields for the compression")
    a = ap.parse_args()
    dev = torch.device("cuda", 0)
    d = build_resident_dictionary(dev)
    srv = Server(d, slots=a.slots, max_series=a.max_series, tuning=json.loads(a.tuning) if a.tuning else None,
                 device=dev)
    # closed loop (everything queued at t=0) -> saturation rate
    warm = request_stream(1, a.warmup, 0.0, max_series=a.max_series, first_id=10_000_000)
    srv.run(warm, realtime=False)
    closed = request_stream(2, a.requests, 0.0, max_series=a.max_series, first_id=20_000_000)
    t = time.perf_counter()
    res = srv.run(closed, realtime=False)
    wall = time.perf_counter() - t
    sat = len(res) / wall
    report = {"dictionary_k": d.size(), "slots": a.slots, "saturation_req_per_s": sat,
              "closed_loop": summarize(res, wall), "rates": []}
    for f in [float(x) for x in a.rates.split(",")]:
        reqs = request_stream(3, a.requests, f * sat, max_series=a.max_series, first_id=30_000_000)
        t = time.perf_counter()
        res = srv.run(reqs, realtime=True)
        wall = time.perf_counter() - t
        s = summarize(res, wall)
        s["rate_req_per_s"] = f * sat
        s["fraction_of_saturation"] = f
        report["rates"].append(s)
    print(json.dumps(report))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
