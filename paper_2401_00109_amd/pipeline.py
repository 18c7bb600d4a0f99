"""Batches in flight: the full step (compress, encode against a resident
dictionary, digitize, reconstruct) driven from several streams at once.

Each buffer set holds its own pieces, symbols, dictionary, encodings,
reconstruction and scratch, and runs every step it is given on its own
stream (default priority).  Consecutive steps go to consecutive sets, so one
batch's compression (FP64-issue bound, a few wavefronts per compute unit)
overlaps the other batches' sort, gathers and reconstruction.  Every step
does all of its work; sets share only the read-only inputs and the resident
dictionary.

The sets are bound to one input batch held in device memory (values,
series_off, t0), as in a throughput measurement or a replay of a resident
batch.  Writing new inputs into those buffers while steps are in flight
would race; a loop that admits new batches is serve.py's.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import api


@dataclass
class BufferSet:
    sz: api.Symbolizer
    pieces: api.Pieces
    enc: torch.Tensor
    rec: api.Reconstructor
    stream: torch.cuda.Stream
    encode_ws: torch.Tensor
    steps: int = field(default=0)


class Pipeline:
    """n_sets buffer sets over one resident input batch.

    values, series_off, t0: the batch on the device.  max_pieces: the
    digitize capacity (the batch's piece count, e.g. from one compress);
    compression itself gets the worst-case capacity sum(n_s - 1).  resident:
    the dictionary the encode step uses.  The constructor compresses and
    digitizes the batch once on each set (current stream) and runs the
    reconstruction's size pass, which synchronises, to allocate its output.
    The sets all hold the same batch, so the first set's symbol count sizes
    the dictionaries of the others."""

    def __init__(self, values: torch.Tensor, series_off: torch.Tensor, t0: torch.Tensor, D: int, tol: float,
                 alpha: float, scl: float, B: int, max_pieces: int, resident: api.Dictionary, n_sets: int = 3,
                 tuning=None, max_len: int = 0):
        if n_sets < 1:
            raise ValueError("n_sets must be >= 1")
        self.values, self.series_off, self.t0 = values, series_off, t0
        self.resident = resident
        self.max_pieces = max(int(max_pieces), 1)
        dev = values.device
        n_series = series_off.numel() - 1
        n_points = values.numel()
        cap = max(n_points, 1)
        self.sets: list[BufferSet] = []
        capacity = self.max_pieces
        for i in range(n_sets):
            sz = api.Symbolizer(n_series, n_points, D, tol, alpha, scl, B, max_len=max_len,
                                max_pieces=self.max_pieces, capacity=capacity, tuning=tuning, device=dev)
            full = api.Pieces(torch.empty(cap, dtype=torch.int32, device=dev),
                              torch.empty(cap, dtype=torch.float64, device=dev),
                              sz.pieces.piece_off, sz.pieces.n_pieces, cap)
            sz.pieces = full
            rec = api.Reconstructor(full.piece_off, series_off, t0, values)
            sz.compress(values, series_off)
            sz.digitize()
            rec.size(sz.symbols, sz.dictionary)
            self.sets.append(BufferSet(sz, full, torch.empty(self.max_pieces, dtype=torch.int32, device=dev), rec,
                                       torch.cuda.Stream(device=dev),
                                       api._ws(api.encode_workspace_bytes(resident.capacity), dev)))
            # every set digitizes the same batch: the first set's symbol count
            # sizes the other sets' dictionaries
            capacity = max(sz.dictionary.size(), 1)

    def step(self, S: BufferSet):
        """Enqueue one full step on set S's stream."""
        st = S.stream
        S.sz.compress(self.values, self.series_off, stream=st)
        api.encode(S.pieces.len, S.pieces.inc, S.pieces.n_pieces, self.max_pieces, self.resident, symbols=S.enc,
                   workspace=S.encode_ws, stream=st)
        S.sz.digitize(stream=st)
        S.rec.run(S.sz.symbols, S.sz.dictionary, stream=st)
        S.steps += 1

    def run(self, n_steps: int, pipelined: bool = True):
        """Enqueue n_steps steps: round robin over the sets, or all on the
        first set when pipelined is False (one batch at a time).  The sets'
        streams wait for the work already on the current stream, and the
        current stream waits for the steps, so callers can time the call with
        events on the current stream."""
        cur = torch.cuda.current_stream()
        ev = torch.cuda.Event()
        ev.record(cur)
        for S in self.sets:
            S.stream.wait_event(ev)
        for i in range(n_steps):
            self.step(self.sets[i % len(self.sets)] if pipelined else self.sets[0])
        for S in self.sets:
            e = torch.cuda.Event()
            e.record(S.stream)
            cur.wait_event(e)
