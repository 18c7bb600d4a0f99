"""Batches in flight: the full step (compress, encode against a resident
dictionary, digitize, reconstruct) driven from several streams at once.

Each buffer set holds its own pieces, symbols, dictionary, encodings,
reconstruction and scratch, and runs every step it is given on its own
stream (default priority).  Consecutive steps go to consecutive sets, so one
batch's compression (FP64-issue bound, a few wavefronts per compute unit)
overlaps the other batches' sort, gathers and reconstruction.  Inside a
step, the encoding needs only the compression's pieces, so it runs on a side
stream shared by the sets while the set's own stream digitizes and
reconstructs; the set's stream waits for it before its next step (whose
compression rewrites the pieces).  Every step does all of its work; sets
share only the read-only inputs and the resident dictionary.

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
    compressed: torch.cuda.Event = field(default_factory=torch.cuda.Event)
    encoded: torch.cuda.Event = field(default_factory=torch.cuda.Event)
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
        self.side = torch.cuda.Stream(device=dev)  # the sets' encodes
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

    def step(self, S: BufferSet, overlap: bool = True):
        """Enqueue one full step on set S's stream (the encoding on the side
        stream when overlap is True)."""
        st = S.stream
        S.sz.compress(self.values, self.series_off, stream=st)
        est = st
        if overlap:
            S.compressed.record(st)
            self.side.wait_event(S.compressed)
            est = self.side
        api.encode(S.pieces.len, S.pieces.inc, S.pieces.n_pieces, self.max_pieces, self.resident, symbols=S.enc,
                   workspace=S.encode_ws, stream=est)
        if overlap:
            S.encoded.record(self.side)
        S.sz.digitize(stream=st)
        S.rec.run(S.sz.symbols, S.sz.dictionary, stream=st)
        if overlap:
            st.wait_event(S.encoded)
        S.steps += 1

    def run(self, n_steps: int, pipelined: bool = True, overlap: bool = True):
        """Enqueue n_steps steps: round robin over the sets, or all on the
        first set when pipelined is False (one batch at a time); overlap
        False keeps each step's encoding on its set's stream (every kernel
        then runs on its own, for per-kernel timing).  The sets' streams and
        the side stream wait for the work already on the current stream, and
        the current stream waits for the steps, so callers can time the call
        with events on the current stream."""
        cur = torch.cuda.current_stream()
        ev = torch.cuda.Event()
        ev.record(cur)
        for S in self.sets:
            S.stream.wait_event(ev)
        self.side.wait_event(ev)
        for i in range(n_steps):
            self.step(self.sets[i % len(self.sets)] if pipelined else self.sets[0], overlap=overlap)
        for S in self.sets:
            e = torch.cuda.Event()
            e.record(S.stream)
            cur.wait_event(e)
