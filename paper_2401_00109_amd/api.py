"""Python face of libjabba: compress / digitize / encode / reconstruct.

Thin marshalling over the C ABI (include/jabba.h).  PyTorch is used only to
hold device memory and to supply the current HIP stream; every step of the
path runs in the library's HIP kernels.  There is no CPU fallback: on a
machine without the built library or without a GPU these calls raise.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

__all__ = [
    "Pieces", "Dictionary", "compress", "compress_plain", "digitize", "encode", "encode_noalloc", "reconstruct",
    "reconstruct_pieces", "reconstruction_mse", "workspace_status", "Plan", "tuning_struct", "Symbolizer", "Reconstructor",
    "timing_enable", "timing_report", "digitize_stats", "digitize_quality", "kmeans", "axis_tolerances",
    "aggregate_points",
]


def _dev(device=None) -> torch.device:
    if device is None:
        device = torch.device("cuda", torch.cuda.current_device())
    return torch.device(device)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def tuning_struct(tuning: dict | None):
    if not tuning:
        return None
    t = L.Tuning()
    for k, v in tuning.items():
        setattr(t, k, int(v))
    return t


def _tref(t):
    return C.byref(t) if t is not None else None


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _as(t, dtype, device):
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    t = t.to(device=device, dtype=dtype)
    return t.contiguous()


def compress_workspace_bytes(n_series: int, total_points: int, D: int) -> int:
    n = C.c_size_t()
    L.check(L.lib().jabba_compress_workspace(n_series, total_points, D, C.byref(n)), "compress_workspace")
    return n.value


def digitize_workspace_bytes(max_pieces: int, B: int) -> int:
    n = C.c_size_t()
    L.check(L.lib().jabba_digitize_workspace(max_pieces, B, C.byref(n)), "digitize_workspace")
    return n.value


def recon_workspace_bytes(n_series: int) -> int:
    n = C.c_size_t()
    L.check(L.lib().jabba_reconstruct_workspace(n_series, C.byref(n)), "reconstruct_workspace")
    return n.value


@dataclass
class Pieces:
    """Compressed pieces on the device (capacity max_pieces, live count in n_pieces)."""
    len: torch.Tensor        # int32[max_pieces]
    inc: torch.Tensor        # float64[max_pieces]
    piece_off: torch.Tensor  # int64[n_series + 1]
    n_pieces: torch.Tensor   # int64[1]
    max_pieces: int
    workspace: torch.Tensor | None = None
    mean: torch.Tensor | None = None         # float64[n_series], z-normalised compression only
    std: torch.Tensor | None = None

    def count(self) -> int:
        return int(self.n_pieces.item())

    def host(self):
        n = self.count()
        return (self.len[:n].cpu().numpy(), self.inc[:n].cpu().numpy(), self.piece_off.cpu().numpy())


class Dictionary:
    """Symbolic centers (jabba_dict) in caller-owned device memory."""

    def __init__(self, capacity: int, device=None):
        dev = _dev(device)
        cap = max(int(capacity), 1)
        self.capacity = cap
        self.params = torch.zeros(4, dtype=torch.float64, device=dev)
        self.k = torch.zeros(1, dtype=torch.int64, device=dev)
        self.center_len = torch.zeros(cap, dtype=torch.float64, device=dev)
        self.center_inc = torch.zeros(cap, dtype=torch.float64, device=dev)
        self.cx = torch.zeros(cap, dtype=torch.float64, device=dev)
        self.cy = torch.zeros(cap, dtype=torch.float64, device=dev)
        self.count = torch.zeros(cap, dtype=torch.int64, device=dev)

    def struct(self) -> L.Dict:
        return L.Dict(self.capacity, self.params.data_ptr(), self.k.data_ptr(), self.center_len.data_ptr(),
                      self.center_inc.data_ptr(), self.cx.data_ptr(), self.cy.data_ptr(), self.count.data_ptr())

    def size(self) -> int:
        return int(self.k.item())

    def encode_workspace(self) -> torch.Tensor:
        """Scratch the encoder orders the centers in (allocated once per dictionary)."""
        if getattr(self, "_enc_ws", None) is None:
            self._enc_ws = _ws(encode_workspace_bytes(self.capacity), self.params.device)
        return self._enc_ws

    def host(self) -> dict:
        k = min(self.size(), self.capacity)
        p = self.params.cpu().numpy()
        return {"k": self.size(), "sigma_len": float(p[0]), "sigma_inc": float(p[1]), "scl": float(p[2]),
                "alpha": float(p[3]), "center_len": self.center_len[:k].cpu().numpy(),
                "center_inc": self.center_inc[:k].cpu().numpy(), "cx": self.cx[:k].cpu().numpy(),
                "cy": self.cy[:k].cpu().numpy(), "count": self.count[:k].cpu().numpy()}

    @classmethod
    def from_host(cls, sigma_len, sigma_inc, scl, alpha, center_len, center_inc, cx, cy, count=None, device=None):
        """Upload a dictionary (for example a saved one) to the device."""
        k = len(center_len)
        d = cls(max(k, 1), device)
        dev = d.params.device
        d.params.copy_(torch.tensor([sigma_len, sigma_inc, scl, alpha], dtype=torch.float64))
        d.k.fill_(k)
        if k:
            d.center_len[:k].copy_(_as(center_len, torch.float64, dev))
            d.center_inc[:k].copy_(_as(center_inc, torch.float64, dev))
            d.cx[:k].copy_(_as(cx, torch.float64, dev))
            d.cy[:k].copy_(_as(cy, torch.float64, dev))
            if count is not None:
                d.count[:k].copy_(_as(count, torch.int64, dev))
        return d

    def save(self, path: str) -> None:
        h = self.host()
        np.savez(path, **{k: np.asarray(v) for k, v in h.items()})

    @classmethod
    def load(cls, path: str, device=None):
        z = np.load(path, allow_pickle=False)
        return cls.from_host(float(z["sigma_len"]), float(z["sigma_inc"]), float(z["scl"]), float(z["alpha"]),
                             z["center_len"], z["center_inc"], z["cx"], z["cy"], z["count"], device)


def digitize_stats(workspace: torch.Tensor, max_pieces: int, B: int, stream=None) -> dict:
    """N, G (Stage I starting points), k, active radix passes, Stage II groups, the bytes per piece
    the radix passes moved and the pieces of oversized prefix groups, for the last digitize on this workspace."""
    arr = (C.c_int64 * 7)()
    L.check(L.lib().jabba_digitize_stats(_p(workspace), int(max_pieces), int(B), _stream(stream), arr),
            "jabba_digitize_stats")
    return {"N": arr[0], "G": arr[1], "k": arr[2], "sort_passes": arr[3], "stage2_groups": arr[4],
            "sort_bytes": arr[5], "sort_large": arr[6]}


def workspace_status(ws: torch.Tensor, stream=None) -> int:
    st = C.c_int32()
    L.check(L.lib().jabba_workspace_status(_p(ws), _stream(stream), C.byref(st)), "workspace_status")
    return st.value


def compress(values: torch.Tensor, series_off: torch.Tensor, D: int, tol: float, max_len: int = 0,
             tuning: dict | None = None, max_pieces: int | None = None, out: Pieces | None = None,
             workspace: torch.Tensor | None = None, stream=None, znorm: bool = False) -> Pieces:
    """Phase I + II of Alg. 1 on the device (see jabba_compress).

    znorm=True compresses the z-normalised series (jabba_compress_znorm); the per-series mean and deviation
    are kept as ``out.mean`` and ``out.std``."""
    dev = values.device
    n_series = series_off.numel() - 1
    total = values.numel()
    cap = int(max_pieces) if max_pieces is not None else max(total, 1)
    if out is None:
        out = Pieces(torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                     torch.empty(max(cap, 1), dtype=torch.float64, device=dev),
                     torch.empty(n_series + 1, dtype=torch.int64, device=dev),
                     torch.empty(1, dtype=torch.int64, device=dev), cap)
    if workspace is None:
        workspace = _ws(compress_workspace_bytes(n_series, total, D), dev)
    out.workspace = workspace
    t = tuning_struct(tuning)
    if znorm:
        out.mean = torch.empty(max(n_series, 1), dtype=torch.float64, device=dev)
        out.std = torch.empty(max(n_series, 1), dtype=torch.float64, device=dev)
        rc = L.lib().jabba_compress_znorm(_p(values), _p(series_off), n_series, total, int(D), float(tol),
                                          int(max_len), _tref(t), _p(out.len), _p(out.inc), _p(out.piece_off),
                                          _p(out.n_pieces), _p(out.mean), _p(out.std), _p(workspace),
                                          workspace.numel(), _stream(stream))
        L.check(rc, "jabba_compress_znorm")
        return out
    rc = L.lib().jabba_compress(_p(values), _p(series_off), n_series, total, int(D), float(tol), int(max_len),
                                _tref(t), _p(out.len), _p(out.inc), _p(out.piece_off), _p(out.n_pieces),
                                _p(workspace), workspace.numel(), _stream(stream))
    L.check(rc, "jabba_compress")
    return out


def compress_plain(values: torch.Tensor, series_off: torch.Tensor, series_off_host: np.ndarray, D: int, tol: float,
                   max_len: int = 0, out: Pieces | None = None, workspace: torch.Tensor | None = None,
                   stream=None) -> Pieces:
    """One launch per series (the per-domain-launch baseline); same outputs as compress."""
    dev = values.device
    so_h = np.ascontiguousarray(series_off_host, dtype=np.int64)
    n_series = so_h.size - 1
    total = int(so_h[-1]) if so_h.size else 0
    cap = max(total, 1)
    if out is None:
        out = Pieces(torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.float64, device=dev),
                     torch.empty(n_series + 1, dtype=torch.int64, device=dev),
                     torch.empty(1, dtype=torch.int64, device=dev), cap)
    if workspace is None:
        workspace = _ws(compress_workspace_bytes(n_series, total, D), dev)
    out.workspace = workspace
    rc = L.lib().jabba_compress_plain(_p(values), _p(series_off), so_h.ctypes.data_as(C.c_void_p), n_series, int(D),
                                      float(tol), int(max_len), _p(out.len), _p(out.inc), _p(out.piece_off),
                                      _p(out.n_pieces), _p(workspace), workspace.numel(), _stream(stream))
    L.check(rc, "jabba_compress_plain")
    return out


def digitize(length: torch.Tensor, inc: torch.Tensor, n_pieces: torch.Tensor, max_pieces: int, alpha: float,
             scl: float = 1.0, B: int = 4096, capacity: int | None = None, tuning: dict | None = None,
             symbols: torch.Tensor | None = None, dictionary: Dictionary | None = None,
             workspace: torch.Tensor | None = None, stream=None, key: str = "norm", axis: torch.Tensor | None = None):
    """Phase III of Alg. 1 (two-stage digitization).  Returns (symbols, Dictionary, workspace).

    key "norm" sorts by sqrt(x^2 + y^2) (jabba_digitize); "pca" by the projection on the principal axis
    (jabba_digitize_pca), which is written to `axis` (2 float64 on the device, allocated when None) and kept as
    ``dictionary.axis``."""
    if key not in ("norm", "pca"):
        raise ValueError(f"key must be 'norm' or 'pca', not {key!r}")
    dev = length.device
    if symbols is None:
        symbols = torch.empty(max(max_pieces, 1), dtype=torch.int32, device=dev)
    if dictionary is None:
        dictionary = Dictionary(capacity if capacity is not None else max(max_pieces, 1), dev)
    if workspace is None:
        workspace = _ws(digitize_workspace_bytes(max_pieces, B), dev)
    d = dictionary.struct()
    t = tuning_struct(tuning)
    if key == "pca":
        if axis is None:
            axis = torch.zeros(2, dtype=torch.float64, device=dev)
        rc = L.lib().jabba_digitize_pca(_p(length), _p(inc), _p(n_pieces), int(max_pieces), float(alpha), float(scl),
                                        int(B), _tref(t), _p(symbols), C.byref(d), _p(axis), _p(workspace),
                                        workspace.numel(), _stream(stream))
        L.check(rc, "jabba_digitize_pca")
        dictionary.axis = axis
        return symbols, dictionary, workspace
    rc = L.lib().jabba_digitize(_p(length), _p(inc), _p(n_pieces), int(max_pieces), float(alpha), float(scl), int(B),
                                _tref(t), _p(symbols), C.byref(d), _p(workspace), workspace.numel(), _stream(stream))
    L.check(rc, "jabba_digitize")
    return symbols, dictionary, workspace


def aggregate_points(x: torch.Tensor, y: torch.Tensor, alpha: float, B: int | None = None,
                     n_points: torch.Tensor | None = None, capacity: int | None = None, workspace=None,
                     stream=None) -> dict:
    """Two-stage aggregation of raw 2-D points (jabba_aggregate_points); B=None is one block (the serial
    greedy).  Returns device tensors labels, cx, cy, count (capacity entries), k (1) and sse (1), and the
    workspace; enqueued on the stream, no synchronisation."""
    dev = x.device
    n = x.numel()
    if y.numel() != n or x.dtype != torch.float64 or y.dtype != torch.float64:
        raise ValueError("x and y: float64 tensors of one size")
    B = max(n, 1) if B is None else int(B)
    cap = max(n, 1) if capacity is None else int(capacity)
    if n_points is None:
        n_points = torch.tensor([n], dtype=torch.int64, device=dev)
    if workspace is None:
        workspace = _ws(digitize_workspace_bytes(n, B), dev)
    labels = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    cx = torch.zeros(max(cap, 1), dtype=torch.float64, device=dev)
    cy = torch.zeros(max(cap, 1), dtype=torch.float64, device=dev)
    count = torch.zeros(max(cap, 1), dtype=torch.int64, device=dev)
    k = torch.zeros(1, dtype=torch.int64, device=dev)
    sse = torch.zeros(1, dtype=torch.float64, device=dev)
    rc = L.lib().jabba_aggregate_points(_p(x), _p(y), _p(n_points), int(n), float(alpha), int(B), _p(labels), cap,
                                        _p(cx), _p(cy), _p(count), _p(k), _p(sse), _p(workspace), workspace.numel(),
                                        _stream(stream))
    L.check(rc, "jabba_aggregate_points")
    return {"labels": labels[:n], "cx": cx, "cy": cy, "count": count, "k": k, "sse": sse, "workspace": workspace}


def axis_tolerances(alpha_len: float, alpha_inc: float, scl: float = 1.0) -> tuple[float, float]:
    """(alpha, scl) for digitize that run the aggregation with separate length and increment tolerances
    (jabba_axis_tolerances, Sec. 3.2 Eq. Var1)."""
    a, s_ = C.c_double(), C.c_double()
    L.check(L.lib().jabba_axis_tolerances(float(alpha_len), float(alpha_inc), float(scl), C.byref(a), C.byref(s_)),
            "jabba_axis_tolerances")
    return a.value, s_.value


def digitize_quality(length: torch.Tensor, inc: torch.Tensor, n_pieces: torch.Tensor, max_pieces: int, alpha: float,
                     B: int, dictionary: Dictionary, workspace: torch.Tensor, stream=None) -> dict:
    """Per-symbol variances and the SSE of the digitization in `workspace` (see jabba_digitize_quality).

    Returns device tensors var_len, var_inc (dictionary capacity entries) and totals = [SSE, max var_len,
    max var_inc]; enqueued on the stream, no synchronisation."""
    dev = length.device
    cap = dictionary.capacity
    var_len = torch.zeros(max(cap, 1), dtype=torch.float64, device=dev)
    var_inc = torch.zeros(max(cap, 1), dtype=torch.float64, device=dev)
    totals = torch.zeros(3, dtype=torch.float64, device=dev)
    d = dictionary.struct()
    rc = L.lib().jabba_digitize_quality(_p(length), _p(inc), _p(n_pieces), int(max_pieces), float(alpha), int(B),
                                        C.byref(d), _p(var_len), _p(var_inc), _p(totals), _p(workspace),
                                        workspace.numel(), _stream(stream))
    L.check(rc, "jabba_digitize_quality")
    return {"var_len": var_len, "var_inc": var_inc, "totals": totals}


def kmeans(length: torch.Tensor, inc: torch.Tensor, n_pieces: torch.Tensor, max_pieces: int, dictionary: Dictionary,
           max_iter: int = 100, symbols: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
           stream=None):
    """Lloyd iterations from the dictionary's initial centers (see jabba_kmeans).

    The dictionary's params (sigma_len, sigma_inc, scl), k and cx/cy are the inputs; its centers and counts
    are overwritten with the result.  Returns (symbols, iterations tensor)."""
    dev = length.device
    if symbols is None:
        symbols = torch.empty(max(max_pieces, 1), dtype=torch.int32, device=dev)
    if workspace is None:
        n = C.c_size_t()
        L.check(L.lib().jabba_kmeans_workspace(int(max_pieces), int(dictionary.capacity), C.byref(n)),
                "jabba_kmeans_workspace")
        workspace = _ws(n.value, dev)
    iters = torch.zeros(1, dtype=torch.int64, device=dev)
    d = dictionary.struct()
    rc = L.lib().jabba_kmeans(_p(length), _p(inc), _p(n_pieces), int(max_pieces), int(max_iter), C.byref(d),
                              _p(symbols), _p(iters), _p(workspace), workspace.numel(), _stream(stream))
    L.check(rc, "jabba_kmeans")
    return symbols, iters


def encode_workspace_bytes(capacity: int) -> int:
    n = C.c_size_t()
    L.check(L.lib().jabba_encode_workspace(int(capacity), C.byref(n)), "encode_workspace")
    return n.value


def encode(length: torch.Tensor, inc: torch.Tensor, n_pieces: torch.Tensor, max_pieces: int, dictionary: Dictionary,
           symbols: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Nearest-center symbols against a resident dictionary (see jabba_encode)."""
    if symbols is None:
        symbols = torch.empty(max(max_pieces, 1), dtype=torch.int32, device=length.device)
    if workspace is None:
        workspace = dictionary.encode_workspace()
    d = dictionary.struct()
    rc = L.lib().jabba_encode(_p(length), _p(inc), _p(n_pieces), int(max_pieces), C.byref(d), _p(symbols),
                              _p(workspace), workspace.numel(), _stream(stream))
    L.check(rc, "jabba_encode")
    return symbols


def encode_noalloc(length: torch.Tensor, inc: torch.Tensor, n_pieces: torch.Tensor, max_pieces: int,
                   dictionary: Dictionary, symbols: torch.Tensor, stream=None) -> torch.Tensor:
    """jabba_encode_noalloc: the same symbols with the library's own per-GPU scratch (no workspace)."""
    d = dictionary.struct()
    rc = L.lib().jabba_encode_noalloc(_p(length), _p(inc), _p(n_pieces), int(max_pieces), C.byref(d), _p(symbols),
                                      _stream(stream))
    L.check(rc, "jabba_encode_noalloc")
    return symbols


def reconstruct(symbols: torch.Tensor, piece_off: torch.Tensor, series_off: torch.Tensor, t0: torch.Tensor,
                dictionary: Dictionary, values: torch.Tensor | None = None, want_lhat: bool = False, stream=None):
    """Inverse symbolization.  Returns dict(out, out_off, lhat, sse, cnt, status); synchronises once for the size."""
    dev = symbols.device
    ns = piece_off.numel() - 1
    ws = _ws(recon_workspace_bytes(ns), dev)
    out_off = torch.empty(ns + 1, dtype=torch.int64, device=dev)
    d = dictionary.struct()
    st = _stream(stream)
    L.check(L.lib().jabba_reconstruct_size(_p(symbols), _p(piece_off), _p(series_off), ns, C.byref(d), _p(out_off),
                                           _p(ws), ws.numel(), st), "jabba_reconstruct_size")
    status = workspace_status(ws, stream)
    total = int(out_off[-1].item())
    out = torch.empty(max(total, 1), dtype=torch.float64, device=dev)
    lhat = torch.empty(max(symbols.numel(), 1), dtype=torch.int64, device=dev) if want_lhat else None
    sse = cnt = None
    if values is not None:
        sse = torch.empty(max(ns, 1), dtype=torch.float64, device=dev)
        cnt = torch.empty(max(ns, 1), dtype=torch.int64, device=dev)
    L.check(L.lib().jabba_reconstruct(_p(symbols), _p(piece_off), _p(series_off), ns, _p(t0), C.byref(d),
                                      _p(out_off), _p(out), _p(lhat), _p(values), _p(sse), _p(cnt), _p(ws),
                                      ws.numel(), st),
            "jabba_reconstruct")
    return {"out": out[:total], "out_off": out_off, "lhat": lhat, "sse": sse, "cnt": cnt, "status": status}


def reconstruction_mse(sse: torch.Tensor, cnt: torch.Tensor, n_series: int, stream=None) -> float:
    """Mean squared error from jabba_reconstruct's per-series outputs (jabba_reconstruct_mse); synchronises."""
    out = torch.empty(1, dtype=torch.float64, device=sse.device)
    L.check(L.lib().jabba_reconstruct_mse(_p(sse), _p(cnt), int(n_series), _p(out), _stream(stream)),
            "jabba_reconstruct_mse")
    return float(out.item())


def reconstruct_pieces(length: torch.Tensor, inc: torch.Tensor, piece_off: torch.Tensor, series_off: torch.Tensor,
                       t0: torch.Tensor, total_out: int | None = None, stream=None):
    """Polyline straight from the pieces.  Returns (out, out_off)."""
    dev = length.device
    ns = piece_off.numel() - 1
    ws = _ws(recon_workspace_bytes(ns), dev)
    out_off = torch.empty(ns + 1, dtype=torch.int64, device=dev)
    cap = total_out if total_out is not None else None
    if cap is None:
        # every series has 1 + sum(len) <= its point count points
        cap = int(series_off[-1].item()) if series_off.numel() else 0
    out = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    L.check(L.lib().jabba_reconstruct_pieces(_p(length), _p(inc), _p(piece_off), _p(series_off), ns, _p(t0),
                                             _p(out_off), _p(out), _p(ws), ws.numel(), _stream(stream)),
            "jabba_reconstruct_pieces")
    return out, out_off


class Plan:
    """Compress + digitize captured once into a HIP graph; run() replays it.

    tuning None lets jabba_plan_create choose the launch shapes (autotune);
    tuning() reports the shapes the graph was captured with."""

    def __init__(self, values: torch.Tensor, series_off: torch.Tensor, D: int, tol: float, alpha: float,
                 scl: float = 1.0, B: int = 4096, max_len: int = 0, max_pieces: int | None = None,
                 capacity: int | None = None, tuning: dict | None = None, buffers: "Symbolizer | None" = None):
        dev = values.device
        self.n_series = series_off.numel() - 1
        self.total = values.numel()
        self.values, self.series_off = values, series_off
        if buffers is not None:
            # share an eager Symbolizer's buffers (sized for its piece count)
            self.max_pieces = buffers.max_pieces
            self.pieces, self.symbols, self.dictionary = buffers.pieces, buffers.symbols, buffers.dictionary
            self.cws, self.dws = buffers.cws, buffers.dws
        else:
            self.max_pieces = int(max_pieces) if max_pieces is not None else max(self.total, 1)
            mp = self.max_pieces
            self.pieces = Pieces(torch.empty(mp, dtype=torch.int32, device=dev),
                                 torch.empty(mp, dtype=torch.float64, device=dev),
                                 torch.empty(self.n_series + 1, dtype=torch.int64, device=dev),
                                 torch.empty(1, dtype=torch.int64, device=dev), mp)
            self.symbols = torch.empty(mp, dtype=torch.int32, device=dev)
            self.dictionary = Dictionary(capacity if capacity is not None else mp, dev)
            self.cws = _ws(compress_workspace_bytes(self.n_series, self.total, D), dev)
            self.dws = _ws(digitize_workspace_bytes(mp, B), dev)
        mp = self.max_pieces
        desc = L.PlanDesc()
        desc.values, desc.series_off = values.data_ptr(), series_off.data_ptr()
        desc.n_series, desc.total_points, desc.D, desc.tol = self.n_series, self.total, int(D), float(tol)
        desc.max_len, desc.alpha, desc.scl, desc.B, desc.max_pieces = int(max_len), float(alpha), float(scl), int(B), mp
        desc.len, desc.inc = self.pieces.len.data_ptr(), self.pieces.inc.data_ptr()
        desc.piece_off, desc.n_pieces = self.pieces.piece_off.data_ptr(), self.pieces.n_pieces.data_ptr()
        desc.symbols = self.symbols.data_ptr()
        desc.dict = self.dictionary.struct()
        desc.compress_ws, desc.compress_ws_bytes = self.cws.data_ptr(), self.cws.numel()
        desc.digitize_ws, desc.digitize_ws_bytes = self.dws.data_ptr(), self.dws.numel()
        t = tuning_struct(tuning)
        if t is not None:
            desc.tuning = C.pointer(t)
        torch.cuda.synchronize(dev)
        h = C.c_void_p()
        L.check(L.lib().jabba_plan_create(C.byref(desc), C.byref(h)), "jabba_plan_create")
        self._h = h

    @classmethod
    def from_symbolizer(cls, sz: "Symbolizer", values: torch.Tensor, series_off: torch.Tensor,
                        tuning: dict | None = None) -> "Plan":
        """A plan over an eager Symbolizer's own buffers (no second set); the
        graph and the Symbolizer then write the same outputs."""
        return cls(values, series_off, sz.D, sz.tol, sz.alpha, sz.scl, sz.B, sz.max_len, tuning=tuning, buffers=sz)

    def tuning(self) -> dict:
        t = L.Tuning()
        L.check(L.lib().jabba_plan_tuning(self._h, C.byref(t)), "jabba_plan_tuning")
        return {"lanes_per_domain": t.lanes_per_domain, "waves_per_block": t.waves_per_block,
                "blocks_per_cu": t.blocks_per_cu, "stage1_waves": t.stage1_waves,
                "segment_intervals": t.segment_intervals}

    def run(self, stream=None) -> None:
        L.check(L.lib().jabba_plan_run(self._h, _stream(stream)), "jabba_plan_run")

    def status(self) -> tuple[int, int]:
        return workspace_status(self.cws), workspace_status(self.dws)

    def close(self) -> None:
        if getattr(self, "_h", None):
            L.lib().jabba_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Symbolizer:
    """Preallocated compress + digitize for one workload shape (eager launches).

    Buffers and workspaces are allocated once; run() only enqueues kernels.
    """

    def __init__(self, n_series: int, total_points: int, D: int, tol: float, alpha: float, scl: float = 1.0,
                 B: int = 4096, max_len: int = 0, max_pieces: int | None = None, capacity: int | None = None,
                 tuning: dict | None = None, device=None):
        dev = _dev(device)
        self.D, self.tol, self.alpha, self.scl, self.B, self.max_len = D, tol, alpha, scl, B, max_len
        self.tuning = tuning
        mp = int(max_pieces) if max_pieces is not None else max(total_points, 1)
        self.max_pieces = mp
        self.pieces = Pieces(torch.empty(mp, dtype=torch.int32, device=dev),
                             torch.empty(mp, dtype=torch.float64, device=dev),
                             torch.empty(n_series + 1, dtype=torch.int64, device=dev),
                             torch.empty(1, dtype=torch.int64, device=dev), mp)
        self.symbols = torch.empty(mp, dtype=torch.int32, device=dev)
        self.dictionary = Dictionary(capacity if capacity is not None else mp, dev)
        self.cws = _ws(compress_workspace_bytes(n_series, total_points, D), dev)
        self.dws = _ws(digitize_workspace_bytes(mp, B), dev)

    def compress(self, values, series_off, stream=None) -> Pieces:
        return compress(values, series_off, self.D, self.tol, self.max_len, self.tuning, self.max_pieces,
                        out=self.pieces, workspace=self.cws, stream=stream)

    def digitize(self, stream=None):
        p = self.pieces
        return digitize(p.len, p.inc, p.n_pieces, self.max_pieces, self.alpha, self.scl, self.B, tuning=self.tuning,
                        symbols=self.symbols, dictionary=self.dictionary, workspace=self.dws, stream=stream)

    def run(self, values, series_off, stream=None):
        self.compress(values, series_off, stream)
        return self.digitize(stream)

    def status(self) -> tuple[int, int]:
        return workspace_status(self.cws), workspace_status(self.dws)

    def stats(self) -> dict:
        return digitize_stats(self.dws, self.max_pieces, self.B)

    def quality(self, stream=None) -> dict:
        """Variances and SSE of the last digitize (call before the next run)."""
        p = self.pieces
        return digitize_quality(p.len, p.inc, p.n_pieces, self.max_pieces, self.alpha, self.B, self.dictionary,
                                self.dws, stream=stream)


class Reconstructor:
    """Preallocated inverse symbolization for a fixed set of series.

    size() runs the size pass and synchronises once to allocate the output;
    run() then enqueues size + fill without any host synchronisation (valid
    while the symbols describe the same total length, e.g. a repeated batch).
    """

    def __init__(self, piece_off: torch.Tensor, series_off: torch.Tensor, t0: torch.Tensor,
                 values: torch.Tensor | None = None):
        dev = piece_off.device
        self.piece_off, self.series_off, self.t0, self.values = piece_off, series_off, t0, values
        self.ns = piece_off.numel() - 1
        self.ws = _ws(recon_workspace_bytes(self.ns), dev)
        self.out_off = torch.empty(self.ns + 1, dtype=torch.int64, device=dev)
        self.sse = torch.empty(max(self.ns, 1), dtype=torch.float64, device=dev)
        self.cnt = torch.empty(max(self.ns, 1), dtype=torch.int64, device=dev)
        self.out = None

    def _size(self, symbols, dictionary, stream=None):
        d = dictionary.struct()
        L.check(L.lib().jabba_reconstruct_size(_p(symbols), _p(self.piece_off), _p(self.series_off), self.ns,
                                               C.byref(d), _p(self.out_off), _p(self.ws), self.ws.numel(),
                                               _stream(stream)), "jabba_reconstruct_size")

    def size(self, symbols, dictionary, stream=None) -> int:
        self._size(symbols, dictionary, stream)
        total = int(self.out_off[-1].item())
        if self.out is None or self.out.numel() < total:
            self.out = torch.empty(max(total, 1), dtype=torch.float64, device=self.piece_off.device)
        return total

    def run(self, symbols, dictionary, stream=None):
        self._size(symbols, dictionary, stream)
        d = dictionary.struct()
        v = self.values
        L.check(L.lib().jabba_reconstruct(_p(symbols), _p(self.piece_off), _p(self.series_off), self.ns, _p(self.t0),
                                          C.byref(d), _p(self.out_off), _p(self.out), None, _p(v),
                                          _p(self.sse) if v is not None else None,
                                          _p(self.cnt) if v is not None else None, _p(self.ws), self.ws.numel(),
                                          _stream(stream)),
                "jabba_reconstruct")

    def mse(self, stream=None) -> float:
        """Sec. 3.3 mean squared error of the last run (jabba_reconstruct_mse); synchronises."""
        return reconstruction_mse(self.sse, self.cnt, self.ns, stream)


def timing_enable(on: bool = True) -> None:
    """Per-kernel HIP-event timing inside the library (see jabba_timing_enable)."""
    L.check(L.lib().jabba_timing_enable(1 if on else 0), "jabba_timing_enable")


def timing_report() -> dict:
    """{kernel name: (total ms, launches)} accumulated since timing_enable(True)."""
    buf = C.create_string_buffer(1 << 16)
    L.check(L.lib().jabba_timing_names(buf, len(buf)), "jabba_timing_names")
    out = {}
    for name in filter(None, buf.value.decode().split(",")):
        ms, n = C.c_double(), C.c_int64()
        L.check(L.lib().jabba_timing_get(name.encode(), C.byref(ms), C.byref(n)), "jabba_timing_get")
        out[name] = (ms.value, n.value)
    return out
