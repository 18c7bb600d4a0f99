"""ctypes wrapper around the plain-C oracle (``jabba_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

The C file is compiled with gcc ``-O2 -ffp-contract=off -fno-fast-math`` so
that each floating-point operation is a single correctly rounded binary64
operation in source order.  Inputs and outputs are numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

__all__ = [
    "build_oracle",
    "lib",
    "OracleError",
    "count_domains",
    "domains",
    "compress",
    "pca_axis",
    "znorm",
    "axis_tolerances",
    "aggregate_points",
    "Aggregated",
    "tree_sum",
    "exact_sum",
    "scaling",
    "sort_order",
    "blocks",
    "aggregate_sorted",
    "digitize",
    "Digitized",
    "reconstruct",
    "reconstruct_pieces",
    "encode",
    "quality",
    "Quality",
    "kmeans",
    "KMeans",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jabba_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "libjabba_oracle.so")
_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-shared", "-fPIC"]
_lock = threading.Lock()
_lib = None


class OracleError(RuntimeError):
    pass


def build_oracle(force: bool = False) -> str:
    """Compile the oracle shared library (always when ``force``).

    ``JABBA_ORACLE_SO`` names a prebuilt oracle library to load instead; the
    mutation tests use it to run the pins against deliberately broken copies.
    """
    override = os.environ.get("JABBA_ORACLE_SO")
    if override and not force:
        return override
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *_FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _SO)
    return _SO


_i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C")


def _nullable(tp):
    base = np.ctypeslib.ndpointer(tp, flags="C")

    class _N(base):  # type: ignore[misc, valid-type]
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return base.from_param(obj)

    return _N


_i64n = _nullable(np.int64)
_f64n = _nullable(np.float64)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build_oracle())
            L.jo_count_domains.restype = C.c_int64
            L.jo_count_domains.argtypes = [_i64p, C.c_int64, C.c_int32]
            L.jo_domains.restype = C.c_int
            L.jo_domains.argtypes = [_i64p, C.c_int64, C.c_int32, _i64p, _i64p, _i64p]
            L.jo_compress.restype = C.c_int64
            L.jo_compress.argtypes = [_f64p, _i64p, C.c_int64, C.c_int32, C.c_double, C.c_int32, _i32p, _f64p,
                                      _i64p]
            L.jo_tree_sum.restype = C.c_double
            L.jo_tree_sum.argtypes = [_f64p, C.c_int64]
            L.jo_exact_sum.restype = C.c_double
            L.jo_exact_sum.argtypes = [_f64p, C.c_int64]
            L.jo_scaling.restype = C.c_int
            L.jo_scaling.argtypes = [_i32p, _f64p, C.c_int64, C.c_double, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), _f64n, _f64n, _f64n]
            L.jo_sort_order.restype = None
            L.jo_sort_order.argtypes = [_f64p, C.c_int64, _i64p]
            L.jo_blocks.restype = C.c_int64
            L.jo_blocks.argtypes = [_f64p, C.c_int64, C.c_int64, _i64p]
            L.jo_aggregate_sorted.restype = None
            L.jo_aggregate_sorted.argtypes = [_f64p, _f64p, _f64p, C.c_int64, C.c_double, _i64p]
            L.jo_digitize.restype = C.c_int64
            L.jo_digitize.argtypes = [_i32p, _f64p, C.c_int64, C.c_double, C.c_double, C.c_int64, C.c_int64,
                                      _i32p, _i64n, _i64n, C.POINTER(C.c_int64), _i64n, _f64n, _f64n, _f64n,
                                      _f64n, _f64n, _i64n, C.POINTER(C.c_int64)]
            L.jo_digitize_key.restype = C.c_int64
            L.jo_digitize_key.argtypes = [_i32p, _f64p, C.c_int64, C.c_double, C.c_double, C.c_int64, C.c_int,
                                          _f64n, C.c_int64, _i32p, _i64n, _i64n, C.POINTER(C.c_int64), _i64n,
                                          _f64n, _f64n, _f64n, _f64n, _f64n, _i64n, C.POINTER(C.c_int64)]
            L.jo_pca_axis.restype = C.c_int
            L.jo_znorm.restype = C.c_int
            L.jo_znorm.argtypes = [_f64p, _i64p, C.c_int64, _f64p, _f64p, _f64p]
            L.jo_aggregate_points.restype = C.c_int64
            L.jo_aggregate_points.argtypes = [_f64p, _f64p, C.c_int64, C.c_double, C.c_int64, C.c_int64, _i32p,
                                              _f64p, _f64p, _i64p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int64)]
            L.jo_pca_axis.argtypes = [_i32p, _f64p, C.c_int64, C.c_double, _f64p]
            L.jo_reconstruct_size.restype = C.c_int
            L.jo_reconstruct_size.argtypes = [_i32p, _i64p, _i64p, C.c_int64, _f64p, C.c_int64, _i64p]
            L.jo_reconstruct.restype = C.c_int
            L.jo_reconstruct.argtypes = [_i32p, _i64p, _i64p, C.c_int64, _f64p, _f64p, _f64p, C.c_int64, _i64p,
                                         _f64p, _i64n, _f64n, _f64n, _i64n]
            L.jo_reconstruct_pieces.restype = C.c_int
            L.jo_reconstruct_pieces.argtypes = [_i32p, _f64p, _i64p, C.c_int64, _f64p, _i64p, _f64p]
            L.jo_encode.restype = C.c_int
            L.jo_encode.argtypes = [_i32p, _f64p, C.c_int64, C.c_double, C.c_double, C.c_double, _f64p, _f64p,
                                    C.c_int64, _i32p]
            L.jo_kmeans.restype = C.c_int
            L.jo_kmeans.argtypes = [_i32p, _f64p, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int64,
                                    C.c_int64, _f64p, _f64p, _f64p, _f64p, _i64p, _i32p, C.POINTER(C.c_int64)]
            L.jo_quality.restype = C.c_int
            L.jo_quality.argtypes = [_i32p, _f64p, _i32p, C.c_int64, C.c_double, C.c_double, C.c_double, _f64p,
                                     _f64p, C.c_int64, _f64p, _f64p, _i64p, C.POINTER(C.c_double)]
            _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc, what):
    if rc < 0:
        raise OracleError(f"{what} failed with status {rc}")
    return rc


def count_domains(series_off, D: int) -> int:
    so = _i64(series_off)
    return int(lib().jo_count_domains(so, so.size - 1, D))


def domains(series_off, D: int):
    """Domain table: (series, first point, number of intervals) per domain."""
    so = _i64(series_off)
    m = count_domains(so, D)
    ds, st, ni = (np.zeros(m, np.int64) for _ in range(3))
    _check(lib().jo_domains(so, so.size - 1, D, ds, st, ni), "domains")
    return ds, st, ni


def compress(values, series_off, D: int, tol: float, max_len: int = 0):
    """Greedy compression of every domain.  Returns (len i32, inc f64, piece_off i64)."""
    v = _f64(values)
    so = _i64(series_off)
    ns = so.size - 1
    cap = int(np.maximum(np.diff(so) - 1, 0).sum())
    ln = np.zeros(max(cap, 1), np.int32)
    inc = np.zeros(max(cap, 1), np.float64)
    po = np.zeros(ns + 1, np.int64)
    n = _check(lib().jo_compress(v, so, ns, int(D), float(tol), int(max_len), ln, inc, po), "compress")
    return ln[:n].copy(), inc[:n].copy(), po


def tree_sum(a) -> float:
    a = _f64(a)
    return float(lib().jo_tree_sum(a, a.size))


def exact_sum(a) -> float:
    a = _f64(a)
    return float(lib().jo_exact_sum(a, a.size))


def scaling(length, inc, scl: float = 1.0):
    """Returns (sigma_len, sigma_inc, x, y, key)."""
    ln, ic = _i32(length), _f64(inc)
    n = ln.size
    sl, si = C.c_double(), C.c_double()
    x, y, k = (np.zeros(n) for _ in range(3))
    _check(lib().jo_scaling(ln, ic, n, float(scl), C.byref(sl), C.byref(si), x, y, k), "scaling")
    return sl.value, si.value, x, y, k


def sort_order(key):
    key = _f64(key)
    perm = np.zeros(key.size, np.int64)
    lib().jo_sort_order(key, key.size, perm)
    return perm


def blocks(sorted_key, B: int):
    sk = _f64(sorted_key)
    bs = np.zeros(sk.size + 2, np.int64)
    m = int(lib().jo_blocks(sk, sk.size, int(B), bs))
    return bs[: m + 1].copy()


def aggregate_sorted(sx, sy, skey, alpha: float):
    """Serial greedy aggregation over presorted arrays; returns start position per point."""
    sx, sy, sk = _f64(sx), _f64(sy), _f64(skey)
    lab = np.zeros(sx.size, np.int64)
    lib().jo_aggregate_sorted(sx, sy, sk, sx.size, float(alpha), lab)
    return lab


@dataclass
class Digitized:
    symbols: np.ndarray
    k: int
    sigma_len: float
    sigma_inc: float
    scl: float
    alpha: float
    center_len: np.ndarray
    center_inc: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    count: np.ndarray
    perm: np.ndarray
    local_start: np.ndarray
    n_starts: int
    gmap: np.ndarray
    n_blocks: int
    axis: np.ndarray | None = None  # unit principal axis (key="pca" only)


KEYS = {"norm": 0, "pca": 1}


def znorm(values, series_off):
    """Per-series z-normalisation (see jo_znorm).  Returns (z f64[total], mean f64[ns], std f64[ns])."""
    v, so = _f64(values), _i64(series_off)
    ns = so.size - 1
    out = np.zeros(max(v.size, 1))
    m, sd = np.zeros(max(ns, 1)), np.zeros(max(ns, 1))
    _check(lib().jo_znorm(v, so, ns, m, sd, out), "znorm")
    return out[:v.size].copy(), m[:ns].copy(), sd[:ns].copy()


def pca_axis(length, inc, scl: float = 1.0) -> np.ndarray:
    """Unit principal axis of the scaled pieces (see jo_pca_axis)."""
    ln, ic = _i32(length), _f64(inc)
    u = np.zeros(2)
    _check(lib().jo_pca_axis(ln, ic, ln.size, float(scl), u), "pca_axis")
    return u


@dataclass
class Aggregated:
    labels: np.ndarray
    k: int
    cx: np.ndarray
    cy: np.ndarray
    count: np.ndarray
    sse: float
    n_starts: int
    n_blocks: int


def aggregate_points(x, y, alpha: float, B: int = 1 << 62) -> Aggregated:
    """Two-stage aggregation of raw 2-D points (see jo_aggregate_points); B >= N is the serial greedy."""
    xs, ys = _f64(x), _f64(y)
    n = xs.size
    lab = np.zeros(max(n, 1), np.int32)
    cx, cy = np.zeros(max(n, 1)), np.zeros(max(n, 1))
    cnt = np.zeros(max(n, 1), np.int64)
    sse, g, nb = C.c_double(), C.c_int64(), C.c_int64()
    k = _check(lib().jo_aggregate_points(xs, ys, n, float(alpha), int(B), max(n, 1), lab, cx, cy, cnt, C.byref(sse),
                                         C.byref(g), C.byref(nb)), "aggregate_points")
    return Aggregated(lab[:n].copy(), int(k), cx[:k].copy(), cy[:k].copy(), cnt[:k].copy(), float(sse.value),
                      int(g.value), int(nb.value))


def axis_tolerances(alpha_len: float, alpha_inc: float, scl: float = 1.0) -> tuple[float, float]:
    """Separate length and increment tolerances (Sec. 3.2, Eq. Var1).

    A piece joins a start when ((x - x_s)/alpha_len)^2 + ((y - y_s)/alpha_inc)^2 <= 1, which is the
    aggregation's test for alpha_len = alpha_inc.  Multiplying x by alpha_inc/alpha_len turns it into the
    disc test of radius alpha_inc, so the variant is the aggregation run with (alpha, scl) returned here."""
    alpha_len, alpha_inc, scl = float(alpha_len), float(alpha_inc), float(scl)
    if not (alpha_len > 0 and alpha_inc > 0 and scl >= 0) or not all(map(np.isfinite, (alpha_len, alpha_inc, scl))):
        raise ValueError("alpha_len, alpha_inc > 0 and scl >= 0, finite")
    return alpha_inc, scl * (alpha_inc / alpha_len)


def digitize(length, inc, alpha: float, scl: float = 1.0, B: int = 4096, capacity: int | None = None,
             key: str = "norm") -> Digitized:
    """Two-stage digitization and dictionary (see jo_digitize_key); key "norm" or "pca"."""
    if key not in KEYS:
        raise ValueError(f"key must be one of {sorted(KEYS)}")
    ln, ic = _i32(length), _f64(inc)
    n = ln.size
    cap = n if capacity is None else int(capacity)
    sym = np.zeros(max(n, 1), np.int32)
    perm = np.zeros(max(n, 1), np.int64)
    lst = np.zeros(max(n, 1), np.int64)
    gmap = np.zeros(max(n, 1), np.int64)
    sig = np.zeros(2)
    cl, ci, cx, cy = (np.zeros(max(cap, 1)) for _ in range(4))
    cnt = np.zeros(max(cap, 1), np.int64)
    g = C.c_int64()
    nb = C.c_int64()
    axis = np.zeros(2)
    k = _check(lib().jo_digitize_key(ln, ic, n, float(alpha), float(scl), int(B), KEYS[key], axis, cap, sym, perm,
                                     lst, C.byref(g), gmap, sig, cl, ci, cx, cy, cnt, C.byref(nb)), "digitize")
    G = g.value
    return Digitized(sym[:n].copy(), int(k), float(sig[0]), float(sig[1]), float(scl), float(alpha),
                     cl[:k].copy(), ci[:k].copy(), cx[:k].copy(), cy[:k].copy(), cnt[:k].copy(), perm[:n].copy(),
                     lst[:n].copy(), int(G), gmap[:G].copy(), int(nb.value), axis if key == "pca" else None)


def reconstruct(symbols, piece_off, series_off, t0, center_len, center_inc, orig=None):
    """Inverse symbolization.  Returns (out f64, out_off i64, lhat i64, sse f64[ns], cnt i64[ns])."""
    sym, po, so = _i32(symbols), _i64(piece_off), _i64(series_off)
    cl, ci, t0 = _f64(center_len), _f64(center_inc), _f64(t0)
    ns = po.size - 1
    k = cl.size
    oo = np.zeros(ns + 1, np.int64)
    _check(lib().jo_reconstruct_size(sym, po, so, ns, cl, k, oo), "reconstruct_size")
    out = np.zeros(max(int(oo[-1]), 1))
    lhat = np.zeros(max(sym.size, 1), np.int64)
    sse = np.zeros(max(ns, 1))
    cnt = np.zeros(max(ns, 1), np.int64)
    og = None if orig is None else _f64(orig)
    _check(lib().jo_reconstruct(sym, po, so, ns, t0, cl, ci, k, oo, out, lhat, og,
                                sse if og is not None else None, cnt if og is not None else None),
           "reconstruct")
    return out[: oo[-1]].copy(), oo, lhat[: sym.size].copy(), sse[:ns].copy(), cnt[:ns].copy()


def reconstruct_pieces(length, inc, piece_off, t0):
    """Polyline straight from (len, inc); returns (out, out_off)."""
    ln, ic, po, t0 = _i32(length), _f64(inc), _i64(piece_off), _f64(t0)
    ns = po.size - 1
    oo = np.zeros(ns + 1, np.int64)
    for s in range(ns):
        a, b = po[s], po[s + 1]
        oo[s + 1] = oo[s] + (1 + int(ln[a:b].sum()) if b > a else 1)
    out = np.zeros(max(int(oo[-1]), 1))
    _check(lib().jo_reconstruct_pieces(ln, ic, po, ns, t0, oo, out), "reconstruct_pieces")
    return out[: oo[-1]].copy(), oo


def encode(length, inc, sigma_len, sigma_inc, scl, cx, cy):
    ln, ic, cx, cy = _i32(length), _f64(inc), _f64(cx), _f64(cy)
    sym = np.zeros(max(ln.size, 1), np.int32)
    _check(lib().jo_encode(ln, ic, ln.size, float(sigma_len), float(sigma_inc), float(scl), cx, cy, cx.size, sym),
           "encode")
    return sym[: ln.size].copy()


@dataclass
class Quality:
    var_len: np.ndarray
    var_inc: np.ndarray
    count: np.ndarray
    sse: float


def quality(length, inc, symbols, sigma_len, sigma_inc, scl, cx, cy) -> Quality:
    """Per-symbol variances and the total SSE in scaled space (see jo_quality)."""
    ln, ic, sym, cx, cy = _i32(length), _f64(inc), _i32(symbols), _f64(cx), _f64(cy)
    k = cx.size
    vl, vi = np.zeros(max(k, 1)), np.zeros(max(k, 1))
    cnt = np.zeros(max(k, 1), np.int64)
    sse = C.c_double()
    _check(lib().jo_quality(ln, ic, sym, ln.size, float(sigma_len), float(sigma_inc), float(scl), cx, cy, k, vl, vi,
                            cnt, C.byref(sse)), "quality")
    return Quality(vl[:k].copy(), vi[:k].copy(), cnt[:k].copy(), float(sse.value))


@dataclass
class KMeans:
    symbols: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    center_len: np.ndarray
    center_inc: np.ndarray
    count: np.ndarray
    iterations: int


def kmeans(length, inc, sigma_len, sigma_inc, scl, cx0, cy0, max_iter) -> KMeans:
    """Lloyd iterations from the given scaled centers (see jo_kmeans)."""
    ln, ic = _i32(length), _f64(inc)
    cx, cy = _f64(cx0).copy(), _f64(cy0).copy()
    k = cx.size
    cl, ci = np.zeros(k), np.zeros(k)
    cnt = np.zeros(k, np.int64)
    sym = np.zeros(max(ln.size, 1), np.int32)
    it = C.c_int64()
    _check(lib().jo_kmeans(ln, ic, ln.size, float(sigma_len), float(sigma_inc), float(scl), k, int(max_iter), cx, cy,
                           cl, ci, cnt, sym, C.byref(it)), "kmeans")
    return KMeans(sym[: ln.size].copy(), cx, cy, cl, ci, cnt, int(it.value))
