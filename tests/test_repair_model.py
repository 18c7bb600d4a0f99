"""The segmented compression (domains compressed as segments in parallel,
then repaired, csrc/compress_repair.h), modelled on the CPU with the kernel's
own header, gives the oracle's domain-by-domain pieces bit for bit for every
segment length: on the workloads, at tol = 0, with max_len, on constant and
straight series and on series whose pieces are long compared with the
segments."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2401_00109_amd.inputs import make_workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    d = tmp_path_factory.mktemp("repair")
    so = d / "repair.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                    "-I", os.path.join(ROOT, "paper_2401_00109_amd", "csrc"), "-o", str(so),
                    os.path.join(ROOT, "tests", "host", "repair_model.cpp")], check=True)
    L = C.CDLL(str(so))
    f64 = np.ctypeslib.ndpointer(np.float64, flags="C")
    i64 = np.ctypeslib.ndpointer(np.int64, flags="C")
    i32 = np.ctypeslib.ndpointer(np.int32, flags="C")
    L.seg_compress.restype = C.c_int64
    L.seg_compress.argtypes = [f64, i64, C.c_int64, C.c_int32, C.c_int32, C.c_double, C.c_int32, i32, f64,
                               C.POINTER(C.c_int64)]

    def run(vals, off, D, G, tol, max_len=0):
        cap = max(int(vals.size), 1)
        ln = np.zeros(cap, np.int32)
        inc = np.zeros(cap)
        nr = C.c_int64()
        n = L.seg_compress(np.ascontiguousarray(vals, np.float64), np.ascontiguousarray(off, np.int64),
                           off.size - 1, D, G, tol, max_len, ln, inc, C.byref(nr))
        assert n >= 0, "repair walk did not end at the domain end"
        return ln[:n], inc[:n], nr.value
    return run


def _same(got, ref):
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1].view(np.uint64), ref[1].view(np.uint64))


@pytest.mark.parametrize("wid,scale", [(1, 1.0), (2, 0.01), (3, 0.002), (4, 1 / 256)])
@pytest.mark.parametrize("G", [1, 2, 3, 7, 32, 128, 1000])
def test_segments_repaired_into_domains(model, wid, scale, G):
    w = make_workload(wid, 0, scale)
    ref = O.compress(w.values, w.series_off, w.D, w.tol)
    got = model(w.values, w.series_off, w.D, G, w.tol)
    _same(got, ref)


@pytest.mark.parametrize("tol,max_len", [(0.0, 0), (0.3, 0), (1.0, 0), (0.5, 5), (5.0, 0), (5.0, 40)])
@pytest.mark.parametrize("G", [1, 5, 32, 64])
def test_long_pieces_and_limits(model, tol, max_len, G):
    rng = np.random.default_rng(int(tol * 10) + max_len)
    walk = np.cumsum(rng.standard_normal(6000))
    line = 0.25 * np.arange(3000.0)
    const = np.full(2000, 1.5)
    steps = np.repeat(rng.integers(-3, 4, 150).astype(np.float64), 20)
    vals = np.concatenate([walk, line, const, steps])
    off = np.array([0, 6000, 9000, 11000, 14000], np.int64)
    for D in (1, 7, 250, 5999):
        ref = O.compress(vals, off, D, tol, max_len)
        got = model(vals, off, D, G, tol, max_len)
        _same(got, ref)


def test_repairs_happen(model):
    # segments shorter than the domains: every domain is repaired
    w = make_workload(1, 0, 1.0)
    _, _, nr = model(w.values, w.series_off, w.D, 32, w.tol)
    assert nr == w.series_off.size - 1


@pytest.mark.parametrize("tol", [0.2, 0.5])
@pytest.mark.parametrize("G", [4, 5, 6])
def test_short_segments_that_need_the_run_moved(model, tol, G):
    # short segments full of short pieces: the pieces recomputed in front of a
    # kept run sometimes do not fit before it, and the run is moved
    rng = np.random.default_rng(1)
    v = np.cumsum(rng.standard_normal(20000))
    off = np.array([0, 20000], np.int64)
    _same(model(v, off, 19999, G, tol), O.compress(v, off, 19999, tol))
