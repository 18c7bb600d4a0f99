"""The compression kernel's decision procedure, modelled on the CPU with the
kernel's own bound (csrc/compress_filter.h), gives the oracle's pieces bit for
bit: on the workloads, on degenerate inputs, and on adversarial near-ties
where the threshold sits within a few ulps of a candidate's sequential sum
(there the bound must leave the candidate undecided and the exact sum
decides)."""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2401_00109_amd.inputs import make_workload, pack

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    d = tmp_path_factory.mktemp("model")
    so = d / "model.so"
    subprocess.run(["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                    "-I", os.path.join(ROOT, "paper_2401_00109_amd", "csrc"), "-o", str(so),
                    os.path.join(ROOT, "tests", "host", "compress_model.cpp")], check=True)
    L = C.CDLL(str(so))
    f64 = np.ctypeslib.ndpointer(np.float64, flags="C")
    i64 = np.ctypeslib.ndpointer(np.int64, flags="C")
    i32 = np.ctypeslib.ndpointer(np.int32, flags="C")
    L.sim_compress.restype = C.c_int64
    L.sim_compress.argtypes = [f64, i64, C.c_int64, C.c_int32, C.c_double, C.c_int32, C.c_int, i32, f64]
    L.get_undecided.restype = C.c_long
    L.get_cand.restype = C.c_long

    def run(vals, off, D, tol, max_len=0, W=4):
        cap = max(int(vals.size), 1)
        ln = np.zeros(cap, np.int32)
        inc = np.zeros(cap)
        L.reset_counts()
        n = L.sim_compress(np.ascontiguousarray(vals, np.float64), np.ascontiguousarray(off, np.int64),
                           off.size - 1, D, tol, max_len, W, ln, inc)
        return ln[:n], inc[:n], L.get_undecided(), L.get_cand()
    return run


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.uint64), b[1].view(np.uint64))


@pytest.mark.parametrize("wid,scale", [(1, 1.0), (2, 0.02), (3, 0.004), (4, 1 / 128)])
def test_model_matches_oracle_on_workloads(model, wid, scale):
    w = make_workload(wid, 0, scale)
    ref = O.compress(w.values, w.series_off, w.D, w.tol)
    for W in (1, 4, 16, 64):
        ln, inc, und, cand = model(w.values, w.series_off, w.D, w.tol, 0, W)
        assert _same((ln, inc), ref)
        assert und <= cand * 1e-4  # the bound decides essentially every candidate


def test_model_degenerate_inputs(model):
    rng = np.random.default_rng(5)
    cases = [
        (pack([3.0 + 0.25 * np.arange(n) for n in (5, 100, 1001, 2)]), 100, 0.0, 0),
        (pack([np.full(300, 2.5), np.zeros(70)]), 64, 0.0, 0),
        (pack([np.cumsum(rng.standard_normal(500)) * 0.01]), 1000, 10.0, 5),
        (pack([np.cumsum(rng.standard_normal(5000)) * 1e-8]), 1000, 1e-9, 0),
        (pack([np.cumsum(rng.standard_normal(5000)) * 1e8]), 1000, 1e7, 0),
        (pack([rng.integers(-3, 4, 3000).astype(float)]), 500, 0.0, 0),
    ]
    for (vals, off), D, tol, ml in cases:
        ref = O.compress(vals, off, D, tol, ml)
        for W in (1, 2, 8, 64):
            assert _same(model(vals, off, D, tol, ml, W)[:2], ref)


def test_model_adversarial_near_ties(model):
    rng = np.random.default_rng(123)
    undecided = 0
    for _ in range(150):
        n = int(rng.integers(20, 300))
        vals = np.cumsum(rng.standard_normal(n)) * float(rng.choice([1e-3, 1.0, 1e3]))
        s = int(rng.integers(0, n // 2))
        c = int(rng.integers(2, min(60, n - s - 1)))
        ts = vals[s]
        b = (vals[s + c] - ts) / c
        acc = 0.0
        for k in range(1, c):
            v = b * k
            v = ts + v
            r = v - vals[s + k]
            acc = acc + r * r
        tol0 = math.sqrt(acc / (c - 1))
        for d in range(-3, 4):
            tol = tol0
            for _ in range(abs(d)):
                tol = math.nextafter(tol, math.inf if d > 0 else -math.inf)
            off = np.array([0, n], np.int64)
            ref = O.compress(vals, off, n, tol)
            for W in (1, 4, 64):
                ln, inc, und, _ = model(vals, off, n, tol, 0, W)
                undecided += und
                assert _same((ln, inc), ref)
    assert undecided > 0  # the near-ties really exercised the exact path
