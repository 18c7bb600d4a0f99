"""The radix sort's pass schedule (csrc/sort_plan.h), modelled on the CPU with
the kernel's own header: stable 8-bit LSD passes over key - kmin that skip
constant digits and carry the keys at the schedule's widths (64-bit, 32-bit
once the digits left fit, none after the last pass; or 32-bit from the start
when key - kmin fits and the keys are kept) give the stable order of the
keys, whatever digits are active.  Also pins the bytes per pair of the
digitization's sort (7 active digits: 128 B, against 168 B with full keys)."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def plan_sort(tmp_path_factory):
    d = tmp_path_factory.mktemp("sortplan")
    so = d / "sortplan.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                    "-I", os.path.join(ROOT, "paper_2401_00109_amd", "csrc"), "-o", str(so),
                    os.path.join(ROOT, "tests", "host", "sort_plan_model.cpp")], check=True)
    L = C.CDLL(str(so))
    u64 = np.ctypeslib.ndpointer(np.uint64, flags="C")
    u32 = np.ctypeslib.ndpointer(np.uint32, flags="C")
    i32 = np.ctypeslib.ndpointer(np.int32, flags="C")
    L.plan_sort.restype = C.c_int
    L.plan_sort.argtypes = [u64, C.c_int64, C.c_int, u32, i32, C.POINTER(C.c_int), C.POINTER(C.c_int64)]

    def run(keys, key_form):
        keys = np.ascontiguousarray(keys, np.uint64)
        order = np.zeros(max(keys.size, 1), np.uint32)
        modes = np.zeros(8, np.int32)
        base, nbytes = C.c_int(), C.c_int64()
        rc = L.plan_sort(keys, keys.size, int(key_form), order, modes, C.byref(base), C.byref(nbytes))
        assert rc != -1, "a pass read keys that no earlier pass wrote"
        assert rc != -3 and rc != -4, "the kept 32-bit keys did not leave sorted"
        assert rc == 0
        return order[:keys.size], modes, base.value, nbytes.value
    return run


def _keys(kind, rng, n):
    if kind == "full":
        return rng.integers(0, 2**63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    if kind == "narrow":
        return np.uint64(0xC000000000000000) + rng.integers(0, 2 ** int(rng.integers(1, 60)), n, dtype=np.uint64)
    if kind == "middle_constant":   # digits 2, 3 and 5 equal in every key
        return (rng.integers(0, 2**62, n, dtype=np.uint64) & np.uint64(0xFFFF00FF0000FFFF)) | np.uint64(1 << 63)
    if kind == "few":
        return rng.integers(0, 4, n, dtype=np.uint64) * np.uint64(1 << int(rng.integers(0, 62)))
    if kind == "norms":             # binary64 norms as the digitization orders them
        f = np.sqrt(rng.integers(1, 25, n) ** 2 * 0.01 + rng.normal(0, 1, n) ** 2)
        return f.view(np.uint64) | np.uint64(1 << 63)
    return np.full(n, 12345, np.uint64)


@pytest.mark.parametrize("kind", ["full", "narrow", "middle_constant", "few", "norms", "constant"])
@pytest.mark.parametrize("key_form", [0, 1])   # order only, 64-bit keys kept
def test_schedule_sorts_stably(plan_sort, kind, key_form):
    rng = np.random.default_rng(7)
    for trial in range(20):
        n = int(rng.integers(0, 3000)) if trial else 0
        keys = _keys(kind, rng, n)
        order, modes, base, _ = plan_sort(keys, key_form)
        np.testing.assert_array_equal(order, np.argsort(keys, kind="stable").astype(np.uint32))
        if key_form == 1:
            assert not modes.any() and base == 0


@pytest.mark.parametrize("span_bits", [1, 8, 17, 24, 31, 32])
def test_kept_32_bit_keys(plan_sort, span_bits):
    # keys whose distance from the smallest fits in 32 bits, as the label
    # propagation's shifted indices: every active pass moves 32-bit keys
    # (4 + 4 + 4 + 4 B per pair) and the keys leave sorted with the order
    rng = np.random.default_rng(span_bits)
    for trial in range(10):
        n = int(rng.integers(1, 3000))
        keys = np.uint64(0x1234_0000_0000) + rng.integers(0, 2 ** span_bits, n, dtype=np.uint64)
        order, modes, base, nbytes = plan_sort(keys, 2)
        np.testing.assert_array_equal(order, np.argsort(keys, kind="stable").astype(np.uint32))
        active = [int(m) for m in modes if m]
        assert all(m == 3 for m in active) and base == 0 and nbytes == 16 * len(active)


def test_bytes_of_the_digitization_sort(plan_sort):
    # 7 active digits (0..6), as for the norm keys of the scale workload:
    # 24 + 24 + 20 + 16 + 16 + 16 + 12 B per pair when only the order is needed
    keys = np.arange(1 << 16, dtype=np.uint64) * np.uint64(0x0101010101)
    keys[0] = np.uint64((1 << 56) - 1)
    order, modes, base, nbytes = plan_sort(keys, 0)
    assert [int(m) for m in modes] == [0, 0, 2, 3, 3, 3, 5, 0] and base == 24 and nbytes == 128
    _, modes_k, _, nbytes_k = plan_sort(keys, 1)
    assert not modes_k.any() and nbytes_k == 168
