"""The C ABI library loads and exports every function include/jabba.h declares
(no compute calls: this runs without a GPU), and host-side argument checks
reject bad input before anything is enqueued."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jabba.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(jabba_\w+)\s*\(", src)))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ["jabba_compress", "jabba_digitize", "jabba_encode", "jabba_reconstruct", "jabba_plan_create"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2401_00109_amd import _lib
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), f"{name} declared in jabba.h but not exported"
    assert L.jabba_abi_version() == 4
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_status_strings():
    from paper_2401_00109_amd import _lib
    assert _lib.status_str(0) == "ok"
    assert _lib.status_str(-4) == "dictionary capacity exceeded"
    assert _lib.status_str(12345) == "unknown status"


def test_host_side_validation_needs_no_gpu():
    from paper_2401_00109_amd import _lib
    L = _lib.lib()
    n = C.c_size_t()
    assert L.jabba_compress_workspace(-1, 10, 5, C.byref(n)) == _lib.JABBA_EINVAL
    assert L.jabba_compress_workspace(2, 10, 0, C.byref(n)) == _lib.JABBA_EINVAL
    assert L.jabba_compress_workspace(2, 10, 5, C.byref(n)) == 0 and n.value > 0
    assert L.jabba_digitize_workspace(100, 0, C.byref(n)) == _lib.JABBA_EINVAL
    assert L.jabba_digitize_workspace(100, 64, C.byref(n)) == 0 and n.value > 0
    # bad tolerance / sizes are refused before any launch (null device pointers are never touched)
    rc = L.jabba_compress(None, None, 1, 10, 5, -1.0, 0, None, None, None, None, None, None, 0, None)
    assert rc == _lib.JABBA_EINVAL
    rc = L.jabba_compress(None, None, 1, 10, 5, float("nan"), 0, None, None, None, None, None, None, 0, None)
    assert rc == _lib.JABBA_EINVAL
    d = _lib.Dict()
    rc = L.jabba_digitize(None, None, None, 10, -0.5, 1.0, 64, None, None, C.byref(d), None, 0, None)
    assert rc == _lib.JABBA_EINVAL
    rc = L.jabba_digitize(None, None, None, 10, 0.5, 1.0, 0, None, None, C.byref(d), None, 0, None)
    assert rc == _lib.JABBA_EINVAL


def test_reconstruct_needs_its_workspace():
    # the fill call takes the reconstruct workspace (it orders the series
    # there): missing or short, it is refused before any launch
    from paper_2401_00109_amd import _lib
    L = _lib.lib()
    n = C.c_size_t()
    assert L.jabba_reconstruct_workspace(1000, C.byref(n)) == 0 and n.value > 0
    fake = C.c_void_p(256)  # never dereferenced on the host
    d = _lib.Dict(capacity=4, center_len=256, center_inc=256)
    args = [fake, fake, fake, 1000, fake, C.byref(d), fake, fake, None, None, None, None]
    assert L.jabba_reconstruct(*args, None, n.value, None) == _lib.JABBA_ENOMEM
    assert L.jabba_reconstruct(*args, fake, n.value - 1, None) == _lib.JABBA_ENOMEM
    assert L.jabba_reconstruct(fake, fake, fake, 0, fake, C.byref(d), fake, fake, None, None, None, None, None, 0,
                               None) == 0  # no series: nothing to do


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2401_00109_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def test_every_export_has_a_ctypes_signature():
    # an entry point without argtypes would fail on its first float argument
    from paper_2401_00109_amd import _lib
    L = _lib.lib()
    for name in _lib.EXPORTS:
        assert getattr(L, name).argtypes is not None, f"{name} has no ctypes signature"


def test_noalloc_encode_limit_is_host_checked():
    # the allocation-free encode's scratch holds the workspace of its maximum
    # capacity, and larger dictionaries are refused before any HIP call
    from paper_2401_00109_amd import _lib
    L = _lib.lib()
    n = C.c_size_t()
    assert L.jabba_encode_workspace(_lib.JABBA_ENCODE_NOALLOC_MAX_CAPACITY, C.byref(n)) == 0
    assert n.value <= 3 << 20
    d = _lib.Dict()
    d.capacity = _lib.JABBA_ENCODE_NOALLOC_MAX_CAPACITY + 1
    fake = C.c_void_p(256)
    d.params = d.k = d.cx = d.cy = fake
    rc = L.jabba_encode_noalloc(fake, fake, fake, 10, C.byref(d), fake, None)
    assert rc == _lib.JABBA_ELIMIT
    assert _lib.status_str(rc).startswith("size above")


def test_device_check_refuses_without_a_gfx950():
    # valid arguments on a machine with no visible GPU: nothing can be
    # enqueued, and the call says why instead of failing inside HIP
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2401_00109_amd import _lib
    L = _lib.lib()
    fake = C.c_void_p(256)
    rc = L.jabba_fp64_selftest(fake, fake, fake, fake, 10, None)
    assert rc == _lib.JABBA_ENODEV
    assert _lib.status_str(rc) == "no gfx950 device"
