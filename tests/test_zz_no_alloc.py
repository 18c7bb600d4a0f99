"""jabba_encode_noalloc (the allocation-free encode, scratch in a file-scope
device array) against jabba_encode with a caller workspace: bit-identical
symbols on two calls in a row, the second with a smaller input, for a
dictionary staged in LDS and one ordered in global memory."""
import numpy as np
import pytest

from gpu_util import DEV, say, to_dev, torch

pytestmark = pytest.mark.gpu


def _dictionary(k, seed):
    import paper_2401_00109_amd as J
    rng = np.random.default_rng(seed)
    cx = rng.integers(1, 30, k) * 0.37
    cy = np.round(rng.standard_normal(k), 2)
    if k > 10:
        cx[k // 2:k // 2 + 5] = cx[0]
        cy[k // 2:k // 2 + 5] = cy[0]  # exact duplicates: the lowest id wins
    return J.Dictionary.from_host(2.7027027027027026, 0.9, 1.0, 0.1, np.ones(k), np.zeros(k), cx, cy, device=DEV)


def _pieces(n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(1, 30, n).astype(np.int32), np.round(rng.standard_normal(n), 2) * 0.9


@pytest.mark.parametrize("k_first,k_second", [(20000, 37), (3000, 20000), (594, 594)])
def test_noalloc_encode_equals_workspace_encode(k_first, k_second):
    import paper_2401_00109_amd as J
    T = torch()
    for call, (k, n) in enumerate([(k_first, 50000), (k_second, 7000)]):
        say(f"encode_noalloc call {call}: k={k} pieces={n}")
        d = _dictionary(k, 10 * call + k)
        ln, inc = _pieces(n, 1000 + call)
        L, I = to_dev(ln), to_dev(inc)
        npc = T.tensor([n], dtype=T.int64, device=DEV)
        exp = J.encode(L, I, npc, n, d)
        got = T.full((n,), -7, dtype=T.int32, device=DEV)
        J.encode_noalloc(L, I, npc, n, d, got)
        T.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), exp[:n].cpu().numpy())


def test_noalloc_encode_rejects_capacity_above_its_maximum():
    import paper_2401_00109_amd as J
    from paper_2401_00109_amd import _lib
    T = torch()
    d = J.Dictionary(_lib.JABBA_ENCODE_NOALLOC_MAX_CAPACITY + 1, device=DEV)
    L = T.ones(4, dtype=T.int32, device=DEV)
    I = T.zeros(4, dtype=T.float64, device=DEV)
    npc = T.tensor([4], dtype=T.int64, device=DEV)
    out = T.empty(4, dtype=T.int32, device=DEV)
    with pytest.raises(_lib.JabbaError) as e:
        J.encode_noalloc(L, I, npc, 4, d, out)
    assert e.value.status == _lib.JABBA_ELIMIT
