"""Host models of the reconstruction producer's and filler's arithmetic.

* Lengths: the running sums of the center lengths are exact integers at
  scale 2^52 (Eq. repolygon, halves away from zero: S_j = (C_j + 2^51) >> 52).
  When every center length of a 64-piece chunk is below 2^25 the kernel
  scans three 32-bit limbs (integer part, two 26-bit halves of the
  fraction) and carries (carryH, carryL) from chunk to chunk; otherwise it
  scans 128-bit values.  The model takes the kernel's steps, chunk by chunk
  and in both forms, with Python integers and checks every S_j against the
  exact rounding of the exact running sum (no limb scan may exceed 2^32).
* Filler: each point's piece by a fixed six-step search over the chunk's 64
  ends (lanes past the last piece hold its end) equals the first piece
  whose end is at or after the point.
"""
import bisect
from fractions import Fraction

import numpy as np
import pytest

F52 = 1 << 52
MASK26 = (1 << 26) - 1


def to_fixed(d: float) -> int:
    f = Fraction(d) * F52
    assert f.denominator == 1
    return f.numerator


def producer(lengths):
    """S_j for every piece, the kernel's chunk steps."""
    carry_h, carry_l = 0, 0
    out = []
    for c0 in range(0, len(lengths), 64):
        lt = [to_fixed(d) for d in lengths[c0:c0 + 64]]
        lt += [0] * (64 - len(lt))
        cnt = min(64, len(lengths) - c0)
        if all(v >> 77 == 0 for v in lt):
            h = [v >> 52 for v in lt]
            m = [(v >> 26) & MASK26 for v in lt]
            q = [v & MASK26 for v in lt]
            hs, ms, qs = np.cumsum(h), np.cumsum(m), np.cumsum(q)
            assert hs[-1] < 1 << 32 and ms[-1] < 1 << 32 and qs[-1] < 1 << 32
            low = [(int(ms[i]) << 26) + int(qs[i]) + carry_l for i in range(64)]
            S = [carry_h + int(hs[i]) + ((low[i] + (1 << 51)) >> 52) for i in range(64)]
            lowc = low[cnt - 1]
            carry_h += int(hs[cnt - 1]) + (lowc >> 52)
            carry_l = lowc & (F52 - 1)
        else:
            base = (carry_h << 52) | carry_l
            C = [base + sum(lt[:i + 1]) for i in range(64)]
            S = [(c + (1 << 51)) >> 52 for c in C]
            cc = C[cnt - 1]
            carry_h, carry_l = cc >> 52, cc & (F52 - 1)
        out.extend(S[:cnt])
    return out


def exact(lengths):
    run = Fraction(0)
    out = []
    for d in lengths:
        run += Fraction(d)
        out.append(int((run * 2 + 1) // 2))  # round halves up (the sums are non-negative)
    return out


@pytest.mark.parametrize("kind", ["small", "halves", "large", "mixed"])
def test_limb_scan_matches_the_exact_rounding(kind):
    rng = np.random.default_rng(["small", "halves", "large", "mixed"].index(kind))
    n = 700
    if kind == "small":
        lengths = [float(1 + rng.integers(0, 2000) / 7.0) for _ in range(n)]
    elif kind == "halves":
        lengths = [float(1 + rng.integers(0, 40) / 2.0) for _ in range(n)]
    elif kind == "large":
        lengths = [float(2 ** 24 + rng.integers(0, 1 << 20) + rng.random()) for _ in range(n)]
    else:
        lengths = [float(2 ** 25 + 0.75) if i % 97 == 5 else float(1 + rng.integers(0, 300) / 3.0) for i in range(n)]
    assert producer(lengths) == exact(lengths)


def fixed_step_search(ends, r):
    L = 0
    step = 32
    while step:
        if ends[L + step - 1] < r:
            L += step
        step >>= 1
    return L


def test_fixed_step_search_equals_lower_bound():
    rng = np.random.default_rng(3)
    for _ in range(3000):
        cnt = int(rng.integers(1, 65))
        lo = int(rng.integers(0, 1000))
        ends = list(lo + np.cumsum(rng.choice([0, 0, 1, 1, 2, 3, 7, 50], size=cnt)))
        hi = ends[-1]
        padded = ends + [hi] * (64 - cnt)
        for r in range(lo + 1, hi + 1):
            assert fixed_step_search(padded, r) == bisect.bisect_left(ends, r)
