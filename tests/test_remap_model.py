"""Host model of the label propagation for large piece counts.

The pairs (canonical index << sh, symbol) are grouped by their two highest
radix digits; the kernels take the digit histograms from a closed form
instead of counting (k_remap_hist), and then scatter each window of
2^(bits - 16) consecutive indices in LDS (k_remap_window), relying on the
window's pairs sitting exactly at the window's own positions.  Both claims are
checked here against brute force: the closed form (transcribed from the
kernel) against a histogram of the actual keys, and the window property
against a stable sort of a random permutation by the same digits.
"""
import numpy as np
import pytest


def remap_hist(n, sh):
    """The kernel's closed form for the digit histograms of {i << sh : i < n}."""
    H = np.zeros((8, 256), np.uint64)
    for d in range(8):
        a = 8 * d - sh
        for b in range(256):
            if a >= 0:
                full = a + 8 >= 64
                S = 1 << a
                P = 0 if full else S << 8
                cycles = 0 if full else n // P
                rem = n if full else n % P
                lo = b * S
                part = (min(rem - lo, S) if rem > lo else 0)
                cnt = cycles * S + part
            elif a > -8:
                P = 1 << (8 + a)
                step = 1 << (-a)
                cnt = 0 if b % step else n // P + (1 if (b // step) < n % P else 0)
            else:
                cnt = n if b == 0 else 0
            H[d, b] = cnt
    return H


def shift_for(n):
    bits = 1
    while bits < 31 and (1 << bits) < n:
        bits += 1
    return bits, 32 - bits


@pytest.mark.parametrize("n,sh", [(1, 0), (1000, 0), (1000, 3), (70_000, 5), (123_457, 7), (5, 1), (300_000, 2),
                                  (1 << 17, 4), ((1 << 17) + 1, 3), (1000, 22), (3, 30)])
def test_closed_form_histogram_matches_counts(n, sh):
    keys = np.arange(n, dtype=np.uint64) << np.uint64(sh)
    brute = np.zeros((8, 256), np.uint64)
    for d in range(8):
        brute[d] = np.bincount(((keys >> np.uint64(8 * d)) & np.uint64(255)).astype(np.int64), minlength=256)
    np.testing.assert_array_equal(remap_hist(n, sh), brute)


def top_two_digit_order(keys, hist):
    """Stable order by the two highest digits that are not constant (the
    radix plan skips constant digits and sorts the top prefix)."""
    active = [d for d in range(8) if np.count_nonzero(hist[d]) > 1]
    used = sorted(active)[-2:]
    order = np.arange(keys.size)
    for d in used:  # LSD over the chosen digits, stable
        dig = (keys[order] >> np.uint64(8 * d)) & np.uint64(255)
        order = order[np.argsort(dig, kind="stable")]
    return order


@pytest.mark.parametrize("n", [(1 << 17) + 12_345, 1 << 18, 3_000_001, 1000])
def test_windows_hold_their_own_indices(n):
    rng = np.random.default_rng(n)
    bits, sh = shift_for(n)
    wlog = max(bits - 16, 0)
    perm = rng.permutation(n).astype(np.uint64)      # canonical index of each sorted position
    keys = perm << np.uint64(sh)
    order = top_two_digit_order(keys, remap_hist(n, sh))
    grouped = (keys[order] >> np.uint64(sh)).astype(np.int64)
    W = 1 << wlog
    for w0 in range(0, n, W):
        m = min(W, n - w0)
        win = grouped[w0:w0 + m]
        assert win.min() >= w0 and win.max() < w0 + m
        assert np.unique(win).size == m          # every slot of the window written once
