"""Host model of the one-lane compression kernel's grouped piece stores.

A lane emits a domain's pieces at staging indices obase, obase + 1, ...;
each piece goes into register slot idx & 3 of a group of four aligned to
the staging index.  A group is written when its slot 3 is filled or the
domain ends: as one 16-byte vector store of lengths (and two of increments)
when the whole group belongs to the domain, else slot by slot from the
domain's first slot in the group (obase & 3 for its first group, 0 after).
The model follows those steps, with the group registers carried over from
one domain to the next as the kernel keeps them, and checks that every
index of every domain is written exactly once, with its own piece, and that
nothing outside the domains' pieces is written.
"""
import numpy as np
import pytest


def run_lane(domains):
    """domains: [(obase, pieces)] in the order one lane takes them."""
    writes = {}
    vector_groups = 0
    g = [None] * 4           # the group registers, never cleared
    for obase, vals in domains:
        gfirst = obase & 3
        for j, v in enumerate(vals):
            idx = obase + j
            slot = idx & 3
            g[slot] = v
            last = j == len(vals) - 1
            if slot == 3 or last:
                g0 = idx - slot
                if gfirst == 0 and slot == 3:
                    assert g0 % 4 == 0
                    vector_groups += 1
                    span = range(0, 4)
                else:
                    span = range(gfirst, slot + 1)
                for u in span:
                    writes.setdefault(g0 + u, []).append(g[u])
                gfirst = 0
    return writes, vector_groups


@pytest.mark.parametrize("seed", range(6))
def test_every_piece_written_once(seed):
    rng = np.random.default_rng(seed)
    # domains of 1..40 intervals laid end to end; a domain of n intervals
    # holds between 1 and n pieces at the start of its staging range
    starts, sizes = [], []
    pos = int(rng.integers(0, 4))
    for _ in range(400):
        n = int(rng.integers(1, 41))
        starts.append(pos)
        sizes.append(n)
        pos += n
    order = rng.permutation(len(starts))  # the queue hands domains to the lane in any order
    expect = {}
    domains = []
    for d in order:
        npieces = int(rng.integers(1, sizes[d] + 1))
        vals = [(int(d), j) for j in range(npieces)]
        domains.append((starts[d], vals))
        for j, v in enumerate(vals):
            expect[starts[d] + j] = v
    writes, vector_groups = run_lane(domains)
    assert set(writes) == set(expect)
    for idx, ws in writes.items():
        assert ws == [expect[idx]], (idx, ws, expect[idx])
    assert vector_groups > 0


def test_single_piece_domains_at_every_alignment():
    for a in range(4):
        writes, _ = run_lane([(8 + a, ["x"]), (20 + a, ["y", "z"])])
        assert writes == {8 + a: ["x"], 20 + a: ["y"], 21 + a: ["z"]}
