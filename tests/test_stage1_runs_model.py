"""Host model of how the aggregation kernels resolve a batch of 64 sorted
points that no active start covers (Stage I and Stage II, pull form).

The sequential greedy (Sec. 3.2, as Sec. 5 runs it inside a block) takes the
points in key order: a point joins the first earlier start that covers it,
else it becomes a start.  The kernel first tests each point of a batch
against the active starts of earlier batches; the points left open are then
resolved in runs: a key more than alpha above the previous point's starts a
new run (keys ascend, so no point reaches across the gap), every run takes
its first open point as a start at each step, that start covers the later
points of its run, and the batch's new starts join the active list in
position order afterwards.  The model follows those steps and is checked
against the plain sequential greedy on clustered, sparse and tie-heavy
points.
"""
import numpy as np
import pytest


def covers(q, p, k, x, y, a):
    return (k[q] - k[p] <= a) and ((x[q] - x[p]) ** 2 + (y[q] - y[p]) ** 2 <= a * a)


def sequential(k, x, y, a):
    owner, starts = [-1] * len(k), []
    for q in range(len(k)):
        for p in starts:
            if covers(q, p, k, x, y, a):
                owner[q] = p
                break
        else:
            owner[q] = q
            starts.append(q)
    return owner


def batched_runs(k, x, y, a, width=64):
    n = len(k)
    owner, active = [-1] * n, []
    for b0 in range(0, n, width):
        lanes = list(range(b0, min(b0 + width, n)))
        is_open = {}
        for q in lanes:  # against the active starts, oldest first
            owner[q] = next((p for p in active if covers(q, p, k, x, y, a)), -1)
            is_open[q] = owner[q] < 0
        head = {}
        for i, q in enumerate(lanes):
            new_run = i == 0 or not (k[q] - k[lanes[i - 1]] <= a)
            head[q] = q if new_run else head[lanes[i - 1]]
        new_starts = []
        pend = [q for q in lanes if is_open[q]]
        while pend:
            first = {q for q in pend if not any(head[q] <= p < q for p in pend)}
            step_start = {q: min(p for p in pend if p >= head[q]) for q in pend}
            for q in pend:
                if q in first:
                    owner[q] = q
                    is_open[q] = False
                    new_starts.append(q)
                elif covers(q, step_start[q], k, x, y, a):
                    owner[q] = step_start[q]
                    is_open[q] = False
            pend = [q for q in lanes if is_open[q]]
        active.extend(sorted(new_starts))
    return owner


@pytest.mark.parametrize("kind", ["clustered", "sparse", "ties", "mixed"])
def test_run_resolution_equals_sequential_greedy(kind):
    rng = np.random.default_rng(["clustered", "sparse", "ties", "mixed"].index(kind))
    a = 0.05
    for _ in range(40):
        n = int(rng.integers(1, 300))
        if kind == "clustered":
            pts = rng.normal(size=(n, 2)) * 0.1
        elif kind == "sparse":
            pts = rng.normal(size=(n, 2)) * 3.0
        elif kind == "ties":
            pts = np.round(rng.normal(size=(n, 2)) * 0.3, 2)
        else:
            pts = np.concatenate([rng.normal(size=(n // 2, 2)) * 0.05, rng.normal(size=(n - n // 2, 2)) * 2.0])
        key = np.hypot(pts[:, 0], pts[:, 1])
        order = np.lexsort((np.arange(n), key))
        k, x, y = key[order], pts[order, 0], pts[order, 1]
        assert batched_runs(k, x, y, a) == sequential(k, x, y, a)
