#!/usr/bin/env python3
"""Throughput of the joint symbolic approximation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload scale]

One step is one pass of the whole path over one batch of synthetic series
that is already resident in HBM:
    compress (Phase I + II) -> two-stage digitize (Phase III: scaling, sort,
    blocks, Stage I, Stage II, label propagation, dictionary) -> encode the
    batch's pieces against a resident dictionary (built once from the
    16 x 1,000 random-walk workload, the serving configuration) ->
    reconstruct the batch (quantization + inverse compression + MSE).
`value` is input points per second of that step.  The JSON line also
carries the symbolization-only rate (compress + digitize), the batched vs
one-launch-per-series compression comparison, the roofline of the dominant
kernel (timed with HIP events on its launch stream) and the CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2401_00109_amd.rocprof_summary import source_hash  # noqa: E402

METRIC = "points symbolized/sec, batched vs per-domain launch; %HBM peak; p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOAD_IDS = {"tiny": 1, "scale": 2, "uneven": 3, "multivar": 4}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic bytes each kernel must move per launch (the data a kernel has
# to read and write at least, whatever its implementation): n = input
# points, N = pieces, G = Stage I starting points, k = symbols,
# nh = reconstructed points.  Only kernels that can be the dominant one are
# listed.
def algorithmic_bytes(name: str, n, N, G, k, nh, sort_bytes, sort_launches):
    if name.startswith("k_compress"):
        return 8.0 * n + 12.0 * N          # read every point once, write (len, inc)
    if name == "k_onesweep":
        # per pair, summed over the active passes: key (8 B, or 4 B once the
        # digits left fit) and value in; key and value out, the value alone
        # in the last pass
        return float(sort_bytes) * N / max(sort_launches, 1)
    if name == "k_stage1":
        return 32.0 * N + 8.0 * G          # sorted key, x, y in; label, flag out; start tags, list
    if name == "k_block_sums":
        return 20.0 * N + 24.0 * G         # label, start index, len, inc in; sums out
    if name == "k_col_greedy":
        return 56.0 * G
    if name == "k_gather":
        return 60.0 * N                    # perm, random 16-byte record in; 6 sorted arrays out
    if name == "k_key":
        return 40.0 * N                    # len, inc in; key, index, record out
    if name == "k_encode" or name.startswith("k_encode<"):
        return 16.0 * N
    if name == "k_recon":                 # symbols, lhat; output points written, originals read for the SSE
        return 12.0 * N + 16.0 * nh
    if name == "k_remap":
        return 24.0 * N
    if name == "k_compact":
        return 24.0 * N
    if name.startswith("k_sum_leaves"):
        return 12.0 * N
    if name == "k_global_hist":
        return 8.0 * N
    return None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scale", choices=sorted(WORKLOAD_IDS))
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the workload's series (tests only)")
    ap.add_argument("--cpu-sample-series", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop latency measurement")
    ap.add_argument("--serving-requests", type=int, default=300)
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph replay (profiler runs)")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="also run a plain 1 GiB copy kernel (for rocprofv3 counter scaling)")
    ap.add_argument("--tuning", default=None, help="JSON dict of jabba_tuning fields")
    ap.add_argument("--pipeline", type=int, default=0,
                    help="buffer sets in flight (one stream each); 0 = 3 up to 2e8 points, else 1")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the library and its benchmark run on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        log("only --gpus 1 is supported: the library and its benchmark are single-GPU")
        return 2

    import torch

    import paper_2401_00109_amd as J
    from paper_2401_00109_amd.inputs import make_workload

    if not torch.cuda.is_available():
        log("no GPU visible")
        return 1
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    tuning = json.loads(args.tuning) if args.tuning else None

    wid = WORKLOAD_IDS[args.workload]
    t = time.time()
    w = make_workload(wid, seed=0, scale=args.scale)
    log(f"workload {w.name}: {w.n_series} series, {w.n_points} points, D={w.D} tol={w.tol} alpha={w.alpha} "
        f"B={w.B} (generated in {time.time() - t:.1f}s)")
    v = torch.from_numpy(w.values).to(dev)
    so = torch.from_numpy(w.series_off).to(dev)
    t0 = torch.from_numpy(np.where(np.diff(w.series_off) > 0, w.values[np.minimum(w.series_off[:-1],
                                                                                  max(w.n_points - 1, 0))],
                                   0.0)).to(dev)

    # resident serving dictionary: built once from the 16 x 1,000 random walks
    from paper_2401_00109_amd.serve import build_resident_dictionary
    w1 = make_workload(1, seed=0)
    resident = build_resident_dictionary(dev)
    log(f"resident dictionary: k={resident.size()}")

    # size the digitize buffers from the actual piece count (one warm-up compress)
    probe = J.compress(v, so, w.D, w.tol, w.max_len, tuning=tuning)
    torch.cuda.synchronize()
    N = probe.count()
    del probe
    # One step = compress, encode against the resident dictionary, digitize,
    # reconstruct, for one batch.  Consecutive steps go to consecutive buffer
    # sets, one stream each, so one batch's compression (a few wavefronts per
    # compute unit) overlaps the others' digitization and reconstruction;
    # every step still does all of its work.  Three streams plus the default
    # one fill the process's four hardware queues; a fourth set in flight
    # measured slower than three.
    from paper_2401_00109_amd.pipeline import Pipeline
    n_sets = args.pipeline if args.pipeline > 0 else (3 if w.n_points <= 200_000_000 else 1)
    pipe = Pipeline(v, so, t0, w.D, w.tol, w.alpha, w.scl, w.B, N, resident, n_sets=n_sets, tuning=tuning,
                    max_len=w.max_len)
    sets = pipe.sets
    S0 = sets[0]
    sz, full, enc, rec = S0.sz, S0.pieces, S0.enc, S0.rec

    def step_sym():
        sz.compress(v, so)
        sz.digitize()

    def run_steps(n, pipelined=True):
        pipe.run(n, pipelined=pipelined)

    run_steps(max(args.warmup, 1) * len(sets))
    torch.cuda.synchronize()
    st = sz.status()
    if st != (0, 0):
        log(f"device status {st}")
        return 1
    k = sz.dictionary.size()
    stats = sz.stats()
    G, active_passes, sort_bytes = stats["G"], stats["sort_passes"], stats["sort_bytes"]
    groups2 = stats["stage2_groups"]
    log(f"N={N} pieces, G={G} starting points, k={k} symbols, {active_passes} radix passes ({sort_bytes} B per piece), "
        f"{groups2} Stage II groups, reconstruction MSE={rec.mse():.4e}")

    # ---------------------------------------------------------------- timed region
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    run_steps(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = w.n_points / (ms_step / 1e3)
    for S in sets[1:]:
        assert torch.equal(S.sz.symbols[:N], sz.symbols[:N]) and torch.equal(S.enc[:N], enc[:N]), \
            "buffer sets disagree"
        assert S.sz.status() == (0, 0)
    ev0.record()
    run_steps(args.steps, pipelined=False)
    ev1.record()
    torch.cuda.synchronize()
    ms_serial = ev0.elapsed_time(ev1) / args.steps
    log(f"full step {ms_step:.3f} ms with {len(sets)} buffer set(s) in flight -> {value:.4e} points/s "
        f"(one batch at a time: {ms_serial:.3f} ms)")

    # symbolization only (compress + digitize), eager and as one graph replay
    ev0.record()
    for _ in range(args.steps):
        step_sym()
    ev1.record()
    torch.cuda.synchronize()
    ms_sym = ev0.elapsed_time(ev1) / args.steps
    plan = J.Plan(v, so, w.D, w.tol, w.alpha, w.scl, w.B, max_pieces=max(w.n_points, 1), capacity=max(N, 1),
                  tuning=tuning) if (w.n_points <= 200_000_000 and not args.no_graph) else None
    ms_graph = None
    if plan is not None:
        plan.run()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            plan.run()
        ev1.record()
        torch.cuda.synchronize()
        ms_graph = ev0.elapsed_time(ev1) / args.steps
        assert plan.status() == (0, 0)
        assert torch.equal(plan.symbols[:N], sz.symbols[:N]), "graph replay differs from eager"
        plan.close()
        del plan
    log(f"symbolize {ms_sym:.3f} ms eager, graph {ms_graph if ms_graph is None else round(ms_graph, 3)} ms")

    # ---------------------------------------------------------------- per-kernel events
    # The roofline is taken one batch at a time, so a kernel's duration is its
    # own (with batches in flight a kernel shares the device with the other
    # batch's kernels; those durations are reported beside it).
    def kernel_times(pipelined):
        J.timing_enable(True)
        run_steps(args.steps, pipelined=pipelined)
        torch.cuda.synchronize()
        rep = J.timing_report()
        J.timing_enable(False)
        return rep

    def roofline_of(rep):
        name = max(rep, key=lambda n: rep[n][0])
        ms, launches = rep[name]
        sort_launches = rep.get("k_onesweep", (0, 1))[1] / args.steps
        alg = algorithmic_bytes(name, w.n_points, N, G, k, n_hat, sort_bytes, sort_launches)
        if alg is None or launches <= 0:
            return None
        avg_ms = ms / launches
        achieved = alg / (avg_ms / 1e3) / 1e9
        return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(name),
                "algorithmic_bytes_per_launch": alg, "avg_launch_ms": round(avg_ms, 5)}

    n_hat = int(rec.out_off[-1].item())
    rep = kernel_times(False)
    per_step = {n: (ms / args.steps, cnt / args.steps) for n, (ms, cnt) in rep.items()}
    roofline = roofline_of(rep)
    top = sorted(per_step.items(), key=lambda kv: -kv[1][0])[:12]
    log("per-step kernel time (one batch at a time): " + ", ".join(f"{n} {ms:.3f}ms" for n, (ms, _) in top))
    in_flight = None
    if len(sets) > 1:
        rf = roofline_of(kernel_times(True))
        if rf is not None:
            in_flight = {"kernel": rf["kernel"], "avg_launch_ms": rf["avg_launch_ms"], "achieved": rf["achieved"],
                         "frac": rf["frac"]}
            log(f"with {len(sets)} batches in flight {rf['kernel']} averages {rf['avg_launch_ms']:.4f} ms per launch")

    # ---------------------------------------------------------------- batched vs plain launches
    plain = None
    if not args.no_plain:
        pp = J.Pieces(torch.empty(max(w.n_points, 1), dtype=torch.int32, device=dev),
                      torch.empty(max(w.n_points, 1), dtype=torch.float64, device=dev),
                      torch.empty(w.n_series + 1, dtype=torch.int64, device=dev),
                      torch.empty(1, dtype=torch.int64, device=dev), max(w.n_points, 1))
        pws = sz.cws
        J.compress_plain(v, so, w.series_off, w.D, w.tol, w.max_len, out=pp, workspace=pws)
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        ev0.record()
        for _ in range(reps):
            J.compress_plain(v, so, w.series_off, w.D, w.tol, w.max_len, out=pp, workspace=pws)
        ev1.record()
        torch.cuda.synchronize()
        ms_plain = ev0.elapsed_time(ev1) / reps
        ev0.record()
        for _ in range(reps):
            sz.compress(v, so)
        ev1.record()
        torch.cuda.synchronize()
        ms_batched = ev0.elapsed_time(ev1) / reps
        same = torch.equal(pp.len[:N], full.len[:N]) and torch.equal(pp.inc[:N], full.inc[:N])
        plain = {"compress_plain_ms": round(ms_plain, 3), "compress_batched_ms": round(ms_batched, 3),
                 "batched_speedup": round(ms_plain / ms_batched, 2), "plain_launches": int(w.n_series),
                 "identical_outputs": bool(same)}
        log(f"compress: plain {ms_plain:.3f} ms ({w.n_series} launches) vs batched {ms_batched:.3f} ms")

    # ---------------------------------------------------------------- digitization quality (not in the step)
    step_sym()
    ev0.record()
    q = sz.quality()
    ev1.record()
    torch.cuda.synchronize()
    qt = q["totals"].cpu().tolist()
    quality = {"sse": qt[0], "max_var_len": qt[1], "max_var_inc": qt[2], "alpha_sq": w.alpha ** 2,
               "sse_bound_two_stage": 4 * w.alpha ** 2 * (N - k), "quality_ms": round(ev0.elapsed_time(ev1), 3)}
    log(f"quality: SSE {qt[0]:.6e} (two-stage bound {quality['sse_bound_two_stage']:.3e}), "
        f"max Var_len {qt[1]:.3e}, max Var_inc {qt[2]:.3e} (alpha^2 {w.alpha ** 2:.3e}), "
        f"{quality['quality_ms']} ms")

    # ---------------------------------------------------------------- pmc calibration copy
    if args.pmc_calibrate:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log("calibration copy kernel: 3 x neg over 1 GiB (read 1 GiB, write 1 GiB per launch)")

    # ---------------------------------------------------------------- serving latency (not in the step)
    # The metric's p99 part: the serving loop with the same resident
    # dictionary, saturation from a closed loop, then Poisson arrivals at half
    # of it; latency is arrival to symbols on the host (H2D and D2H included).
    serving = None
    if not args.no_serving:
        from paper_2401_00109_amd.inputs import request_stream
        from paper_2401_00109_amd.serve import Server, summarize
        srv = Server(resident, slots=4, max_series=256, device=dev)
        srv.run(request_stream(1, 20, 0.0, max_series=256, first_id=10_000_000), realtime=False)
        closed = request_stream(2, args.serving_requests, 0.0, max_series=256, first_id=20_000_000)
        t = time.perf_counter()
        res = srv.run(closed, realtime=False)
        sat = len(res) / (time.perf_counter() - t)
        reqs = request_stream(3, args.serving_requests, 0.5 * sat, max_series=256, first_id=30_000_000)
        t = time.perf_counter()
        res = srv.run(reqs, realtime=True)
        sm = summarize(res, time.perf_counter() - t)
        serving = {"saturation_req_per_s": round(sat, 1), "rate_req_per_s": round(0.5 * sat, 1),
                   "requests": sm["requests"], "p50_ms": round(sm["p50_ms"], 3), "p99_ms": round(sm["p99_ms"], 3),
                   "points_per_s": round(sm["points_per_s"], 1),
                   "requests_shape": "1-256 random walks of 500-50,000 points, four slots",
                   "latency": "arrival to symbols on the host, H2D and D2H included"}
        log(f"serving: saturation {sat:.0f} req/s; at half of it p50 {sm['p50_ms']:.2f} ms, "
            f"p99 {sm['p99_ms']:.2f} ms")
        del srv

    # ---------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(w, w1, args.cpu_sample_series)
        log(f"cpu oracle: {cpu['value']:.4e} points/s on {cpu['sample']}")

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_one_batch_at_a_time": round(ms_serial, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n_series} series x {w.n_points // max(w.n_series, 1)} points "
                               f"(3-way random walk / sinusoid / piecewise-linear mix), {w.D}-interval domains, "
                               f"tol={w.tol}, alpha={w.alpha}, B={w.B}",
                   "points": w.n_points, "pieces": N, "symbols": k, "starting_points": G,
                   "stage2_groups": groups2,
                   "step": "compress+digitize+encode(resident k=%d)+reconstruct" % resident.size(),
                   "batches_in_flight": len(sets)},
        "symbolize_points_per_s": round(w.n_points / (ms_sym / 1e3), 1),
        "symbolize_ms": round(ms_sym, 4),
        "symbolize_graph_ms": None if ms_graph is None else round(ms_graph, 4),
        "kernel_ms_per_step": {n: round(ms, 4) for n, (ms, _) in top},
        "roofline": roofline,
        "dominant_kernel_with_batches_in_flight": in_flight,
        "batched_vs_plain": plain,
        "serving": serving,
        "cpu_baseline": cpu,
        "reconstruction_mse": rec.mse(),
        "digitization_quality": quality,
        "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)
    return 0


def _traffic(kernel: str):
    """Measured HBM bytes per launch from the committed counter summary, if the
    kernel sources have not changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except Exception:
        return None
    if t.get("source_hash") != source_hash():
        return None
    e = t.get("kernels", {}).get(kernel)
    return None if e is None else e.get("bytes_per_launch")


def _cpu_baseline(w, w1, n_sample: int):
    """The oracle, single-threaded, over one in (n_series / n_sample) series
    (all of them when n_sample covers the workload)."""
    import oracle as O
    from paper_2401_00109_amd.inputs import pack
    stride = max(1, w.n_series // max(n_sample, 1))
    idx = np.arange(0, w.n_series, stride)[:n_sample]
    ser = [w.values[w.series_off[i]:w.series_off[i + 1]] for i in idx]
    vals, off = pack(ser)
    l1, i1, _ = O.compress(w1.values, w1.series_off, w1.D, w1.tol)
    d1 = O.digitize(l1, i1, w1.alpha, w1.scl, w1.B)
    t = time.perf_counter()
    ln, inc, po = O.compress(vals, off, w.D, w.tol)
    d = O.digitize(ln, inc, w.alpha, w.scl, w.B)
    O.encode(ln, inc, d1.sigma_len, d1.sigma_inc, d1.scl, d1.cx, d1.cy)
    t0 = np.where(np.diff(off) > 0, vals[np.minimum(off[:-1], max(vals.size - 1, 0))], 0.0)
    O.reconstruct(d.symbols, po, off, t0, d.center_len, d.center_inc, orig=vals)
    el = time.perf_counter() - t
    return {"value": round(vals.size / el, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": (f"all {w.n_series} series" if idx.size == w.n_series else
                       f"{idx.size} of {w.n_series} series (one in {stride})") +
                      f", {vals.size} points, same step: compress+digitize+encode+reconstruct, {el:.1f} s"}


if __name__ == "__main__":
    sys.exit(main())
