#!/usr/bin/env python3
"""Throughput of the joint symbolic approximation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload uneven]

One step is one pass of the whole path over one batch of synthetic series
that is already resident in HBM:
    compress (Phase I + II) -> two-stage digitize (Phase III: scaling, sort,
    blocks, Stage I, Stage II, label propagation, dictionary) -> encode the
    batch's pieces against a resident dictionary (built once from the
    16 x 1,000 random-walk workload, the serving configuration) ->
    reconstruct the batch (quantization + inverse compression + MSE).
The headline workload is the uneven one: 50,000 series of log-uniform length
in [100, 100,000] (7.2e8 points), 2,000-interval domains.  `value` is input
points per second of that step.  The JSON line also carries:
  * the path's roofline: the algorithmic bytes of the step over its time,
    against the 8 TB/s HBM peak, and the dominant kernel's roofline (timed
    with HIP events on its launch stream);
  * compress + digitize alone, eager and as one captured-graph replay;
  * batched (one persistent launch, length-ordered queue) against plain
    launches: one launch per series over the whole workload, and one launch
    per domain timed on a sample of series and scaled to all domains;
  * the serving loop at three arrival rates (p50, p99, points/s);
  * the CPU oracle on a sample of the same workload, one core, and its
    compression over all host cores (speed-up and efficiency);
  * the 4,096 x 10,000 workload as a second line item.
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
WORKLOAD_TEXT = {
    1: "16 random walks x 1,000 points, one domain per series",
    2: "4,096 series x 10,000 points (3-way random walk / sinusoid / piecewise-linear mix), 1,000-interval domains",
    3: "50,000 series of log-uniform length in [100, 100,000] (3-way random walk / sinusoid / piecewise-linear "
       "mix), 2,000-interval domains",
    4: "1,024 samples x 64 correlated channels x 5,000 points, one domain per channel, one joint dictionary",
}


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
    if name == "k_bucket_local":
        return 60.0 * N                    # index, its 16-byte record in; 6 sorted arrays (40 B) out
    if name == "k_key":
        return 40.0 * N                    # len, inc in; key, index, record out
    if name == "k_encode" or name.startswith("k_encode<"):
        return 16.0 * N
    if name == "k_recon":                 # symbols, lhat; output points written, originals read for the SSE
        return 12.0 * N + 16.0 * nh
    if name == "k_remap":
        return 24.0 * N                    # index, local start, start map in; symbol scattered out
    if name == "k_remap_scatter":
        return 16.0 * N                    # (index, symbol) pairs in; symbol out
    if name == "k_remap_pairs":
        return 24.0 * N                    # index, local start in; (index, symbol) pairs out
    if name == "k_compact":
        return 24.0 * N
    if name.startswith("k_sum_leaves"):
        return 12.0 * N
    if name == "k_global_hist":
        return 8.0 * N
    return None


def path_bytes(n: int, N: int) -> float:
    """Algorithmic bytes of one step: compress 8n + 12N (points in, pieces
    out); digitize 12N + 4N (pieces in, symbols out); encode 12N + 4N;
    reconstruct 4N + 8n (symbols in, points out)."""
    return 16.0 * n + 48.0 * N


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uneven", choices=sorted(WORKLOAD_IDS))
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the workload's series (tests only)")
    ap.add_argument("--secondary", default="scale", help="second workload reported beside the headline ('' = none)")
    ap.add_argument("--cpu-sample-points", type=float, default=5e7,
                    help="points of the oracle's timed sample (whole series, evenly spaced)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-domain-sample", type=int, default=64,
                    help="one-launch-per-domain leg: one series in this many")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop latency measurement")
    ap.add_argument("--serving-requests", type=int, default=2000, help="measured requests per arrival rate")
    ap.add_argument("--serving-pool", type=int, default=256, help="distinct request bodies the stream cycles over")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph replay (profiler runs)")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="also run a plain 1 GiB copy kernel (for rocprofv3 counter scaling)")
    ap.add_argument("--tuning", default=None, help="JSON dict of jabba_tuning fields")
    ap.add_argument("--pipeline", type=int, default=0,
                    help="buffer sets in flight (one stream each); 0 = 3 up to 2e8 points, else 2 (fewer when "
                         "device memory runs out)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the library and its benchmark run on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        log("only --gpus 1 is supported: the library and its benchmark are single-GPU")
        return 2

    import torch

    from paper_2401_00109_amd.inputs import make_workload
    from paper_2401_00109_amd.serve import build_resident_dictionary

    if not torch.cuda.is_available():
        log("no GPU visible")
        return 1
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    tuning = json.loads(args.tuning) if args.tuning else None

    # resident serving dictionary: built once from the 16 x 1,000 random walks
    resident = build_resident_dictionary(dev)
    log(f"resident dictionary: k={resident.size()}")

    wid = WORKLOAD_IDS[args.workload]
    t = time.time()
    w = make_workload(wid, seed=0, scale=args.scale)
    log(f"workload {w.name}: {w.n_series} series, {w.n_points} points, D={w.D} tol={w.tol} alpha={w.alpha} "
        f"B={w.B} (generated in {time.time() - t:.1f}s)")
    head = measure(w, dev, resident, args, tuning, primary=True)

    secondary = None
    if args.secondary and args.secondary != args.workload:
        torch.cuda.empty_cache()
        w2 = make_workload(WORKLOAD_IDS[args.secondary], seed=0)
        log(f"secondary workload {w2.name}: {w2.n_series} series, {w2.n_points} points")
        sec = measure(w2, dev, resident, args, tuning, primary=False)
        secondary = {"workload": f"{w2.name}: {WORKLOAD_TEXT[w2.workload_id]}, tol={w2.tol}, alpha={w2.alpha}, "
                                 f"B={w2.B}",
                     "value": sec["value"], "unit": "points/s", "ms_per_step": sec["ms_per_step"],
                     "ms_per_step_one_batch_at_a_time": sec["ms_serial"], "batches_in_flight": sec["n_sets"],
                     "points": w2.n_points, "pieces": sec["N"], "symbols": sec["k"],
                     "symbolize_ms": sec["symbolize_ms"], "symbolize_graph_ms": sec["graph_ms"],
                     "path_roofline": sec["path_roofline"], "roofline": sec["roofline"],
                     "kernel_ms_per_step": sec["kernel_ms_per_step"]}
        del w2

    serving = None if args.no_serving else serving_leg(resident, dev, args)
    copy = copy_ceiling(dev)
    log(f"copy ceiling: {copy['achieved']:.0f} GB/s ({100 * copy['frac']:.1f} % of {HBM_PEAK_GBS:.0f})")

    cpu = None
    if not args.no_cpu_baseline:
        w1 = make_workload(1, seed=0)
        cpu = cpu_baseline(w, w1, args.cpu_sample_points)
        log(f"cpu oracle: {cpu['value']:.4e} points/s ({cpu['cores']} core) on {cpu['sample']}; compression over "
            f"{cpu['all_cores']['threads']} threads: speed-up {cpu['all_cores']['speedup']:.2f}, efficiency "
            f"{cpu['all_cores']['efficiency']:.2f}")

    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_one_batch_at_a_time": head["ms_serial"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {WORKLOAD_TEXT[w.workload_id]}, tol={w.tol}, alpha={w.alpha}, B={w.B}",
                   "points": w.n_points, "series": w.n_series, "pieces": head["N"], "symbols": head["k"],
                   "starting_points": head["G"], "stage2_groups": head["groups2"],
                   "step": "compress+digitize+encode(resident k=%d)+reconstruct" % resident.size(),
                   "batches_in_flight": head["n_sets"]},
        "path_roofline": head["path_roofline"],
        "roofline": head["roofline"],
        "copy_ceiling": copy,
        "dominant_kernel_with_batches_in_flight": head["in_flight"],
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "symbolize_points_per_s": head["symbolize_points_per_s"],
        "symbolize_ms": head["symbolize_ms"],
        "symbolize_graph_ms": head["graph_ms"],
        "graph_tuning": head["graph_tuning"],
        "batched_vs_plain": head["plain"],
        "serving": serving,
        "cpu_baseline": cpu,
        "reconstruction_mse": head["mse"],
        "digitization_quality": head["quality"],
        "secondary": secondary,
        "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)
    return 0


def measure(w, dev, resident, args, tuning, primary: bool) -> dict:
    """Time the full step on workload w; the primary workload also gets the
    plain-launch comparison and the quality figures."""
    import torch

    import paper_2401_00109_amd as J
    from paper_2401_00109_amd.pipeline import Pipeline

    v = torch.from_numpy(w.values).to(dev)
    so = torch.from_numpy(w.series_off).to(dev)
    t0 = torch.from_numpy(np.where(np.diff(w.series_off) > 0, w.values[np.minimum(w.series_off[:-1],
                                                                                  max(w.n_points - 1, 0))],
                                   0.0)).to(dev)
    # size the digitize buffers from the actual piece count (one warm-up compress)
    probe = J.compress(v, so, w.D, w.tol, w.max_len, tuning=tuning)
    torch.cuda.synchronize()
    N = probe.count()
    del probe
    torch.cuda.empty_cache()
    # One step = compress, encode against the resident dictionary, digitize,
    # reconstruct, for one batch.  Consecutive steps go to consecutive buffer
    # sets, one stream each, so one batch's compression overlaps the others'
    # digitization and reconstruction; every step still does all of its work.
    n_sets = args.pipeline if args.pipeline > 0 else (3 if w.n_points <= 200_000_000 else 2)
    while True:
        try:
            pipe = Pipeline(v, so, t0, w.D, w.tol, w.alpha, w.scl, w.B, N, resident, n_sets=n_sets, tuning=tuning,
                            max_len=w.max_len)
            break
        except torch.OutOfMemoryError:
            if n_sets == 1:
                raise
            pipe = None
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            log(f"{n_sets} buffer sets do not fit in device memory; trying {n_sets - 1}")
            n_sets -= 1
    sets = pipe.sets
    S0 = sets[0]
    sz, full, enc, rec = S0.sz, S0.pieces, S0.enc, S0.rec

    def run_steps(n, pipelined=True, overlap=True):
        pipe.run(n, pipelined=pipelined, overlap=overlap)

    run_steps(max(args.warmup, 1) * len(sets))
    torch.cuda.synchronize()
    st = sz.status()
    if st != (0, 0):
        raise RuntimeError(f"device status {st}")
    k = sz.dictionary.size()
    stats = sz.stats()
    G, active_passes, sort_bytes = stats["G"], stats["sort_passes"], stats["sort_bytes"]
    groups2 = stats["stage2_groups"]
    mse = rec.mse()
    log(f"N={N} pieces, G={G} starting points, k={k} symbols, {active_passes} radix passes ({sort_bytes} B per piece), "
        f"{groups2} Stage II groups, reconstruction MSE={mse:.4e}")

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
    if len(sets) > 1:
        ev0.record()
        run_steps(args.steps, pipelined=False)
        ev1.record()
        torch.cuda.synchronize()
        ms_serial = ev0.elapsed_time(ev1) / args.steps
    else:
        ms_serial = ms_step
    pb = path_bytes(w.n_points, N)
    path_rf = {"bound": "hbm", "bytes_per_step": pb, "achieved": round(pb / (ms_step / 1e3) / 1e9, 2),
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(pb / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
               "bytes": "16 n + 48 N: compress 8n + 12N, digitize 16N, encode 16N, reconstruct 4N + 8n"}
    log(f"full step {ms_step:.3f} ms with {len(sets)} buffer set(s) in flight -> {value:.4e} points/s "
        f"(one batch at a time: {ms_serial:.3f} ms); path {path_rf['achieved']:.0f} GB/s = "
        f"{100 * path_rf['frac']:.1f} % of HBM peak")

    # symbolization only (compress + digitize), eager and as one graph replay
    ev0.record()
    for _ in range(args.steps):
        sz.run(v, so)
    ev1.record()
    torch.cuda.synchronize()
    ms_sym = ev0.elapsed_time(ev1) / args.steps
    ev0.record()
    for _ in range(args.steps):
        sz.compress(v, so)
    ev1.record()
    torch.cuda.synchronize()
    ms_comp = ev0.elapsed_time(ev1) / args.steps
    ms_graph, graph_tuning = None, None
    if not args.no_graph:
        plan = J.Plan.from_symbolizer(sz, v, so, tuning=tuning)
        graph_tuning = plan.tuning()
        plan.run()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            plan.run()
        ev1.record()
        torch.cuda.synchronize()
        ms_graph = ev0.elapsed_time(ev1) / args.steps
        assert plan.status() == (0, 0)
        ref = sz.symbols[:N].clone()
        sz.run(v, so)
        torch.cuda.synchronize()
        assert torch.equal(ref, sz.symbols[:N]), "graph replay differs from eager"
        plan.close()
        del plan
    log(f"symbolize {ms_sym:.3f} ms eager (compress {ms_comp:.3f} ms), graph "
        f"{ms_graph if ms_graph is None else round(ms_graph, 3)} ms (tuning {graph_tuning})")

    # ---------------------------------------------------------------- per-kernel events
    # The roofline is taken one batch at a time with each step's encoding on
    # the step's own stream, so a kernel's duration is its own (with batches
    # in flight a kernel shares the device with the other batch's kernels and
    # the encodings; those durations are reported beside it).
    def kernel_times(pipelined):
        J.timing_enable(True)
        run_steps(args.steps, pipelined=pipelined, overlap=pipelined)
        torch.cuda.synchronize()
        rep = J.timing_report()
        J.timing_enable(False)
        return rep

    n_hat = int(rec.out_off[-1].item())

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
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(name, w.name),
                "algorithmic_bytes_per_launch": alg, "avg_launch_ms": round(avg_ms, 5)}

    rep = kernel_times(False)
    per_step = {n: (ms / args.steps, cnt / args.steps) for n, (ms, cnt) in rep.items()}
    roofline = roofline_of(rep)
    top = sorted(per_step.items(), key=lambda kv: -kv[1][0])[:14]
    log("per-step kernel time (one batch at a time): " + ", ".join(f"{n} {ms:.3f}ms" for n, (ms, _) in top))
    in_flight = None
    if len(sets) > 1:
        rf = roofline_of(kernel_times(True))
        if rf is not None:
            in_flight = {"kernel": rf["kernel"], "avg_launch_ms": rf["avg_launch_ms"], "achieved": rf["achieved"],
                         "frac": rf["frac"]}
            log(f"with {len(sets)} batches in flight {rf['kernel']} averages {rf['avg_launch_ms']:.4f} ms per launch")

    out = {"value": round(value, 1), "ms_per_step": round(ms_step, 4), "ms_serial": round(ms_serial, 4),
           "n_sets": len(sets), "N": N, "k": k, "G": G, "groups2": groups2, "mse": mse,
           "path_roofline": path_rf, "roofline": roofline, "in_flight": in_flight,
           "kernel_ms_per_step": {n: round(ms, 4) for n, (ms, _) in top},
           "symbolize_points_per_s": round(w.n_points / (ms_sym / 1e3), 1), "symbolize_ms": round(ms_sym, 4),
           "graph_ms": None if ms_graph is None else round(ms_graph, 4), "graph_tuning": graph_tuning,
           "plain": None, "quality": None}
    if not primary:
        return out

    # ---------------------------------------------------------------- batched vs plain launches
    if not args.no_plain:
        out["plain"] = plain_leg(w, v, so, sz, full, N, ms_comp, ms_sym, ms_graph, args, dev)

    # ---------------------------------------------------------------- digitization quality (not in the step)
    sz.run(v, so)
    ev0.record()
    q = sz.quality()
    ev1.record()
    torch.cuda.synchronize()
    qt = q["totals"].cpu().tolist()
    out["quality"] = {"sse": qt[0], "max_var_len": qt[1], "max_var_inc": qt[2], "alpha_sq": w.alpha ** 2,
                      "sse_bound_two_stage": 4 * w.alpha ** 2 * (N - k), "quality_ms": round(ev0.elapsed_time(ev1), 3)}
    log(f"quality: SSE {qt[0]:.6e} (two-stage bound {out['quality']['sse_bound_two_stage']:.3e}), "
        f"max Var_len {qt[1]:.3e}, max Var_inc {qt[2]:.3e} (alpha^2 {w.alpha ** 2:.3e})")

    # ---------------------------------------------------------------- pmc calibration copy
    if args.pmc_calibrate:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy kernel: 3 x neg over 1 GiB (read 1 GiB, write 1 GiB per launch)")
    del pipe, sets, S0, sz, full, enc, rec, v, so, t0
    torch.cuda.empty_cache()
    return out


def plain_leg(w, v, so, sz, full, N, ms_comp, ms_sym, ms_graph, args, dev) -> dict:
    """Batched compression against plain launches of the same kernel (one
    wavefront per domain, no queue, no graph): one launch per series over
    the whole workload, and one launch per domain on a sample of series."""
    import torch

    import paper_2401_00109_amd as J

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cap = max(w.n_points, 1)
    pp = J.Pieces(torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.float64, device=dev),
                  torch.empty(w.n_series + 1, dtype=torch.int64, device=dev),
                  torch.empty(1, dtype=torch.int64, device=dev), cap)
    # warm the plain path on one series, then time it once over all series
    J.compress_plain(v, so[:2], w.series_off[:2], w.D, w.tol, w.max_len, out=pp, workspace=sz.cws)
    torch.cuda.synchronize()
    reps = 1 if w.n_points > 200_000_000 else max(1, min(args.steps, 3))
    ev0.record()
    for _ in range(reps):
        J.compress_plain(v, so, w.series_off, w.D, w.tol, w.max_len, out=pp, workspace=sz.cws)
    ev1.record()
    torch.cuda.synchronize()
    ms_plain = ev0.elapsed_time(ev1) / reps
    same = (int(pp.n_pieces.item()) == N and torch.equal(pp.len[:N], full.len[:N])
            and torch.equal(pp.inc[:N], full.inc[:N]) and torch.equal(pp.piece_off, full.piece_off))
    del pp
    # one launch per domain: every domain of the sampled series becomes a
    # series of its own (its D + 1 points, end points repeated), compressed by
    # the plain path, which then launches once per domain
    stride = max(1, args.plain_domain_sample)
    idx = np.arange(0, w.n_series, stride)
    parts, offs = [], [0]
    for s in idx:
        a, b = int(w.series_off[s]), int(w.series_off[s + 1])
        for d0 in range(a, b - 1, w.D):
            seg = w.values[d0:min(d0 + w.D, b - 1) + 1]
            parts.append(seg)
            offs.append(offs[-1] + seg.size)
    dv = torch.from_numpy(np.concatenate(parts)).to(dev)
    doff_h = np.asarray(offs, np.int64)
    doff = torch.from_numpy(doff_h).to(dev)
    n_dom = doff_h.size - 1
    dws = J.api._ws(J.api.compress_workspace_bytes(n_dom, int(doff_h[-1]), w.D), dev)
    J.compress_plain(dv, doff[:2], doff_h[:2], w.D, w.tol, w.max_len, workspace=dws)
    torch.cuda.synchronize()
    ev0.record()
    J.compress_plain(dv, doff, doff_h, w.D, w.tol, w.max_len, workspace=dws)
    ev1.record()
    torch.cuda.synchronize()
    ms_dom_sample = ev0.elapsed_time(ev1)
    total_domains = int(sum(max(0, (int(n) - 1 + w.D - 1) // w.D) for n in np.diff(w.series_off)))
    ms_dom = ms_dom_sample / n_dom * total_domains
    del dv, doff, dws
    torch.cuda.empty_cache()
    ms_digitize = ms_sym - ms_comp
    batched_e2e = ms_graph if ms_graph is not None else ms_sym
    res = {"compress_batched_ms": round(ms_comp, 3),
           "compress_plain_per_series_ms": round(ms_plain, 3), "plain_per_series_launches": int(w.n_series),
           "compress_speedup_vs_per_series": round(ms_plain / ms_comp, 2),
           "compress_plain_per_domain_ms": round(ms_dom, 3), "plain_per_domain_launches": total_domains,
           "plain_per_domain_timed_on": f"{n_dom} domains of {idx.size} series (one in {stride}), "
                                        f"{ms_dom_sample:.1f} ms, scaled by {total_domains}/{n_dom}",
           "compress_speedup_vs_per_domain": round(ms_dom / ms_comp, 2),
           "symbolize_batched_ms": round(batched_e2e, 3),
           "symbolize_plain_per_series_ms": round(ms_plain + ms_digitize, 3),
           "end_to_end_speedup_vs_per_series": round((ms_plain + ms_digitize) / batched_e2e, 2),
           "end_to_end_speedup_vs_per_domain": round((ms_dom + ms_digitize) / batched_e2e, 2),
           "identical_outputs": bool(same)}
    log(f"compress: batched {ms_comp:.3f} ms; plain {ms_plain:.1f} ms ({w.n_series} launches, one per series); "
        f"one per domain {ms_dom:.1f} ms ({total_domains} launches, timed on {n_dom}); end to end "
        f"{res['end_to_end_speedup_vs_per_series']}x / {res['end_to_end_speedup_vs_per_domain']}x")
    return res


def serving_leg(resident, dev, args) -> dict:
    """The metric's p99 part: the serving loop with the resident dictionary.
    Saturation from a closed loop (every request queued at once), then
    Poisson arrivals at 0.25, 0.5 and 0.9 of it; latency is arrival to
    symbols on the host (H2D and D2H included)."""
    from paper_2401_00109_amd.inputs import request_pool, request_stream
    from paper_2401_00109_amd.serve import Server, summarize
    t = time.time()
    pool = request_pool(7, args.serving_pool, max_series=256)
    log(f"serving: {len(pool)} request bodies ({sum(p[0].size for p in pool) / len(pool):.3g} points each on "
        f"average) generated in {time.time() - t:.1f} s")
    srv = Server(resident, slots=4, max_series=256, device=dev)
    srv.run(request_stream(1, 200, 0.0, first_id=10_000_000, pool=pool), realtime=False)
    n_closed = max(1000, args.serving_requests // 2)
    closed = request_stream(2, n_closed, 0.0, first_id=20_000_000, pool=pool)
    t = time.perf_counter()
    res = srv.run(closed, realtime=False)
    wall = time.perf_counter() - t
    sat = len(res) / wall
    closed_sm = summarize(res, wall)
    rates = []
    for i, f in enumerate((0.25, 0.5, 0.9)):
        reqs = request_stream(3 + i, args.serving_requests, f * sat, first_id=30_000_000 + 10_000 * i, pool=pool)
        t = time.perf_counter()
        res = srv.run(reqs, realtime=True)
        sm = summarize(res, time.perf_counter() - t)
        rates.append({"fraction_of_saturation": f, "rate_req_per_s": round(f * sat, 1), "requests": sm["requests"],
                      "p50_ms": round(sm["p50_ms"], 3), "p99_ms": round(sm["p99_ms"], 3),
                      "points_per_s": round(sm["points_per_s"], 1), "peak_in_flight": srv.peak_in_flight})
        log(f"serving at {f} x saturation ({f * sat:.0f} req/s): p50 {sm['p50_ms']:.2f} ms, p99 {sm['p99_ms']:.2f} ms, "
            f"{sm['points_per_s']:.3e} points/s, up to {srv.peak_in_flight} requests in flight")
    del srv
    return {"saturation_req_per_s": round(sat, 1), "saturation_points_per_s": round(closed_sm["points_per_s"], 1),
            "closed_loop_requests": n_closed, "rates": rates,
            "requests_shape": "1-256 random walks of 500-50,000 points (log-uniform), cycling over "
                              f"{len(pool)} distinct request bodies; four slots; 200 warm-up requests",
            "latency": "arrival to symbols on the host, H2D and D2H included"}


def copy_ceiling(dev, gib: int = 2, reps: int = 10) -> dict:
    """What a plain device copy reaches on this GPU: torch's copy kernel over
    `gib` GiB of float64 (that much read and written per launch), timed with
    events over `reps` launches after a warm-up."""
    import torch
    n = (gib << 30) // 8
    a = torch.empty(n, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2.0 * n * 8
    del a, b
    torch.cuda.empty_cache()
    gbs = moved / (ms / 1e3) / 1e9
    return {"kernel": f"torch copy_ of {gib} GiB float64", "bytes_per_launch": moved, "avg_launch_ms": round(ms, 4),
            "achieved": round(gbs, 1), "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def _traffic(kernel: str, workload: str):
    """Measured HBM bytes per launch from the committed counter summary of this
    workload, if the kernel sources have not changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
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


def _cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, w1, sample_points: float) -> dict:
    """The oracle, single-threaded, over evenly spaced whole series of about
    `sample_points` points (the same step: compress, digitize, encode,
    reconstruct); then its compression of the same sample over all host
    cores (series split into chunks, one thread each), for the speed-up and
    efficiency of the paper's domain-parallel compression."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O
    from paper_2401_00109_amd.inputs import pack
    stride = max(1, int(round(w.n_points / max(sample_points, 1.0))))
    idx = np.arange(0, w.n_series, stride)
    ser = [w.values[w.series_off[i]:w.series_off[i + 1]] for i in idx]
    vals, off = pack(ser)
    l1, i1, _ = O.compress(w1.values, w1.series_off, w1.D, w1.tol)
    d1 = O.digitize(l1, i1, w1.alpha, w1.scl, w1.B)
    t = time.perf_counter()
    ln, inc, po = O.compress(vals, off, w.D, w.tol)
    t_comp1 = time.perf_counter() - t
    d = O.digitize(ln, inc, w.alpha, w.scl, w.B)
    O.encode(ln, inc, d1.sigma_len, d1.sigma_inc, d1.scl, d1.cx, d1.cy)
    t0 = np.where(np.diff(off) > 0, vals[np.minimum(off[:-1], max(vals.size - 1, 0))], 0.0)
    O.reconstruct(d.symbols, po, off, t0, d.center_len, d.center_inc, orig=vals)
    el = time.perf_counter() - t
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    ns = off.size - 1
    cuts = np.unique(np.linspace(0, ns, min(ns, 4 * cores) + 1).astype(np.int64))

    def run(i):
        a, b = int(cuts[i]), int(cuts[i + 1])
        return O.compress(vals[off[a]:off[b]], off[a:b + 1] - off[a], w.D, w.tol)[0].size

    with ThreadPoolExecutor(cores) as ex:
        t = time.perf_counter()
        n_par = sum(ex.map(run, range(cuts.size - 1)))
        t_compM = time.perf_counter() - t
    assert n_par == ln.size
    phi = t_comp1 / t_compM
    return {"value": round(vals.size / el, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
            "cpu": _cpu_model(), "host_cores": cores,
            "sample": f"{idx.size} of {w.n_series} series (one in {stride}), {vals.size} points, same step: "
                      f"compress+digitize+encode+reconstruct, {el:.1f} s",
            "all_cores": {"threads": cores, "compress_1_thread_s": round(t_comp1, 3),
                          "compress_all_threads_s": round(t_compM, 3),
                          "compress_points_per_s": round(vals.size / t_compM, 1),
                          "speedup": round(phi, 3), "efficiency": round(phi / cores, 3),
                          "note": "the oracle's compression over chunks of whole series, one thread each; "
                                  "digitization stays sequential"}}


if __name__ == "__main__":
    sys.exit(main())
