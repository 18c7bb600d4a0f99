"""Condense rocprofv3 output into the short text summaries kept under profiles/.

    python -m paper_2401_00109_amd.rocprof_summary \\
        --trace <dir with *_kernel_stats.csv> --fetch <FETCH_SIZE counter csv> \\
        --write <WRITE_SIZE counter csv> --workload scale --command "<cmd>" --out profiles
    python -m paper_2401_00109_amd.rocprof_summary --sq <SQ counter csvs> --command "<cmd>" --out profiles

HBM traffic per dispatch comes from two counter runs (FETCH_SIZE, then
WRITE_SIZE, in KiB per dispatch).  Each counter is scaled by what it reads
for a plain copy kernel of known size that the benchmark launches in the
same run (``--pmc-calibrate``: torch.neg over 1 GiB, reading and writing
1 GiB), so the factor corrects the counter's granularity on this device.
traffic_<workload>.json records the source hash of the kernels; the
benchmark ignores it once the kernel sources change.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
CAL_BYTES = float(1 << 30)
PEAK_GBS = 8000.0  # MI355X HBM3E


def _code_only(text: str) -> str:
    """The source without comments and with whitespace collapsed, so that an
    edit of comments alone leaves the hash (and the measurements) valid."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash() -> str:
    """Hash of the HIP sources' code; identifies the kernels a measurement belongs to."""
    h = hashlib.sha256()
    d = os.path.join(PKG, "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            h.update(f.encode() + _code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def timing_name(kernel: str) -> str:
    """rocprof's demangled kernel name -> the library's timing name."""
    m = re.search(r"::(k_[A-Za-z0-9_]+)(<[^()]*>)?\(", kernel)
    if not m:
        return kernel.split("(")[0][-60:]
    base, targs = m.group(1), (m.group(2) or "")
    if base == "k_compress1":  # <Norm, Grouped>
        norm = targs.strip("<>").split(",")[0].strip()
        return "k_compress_znorm" if norm in ("true", "(bool)1") else "k_compress<W>"
    if base == "k_compress":
        return "k_compress_znorm" if ("true" in targs or "(bool)1" in targs) else "k_compress<W>"
    if base == "k_onesweep":  # <0, ...>: the main sort's passes; the others: every other radix sort
        return base + ("" if targs.startswith("<0") else "_aux")
    if base in ("k_key", "k_bucket_local", "k_large_collect", "k_large_emit"):
        return base + ("_pca" if targs == "<1>" else "")
    if base == "k_recon":
        return "k_recon" if ("true" in targs or "(bool)1" in targs) else "k_recon_pieces"
    return base + targs


def load_counter(path: str, counter: str):
    per = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") == counter:
                per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def calibration(per: dict) -> float | None:
    vals = [v for name, vs in per.items() if "neg_kernel" in name for v in vs]
    if not vals:
        return None
    return CAL_BYTES / (sum(vals) / len(vals) * 1024.0)


SQ_SHOWN = ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU",
            "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_LDS", "SQ_INSTS_VALU", "SQ_INSTS_LDS",
            "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"]


def sq_table(args) -> int:
    """Median per-dispatch SQ counters of the kernels with the most wave cycles
    in total, with the share of wave cycles spent waiting and issuing VALU work."""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in args.sq:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if "jabba" in r["Kernel_Name"]:
                    per[timing_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))

    def med(v):
        v = sorted(v)
        return v[len(v) // 2] if v else None

    rows = sorted(per.items(), key=lambda kv: -sum(kv[1].get("SQ_WAVE_CYCLES", [])))[:10]
    shown = [c for c in SQ_SHOWN if any(c in d for _, d in rows)]
    lines = [f"# SQ counters of the largest kernels, workload `{args.workload}`", "",
             f"Command: `{args.command}`", "",
             f"Source hash of the kernels: `{source_hash()}`", "",
             "Median over the kernel's dispatches (skipped radix passes included), summed over the device. "
             "wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES, valu = SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES.", "",
             "| kernel | wait | valu | " + " | ".join(shown) + " |",
             "|---|---|---|" + "---|" * len(shown)]
    for name, d in rows:
        m = {c: med(d.get(c, [])) for c in shown}
        wc = m.get("SQ_WAVE_CYCLES")
        wait = f"{m['SQ_WAIT_ANY'] / wc:.2f}" if wc and m.get("SQ_WAIT_ANY") is not None else ""
        valu = f"{m['SQ_ACTIVE_INST_VALU'] / wc:.2f}" if wc and m.get("SQ_ACTIVE_INST_VALU") is not None else ""
        lines.append(f"| {name} | {wait} | {valu} | " +
                     " | ".join("" if m[c] is None else f"{m[c]:.3g}" for c in shown) + " |")
    path = os.path.join(args.out, f"sq_counters_{args.workload}.md")
    os.makedirs(args.out, exist_ok=True)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(path)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq", nargs="*", default=None,
                    help="counter-collection csvs of SQ counter runs: writes sq_counters_<workload>.md instead")
    ap.add_argument("--workload", default="scale")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default="profiles")
    args = ap.parse_args()
    if args.sq:
        return sq_table(args)
    if not args.trace or not args.fetch or not args.write:
        ap.error("--trace, --fetch and --write are required without --sq")

    stats_csv = glob.glob(os.path.join(args.trace, "*kernel_stats.csv"))[0]
    with open(stats_csv) as fh:
        stats = list(csv.DictReader(fh))
    fetch = load_counter(args.fetch, "FETCH_SIZE")
    write = load_counter(args.write, "WRITE_SIZE")
    ff, wf = calibration(fetch), calibration(write)

    # per kernel as rocprof names it (template forms apart); a timing name
    # that covers several forms keeps the one launched most often
    by_name = {}
    for name in set(fetch) | set(write):
        if "jabba" not in name:
            continue
        f = fetch.get(name, [])
        w = write.get(name, [])
        fb = (sum(f) / len(f) * 1024.0 * ff) if (f and ff) else None
        wb = (sum(w) / len(w) * 1024.0 * wf) if (w and wf) else None
        by_name[name] = {"rocprof_name": name[:name.find("(", name.find("::k_"))] if "::k_" in name else name[:80],
                         "dispatches": len(f),
                         "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                         "bytes_per_launch": (fb or 0.0) + (wb or 0.0) if (fb is not None and wb is not None)
                         else None}
    traffic = {}
    for name, e in sorted(by_name.items()):
        tn = timing_name(name)
        if tn not in traffic or e["dispatches"] > traffic[tn]["dispatches"]:
            traffic[tn] = e

    os.makedirs(args.out, exist_ok=True)
    with open(os.path.join(args.out, f"traffic_{args.workload}.json"), "w") as fh:
        json.dump({"source_hash": source_hash(), "workload": args.workload, "fetch_factor": ff, "write_factor": wf,
                   "calibration": "torch.neg over 1 GiB of float64 (1 GiB read + 1 GiB written per launch)",
                   "kernels": traffic}, fh, indent=1, sort_keys=True)

    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    # counted HBM bytes over kernel time, per kernel and weighted by time over
    # every kernel of the library that has both figures
    tot_bytes = tot_ns = 0.0
    for r in stats:
        t = by_name.get(r["Name"]) or traffic.get(timing_name(r["Name"]), {})
        if "jabba" in r["Name"] and t.get("bytes_per_launch") is not None:
            tot_bytes += t["bytes_per_launch"] * float(r["Calls"])
            tot_ns += float(r["TotalDurationNs"])
    weighted = (f"Time-weighted over the library's kernels: {tot_bytes / tot_ns:.0f} GB/s of counted traffic, "
                f"{100 * tot_bytes / tot_ns / PEAK_GBS:.1f} % of {PEAK_GBS:.0f} GB/s" if tot_ns > 0 else
                "Time-weighted counted traffic: not available")
    lines = [f"# Kernel time and HBM traffic, workload `{args.workload}`", "",
             f"Command: `{args.command}`", "",
             f"Source hash of the kernels: `{source_hash()}`", "",
             f"Counter scaling from the 1 GiB copy kernel: FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {wf:.4f}"
             if ff and wf else "Counter scaling: calibration kernel missing", "",
             weighted, "",
             "| kernel | calls | total ms | avg us | % | fetch MB/launch | write MB/launch | counted GB/s | % of peak |",
             "|---|---|---|---|---|---|---|---|---|"]
    for r in stats[:24]:
        tn = timing_name(r["Name"])
        t = by_name.get(r["Name"]) or traffic.get(tn, {})
        fb, wb = t.get("fetch_bytes_per_launch"), t.get("write_bytes_per_launch")
        bl = t.get("bytes_per_launch")
        avg_ns = float(r["AverageNs"])
        gbs = bl / avg_ns if (bl is not None and avg_ns > 0) else None
        lines.append(f"| {tn} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{avg_ns / 1e3:.2f} | {float(r['Percentage']):.1f} | "
                     f"{'' if fb is None else f'{fb / 1e6:.1f}'} | {'' if wb is None else f'{wb / 1e6:.1f}'} | "
                     f"{'' if gbs is None else f'{gbs:.0f}'} | {'' if gbs is None else f'{100 * gbs / PEAK_GBS:.1f}'} |")
    path = os.path.join(args.out, f"kernels_{args.workload}.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(path)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
