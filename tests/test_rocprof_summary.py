"""Host checks of the profile summariser: rocprof's demangled kernel names map
to the names the library times its launches under, and the source hash that
ties a measurement to the kernels ignores comments but not code."""
import os
import shutil

import pytest

from paper_2401_00109_amd import rocprof_summary as R

NS = "void jabba::(anonymous namespace)::"


@pytest.mark.parametrize("kernel,name", [
    (NS + "k_compress1<false, true>(double const*, long)", "k_compress<W>"),
    (NS + "k_compress1<false, false>(double const*, long)", "k_compress<W>"),
    (NS + "k_compress1<true, false>(double const*, long)", "k_compress_znorm"),
    (NS + "k_compress1<true, true>(double const*, long)", "k_compress_znorm"),
    (NS + "k_compress<4, false>(double const*, long)", "k_compress<W>"),
    (NS + "k_compress<4, true>(double const*, long)", "k_compress_znorm"),
    (NS + "k_onesweep<0, false>(unsigned int const*)", "k_onesweep"),
    (NS + "k_onesweep<1, true>(unsigned int const*)", "k_onesweep_aux"),
    (NS + "k_bucket_local<0>(unsigned int const*)", "k_bucket_local"),
    (NS + "k_bucket_local<1>(unsigned int const*)", "k_bucket_local_pca"),
    (NS + "k_recon<true>(jabba::Src, long const*)", "k_recon"),
    (NS + "k_recon<false>(jabba::Src, long const*)", "k_recon_pieces"),
    (NS + "k_stage1(long const*, long)", "k_stage1"),
])
def test_timing_names(kernel, name):
    assert R.timing_name(kernel) == name


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    pkg = tmp_path / "pkg"
    shutil.copytree(os.path.join(R.PKG, "csrc"), pkg / "csrc")
    monkeypatch.setattr(R, "PKG", str(pkg))
    h0 = R.source_hash()
    f = pkg / "csrc" / "reconstruct.hip"
    text = f.read_text()
    f.write_text("// a new comment line\n" + text.replace("namespace jabba {", "namespace jabba {  /* note */"))
    assert R.source_hash() == h0
    f.write_text(text.replace("constexpr int kTagAhead = 3;", "constexpr int kTagAhead = 3; int unused_x = 0;"))
    assert R.source_hash() != h0


def test_forms_sharing_a_timing_name_keep_their_own_traffic(tmp_path, monkeypatch):
    # a timing name covering two template forms: the table reads each form's
    # own counters, and the traffic file keeps the form launched most often
    import csv
    import json
    import sys
    big = NS + "k_compress1<false, true>(double const*, long)"
    small = NS + "k_compress1<false, false>(double const*, long)"
    cal = "void at::native::neg_kernel(float*)"
    (tmp_path / "trace").mkdir()
    with open(tmp_path / "trace" / "t_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": big, "Calls": 3, "TotalDurationNs": 3e6, "AverageNs": 1e6, "Percentage": 90})
        w.writerow({"Name": small, "Calls": 1, "TotalDurationNs": 1e3, "AverageNs": 1e3, "Percentage": 10})
    for counter, fname in (("FETCH_SIZE", "f.csv"), ("WRITE_SIZE", "w.csv")):
        with open(tmp_path / fname, "w", newline="") as fh:
            w = csv.DictWriter(fh, ["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            w.writerow({"Kernel_Name": cal, "Counter_Name": counter, "Counter_Value": 1 << 20})  # 1 GiB in KiB
            for _ in range(3):
                w.writerow({"Kernel_Name": big, "Counter_Name": counter, "Counter_Value": 1000.0})
            w.writerow({"Kernel_Name": small, "Counter_Name": counter, "Counter_Value": 1.0})
    out = tmp_path / "out"
    monkeypatch.setattr(sys, "argv", ["x", "--trace", str(tmp_path / "trace"), "--fetch", str(tmp_path / "f.csv"),
                                      "--write", str(tmp_path / "w.csv"), "--workload", "t", "--out", str(out)])
    assert R.main() == 0
    k = json.load(open(out / "traffic_t.json"))["kernels"]["k_compress<W>"]
    assert k["dispatches"] == 3 and k["fetch_bytes_per_launch"] == 1000.0 * 1024
    table = (out / "kernels_t.md").read_text().splitlines()
    rows = [r for r in table if r.startswith("| k_compress<W>")]
    assert [r.split("|")[6].strip() for r in rows] == ["1.0", "0.0"]  # fetch MB per launch of each form
