"""bench.py host logic: the HBM-traffic summary of profiler counter runs (copy-calibrated) and the
source-hash gate that withholds a traffic figure once a kernel's sources have changed."""

import csv
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            r = {k: 0 for k in FIELDS}
            r.update(Kernel_Name=name, Counter_Name=counter, Counter_Value=value, Dispatch_Id=i + 1)
            w.writerow(r)


def test_counter_summary_scales_by_the_copy_calibration(tmp_path):
    kern = "void ridg::predict_plans_nr_kernel<2, 4, 3, 8>(ridg::DevGeom, double)"
    copy = "void at::native::vectorized_elementwise_kernel<4, Mul>(int)"
    # the copy moves 256 MiB each way; FETCH_SIZE reads half of it, WRITE_SIZE all of it
    _csv(tmp_path / "cf.csv", "FETCH_SIZE", [("fill", 16.0), (copy, 131072.0)])
    _csv(tmp_path / "cw.csv", "WRITE_SIZE", [(copy, 262144.0)])
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(kern, 1000.0), (kern, 3000.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(kern, 500.0), (kern, 500.0)])
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--counter-summary",
                          str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                          str(tmp_path / "cw.csv"), "--title", "t", "--commands", "c1;;c2"],
                         capture_output=True, text=True, check=True).stdout
    recs = [json.loads(line[len(bench.RECORD_TAG):]) for line in out.splitlines() if line.startswith(bench.RECORD_TAG)]
    assert len(recs) == 1
    rec = recs[0]
    assert rec["kernel"] == "ridg::predict_plans_nr_kernel<2, 4, 3, 8>"
    assert rec["dispatches"] == 2
    assert rec["fetch_bytes"] == round(2000.0 * 1024 * 2.0)  # mean 2000 KiB, factor 2
    assert rec["write_bytes"] == round(500.0 * 1024 * 1.0)
    assert rec["src"] == bench.kernel_source_hash(rec["kernel"])
    assert "c1" in out and "c2" in out


def test_traffic_is_withheld_when_sources_differ(tmp_path, monkeypatch):
    kern = "ridg::tap_update_kernel<3, 10, 10>"
    good = bench.kernel_source_hash(kern)
    assert good is not None and bench.kernel_source_hash("ridg::unknown_kernel<1>") is None
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": kern, "src": good, "fetch_bytes": 10, "write_bytes": 5, "dispatches": 1}
    (prof / "x.md").write_text(bench.RECORD_TAG + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    # kernel_source_hash reads the sources relative to HERE: point it back at the repository's
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k, _h=good: _h if k == kern else None)
    assert bench.traffic_from_profiles(kern)["bytes"] == 15
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: "0" * 16)
    assert bench.traffic_from_profiles(kern) is None
    # a record of the same kernel with further template arguments matches; another kernel does not
    mk = "ridg::tap_mfma_kernel<10, 10>"
    rec2 = {"kernel": "ridg::tap_mfma_kernel<10, 10, true>", "src": "h", "fetch_bytes": 1, "write_bytes": 2,
            "dispatches": 1}
    rec3 = {"kernel": "ridg::tap_mfma_kernel<10, 15, true>", "src": "h", "fetch_bytes": 7, "write_bytes": 7,
            "dispatches": 1}
    (prof / "y.md").write_text("\n".join(bench.RECORD_TAG + json.dumps(r) for r in (rec3, rec2)) + "\n")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: "h")
    assert bench.traffic_from_profiles(mk)["bytes"] == 3


def test_dominant_kernel_names_follow_the_options():
    class Info:
        theta, theta_t, solver = 10, 20, 2  # 2D order 4, REGION

    assert bench.dominant_kernel(Info(), {"plan_layout": 4}, "fp64") == "ridg::predict_plans_nr_kernel<2, 4, 3, 8>"
    assert bench.dominant_kernel(Info(), {"plan_layout": 3}, "fp64") == "ridg::predict_plans_nr_kernel<2, 4, 2, 10>"
    assert bench.dominant_kernel(Info(), {"plan_layout": 0}, "fp32") == "ridg::predict_plans_kernel<2, 4, false, true>"
    # static pivots at 2D order 4: two rows per lane in 10-lane segments
    assert bench.dominant_kernel(Info(), {"plan_layout": 5}, "fp64") == "ridg::predict_plans_sp_kernel<2, 4, 2, 10, false>"

    class Info3:
        theta, theta_t, solver = 10, 15, 1  # 3D order 3, PREFACTORED

    assert bench.dominant_kernel(Info3(), {"composite": 1}, "fp64") == "ridg::tap_update_kernel<3, 10, 10>"
    # two z-neighbours per thread where n[2] is even; one element per thread otherwise
    assert bench.dominant_kernel(Info3(), {"composite": 1}, "fp64", (128, 128, 128)) == "ridg::tap_z2_kernel<10>"
    assert bench.dominant_kernel(Info3(), {"composite": 1}, "fp64", (12, 12, 13)) == "ridg::tap_update_kernel<3, 10, 10>"

    class Info2:
        theta, theta_t, solver = 6, 10, 1  # 2D order 3, PREFACTORED

    assert bench.dominant_kernel(Info2(), {"composite": 3}, "fp64", (256, 256)) == "ridg::tap_tblock_kernel<6>"
    assert bench.dominant_kernel(Info3(), {"composite": 1, "mfma": 1}, "fp64") == "ridg::tap_mfma_kernel<10, 10>"
    assert bench.dominant_kernel(Info3(), {"mfma": 1}, "fp64") == "ridg::tap_mfma_kernel<15, 10>"
