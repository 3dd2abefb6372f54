"""Host-side logic of bench.py (no GPU): the counter summary with its copy
calibration, the traffic lookup and its staleness check, the workload table."""
import csv
import os

import pytest

import bench

HDR = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
       "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
       "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
       "Counter_Value", "Start_Timestamp", "End_Timestamp"]
KERNEL = "void gpcg::step_kernel<double, true, false>(gpcg::StepLaunch)"


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for i, (name, val) in enumerate(rows):
            w.writerow([i, i, 0, 0, 0, 0, 1, 1, name, 256, 0, 0, 8, 0, 8, counter, val, 0, 1])


def test_counter_summary_and_traffic(tmp_path, monkeypatch):
    big = bench.COPY_CALIB_BYTES / 1024.0
    # copy kernel: one calibration dispatch (half the fetch counted) and a small copy
    _write(tmp_path / "f", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", big / 2),
                                          ("__amd_rocclr_copyBuffer", 100.0),
                                          (KERNEL, 1000.0), (KERNEL, 1002.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", big),
                                          ("__amd_rocclr_copyBuffer", 200.0),
                                          (KERNEL, 500.0), (KERNEL, 500.0)])
    txt = bench.counters_summary(str(tmp_path / "f"), str(tmp_path / "w"))
    assert "calib_factor_fetch: 2.0" in txt and "calib_factor_write: 1.0" in txt
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_wl.md").write_text("# note\n\n```\n" + txt + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for rel in bench.KERNEL_SOURCES:  # the digest is taken over these files
        p = tmp_path / rel
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_text(open(os.path.join(os.path.dirname(bench.__file__), rel)).read())
    # regenerate with the digest of the copied sources
    txt = bench.counters_summary(str(tmp_path / "f"), str(tmp_path / "w"))
    (prof / "traffic_wl.md").write_text("```\n" + txt + "\n```\n")
    got = bench.traffic_from_profile("wl", "step_kernel<double, true, false>")
    assert got == pytest.approx((1001.0 * 2.0 + 500.0) * 1024.0)
    # a change to the kernel sources makes the summary stale
    src = tmp_path / bench.KERNEL_SOURCES[0]
    src.write_text(src.read_text() + "\n// changed\n")
    assert bench.traffic_from_profile("wl", "step_kernel<double, true, false>") is None
    assert bench.traffic_from_profile("absent", "step_kernel") is None


def test_workload_table():
    for name, (key, opts, desc) in bench.WORKLOADS.items():
        inst = bench.make_instance(key)
        assert inst.n > 0 and desc
    assert bench.make_instance("obstacle_ub_1024").N == 1024


def test_cpu_baseline_reports_one_thread_and_all_cores():
    """The oracle baseline states the threads it used, the host, and an
    all-cores figure (the oracle has no threaded code: for one solve both
    figures are the same)."""
    import instances
    r = bench.cpu_baseline_whole(instances.obstacle50(0), budget_s=0.2)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0
    assert r["all_cores"]["value"] == r["value"] and r["all_cores"]["cores"] == 1
    assert "cpu_model" in r and r["cpus_available"] >= 1
