"""bench.py host behaviour that needs no GPU: more than one GPU is refused before any
device work, with a JSON error line and exit status 2; the counter summary of a run
directory is computed from its CSV files."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_counter_summary_scales_by_the_copy_calibration(tmp_path):
    sys.path.insert(0, ROOT)
    import bench

    def write(sub, kernel, counter, value):
        d = tmp_path / sub
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for v in (value, value):
                w.writerow({"Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": v})

    fwd = "void abg::(anonymous namespace)::forward_kernel<float>(float const*)"
    write("fetch", fwd, "FETCH_SIZE", 1000.0)
    write("write", fwd, "WRITE_SIZE", 300.0)
    write("cfetch", "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0)
    write("cwrite", "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0)
    text = bench.summarize_counters(str(tmp_path))
    data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    assert data["fetch_scale"] == 2.0 and data["write_scale"] == 1.0
    assert data["traffic_bytes_per_launch"] == 1024 * (1000 * 2 + 300)
    assert data["source_hash"] == bench.forward_source_hash()
    assert "valu_wave_insts_per_dispatch" not in data
    write("sq", fwd, "SQ_INSTS_VALU", 5000.0)
    text = bench.summarize_counters(str(tmp_path))
    data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    assert data["valu_wave_insts_per_dispatch"] == 5000.0


def test_kernel_stats_summary(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    with open(tmp_path / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": "void abg::(anonymous namespace)::forward_kernel<double>(double const*)",
                    "Calls": 3, "TotalDurationNs": 15000000, "AverageNs": 5000000, "Percentage": 75.0})
        w.writerow({"Name": "abg::(anonymous namespace)::ncp_dist_kernel(double const*)",
                    "Calls": 2, "TotalDurationNs": 5000000, "AverageNs": 2500000, "Percentage": 25.0})
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for start, end in ((0, 4000000), (10, 6000010), (20, 3020)):   # the last one < 20 us
            w.writerow({"Kernel_Name": "void abg::(anonymous namespace)::forward_kernel<double>(x)",
                        "Start_Timestamp": start, "End_Timestamp": end})
    text = bench.summarize_kernel_stats(str(tmp_path), "t", "cmd")
    lines = text.splitlines()
    assert lines[0] == "# t" and "    cmd" in lines
    row = [ln for ln in lines if ln.startswith("forward_kernel<double>") and "%" in ln][0]
    assert row.split()[1:] == ["3", "5000.0", "15.00", "75.0%"]
    assert "forward_kernel<double>: 2 launches > 20 us, average 5000.0 us" in lines
