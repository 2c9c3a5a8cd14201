"""The rocprofv3 summarizer behind profiles/ (CPU, synthetic counter files):
the copy calibration, the steady-state averages over the last dispatches,
the most dispatched template variant of a kernel, and the stats table."""
import csv
import os

from paper_1903_02118_amd import profsum


def _counters(d, rows):
    os.makedirs(os.path.join(d, "host", "1"), exist_ok=True)
    with open(os.path.join(d, "host", "1", "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": "X", "Counter_Value": v})


def test_traffic_calibration_tail_average_and_variant_choice(tmp_path):
    gib = 1 << 30
    fetch = [("__amd_rocclr_copyBuffer", 16.0), ("__amd_rocclr_copyBuffer", gib / 1024 / 2)]  # the counter halves reads
    fetch += [("void bie::k_near<double, 128, 16, 2>(...)", 999.0)] * 2  # autotuner variant, fewer dispatches
    fetch += [("void bie::k_near<double, 128, 8, 2>(...)", v) for v in (100.0, 200.0, 300.0, 400.0, 500.0)]
    fetch += [("void bie::k_recv<double>(...)", 10.0)] * 3
    write = [("__amd_rocclr_copyBuffer", 8.0), ("__amd_rocclr_copyBuffer", gib / 1024)]
    write += [("void bie::k_near<double, 128, 16, 2>(...)", 1.0)] * 2
    write += [("void bie::k_near<double, 128, 8, 2>(...)", v) for v in (1.0, 2.0, 3.0, 4.0, 6.0)]
    write += [("void bie::k_recv<double>(...)", 0.5)] * 3
    _counters(str(tmp_path / "f"), fetch)
    _counters(str(tmp_path / "w"), write)
    t = profsum.traffic(str(tmp_path / "f"), str(tmp_path / "w"), gib, last=2)
    assert t["scale_fetch"] == 2.0 and t["scale_write"] == 1.0
    k = t["kernels"]["k_near"]
    assert k["name"] == "k_near<double, 128, 8, 2>" and k["dispatches"] == 5
    assert k["fetch_kib"] == 450.0 and k["write_kib"] == 5.0
    assert k["hbm_bytes"] == (450.0 * 2.0 + 5.0) * 1024.0
    assert t["kernels"]["k_recv"]["hbm_bytes"] == (10.0 * 2.0 + 0.5) * 1024.0
    assert t["source_hash"] == profsum.source_hash()
    md = profsum.traffic_md(dict(t, command_fetch="cf", command_write="cw"), "T", alg_bytes=(450.0 * 2.0) * 1024.0)
    assert "above it" in md and "cf" in md


def test_stats_table_with_tail_average(tmp_path):
    st = tmp_path / "stats.csv"
    with open(st, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": "void bie::k_near<float, 128, 8, 4>(...)", "Calls": 4, "AverageNs": 2500.0,
                    "MinNs": 1000.0, "MaxNs": 4000.0, "Percentage": 90.0})
        w.writerow({"Name": "k_fdph_update", "Calls": 1, "AverageNs": 500.0, "MinNs": 500.0, "MaxNs": 500.0,
                    "Percentage": 10.0})
    tr = tmp_path / "trace.csv"
    with open(tr, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for d in (1000, 2000, 3000, 4000):
            w.writerow({"Kernel_Name": "void bie::k_near<float, 128, 8, 4>(...)", "Start_Timestamp": 0,
                        "End_Timestamp": d})
        w.writerow({"Kernel_Name": "k_fdph_update", "Start_Timestamp": 0, "End_Timestamp": 500})
    md = profsum.stats_md(str(st), "cmd", str(tr), tail=2).splitlines()
    assert md[0].endswith("avg of last 2 us |")
    assert md[2] == "| `k_near<float, 128, 8, 4>` | 4 | 2.5 | 1.0 | 4.0 | 90.00 | 3.5 |"
    assert md[3].endswith("| 10.00 | |")  # fewer dispatches than the tail: no tail average


def test_traffic_reads_calibrated_on_the_read_probe(tmp_path):
    """With the probe's known byte count, FETCH_SIZE is scaled by the probe's
    own reading (same loads as the near kernel), WRITE_SIZE by the copy."""
    gib = 1 << 30
    fetch = [("__amd_rocclr_copyBuffer", gib / 1024 / 2), ("k_hbm_read(double2 const*, long, double*)", gib / 1024 / 1.9)]
    fetch += [("void bie::k_near<double, 128, 8, 2>(...)", 100.0)] * 3
    write = [("__amd_rocclr_copyBuffer", gib / 1024), ("k_hbm_read(double2 const*, long, double*)", 0.0)]
    write += [("void bie::k_near<double, 128, 8, 2>(...)", 1.0)] * 3
    _counters(str(tmp_path / "f"), fetch)
    _counters(str(tmp_path / "w"), write)
    t = profsum.traffic(str(tmp_path / "f"), str(tmp_path / "w"), gib, last=3, probe_bytes=gib)
    assert abs(t["scale_fetch"] - 1.9) < 1e-12 and t["scale_write"] == 1.0
    assert t["probe_calibration"]["bytes_read"] == gib
    md = profsum.traffic_md(dict(t, command_fetch="cf", command_write="cw"), "T")
    assert "k_hbm_read" in md

