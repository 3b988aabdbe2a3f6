"""The rocprofv3 summaries (profsum) on small synthetic CSV files (CPU only):
the traffic scale comes from the calibration copy, the per-launch bytes are
the traversal's mean per dispatch times that scale, the record round-trips
through read_record, and the kernel table keeps rocprofv3's figures."""
import csv
import json

from paper_2411_11244_amd import profsum


def _counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, v in rows:
            # two rows per dispatch (e.g. two XCD instances): the summary adds them
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v / 2})
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v / 2})


def test_pmc_scales_by_the_calibration_copy(tmp_path):
    calib = 1 << 30
    trav = "void gd::k_traverse<true>(gd::TravParams)"
    cal = "void at::native::elementwise_kernel<128, 4>(...)"
    # FETCH_SIZE reads half the true bytes of the copy, WRITE_SIZE all of them
    _counters(tmp_path / "f.csv", "FETCH_SIZE", [(1, trav, 1000.0), (2, trav, 3000.0), (3, cal, calib / 2048.0),
                                                 (4, "other", 9e9)])
    _counters(tmp_path / "w.csv", "WRITE_SIZE", [(1, trav, 500.0), (2, trav, 500.0), (3, cal, calib / 1024.0)])
    md = profsum.pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "cmd", "title", calib)
    p = tmp_path / "s.md"
    p.write_text(md)
    rec = profsum.read_record(str(p))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_bytes_per_launch"] == 2000 * 1024 * 2
    assert rec["write_bytes_per_launch"] == 500 * 1024
    assert rec["traffic_bytes_per_launch"] == 2000 * 1024 * 2 + 500 * 1024
    assert rec["dispatches"] == [2, 2]
    assert rec["sources_sha256"] == profsum.sources_sha256()


def test_stats_table_and_bench_line(tmp_path):
    stats = tmp_path / "k.csv"
    with open(stats, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                                          "MaxNs", "StdDev"])
        w.writeheader()
        w.writerow({"Name": "void gd::k_traverse<true>(gd::TravParams)", "Calls": 3, "TotalDurationNs": 81e6,
                    "AverageNs": 27e6, "Percentage": 94.0, "MinNs": 10e6, "MaxNs": 45e6, "StdDev": 1})
    log = tmp_path / "run.log"
    log.write_text("noise\n" + json.dumps({"metric": "m", "value": 500.0, "unit": "queries/s", "ms_per_step": 200.0,
                                           "roofline": {"frac": 1.0}, "other": 1}) + "\n")
    md = profsum.stats(str(stats), str(log), "cmd", "title")
    assert "| void gd::k_traverse<true> | 3 | 81.000 | 27000.0 | 10000.0 | 45000.0 | 94.00 |" in md
    assert '"value": 500.0' in md and '"other"' not in md


def test_counters_summary(tmp_path):
    """Per-dispatch means of several counters for the traversal only, and the
    derived hit rates from their definitions."""
    p = tmp_path / "c.csv"
    rows = []
    for d, name in ((1, "k_traverse<true>"), (2, "k_refit_leaves_batch"), (3, "k_traverse<true>")):
        for cn, v in (("TCC_HIT_sum", 300.0 * d), ("TCC_MISS_sum", 100.0 * d), ("SQ_WAVES", 10.0),
                      ("SQ_INSTS_VALU", 1000.0 * d)):
            rows.append((d, name, cn, v))
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, cn, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": cn, "Counter_Value": v})
    out = profsum.counters([str(p)], "cmd", "title")
    assert "| TCC_HIT_sum | 600 | 2 |" in out          # mean of dispatches 1 and 3: (300 + 900) / 2
    assert "| L2 hit rate | 0.75 |" in out
    assert "| VALU instructions per wave | 200 |" in out
