"""Summaries of rocprofv3 output for the traversal kernel (text for profiles/).

    python -m paper_2411_11244_amd.profsum stats  <kernel_stats.csv> <bench log> "<command>" "<title>"
    python -m paper_2411_11244_amd.profsum pmc    <fetch counter csv> <write counter csv> "<commands>" "<title>" <calibration bytes>
    python -m paper_2411_11244_amd.profsum counters "<commands>" "<title>" <counter csv> [<counter csv> ...]

``stats`` turns a ``--kernel-trace --stats`` kernel table into a markdown
table and appends the bench.py line the same run printed.

``pmc`` reads two ``--pmc`` runs of bench.py (one with FETCH_SIZE, one with
WRITE_SIZE; both in KiB per dispatch) that also ran its calibration copy (a
plain elementwise kernel reading and writing a known number of bytes).  The
copy's counters give the scale from counter units to bytes; the traversal
kernel's average per dispatch, scaled, is its HBM traffic per launch.  The
summary records a hash of the kernel's sources, so that bench.py reports the
traffic only while the kernel is unchanged.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# the kernel and the launch configuration bench.py applies (the tuning file)
KERNEL_SOURCES = ("csrc/traverse.hip", "csrc/gdist_dev.hpp", "csrc/internal.hpp", "tuning/rings_mi355x.json")
CALIB_MARK = "elementwise"          # the calibration copy is torch's elementwise kernel
TRAVERSE = "k_traverse"
XCDS, CUS, SIMDS = 8, 256, 1024    # MI355X


def sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counter_means(path: str, counter: str):
    """Mean counter value per dispatch for the traversal and calibration kernels."""
    per = defaultdict(dict)  # dispatch -> (name, value summed over rows)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            d = r["Dispatch_Id"]
            per[d]["name"] = r["Kernel_Name"]
            per[d]["v"] = per[d].get("v", 0.0) + float(r["Counter_Value"])
    trav = [e["v"] for e in per.values() if TRAVERSE in e["name"]]
    cal = [e["v"] for e in per.values() if CALIB_MARK in e["name"]]
    if not trav or not cal:
        raise SystemExit(f"{path}: no {TRAVERSE} or calibration dispatches with {counter}")
    return sum(trav) / len(trav), len(trav), max(cal)


def pmc(fetch_csv: str, write_csv: str, cmds: str, title: str, calib_bytes: int) -> str:
    f_trav, n_f, f_cal = _counter_means(fetch_csv, "FETCH_SIZE")
    w_trav, n_w, w_cal = _counter_means(write_csv, "WRITE_SIZE")
    f_scale = calib_bytes / (f_cal * 1024.0)
    w_scale = calib_bytes / (w_cal * 1024.0)
    fetch_b = f_trav * 1024.0 * f_scale
    write_b = w_trav * 1024.0 * w_scale
    rec = {"kernel": TRAVERSE, "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
           "traffic_bytes_per_launch": round(fetch_b + write_b), "dispatches": [n_f, n_w],
           "calibration_bytes": calib_bytes, "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5),
           "sources_sha256": sources_sha256()}
    out = [f"# {title}", "", "Commands (run from the repository root on one MI355X):", "", "```", cmds, "```", "",
           "Calibration: a torch elementwise copy of float32 data reading and writing "
           f"{calib_bytes} bytes each, in the same process.  Scale = known bytes / counter bytes.", "",
           "| | counter KiB per dispatch (k_traverse) | calibration KiB | scale | bytes per launch |",
           "|---|---|---|---|---|",
           f"| FETCH_SIZE | {f_trav:.1f} | {f_cal:.1f} | {f_scale:.4f} | {fetch_b:.4g} |",
           f"| WRITE_SIZE | {w_trav:.1f} | {w_cal:.1f} | {w_scale:.4f} | {write_b:.4g} |", "",
           "Record read by bench.py (traffic is reported only while the kernel's sources hash the same):", "",
           "```", "PMC_RECORD " + json.dumps(rec), "```"]
    return "\n".join(out)


def counters(csvs, cmds: str, title: str) -> str:
    """Per-dispatch means of every counter in one or more ``--pmc`` runs, for
    the traversal kernel, with the derived utilisations computed from them."""
    vals = {}
    res = {}   # launch resources of the traversal's dispatches, as the profiler records them
    for path in csvs:
        per = defaultdict(lambda: defaultdict(float))   # counter -> dispatch -> value
        names = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                d = r["Dispatch_Id"]
                names[d] = r["Kernel_Name"]
                per[r["Counter_Name"]][d] += float(r["Counter_Value"])
                if TRAVERSE in r["Kernel_Name"] and not res:
                    res = {k: r[k] for k in ("Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count",
                                             "LDS_Block_Size", "Workgroup_Size", "Grid_Size") if k in r}
        for cn, byd in per.items():
            tv = [v for d, v in byd.items() if TRAVERSE in names[d]]
            if tv:
                vals[cn] = (sum(tv) / len(tv), len(tv))
    out = [f"# {title}", "", "Commands (run from the repository root on one MI355X):", "", "```", cmds, "```", "",
           "| counter | mean per k_traverse dispatch | dispatches |", "|---|---|---|"]
    for cn in sorted(vals):
        out.append(f"| {cn} | {vals[cn][0]:.6g} | {vals[cn][1]} |")
    der = []
    v = {k: x[0] for k, x in vals.items()}
    if "SQ_INSTS_VALU" in v and "SQ_WAVES" in v:
        der.append(("VALU instructions per wave", v["SQ_INSTS_VALU"] / max(1.0, v["SQ_WAVES"])))
    if "TCC_HIT_sum" in v and "TCC_MISS_sum" in v:
        der.append(("L2 hit rate", v["TCC_HIT_sum"] / max(1.0, v["TCC_HIT_sum"] + v["TCC_MISS_sum"])))
    # MI355X: 8 XCDs (GRBM_GUI_ACTIVE is their sum), 256 CUs, 1,024 SIMDs; the
    # SQ cycle counters count 4-cycle units
    if "SQ_ACTIVE_INST_VALU" in v and "GRBM_GUI_ACTIVE" in v:
        cyc = v["GRBM_GUI_ACTIVE"] / XCDS
        der.append(("VALU busy (SQ_ACTIVE_INST_VALU x 4 / 1024 SIMDs / GPU cycles)",
                    v["SQ_ACTIVE_INST_VALU"] * 4.0 / SIMDS / max(1.0, cyc)))
        if "TA_TA_BUSY_sum" in v:
            der.append(("texture address unit busy (TA_TA_BUSY / 256 CUs / GPU cycles)",
                        v["TA_TA_BUSY_sum"] / CUS / max(1.0, cyc)))
        if "TCP_PENDING_STALL_CYCLES_sum" in v:
            der.append(("L1 stalled on pending misses (per CU / GPU cycles)",
                        v["TCP_PENDING_STALL_CYCLES_sum"] / CUS / max(1.0, cyc)))
    if "SQ_THREAD_CYCLES_VALU" in v and "SQ_ACTIVE_INST_VALU" in v:
        der.append(("lanes active per VALU instruction", v["SQ_THREAD_CYCLES_VALU"] / max(1.0, 64.0 * v["SQ_ACTIVE_INST_VALU"])))
    if "TCP_TCC_READ_REQ_sum" in v and "TCP_TOTAL_CACHE_ACCESSES_sum" in v:
        der.append(("L1 hit rate (1 - L1-to-L2 reads / L1 accesses)",
                    1.0 - v["TCP_TCC_READ_REQ_sum"] / max(1.0, v["TCP_TOTAL_CACHE_ACCESSES_sum"])))
    if der:
        out += ["", "| derived | value |", "|---|---|"] + [f"| {k} | {x:.4g} |" for k, x in der]
    if res:
        out += ["", "| k_traverse launch resource (profiler record) | value |", "|---|---|"]
        out += [f"| {k} | {x} |" for k, x in res.items()]
    return "\n".join(out)


def read_record(path: str):
    """The PMC_RECORD of a summary, or None."""
    try:
        with open(path) as f:
            m = re.search(r"^PMC_RECORD (\{.*\})$", f.read(), re.M)
    except OSError:
        return None
    return json.loads(m.group(1)) if m else None


def stats(stats_csv: str, log: str, cmd: str, title: str) -> str:
    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    out = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "", "```", cmd, "```", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:16]:
        name = r["Name"].split("(")[0]
        out.append(f"| {name} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    with open(log) as f:
        m = re.search(r'\{"metric".*\}', f.read())
    if m:
        j = json.loads(m.group(0))
        keep = {k: j[k] for k in ("value", "unit", "ms_per_step", "roofline", "refit") if k in j}
        out += ["", "bench.py line printed by the same run (live HIP-event measurement of the same launches):", "",
                "```", json.dumps(keep, indent=1), "```"]
    return "\n".join(out)


def main(argv=None) -> int:
    a = sys.argv[1:] if argv is None else argv
    if len(a) >= 5 and a[0] == "stats":
        print(stats(a[1], a[2], a[3], a[4]))
        return 0
    if len(a) >= 4 and a[0] == "counters":
        print(counters(a[3:], a[1], a[2]))
        return 0
    if len(a) >= 6 and a[0] == "pmc":
        print(pmc(a[1], a[2], a[3], a[4], int(a[5])))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    raise SystemExit(main())
