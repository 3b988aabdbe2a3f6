"""bench.py's roofline arithmetic and its use of the committed PMC record
(CPU only: synthetic statistics, no GPU)."""
import bench
from paper_2411_11244_amd import profsum


def test_roofline_scales_counted_bytes_to_the_timed_launches():
    # two timed calls of 2 launches each (statistics off: no byte counts) and
    # one counted call of the same work with them on
    timed = [{"ms_traverse_kernel": 5.0, "traverse_launches": 2, "bytes_traversal": 0, "bytes_narrow": 0}] * 2
    counted = [{"ms_traverse_kernel": 5.5, "traverse_launches": 2, "bytes_traversal": 40_000_000_000,
                "bytes_narrow": 20_000_000_000}]
    r = bench.trav_roofline(timed, copy_gbs=5000.0, counted=counted)
    # 3e10 bytes per launch, 4 launches in 10 ms: 12 TB/s (made-up numbers:
    # only the arithmetic is checked here)
    assert r["algorithmic_bytes_per_launch"] == 30_000_000_000
    assert r["launches"] == 4 and r["avg_ms_per_launch"] == 2.5
    assert r["achieved"] == 12000.0 and r["frac"] == 1.5 and r["frac_of_copy"] == 2.4
    assert r["bytes_traversal_per_launch"] == 20_000_000_000 and r["bytes_narrow_per_launch"] == 10_000_000_000
    assert r["peak"] == bench.HBM_PEAK_GBS == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"


def test_roofline_without_counted_calls_uses_the_timed_ones():
    timed = [{"ms_traverse_kernel": 20.0, "traverse_launches": 5, "bytes_traversal": 10 ** 11,
              "bytes_narrow": 6 * 10 ** 10}]
    r = bench.trav_roofline(timed)
    assert r["achieved"] == 8000.0 and r["frac"] == 1.0 and "frac_of_copy" not in r
    assert r["algorithmic_bytes_per_launch"] == 32_000_000_000


def test_traffic_record_follows_the_kernel_sources(monkeypatch):
    rec = bench.traffic_record()
    if rec is not None:   # the committed summary was taken on the current sources
        assert rec["sources_sha256"] == profsum.sources_sha256()
        total = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
        assert abs(rec["traffic_bytes_per_launch"] - total) <= 2   # each rounded to whole bytes
    monkeypatch.setattr(profsum, "sources_sha256", lambda: "0" * 64)
    assert bench.traffic_record() is None
