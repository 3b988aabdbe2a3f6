"""Benchmark of the mesh-distance hot path on one MI355X.

Headline workload ("rings"): two interlocked tori of 7,502,120 FP32 triangles
each (2740 x 1369 grid, R = 1, r = 0.1; one mesh handle used twice), B
rotated about the world z axis by 0.5 degrees per frame, 100 frames.  The
tree is built once before timing (the meshes are resident in HBM).

A step is one pass of the whole hot path over the 100-frame batch: per query
the refit of B's tree into A's frame, the persistent traversal with its
narrow phase, and the FP64 re-evaluation, all 100 queries in one batched
call.  value = queries per second over the K timed steps.

Beside it, on the same GPU:
  * latency: p50 / p99 of the same frames issued one query per call
    (gdist_query, host wall clock including launch and copy-back);
  * roofline of the dominant kernel (k_traverse): algorithmic bytes counted
    in the kernel (16 B per entry popped + 24 B per child box read, i.e.
    2^kA + 2^kB per popped entry + 16 B per entry pushed; 16 B per leaf pair +
    36 B per triangle read, i.e. tA + tB per leaf pair) per launch, over the
    launch's average duration from HIP events on the library's stream, against
    8 TB/s and against a copy kernel measured in the same process;
  * cpu_baseline: the FP64 CPU oracle on the host's cores (one Rings frame
    per worker process, all workers at once), with the CPU model;
  * legs for the other workloads: tiny (2 x 2,048-triangle tori, latency and
    error against the oracle's brute force), batched (256 mesh pairs of 1K-500K
    triangles in one call), hard (two concentric noisy spheres of 1,997,120
    triangles, min and max, FP32 vs FP64 error), serving (64 resident meshes,
    Poisson arrivals at several rates, served vs plain under the same
    arrivals, every served result equal to the plain one).

Prints ONE JSON line.
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

HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden")
TUNING = os.path.join(ROOT, "paper_2411_11244_amd", "tuning")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--latency-frames", type=int, default=100)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="oracle worker processes of the CPU baseline, one Rings frame each "
                         "(capped by the host's CPUs; 0 = skip)")
    ap.add_argument("--nu", type=int, default=2740)
    ap.add_argument("--nv", type=int, default=1369)
    ap.add_argument("--tuning", default=os.path.join(TUNING, "rings_mi355x.json"),
                    help="launch options tuned for this workload ('' = library defaults)")
    ap.add_argument("--legs", default="tiny,batched,hard,serving",
                    help="comma-separated legs beside the headline ('' = none)")
    ap.add_argument("--serving-queries", type=int, default=20000, help="queries per arrival rate")
    ap.add_argument("--serving-rates", default="5000,10000,20000,50000",
                    help="offered queries/s of the served form")
    ap.add_argument("--plain-rate", type=float, default=2000.0,
                    help="offered queries/s at which the plain and served forms run the same arrivals")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the measured copy kernel")
    ap.add_argument("--stats-in-timed-steps", type=int, default=0,
                    help="1: the timed steps also count the work statistics")
    ap.add_argument("--count-steps", type=int, default=1,
                    help="steps run after the timed ones with the work statistics on (byte counts)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the timed steps, run one elementwise copy reading and writing this many MiB "
                         "(the scale for rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def pct(x, q):
    return round(float(np.percentile(np.asarray(x), q)), 4) if len(x) else None


def load_golden(name):
    p = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)["records"]


def copy_peak_gbs(mib: int) -> dict:
    """Device copy of `mib` MiB (read + write), median of 5, HIP events on
    torch's stream: the achievable streaming rate on this machine."""
    import torch
    n = mib << 18
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    del src, dst
    ms = float(np.median(ts))
    return {"gbs": round(2 * (mib << 20) / (ms * 1e-3) / 1e9, 1), "mib": mib, "ms": round(ms, 4)}


def trav_roofline(stats, copy_gbs=None, counted=None) -> dict:
    """k_traverse roofline from the kernel's own counters and HIP events.
    `stats`: the timed calls (launch times); `counted`: calls of the same work
    run with the statistics on, whose byte counts give the bytes per launch
    (default: the timed calls themselves)."""
    ms = sum(s["ms_traverse_kernel"] for s in stats)
    launches = sum(s["traverse_launches"] for s in stats)
    cnt = counted if counted else stats
    c_launches = max(1, sum(s["traverse_launches"] for s in cnt))
    b_trav = sum(s["bytes_traversal"] for s in cnt) / c_launches * launches
    b_narrow = sum(s["bytes_narrow"] for s in cnt) / c_launches * launches
    avg = ms / max(1, launches)
    gbs = (b_trav + b_narrow) / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    out = {"bound": "hbm", "kernel": "k_traverse", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4),
           "algorithmic_bytes_per_launch": int((b_trav + b_narrow) / max(1, launches)),
           "bytes_traversal_per_launch": int(b_trav / max(1, launches)),
           "bytes_narrow_per_launch": int(b_narrow / max(1, launches)),
           "avg_ms_per_launch": round(avg, 5), "launches": int(launches)}
    if copy_gbs:
        out["copy_peak_gbs"] = copy_gbs
        out["frac_of_copy"] = round(gbs / copy_gbs, 4)
    return out


def traffic_record():
    """HBM bytes per k_traverse launch from the committed rocprofv3 PMC summary,
    or None when the kernel or its launch configuration changed since."""
    from paper_2411_11244_amd import profsum
    rec = profsum.read_record(os.path.join(ROOT, "profiles", "k_traverse_rings_traffic.md"))
    if not rec or rec.get("sources_sha256") != profsum.sources_sha256():
        return None
    return rec


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rings_frame(args):
    """One Rings frame by the FP64 BVH oracle in a worker process (builds its
    own trees; single thread)."""
    frame, nu, nv = args
    import meshgen as g
    import oracle
    m = g.rings(frames=1, nu=nu, nv=nv).meshes[0]
    t = time.perf_counter()
    r = oracle.query(m.verts, m.tris, g.pose_to_flat(g.identity_pose()), m.verts, m.tris,
                     g.pose_to_flat(g.rings_pose_b(frame)), 0, "bvh")
    return frame, time.perf_counter() - t, r["distance"], r["tri_a"], r["tri_b"], r["n_ties"]


def cpu_baseline(workers: int, nu: int, nv: int) -> dict:
    """The oracle as it stands on the host's cores: `workers` processes, each
    one Rings frame (frames 0 .. workers-1), all at once; throughput =
    frames / wall time.  Also the single-thread time per query."""
    from concurrent.futures import ProcessPoolExecutor
    import oracle
    oracle.build_oracle(force=False)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    n = max(1, min(workers, avail))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(n) as ex:
        rows = list(ex.map(_oracle_rings_frame, [(f, nu, nv) for f in range(n)]))
    wall = time.perf_counter() - t0
    per = [r[1] for r in rows]
    return {"value": round(n / wall, 5), "unit": "queries/s", "cores": n, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus_available": avail,
            "single_thread_s_per_query": round(float(np.median(per)), 3),
            "sample": f"Rings frames 0-{n - 1}, one per worker process, FP64 BVH oracle (its own tree builds "
                      f"included), {n} processes at once, {wall:.1f} s wall",
            "results": {r[0]: {"distance": r[2], "pair": [r[3], r[4]], "n_ties": r[5]} for r in rows}}


def build_timing(mesh, reps: int = 3) -> dict:
    """gdist_build of the Rings mesh from device-resident arrays (torch
    tensors), the library's allocations served by torch's caching allocator,
    median wall time of `reps` builds after one warm-up build."""
    import torch
    from paper_2411_11244_amd import gdist
    ctx = gdist.gdist_create(0)
    live = {}

    def alloc(n, user):
        p = torch.cuda.caching_allocator_alloc(int(n))
        live[p] = int(n)
        return p

    def free(p, user):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    keep = gdist.gdist_set_allocator(ctx, alloc, free)
    ts = []
    try:
        v = torch.from_numpy(mesh.verts).cuda()
        f = torch.from_numpy(mesh.tris.astype(np.int32)).cuda()
        for i in range(reps + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            h = gdist.gdist_build(ctx, v, f)
            ts.append((time.perf_counter() - t) * 1e3)
            gdist.gdist_release(ctx, h)
        del v, f
    finally:
        gdist.gdist_destroy(ctx)
    del keep
    return {"ms": round(float(np.median(ts[1:])), 3), "tris": int(mesh.n_tris),
            "input": "device-resident arrays; synchronous call (vertex pass, key pass, one-sweep radix sort over "
                     "the Morton bits, tree emitted with its boxes, three small copies back)"}


# ---------------------------------------------------------------- legs
def leg_tiny(copy_gbs) -> dict:
    import meshgen as g
    import oracle
    from paper_2411_11244_amd import gdist
    ctx = gdist.gdist_create(0)
    gdist.gdist_set_option(ctx, "stats", 0)
    rows = []
    try:
        for seed in range(10):
            w = g.tiny(seed)
            m, q = w.meshes[0], w.queries[0]
            h = gdist.gdist_build(ctx, m.verts, m.tris)
            for _ in range(10):
                gdist.gdist_query(ctx, h, h, q.pose_a, q.pose_b, 0)
            lat = []
            for _ in range(20):
                t = time.perf_counter()
                r = gdist.gdist_query(ctx, h, h, q.pose_a, q.pose_b, 0)
                lat.append((time.perf_counter() - t) * 1e3)
            dev = gdist.gdist_last_stats(ctx)["ms_total"]
            t = time.perf_counter()
            ref = oracle.query(m.verts, m.tris, g.pose_to_flat(q.pose_a), m.verts, m.tris,
                               g.pose_to_flat(q.pose_b), 0, "brute")
            cpu_s = time.perf_counter() - t
            gdist.gdist_release(ctx, h)
            rows.append({"seed": seed, "p50_ms": pct(lat, 50), "device_ms": round(dev, 4),
                         "abs_err_vs_oracle": abs(r["distance"] - ref["distance"]),
                         "pair_in_ties": [r["tri_a"], r["tri_b"]] in ref["ties"].tolist(),
                         "oracle_brute_s": round(cpu_s, 3)})
    finally:
        gdist.gdist_destroy(ctx)
    return {"workload": "tiny: two 2,048-triangle tori (32x32, R=1, r=0.25), seeds 0-9, one query per call",
            "p50_ms": pct([x["p50_ms"] for x in rows], 50), "p99_ms_over_seeds": pct([x["p50_ms"] for x in rows], 99),
            "max_abs_err_vs_oracle": max(x["abs_err_vs_oracle"] for x in rows),
            "all_pairs_in_ties": all(x["pair_in_ties"] for x in rows),
            "oracle_brute_s_median": pct([x["oracle_brute_s"] for x in rows], 50),
            "oracle_threads": min(16, os.cpu_count() or 1), "tri_tri_tests_per_query": 2048 * 2048,
            "seeds": rows}


def leg_batched(copy_gbs) -> dict:
    import meshgen as g
    from paper_2411_11244_amd import gdist
    gold = {r["pair"]: r for r in (load_golden("batched_all") or [])}
    ctx = gdist.gdist_create(0)
    tuned = None
    try:
        path = os.path.join(TUNING, "batched_mi355x.json")
        if os.path.exists(path):
            from paper_2411_11244_amd import tune
            tuned = tune.apply(ctx, path).get("best")
        hs, descs, total = [], [], 0
        for p in range(256):
            ma, mb, pa, pb, _ = g.batched_pair(1, p)
            ha, hb = gdist.gdist_build(ctx, ma.verts, ma.tris), gdist.gdist_build(ctx, mb.verts, mb.tris)
            total += ma.n_tris + mb.n_tris
            descs.append(gdist.make_desc(ha, hb, pa, pb, 0))
        gdist.gdist_set_option(ctx, "stats", 0)
        for _ in range(2):
            gdist.gdist_query_batch(ctx, descs)
        ts, stats = [], []
        for _ in range(5):
            t = time.perf_counter()
            res = gdist.gdist_query_batch(ctx, descs)
            ts.append(time.perf_counter() - t)
            stats.append(gdist.gdist_last_stats(ctx))
        lat, plain = [], []
        for d in descs:
            t = time.perf_counter()
            r = gdist.gdist_query(ctx, d.a, d.b, (np.array(d.pa.R).reshape(3, 3), np.array(d.pa.t)),
                                  (np.array(d.pb.R).reshape(3, 3), np.array(d.pb.t)), 0)
            lat.append((time.perf_counter() - t) * 1e3)
            plain.append(r)
        # one more call with the work statistics on: the byte and work counts
        gdist.gdist_set_option(ctx, "stats", 1)
        gdist.gdist_query_batch(ctx, descs)
        counted = [gdist.gdist_last_stats(ctx)]
    finally:
        gdist.gdist_destroy(ctx)
    ms = float(np.median(ts)) * 1e3
    errs = [abs(r["distance"] - gold[p]["distance"]) for p, r in enumerate(res) if p in gold]
    pairs = [(r["tri_a"], r["tri_b"]) == (gold[p]["tri_a"], gold[p]["tri_b"]) for p, r in enumerate(res) if p in gold]
    st = counted[-1]
    return {"workload": "batched: 256 mesh pairs (seed 1), 1K-500K triangles each, one gdist_query_batch call",
            "launch_options": tuned, "tris_total": total, "ms_per_call": round(ms, 3), "queries_per_s": round(256 / (ms * 1e-3), 1),
            "plain_p50_ms": pct(lat, 50), "plain_p99_ms": pct(lat, 99),
            "plain_queries_per_s": round(256 / (sum(lat) * 1e-3), 1),
            "batched_equals_plain": all(a["distance"] == b["distance"] and (a["tri_a"], a["tri_b"]) ==
                                        (b["tri_a"], b["tri_b"]) for a, b in zip(res, plain)),
            "oracle_checked": len(errs), "max_abs_err_vs_oracle": max(errs) if errs else None,
            "pairs_equal_oracle": all(pairs) if pairs else None,
            "roofline": trav_roofline(stats, copy_gbs, counted),
            "counts": {k: st[k] for k in ("rounds", "entries_popped", "child_pairs", "child_boxes", "entries_pushed",
                                          "leaf_pairs", "leaf_tris", "tri_pairs", "tri_full", "candidates")}}


def leg_hard(copy_gbs) -> dict:
    import meshgen as g
    from paper_2411_11244_amd import gdist
    w = g.hard(seed=4, n=316)
    A, B = w.meshes
    out = {"workload": f"hard: two concentric noisy geodesic spheres, {A.n_tris:,} triangles each, radii 1 and "
                       "1.0001, radial noise U[-2e-5, 2e-5] (seed 4)"}
    ctx = gdist.gdist_create(0)
    try:
        ha, hb = gdist.gdist_build(ctx, A.verts, A.tris), gdist.gdist_build(ctx, B.verts, B.tris)
        for mode, name, reps in ((0, "min", 5), (1, "max", 3)):
            q = w.queries[mode]
            gdist.gdist_set_option(ctx, "stats", 0)
            gdist.gdist_query(ctx, ha, hb, q.pose_a, q.pose_b, mode)
            ts, stats = [], []
            for _ in range(reps):
                t = time.perf_counter()
                r = gdist.gdist_query(ctx, ha, hb, q.pose_a, q.pose_b, mode)
                ts.append((time.perf_counter() - t) * 1e3)
                stats.append(gdist.gdist_last_stats(ctx))
            gdist.gdist_set_option(ctx, "stats", 1)   # one counted call: the byte and work counts
            gdist.gdist_query(ctx, ha, hb, q.pose_a, q.pose_b, mode)
            counted = [gdist.gdist_last_stats(ctx)]
            gold = (load_golden("hard_max" if mode else "hard_min") or [None])[0]
            st = stats[-1]
            out[name] = {"ms_median": pct(ts, 50), "device_ms": round(st["ms_total"], 3), "rounds": st["rounds"],
                         "front_peak": st["front_peak"], "distance": r["distance"],
                         "fp32_minus_fp64": r["distance_fp32"] - r["distance"],
                         "abs_err_vs_oracle": abs(r["distance"] - gold["distance"]) if gold else None,
                         "pair_equals_oracle": ((r["tri_a"], r["tri_b"]) == (gold["tri_a"], gold["tri_b"]))
                                               if gold else None,
                         "n_ties": r["n_ties"], "roofline": trav_roofline(stats, copy_gbs, counted)}
    finally:
        gdist.gdist_destroy(ctx)
    return out


def leg_serving(n_queries: int, rates, plain_rate: float) -> dict:
    """The serving configuration on its own context: 64 resident meshes, one
    seeded stream (seed 3) replayed at each offered rate by the tuned server;
    at `plain_rate` the plain form runs the same open-loop arrivals; every
    served result must equal the plain one."""
    import meshgen as g
    from paper_2411_11244_amd import gdist, tune
    from paper_2411_11244_amd.serve import compare, run_plain_stream, run_stream
    path = os.path.join(TUNING, "serving_mi355x.json")
    pool = g.serving_pool(2, 64)
    base = 1000.0
    qs = g.serving_stream(pool, base, n_queries, seed=3)
    ctx = gdist.gdist_create(0)
    rows = []
    try:
        tune.apply(ctx, path)
        gdist.gdist_set_option(ctx, "stats", 0)
        sc = tune.server_config(path)
        hs = [gdist.gdist_build(ctx, m.verts, m.tris) for m in pool]
        cmp = compare(ctx, hs, qs, None, keep_plain=True)
        plain_ref = cmp.pop("plain_results")

        def same(a, b):
            return a["distance"] == b["distance"] and (a["tri_a"], a["tri_b"]) == (b["tri_a"], b["tri_b"])

        for rate in [plain_rate] + list(rates):
            out = run_stream(ctx, hs, qs, sc.get("max_slots", 64), sc.get("rounds_per_step", 4),
                             time_scale=base / rate, timeout_s=300)
            lat = out["latency_ms"]
            row = {"offered_qps": rate, "form": "served", "completed_qps": round(n_queries / out["wall_s"], 1),
                   "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                   "served_equal_plain": all(same(a, b) for a, b in zip(out["results"], plain_ref)),
                   "all_ok": all(r["status"] == 0 for r in out["results"]), "steps": out["stats"]["steps"]}
            rows.append(row)
            if rate == plain_rate:
                po = run_plain_stream(ctx, hs, qs, time_scale=base / rate, timeout_s=300)
                rows.append({"offered_qps": rate, "form": "plain (one gdist_query per arrival)",
                             "completed_qps": round(n_queries / po["wall_s"], 1),
                             "p50_ms": pct(po["latency_ms"], 50), "p99_ms": pct(po["latency_ms"], 99)})
    finally:
        gdist.gdist_destroy(ctx)
    return {"workload": "serving: 64 resident meshes (pool seed 2, 10K-2M triangles), Poisson arrivals (stream "
                        "seed 3), uniform random pairs and poses, half max mode, 10% overlapping",
            "pool_tris": sum(m.n_tris for m in pool), "queries_per_rate": n_queries, "server": sc,
            "rates": rows, "closed_loop": cmp}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)

    # the CPU baseline's worker processes are forked before this process
    # touches the GPU
    cpu = cpu_baseline(args.cpu_workers, args.nu, args.nv) if args.cpu_workers > 0 else None
    print("[bench] cpu baseline done", file=sys.stderr, flush=True)

    import torch

    import meshgen as g
    from paper_2411_11244_amd import gdist

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.init()
    w = g.rings(frames=args.frames, nu=args.nu, nv=args.nv)
    mesh = w.meshes[0]
    ctx = gdist.gdist_create(0)
    tuned = None
    if args.tuning:
        from paper_2411_11244_amd import tune
        tuned = tune.apply(ctx, args.tuning).get("best")
    h = gdist.gdist_build(ctx, mesh.verts, mesh.tris)
    info = gdist.gdist_mesh_info(ctx, h)
    descs = [gdist.make_desc(h, h, q.pose_a, q.pose_b, gdist.GDIST_MIN) for q in w.queries]
    # timed steps without the work statistics (diagnostic counters, not part
    # of the method); the same step is then run --count-steps times with them
    # on for the byte and work counts
    gdist.gdist_set_option(ctx, "stats", 1 if args.stats_in_timed_steps else 0)

    # ---- warmup + timed steps: one batched call over all frames per step
    for _ in range(args.warmup):
        gdist.gdist_query_batch(ctx, descs)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = gdist.gdist_query_batch(ctx, descs)
        stats.append(gdist.gdist_last_stats(ctx))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    qps = args.frames * args.steps / (t1 - t0)
    counted = []
    if args.count_steps > 0:
        gdist.gdist_set_option(ctx, "stats", 1)
        for _ in range(args.count_steps):
            gdist.gdist_query_batch(ctx, descs)
            counted.append(gdist.gdist_last_stats(ctx))
        gdist.gdist_set_option(ctx, "stats", 1 if args.stats_in_timed_steps else 0)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    copy = copy_peak_gbs(args.copy_mib) if args.copy_mib > 0 else None
    copy_gbs = copy["gbs"] if copy else None

    # ---- dominant kernel: k_traverse, timed by the library's HIP events
    # around each of its launches on the library's stream (the timed steps only)
    roof = trav_roofline(stats, copy_gbs, counted)
    pmc = traffic_record()
    avg_s = roof["avg_ms_per_launch"] * 1e-3
    roof["traffic"] = pmc["traffic_bytes_per_launch"] if pmc else None
    roof["traffic_gbs"] = round(pmc["traffic_bytes_per_launch"] / avg_s / 1e9, 1) if pmc else None
    roof["traffic_note"] = ("HBM bytes per launch, rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by a copy kernel "
                            "(profiles/k_traverse_rings_traffic.md)") if pmc else \
        "null: no PMC summary for the current kernel sources and launch options"
    roof["frac_le_1"] = roof["frac"] <= 1.0
    N, L = info["n_tris"], info["n_leaves"]
    refit_bytes = 36 * N + 24 * (2 * L - 1)
    refit_ms = float(np.mean([s["ms_refit"] for s in stats])) / args.frames
    refit = {"kernel": "k_refit_leaves_batch + k_reduce_batch (per 7.5M-triangle tree)",
             "achieved": round(refit_bytes / (refit_ms * 1e-3) / 1e9, 1), "unit": "GB/s",
             "frac": round(refit_bytes / (refit_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "algorithmic_bytes_per_tree": refit_bytes, "avg_ms_per_tree": round(refit_ms, 5)}

    # ---- plain form: one query per call, per-frame latency
    lat, plain_res = [], []
    for q in w.queries[: args.latency_frames]:
        ta = time.perf_counter()
        r = gdist.gdist_query(ctx, h, h, q.pose_a, q.pose_b, gdist.GDIST_MIN)
        lat.append((time.perf_counter() - ta) * 1e3)
        plain_res.append(r)
    agree = all(a["distance"] == b["distance"] and (a["tri_a"], a["tri_b"]) == (b["tri_a"], b["tri_b"])
                for a, b in zip(res, plain_res))
    gdist.gdist_destroy(ctx)
    build = build_timing(mesh)

    # ---- stored oracle results of the Rings frames (tests/golden, written by the oracle)
    verify = None
    gold = load_golden("rings_frames")
    if gold and args.frames == 100 and (args.nu, args.nv) == (2740, 1369):
        errs = [abs(res[r["frame"]]["distance"] - r["distance"]) for r in gold]
        pairs = [(res[r["frame"]]["tri_a"], res[r["frame"]]["tri_b"]) == (r["tri_a"], r["tri_b"]) for r in gold]
        verify = {"frames": [r["frame"] for r in gold], "max_abs_err": max(errs), "pairs_match": all(pairs)}

    legs = {}
    for leg in [x for x in args.legs.split(",") if x]:
        try:
            if leg == "tiny":
                legs[leg] = leg_tiny(copy_gbs)
            elif leg == "batched":
                legs[leg] = leg_batched(copy_gbs)
            elif leg == "hard":
                legs[leg] = leg_hard(copy_gbs)
            elif leg == "serving":
                legs[leg] = leg_serving(args.serving_queries, [float(x) for x in args.serving_rates.split(",") if x],
                                        args.plain_rate)
        except Exception as e:   # the headline line is printed regardless
            legs[leg] = {"error": f"{type(e).__name__}: {e}"}
        print(f"[bench] leg {leg} done", file=sys.stderr, flush=True)

    if cpu is not None:
        if verify is not None:
            verify["cpu_frames_max_abs_err"] = max(abs(res[f]["distance"] - r["distance"])
                                                   for f, r in cpu["results"].items() if f < len(res))
        cpu.pop("results")

    out = {
        "metric": "distance queries/sec at 2x7.5M tris (1 GPU) + p50/p99 latency; HBM GB/s frac",
        "value": round(qps, 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "rings", "tris_per_mesh": N, "frames_per_step": args.frames,
                   "grid": [args.nu, args.nv], "mode": "min", "form": "batched (one call per step)",
                   "launch_options": tuned},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "form": "plain (one query per call)",
                       "plain_queries_per_s": round(1e3 / float(np.mean(lat)), 3) if lat else None},
        "roofline": roof,
        "copy_kernel": copy,
        "refit": refit,
        "build": build,
        "stats_in_timed_steps": bool(args.stats_in_timed_steps),
        "stats_last_step": counted[-1] if counted else stats[-1],
        "batched_equals_plain": agree,
        "cpu_baseline": cpu,
        "verify": verify,
        "legs": legs,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
