"""Open-loop serving driver for the continuous-batching server (gdist_server_*).

Queries arrive as a Poisson stream (seeded; meshgen.serving_stream) over a
pool of meshes whose sizes are log-uniform; each is submitted at its arrival
time and the completions are polled as they come.  Reported: completed
queries/s over the run, and p50/p99 of the latency from submit to the result
in host memory (the server's own steady-clock stamps).  With --compare, the
same queries are also run in the plain form (one gdist_query per query, back
to back: queries/s and per-call latency) and as one gdist_query_batch call,
and every served result is checked against its plain result.

    python -m paper_2411_11244_amd.serve --rate 5000 --queries 2000 --pool 64 --compare

All distance work runs in libgdist.so; this file only schedules submissions.
"""
from __future__ import annotations

import argparse
import gc
import json
import time
from typing import List, Sequence

import numpy as np

from . import gdist


def run_stream(ctx: int, handles: Sequence[int], queries, max_slots: int = 64, rounds_per_step: int = 4,
               front_capacity: int = 0, cand_per_slot: int = 0, time_scale: float = 1.0,
               timeout_s: float = 300.0, stack_capacity: int = 0, direct: bool = False) -> dict:
    """Submit ``queries`` (meshgen.Query with .arrival seconds) at their arrival
    times (scaled by ``time_scale``; 0 submits everything at once) and collect
    every completion.  Returns {"results": [dict per query, in query order],
    "latency_ms": np.ndarray, "wall_s": float, "stats": server stats}.
    ``direct`` launches each step's kernels one by one instead of replaying
    the step graph.  Python's cyclic garbage collector is off while the
    stream runs: a collection pause (tens of ms once the results pile up)
    would hold back the arrivals due meanwhile and submit them as one burst,
    a queueing delay made by the driver, not the server."""
    srv = gdist.gdist_server_start(ctx, max_slots, rounds_per_step, front_capacity, cand_per_slot, 0,
                                   stack_capacity, gdist.GDIST_SERVER_DIRECT if direct else 0)
    n = len(queries)
    results: List[dict] = [None] * n  # type: ignore
    got = 0
    gc_on = gc.isenabled()
    try:
        descs = [gdist.make_desc(handles[q.a], handles[q.b], q.pose_a, q.pose_b, q.mode) for q in queries]
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        nxt = 0
        deadline = t0 + timeout_s
        while got < n:
            now = time.perf_counter()
            while nxt < n and (time_scale == 0 or queries[nxt].arrival * time_scale <= now - t0):
                gdist.gdist_server_submit(srv, descs[nxt], nxt)
                nxt += 1
            for c in gdist.gdist_server_poll(srv, 1024):
                results[c["tag"]] = c
                got += 1
            if now > deadline:
                raise TimeoutError(f"server finished {got} of {n} queries in {timeout_s} s")
            if got < n:
                time.sleep(0.0002)
        wall = time.perf_counter() - t0
        stats = gdist.gdist_server_stats(srv)
    finally:
        if gc_on:
            gc.enable()
        gdist.gdist_server_stop(srv)
    lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) * 1e-6 for r in results])
    return {"results": results, "latency_ms": lat, "wall_s": wall, "stats": stats}


def run_plain_stream(ctx: int, handles: Sequence[int], queries, time_scale: float = 1.0,
                     timeout_s: float = 300.0) -> dict:
    """The plain form under the same open-loop arrivals: one gdist_query per
    query, issued at its arrival time (or as soon as the previous call
    returns, if that is later).  Latency = completion - arrival, so it
    includes the time a query waited behind earlier ones.  As in run_stream,
    Python's cyclic garbage collector is off while the stream runs.  Returns
    {"results", "latency_ms", "wall_s"}."""
    n = len(queries)
    results: List[dict] = []
    lat = np.zeros(n)
    gc.collect()
    gc_on = gc.isenabled()
    gc.disable()
    try:
        return _plain_stream(ctx, handles, queries, time_scale, timeout_s, results, lat)
    finally:
        if gc_on:
            gc.enable()


def _plain_stream(ctx, handles, queries, time_scale, timeout_s, results, lat) -> dict:
    n = len(queries)
    t0 = time.perf_counter()
    deadline = t0 + timeout_s
    for i, q in enumerate(queries):
        due = t0 + q.arrival * time_scale
        while True:
            now = time.perf_counter()
            if now >= due:
                break
            if due - now > 0.0005:
                time.sleep(0.0002)
        results.append(gdist.gdist_query(ctx, handles[q.a], handles[q.b], q.pose_a, q.pose_b, q.mode))
        lat[i] = (time.perf_counter() - due) * 1e3
        if time.perf_counter() > deadline:
            raise TimeoutError(f"plain stream finished {i + 1} of {n} queries in {timeout_s} s")
    return {"results": results, "latency_ms": lat, "wall_s": time.perf_counter() - t0}


def main(argv=None) -> int:
    import meshgen as g

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--rate", type=float, default=400.0, help="arrivals per second")
    ap.add_argument("--queries", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=16, help="meshes in the pool")
    ap.add_argument("--tmin", type=float, default=1e4)
    ap.add_argument("--tmax", type=float, default=2e6)
    ap.add_argument("--slots", type=int, default=0, help="server slots (0: the tuning file's, else 64)")
    ap.add_argument("--rounds", type=int, default=0, help="rounds per step (0: the tuning file's, else 4)")
    ap.add_argument("--tuning", default="", help="tuning file written by tune.py --workload serving")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--direct", action="store_true", help="launch each step's kernels one by one (no graph)")
    ap.add_argument("--compare", action="store_true",
                    help="also run the queries in the plain form and as one batch, and check the served results")
    a = ap.parse_args(argv)
    pool = g.serving_pool(a.seed, a.pool, a.tmin, a.tmax)
    qs = g.serving_stream(pool, a.rate, a.queries, seed=a.seed + 1)
    ctx = gdist.gdist_create(0)
    try:
        gdist.gdist_set_option(ctx, "stats", 0)   # diagnostic counters off while serving
        tuned = {}
        if a.tuning:
            from . import tune
            tune.apply(ctx, a.tuning)
            tuned = tune.server_config(a.tuning)
        a.slots = a.slots or tuned.get("max_slots", 64)
        a.rounds = a.rounds or tuned.get("rounds_per_step", 4)
        handles = [gdist.gdist_build(ctx, m.verts, m.tris) for m in pool]
        out = run_stream(ctx, handles, qs, a.slots, a.rounds, direct=a.direct)
        cmp = compare(ctx, handles, qs, out["results"]) if a.compare else None
    finally:
        gdist.gdist_destroy(ctx)
    lat = out["latency_ms"]
    ok = sum(1 for r in out["results"] if r["status"] == gdist.GDIST_OK)
    print(json.dumps({"completed_qps": round(len(qs) / out["wall_s"], 2), "ok": ok, "n": len(qs),
                      "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3),
                      "offered_rate": a.rate, "pool": a.pool, "pool_tris": sum(m.n_tris for m in pool),
                      "slots": a.slots, "rounds_per_step": a.rounds, "stats": out["stats"], "compare": cmp}))
    return 0


def compare(ctx: int, handles: Sequence[int], queries, served: List[dict] = None, keep_plain: bool = False) -> dict:
    """The same queries in the plain form (one gdist_query each, back to back)
    and as one gdist_query_batch call; every served result (if given) must
    equal its plain result (same FP64 distance bits and pair).  keep_plain
    adds the plain results under "plain_results"."""
    plain, lat = [], []
    t0 = time.perf_counter()
    for q in queries:
        t = time.perf_counter()
        plain.append(gdist.gdist_query(ctx, handles[q.a], handles[q.b], q.pose_a, q.pose_b, q.mode))
        lat.append((time.perf_counter() - t) * 1e3)
    plain_s = time.perf_counter() - t0
    descs = [gdist.make_desc(handles[q.a], handles[q.b], q.pose_a, q.pose_b, q.mode) for q in queries]
    gdist.gdist_query_batch(ctx, descs)   # warm: grows the batch storage once
    t0 = time.perf_counter()
    batch = gdist.gdist_query_batch(ctx, descs)
    batch_s = time.perf_counter() - t0

    def same(r, a):
        return r["distance"] == a["distance"] and (r["tri_a"], r["tri_b"]) == (a["tri_a"], a["tri_b"])

    lat = np.array(lat)
    out = {"plain_qps": round(len(queries) / plain_s, 2), "plain_p50_ms": round(float(np.percentile(lat, 50)), 3),
           "plain_p99_ms": round(float(np.percentile(lat, 99)), 3),
           "batch_qps": round(len(queries) / batch_s, 2), "batch_ms": round(batch_s * 1e3, 2),
           "batch_equal_plain": all(same(r, a) for r, a in zip(batch, plain))}
    if served is not None:
        out["served_equal_plain"] = all(same(r, a) for r, a in zip(served, plain))
    if keep_plain:
        out["plain_results"] = plain
    return out


if __name__ == "__main__":
    raise SystemExit(main())
