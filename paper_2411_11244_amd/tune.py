"""Autotuner for the traversal's launch parameters.

Sweeps the adaptive-depth budget C ("expand_budget": k is the largest value
with 4^k n < C), the per-round depth cap ("k_cap"), the persistent grid size
("blocks_per_cu"), the front buffers ("front_capacity", which also bounds the
entries a round expands; the leaf-pair buffers follow it) and the queries
traversed per launch ("group_size") on a set of sample queries, and keeps the
setting with the lowest median device time.  The choice never changes a
result, only the amount of work per round, the number of rounds and the
locality of the trees' boxes in the caches.

    python -m paper_2411_11244_amd.tune --out tune.json   (needs the GPU)

``apply(ctx, path)`` sets the options stored in a tuning file on a context.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time
from typing import Dict, Iterable, List

import numpy as np

from . import gdist

KEYS = ("expand_budget", "k_cap", "blocks_per_cu", "front_capacity", "group_size")


def _set(ctx: int, k: str, v) -> None:
    gdist.gdist_set_option(ctx, k, float(v))
    if k == "front_capacity":
        gdist.gdist_set_option(ctx, "leaf_capacity", float(v))


def apply(ctx: int, path_or_dict) -> Dict:
    cfg = path_or_dict
    if isinstance(path_or_dict, str):
        with open(path_or_dict) as f:
            cfg = json.load(f)
    best = cfg.get("best", cfg)
    for k in KEYS:
        if k in best:
            _set(ctx, k, best[k])
    return cfg


def time_setting(ctx: int, descs: List, reps: int) -> float:
    """Median device time (ms) of a batched call over `descs`."""
    gdist.gdist_query_batch(ctx, descs)          # warm: capacities settle
    ts = []
    for _ in range(reps):
        gdist.gdist_query_batch(ctx, descs)
        ts.append(gdist.gdist_last_stats(ctx)["ms_total"])
    return float(np.median(ts))


def tune(ctx: int, descs: List, grid: Dict[str, Iterable], reps: int = 3, log=print) -> Dict:
    names = list(grid)
    results = []
    for values in itertools.product(*(grid[n] for n in names)):
        setting = dict(zip(names, values))
        for k, v in setting.items():
            _set(ctx, k, v)
        ms = time_setting(ctx, descs, reps)
        results.append({**setting, "ms": ms})
        log(f"tune {setting} -> {ms:.4f} ms")
    best = min(results, key=lambda r: r["ms"])
    for k in names:
        _set(ctx, k, best[k])
    return {"best": {k: best[k] for k in names}, "ms": best["ms"], "results": results}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rings", choices=["rings", "tiny"])
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--out", default="")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import meshgen as g
    if args.workload == "rings":
        w = g.rings(frames=args.frames)
        sel = np.linspace(0, 99, args.frames).astype(int)
        queries = [g.Query(0, 0, g.identity_pose(), g.rings_pose_b(int(f)), 0) for f in sel]
        w.queries = queries
    else:
        w = g.tiny(0)
    ctx = gdist.gdist_create(0)
    hs = [gdist.gdist_build(ctx, m.verts, m.tris) for m in w.meshes]
    descs = [gdist.make_desc(hs[q.a], hs[q.b], q.pose_a, q.pose_b, q.mode) for q in w.queries]
    grid = {"expand_budget": [1 << 20, 1 << 22], "k_cap": [5, 7], "blocks_per_cu": [0],
            "front_capacity": [1 << 27], "group_size": [16, 12, 10, 8]}
    t = time.time()
    res = tune(ctx, descs, grid, args.reps)
    res["workload"] = args.workload
    res["seconds"] = time.time() - t
    print(json.dumps(res["best"]), res["ms"])
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    gdist.gdist_destroy(ctx)


if __name__ == "__main__":
    main()
