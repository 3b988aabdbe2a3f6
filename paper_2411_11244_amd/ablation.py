"""Ablations of the traversal (gDist Sec. 7, "Ablation Studies").

Three variants run on the same queries:
  gdist     enhanced upper bounds (Sec. 4) and adaptive expansion depth (Sec. 5);
  v1        conventional bounds only (option bounds=1): the enhanced bound
            computation is off;
  v2        no adaptive depth (option k_cap=1): every round expands one level
            per side, as in a plain breadth-first BVTT traversal.
Reported per workload: device time of the batched call and the BVTT node
counts (child pairs evaluated, pairs pushed, leaf pairs), each as a ratio to
gdist (time) or of gdist to v1 (nodes: the paper's enhanced/conventional
ratio).  The distances must not change.

    python -m paper_2411_11244_amd.ablation --workloads rings,batched,hard_min
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from typing import Dict, List, Tuple

import numpy as np

from . import gdist, tune

HERE = os.path.dirname(os.path.abspath(__file__))
VARIANTS = (("gdist", {}), ("v1", {"bounds": 1}), ("v2", {"k_cap": 1}))
NODES = ("child_pairs", "entries_pushed", "leaf_pairs")
DEFAULT_K_CAP = 8   # the library's default


def _workload(name: str, ctx: int) -> Tuple[List, List[int]]:
    sys.path.insert(0, os.path.dirname(HERE))
    import meshgen as g
    if name == "rings":
        w = g.rings(frames=100)
        hs = [gdist.gdist_build(ctx, m.verts, m.tris) for m in w.meshes]
        return [gdist.make_desc(hs[0], hs[0], q.pose_a, q.pose_b, 0) for q in w.queries], hs
    if name == "batched":
        descs, hs = [], []
        for p in range(256):
            ma, mb, pa, pb, _ = g.batched_pair(1, p)
            ha, hb = gdist.gdist_build(ctx, ma.verts, ma.tris), gdist.gdist_build(ctx, mb.verts, mb.tris)
            hs += [ha, hb]
            descs.append(gdist.make_desc(ha, hb, pa, pb, 0))
        return descs, hs
    if name in ("hard_min", "hard_max"):
        w = g.hard(seed=4, n=316)
        hs = [gdist.gdist_build(ctx, m.verts, m.tris) for m in w.meshes]
        mode = 0 if name == "hard_min" else 1
        q = w.queries[mode]
        return [gdist.make_desc(hs[0], hs[1], q.pose_a, q.pose_b, mode)], hs
    raise ValueError(f"unknown workload {name}")


def _run(ctx: int, descs: List, opts: Dict, reps: int) -> Dict:
    for k, v in opts.items():
        gdist.gdist_set_option(ctx, k, float(v))
    res = gdist.gdist_query_batch(ctx, descs)      # warm: capacities settle
    ms = []
    for _ in range(reps):
        res = gdist.gdist_query_batch(ctx, descs)
        ms.append(gdist.gdist_last_stats(ctx)["ms_total"])
    st = gdist.gdist_last_stats(ctx)
    return {"ms": float(np.median(ms)), **{k: int(st[k]) for k in NODES},
            "distances": [r["distance"] for r in res]}


def ablate(names: List[str], reps: int = 3, log=print) -> Dict:
    out = {}
    for name in names:
        ctx = gdist.gdist_create(0)
        try:
            tuned = {}
            if name == "rings":
                tuned = tune.apply(ctx, os.path.join(HERE, "tuning", "rings_mi355x.json"))["best"]
            base = {"bounds": 0, "k_cap": tuned.get("k_cap", DEFAULT_K_CAP)}
            descs, hs = _workload(name, ctx)
            rec = {}
            for vname, opts in VARIANTS:
                for k, v in base.items():
                    gdist.gdist_set_option(ctx, k, float(v))
                rec[vname] = _run(ctx, descs, opts, reps)
            g0 = rec["gdist"]
            summary = {"queries": len(descs),
                       "same_distances": all(rec[v]["distances"] == g0["distances"] for v in ("v1", "v2"))}
            for vname, _ in VARIANTS:
                r = rec[vname]
                summary[vname] = {"ms": round(r["ms"], 3), "time_ratio": round(r["ms"] / g0["ms"], 3),
                                  **{k: r[k] for k in NODES}}
            summary["nodes_gdist_over_v1"] = {k: round(g0[k] / max(1, rec["v1"][k]), 4) for k in NODES}
            out[name] = summary
            log(json.dumps({name: summary}))
        finally:
            gdist.gdist_destroy(ctx)
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workloads", default="rings,batched,hard_min")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    res = ablate(a.workloads.split(","), a.reps)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
