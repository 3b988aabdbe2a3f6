"""Write the stored expected values of the full-size parity tests.

Calls only the FP64 CPU oracle (oracle/) and the seeded input generators
(meshgen/); nothing here touches the GPU library.  Each record holds the
oracle's optimum, its canonical pair (lexicographically smallest pair within
tau of the optimum), the size of that tie set and the tolerance tau.

    python tests/golden/make_golden.py [rings] [hard_min] [hard_max] [batched] [batched_all] [serving]

Writes tests/golden/<name>.json.  Run times on 8 host cores: rings about a
minute, hard_min a few minutes, hard_max about ten minutes (10^12 vertex
pairs), batched a few minutes, batched_all and serving some minutes each
(independent queries run in parallel worker processes, one thread each).
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import meshgen as g  # noqa: E402
import oracle  # noqa: E402

RINGS_FRAMES = [0, 37, 99]
BATCHED_PAIRS = list(range(12))
HARD = dict(seed=4, n=316)
# serving stream (pool seed 2, 64 meshes; stream seed 3): the first 200
# queries (about half in max mode, 10 overlapping, 15 on the largest mesh of
# about 1.9M triangles)
SERVING = dict(pool_seed=2, n_meshes=64, stream_seed=3, rate=5000.0, stream_len=200)
SERVING_QUERIES = list(range(200))
WORKERS = max(1, min(8, os.cpu_count() or 1))


def record(name, mode, res, seconds, **extra):
    return {"name": name, "mode": mode, "distance": res["distance"], "tri_a": res["tri_a"],
            "tri_b": res["tri_b"], "n_ties": res["n_ties"], "tau": res["tau"],
            "method": res["method"], "seconds": round(seconds, 2), **extra}


def write(name, recs):
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump({"generator": "tests/golden/make_golden.py", "records": recs}, f, indent=1)
    print("wrote", name, len(recs), "records", flush=True)


def rings():
    w = g.rings(frames=1)
    m = w.meshes[0]
    recs = []
    for f in RINGS_FRAMES:
        pa, pb = g.identity_pose(), g.rings_pose_b(f)
        t = time.time()
        r = oracle.query(m.verts, m.tris, g.pose_to_flat(pa), m.verts, m.tris, g.pose_to_flat(pb), 0, "bvh")
        recs.append(record("rings", 0, r, time.time() - t, frame=f))
        print(recs[-1], flush=True)
    write("rings_frames", recs)


def hard(mode):
    w = g.hard(**HARD)
    A, B = w.meshes
    q = w.queries[mode]
    t = time.time()
    if mode == 0:
        r = oracle.query(A.verts, A.tris, g.pose_to_flat(q.pose_a), B.verts, B.tris, g.pose_to_flat(q.pose_b),
                         0, "bvh")
    else:
        r = oracle.max_by_vertices(A.verts, A.tris, g.pose_to_flat(q.pose_a), B.verts, B.tris,
                                   g.pose_to_flat(q.pose_b), threads=os.cpu_count() or 8)
    rec = record("hard", mode, r, time.time() - t, **HARD)
    print(rec, flush=True)
    write("hard_max" if mode else "hard_min", [rec])


def batched():
    recs = []
    for p in BATCHED_PAIRS:
        ma, mb, pa, pb, gap = g.batched_pair(1, p)
        t = time.time()
        r = oracle.query(ma.verts, ma.tris, g.pose_to_flat(pa), mb.verts, mb.tris, g.pose_to_flat(pb), 0)
        recs.append(record("batched", 0, r, time.time() - t, seed=1, pair=p, gap=gap,
                           tris=[ma.n_tris, mb.n_tris]))
        print(recs[-1], flush=True)
    write("batched_pairs", recs)


def _one_query(args):
    """One oracle query in a worker process (single thread): min mode by the
    oracle's BVH (brute force for small pair counts), max mode by the BVH or,
    for pairs whose max-mode culling is weak, by vertex pairs."""
    va, fa, pa, vb, fb, pb, mode = args
    t = time.time()
    if mode == 0:
        r = oracle.query(va, fa, pa, vb, fb, pb, 0, "auto", threads=1)
    else:
        r = oracle.query(va, fa, pa, vb, fb, pb, 1, "auto" if len(fa) * len(fb) <= 8_000_000 else "bvh",
                         threads=1)
    return r, time.time() - t


def batched_all():
    """Every pair of the 256-pair batched workload (seed 1)."""
    jobs, meta = [], []
    for p in range(256):
        ma, mb, pa, pb, gap = g.batched_pair(1, p)
        jobs.append((ma.verts, ma.tris, g.pose_to_flat(pa), mb.verts, mb.tris, g.pose_to_flat(pb), 0))
        meta.append(dict(seed=1, pair=p, gap=gap, tris=[ma.n_tris, mb.n_tris]))
    recs = []
    with ProcessPoolExecutor(WORKERS) as ex:
        for (r, dt), m in zip(ex.map(_one_query, jobs), meta):
            recs.append(record("batched", 0, r, dt, **m))
            print(recs[-1], flush=True)
    write("batched_all", recs)


def serving():
    pool = g.serving_pool(SERVING["pool_seed"], SERVING["n_meshes"])
    qs = g.serving_stream(pool, SERVING["rate"], SERVING["stream_len"], seed=SERVING["stream_seed"])
    jobs, meta = [], []
    for i in SERVING_QUERIES:
        q = qs[i]
        ma, mb = pool[q.a], pool[q.b]
        jobs.append((ma.verts, ma.tris, g.pose_to_flat(q.pose_a), mb.verts, mb.tris, g.pose_to_flat(q.pose_b),
                     q.mode))
        meta.append(dict(query=i, a=q.a, b=q.b, gap=q.gap, tris=[ma.n_tris, mb.n_tris], **SERVING))
    recs = []
    with ProcessPoolExecutor(WORKERS) as ex:
        for (r, dt), m, i in zip(ex.map(_one_query, jobs), meta, SERVING_QUERIES):
            recs.append(record("serving", qs[i].mode, r, dt, **m))
            print(recs[-1], flush=True)
    write("serving_stream", recs)


if __name__ == "__main__":
    oracle.build_oracle(force=False)
    todo = sys.argv[1:] or ["rings", "hard_min", "hard_max", "batched"]
    for job in todo:
        {"rings": rings, "hard_min": lambda: hard(0), "hard_max": lambda: hard(1), "batched": batched,
         "batched_all": batched_all, "serving": serving}[job]()
