"""Full-size parity: the GPU path against stored FP64 oracle results.

The expected values in tests/golden/*.json were written by
tests/golden/make_golden.py, which calls only the CPU oracle and the seeded
generators.  The workloads are the full-size configurations: the Rings
sequence (two 7.5M-triangle tori, frames 0, 37 and 99), the Hard pair (two
concentric noisy geodesic spheres of about 2M triangles each, min and max),
the first twelve pairs of the batched workload (sizes log-uniform in
[1e3, 5e5] triangles) and all 256 of its pairs in one call, and the first
200 queries of the serving stream (64 resident meshes of 10K-2M triangles,
half in max mode, some overlapping), served and batched.

Bar: distance within 1e-6 absolute or 1e-5 relative of the oracle's; the
reported pair is in the tie set (its own FP64 distance within tau of the
oracle's optimum) and equals the oracle's canonical pair (the lexicographically
smallest pair of the tie set); the tie counts agree; the points lie on the
pair's triangles and realise its distance.
"""
import json
import os

import numpy as np
import pytest

import meshgen as g
from gpu_common import on_triangle, world_tri
from paper_2411_11244_amd import gdist

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)["records"]


def check_golden(orc, r, rec, ma, pa, mb, pb, mode):
    D = rec["distance"]
    assert r["status"] == 0, r
    assert abs(r["distance"] - D) <= max(1e-6, 1e-5 * abs(D)), (r["distance"], D)
    Pa, Pb = world_tri(ma, pa, r["tri_a"]), world_tri(mb, pb, r["tri_b"])
    dp = (orc.tri_tri_max if mode else orc.tri_tri_min)(Pa, Pb)[0]
    assert abs(dp - D) <= rec["tau"] + 1e-14 * max(1.0, abs(D)), ("pair not in tie set", dp, D)
    assert (r["tri_a"], r["tri_b"]) == (rec["tri_a"], rec["tri_b"])
    assert r["n_ties"] == rec["n_ties"]
    assert bool(r["flags"] & gdist.GDIST_F_TIED) == (rec["n_ties"] > 1)
    tol = 1e-9 * max(1.0, float(np.abs(Pa).max()), float(np.abs(Pb).max()))
    xa, xb = np.asarray(r["point_a"]), np.asarray(r["point_b"])
    assert on_triangle(xa, Pa, tol) and on_triangle(xb, Pb, tol)
    assert abs(np.linalg.norm(xa - xb) - dp) <= tol


@pytest.fixture(scope="module")
def rings_mesh(gctx):
    m = g.rings(frames=1).meshes[0]
    h = gdist.gdist_build(gctx, m.verts, m.tris)
    yield m, h
    gdist.gdist_release(gctx, h)


@pytest.mark.parametrize("rec", _load("rings_frames"), ids=lambda r: f"frame{r['frame']}")
def test_rings_frame(orc, gctx, rings_mesh, rec):
    m, h = rings_mesh
    pa, pb = g.identity_pose(), g.rings_pose_b(rec["frame"])
    r = gdist.gdist_query(gctx, h, h, pa, pb, 0)
    check_golden(orc, r, rec, m, pa, m, pb, 0)


def test_rings_frames_batched(orc, gctx, rings_mesh):
    """The three frames in one gdist_query_batch call (the launch shape of the
    throughput measurement) give the same answers."""
    m, h = rings_mesh
    recs = _load("rings_frames")
    descs = [gdist.make_desc(h, h, g.identity_pose(), g.rings_pose_b(rec["frame"]), 0) for rec in recs]
    out = gdist.gdist_query_batch(gctx, descs)
    for r, rec in zip(out, recs):
        check_golden(orc, r, rec, m, g.identity_pose(), m, g.rings_pose_b(rec["frame"]), 0)


@pytest.fixture(scope="module")
def hard_pair(gctx):
    rec = _load("hard_min")[0]
    w = g.hard(seed=rec["seed"], n=rec["n"])
    A, B = w.meshes
    ha, hb = gdist.gdist_build(gctx, A.verts, A.tris), gdist.gdist_build(gctx, B.verts, B.tris)
    yield w, ha, hb
    gdist.gdist_release(gctx, ha)
    gdist.gdist_release(gctx, hb)


@pytest.mark.parametrize("name", ["hard_min", "hard_max"])
def test_hard(orc, gctx, hard_pair, name):
    rec = _load(name)[0]
    w, ha, hb = hard_pair
    A, B = w.meshes
    q = w.queries[rec["mode"]]
    r = gdist.gdist_query(gctx, ha, hb, q.pose_a, q.pose_b, rec["mode"])
    check_golden(orc, r, rec, A, q.pose_a, B, q.pose_b, rec["mode"])


def test_batched_pairs(orc, gctx):
    recs = _load("batched_pairs")
    meshes, handles, descs = [], [], []
    try:
        for rec in recs:
            ma, mb, pa, pb, gap = g.batched_pair(rec["seed"], rec["pair"])
            assert [ma.n_tris, mb.n_tris] == rec["tris"]
            ha, hb = gdist.gdist_build(gctx, ma.verts, ma.tris), gdist.gdist_build(gctx, mb.verts, mb.tris)
            handles += [ha, hb]
            meshes.append((ma, pa, mb, pb))
            descs.append(gdist.make_desc(ha, hb, pa, pb, 0))
        out = gdist.gdist_query_batch(gctx, descs)
        for r, rec, (ma, pa, mb, pb) in zip(out, recs, meshes):
            check_golden(orc, r, rec, ma, pa, mb, pb, 0)
            assert r["distance"] >= rec["gap"] - 1e-9
    finally:
        for h in handles:
            gdist.gdist_release(gctx, h)


def test_batched_all_pairs(orc, gctx):
    """All 256 pairs of the batched workload in one gdist_query_batch call
    (the workload's launch shape) against the stored oracle results."""
    recs = _load("batched_all")
    assert len(recs) == 256
    meshes, handles, descs = [], [], []
    try:
        for rec in recs:
            ma, mb, pa, pb, gap = g.batched_pair(rec["seed"], rec["pair"])
            assert [ma.n_tris, mb.n_tris] == rec["tris"]
            ha, hb = gdist.gdist_build(gctx, ma.verts, ma.tris), gdist.gdist_build(gctx, mb.verts, mb.tris)
            handles += [ha, hb]
            meshes.append((ma, pa, mb, pb))
            descs.append(gdist.make_desc(ha, hb, pa, pb, 0))
        out = gdist.gdist_query_batch(gctx, descs)
        for r, rec, (ma, pa, mb, pb) in zip(out, recs, meshes):
            check_golden(orc, r, rec, ma, pa, mb, pb, 0)
            assert r["distance"] >= rec["gap"] - 1e-9
    finally:
        for h in handles:
            gdist.gdist_release(gctx, h)


@pytest.fixture(scope="module")
def serving_ctx():
    """The serving configuration on a context of its own (its tuned launch
    options stay off the shared context): 64 resident meshes of 10K-2M
    triangles (pool seed 2) and the stored queries of its stream (seed 3)."""
    from paper_2411_11244_amd import tune
    recs = _load("serving_stream")
    cfg = {k: recs[0][k] for k in ("pool_seed", "n_meshes", "stream_seed", "rate", "stream_len")}
    pool = g.serving_pool(cfg["pool_seed"], cfg["n_meshes"])
    qs = g.serving_stream(pool, cfg["rate"], cfg["stream_len"], seed=cfg["stream_seed"])
    path = os.path.join(os.path.dirname(GOLDEN), "..", "paper_2411_11244_amd", "tuning", "serving_mi355x.json")
    ctx = gdist.gdist_create(0)
    try:
        tune.apply(ctx, path)
        handles = [gdist.gdist_build(ctx, m.verts, m.tris) for m in pool]
        yield ctx, pool, handles, [qs[r["query"]] for r in recs], recs, tune.server_config(path)
    finally:
        gdist.gdist_destroy(ctx)


def _check_serving(orc, out, pool, qs, recs):
    for r, q, rec in zip(out, qs, recs):
        assert (q.a, q.b, q.mode) == (rec["a"], rec["b"], rec["mode"])
        check_golden(orc, r, rec, pool[q.a], q.pose_a, pool[q.b], q.pose_b, q.mode)


def test_serving_stream_served(orc, serving_ctx):
    """The stored stream queries, submitted at their Poisson arrival times to
    the tuned continuous-batching server, against the oracle."""
    from paper_2411_11244_amd.serve import run_stream
    ctx, pool, handles, qs, recs, sc = serving_ctx
    out = run_stream(ctx, handles, qs, sc.get("max_slots", 64), sc.get("rounds_per_step", 4), timeout_s=120)
    _check_serving(orc, out["results"], pool, qs, recs)


def test_serving_stream_batched(orc, serving_ctx):
    """The same queries as one gdist_query_batch call, against the oracle."""
    ctx, pool, handles, qs, recs, _ = serving_ctx
    descs = [gdist.make_desc(handles[q.a], handles[q.b], q.pose_a, q.pose_b, q.mode) for q in qs]
    _check_serving(orc, gdist.gdist_query_batch(ctx, descs), pool, qs, recs)
