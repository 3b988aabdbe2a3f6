"""Continuous-batching server (gdist_server_*) through the C ABI.

A query served alongside others, admitted between traversal steps and
completed when its own traversal drains, must give exactly what gdist_query
gives for it alone: same FP64 distance bits, same pair, same tie count (the
FP64 re-evaluation decides all three from candidates that the conservative
FP32 window never drops).  A sample is also checked against the FP64 oracle.

Each device step after admission is replayed from a HIP graph (every step of
a run is one replay, with the admission's launches and host work between
replays); the same stream with the kernels launched one by one
(GDIST_SERVER_DIRECT) must give the same results.
"""
import numpy as np
import pytest

import meshgen as g
from gpu_common import check_against_oracle, oracle_query
from paper_2411_11244_amd import gdist
from paper_2411_11244_amd.serve import run_stream

pytestmark = pytest.mark.gpu


def _pool(rng):
    return [g.torus(40, 20, 1.0, 0.3), g.icosphere(8, 1.0, 1e-3, rng), g.random_soup(rng, 1500, 1.0, 0.1),
            g.heightfield(30, 0.02, rng), g.ellipsoid(20, 40, (1.2, 0.6, 0.9)), g.random_soup(rng, 333, 0.5, 0.2),
            g.torus(64, 32, 1.0, 0.25), g.icosphere(12, 0.7, 0.0, rng)]


def _alone(ctx, handles, qs):
    return [gdist.gdist_query(ctx, handles[q.a], handles[q.b], q.pose_a, q.pose_b, q.mode) for q in qs]


def _same(r, a):
    assert r["status"] == 0 and a["status"] == 0, (r, a)
    assert r["distance"] == a["distance"], (r["distance"], a["distance"])
    assert (r["tri_a"], r["tri_b"]) == (a["tri_a"], a["tri_b"])
    assert r["n_ties"] == a["n_ties"]
    assert np.array_equal(r["point_a"], a["point_a"]) and np.array_equal(r["point_b"], a["point_b"])


@pytest.fixture(scope="module")
def served(gctx):
    rng = np.random.default_rng(77)
    pool = _pool(rng)
    handles = [gdist.gdist_build(gctx, m.verts, m.tris) for m in pool]
    qs = g.serving_stream(pool, 2000.0, 96, seed=78)
    alone = _alone(gctx, handles, qs)
    yield pool, handles, qs, alone
    for h in handles:
        gdist.gdist_release(gctx, h)


def _graph_used(st, direct):
    if direct:
        assert st["graph_mode"] == 0 and st["graph_steps"] == 0
    else:
        assert st["graph_mode"] == 1 and st["graph_steps"] == st["steps"]


@pytest.mark.parametrize("slots,rounds,scale,direct", [(8, 1, 0.0, False), (32, 3, 0.0, False), (64, 4, 1.0, False),
                                                       (32, 3, 0.0, True)])
def test_server_equals_alone(gctx, served, slots, rounds, scale, direct):
    pool, handles, qs, alone = served
    out = run_stream(gctx, handles, qs, max_slots=slots, rounds_per_step=rounds, time_scale=scale, timeout_s=120,
                     direct=direct)
    for r, a in zip(out["results"], alone):
        _same(r, a)
    st = out["stats"]
    assert st["submitted"] == len(qs) and st["completed"] == len(qs) and st["failed"] == 0
    assert st["steps"] >= 1 and st["rounds"] >= 1
    _graph_used(st, direct)
    assert np.all(out["latency_ms"] >= 0)


def test_server_sample_vs_oracle(orc, gctx, served):
    pool, handles, qs, _ = served
    sample = qs[:12]
    out = run_stream(gctx, handles, sample, max_slots=4, rounds_per_step=2, time_scale=0.0, timeout_s=120)
    for q, r in zip(sample, out["results"]):
        ref = oracle_query(orc, pool[q.a], q.pose_a, pool[q.b], q.pose_b, q.mode)
        check_against_oracle(orc, r, ref, pool[q.a], q.pose_a, pool[q.b], q.pose_b, q.mode)


def test_server_storage_growth(gctx, served):
    """Front and spill stack far too small: rounds expand few entries, the
    stack overflows, queries are requeued, the stack grows, and every result
    still equals the result alone."""
    pool, handles, qs, alone = served
    gdist.gdist_set_option(gctx, "expand_budget", 4)   # rounds of at most 4,096 entries
    try:
        out = run_stream(gctx, handles, qs[:24], max_slots=16, rounds_per_step=2, front_capacity=64,
                         time_scale=0.0, timeout_s=120, stack_capacity=256)
    finally:
        gdist.gdist_set_option(gctx, "expand_budget", 1 << 22)
    for r, a in zip(out["results"], alone[:24]):
        _same(r, a)
    assert out["stats"]["requeued"] > 0
    _graph_used(out["stats"], False)   # rebuilt for the grown stack


def test_server_candidate_overflow(gctx):
    """Identical meshes at the same pose touch along every face: far more
    candidates than a region of 64 holds.  That query is re-run alone through
    the batched path and still returns what gdist_query returns; a separated
    query in the same stream is served normally."""
    w = g.tiny(3, identity_rotation=True)
    m = w.meshes[0]
    h = gdist.gdist_build(gctx, m.verts, m.tris)
    try:
        I = g.identity_pose()
        far = w.queries[0]
        qs = [g.Query(0, 0, I, I, 0), g.Query(0, 0, far.pose_a, far.pose_b, 0)]
        alone = [gdist.gdist_query(gctx, h, h, q.pose_a, q.pose_b, 0) for q in qs]
        assert alone[0]["distance"] == 0.0 and alone[0]["n_candidates"] > 64
        out = run_stream(gctx, [h], qs, max_slots=4, rounds_per_step=2, cand_per_slot=64, time_scale=0.0,
                         timeout_s=60)
        for r, a in zip(out["results"], alone):
            _same(r, a)
        assert out["stats"]["fallbacks"] >= 1
    finally:
        gdist.gdist_release(gctx, h)


def test_server_busy_and_errors(gctx):
    m = g.torus(16, 8, 1.0, 0.3)
    h = gdist.gdist_build(gctx, m.verts, m.tris)
    srv = gdist.gdist_server_start(gctx, 4, 2)
    try:
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_query(gctx, h, h, g.identity_pose(), g.identity_pose(), 0)
        assert e.value.status == gdist.GDIST_E_BUSY
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_server_start(gctx, 4, 2)
        assert e.value.status == gdist.GDIST_E_BUSY
        bad = gdist.make_desc(h, h + 999, g.identity_pose(), g.identity_pose(), 0)
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_server_submit(srv, bad, 0)
        assert e.value.status == gdist.GDIST_E_HANDLE
        big = g.torus(64, 64, 1.0, 0.3)
    finally:
        gdist.gdist_server_stop(srv)
    # after stop the context serves plain queries again, and a query whose
    # smaller mesh (the one it refits) exceeds max_tris is refused at submit
    hb = gdist.gdist_build(gctx, big.verts, big.tris)
    srv = gdist.gdist_server_start(gctx, 4, 2, 0, 0, m.n_tris)
    try:
        d = gdist.make_desc(hb, hb, g.identity_pose(), (np.eye(3), np.array([5.0, 0, 0])), 0)
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_server_submit(srv, d, 1)
        assert e.value.status == gdist.GDIST_E_CAPACITY
    finally:
        gdist.gdist_server_stop(srv)
    r = gdist.gdist_query(gctx, h, h, g.identity_pose(), (np.eye(3), np.array([5.0, 0, 0])), 0)
    assert r["status"] == 0
    gdist.gdist_release(gctx, hb)
    gdist.gdist_release(gctx, h)
