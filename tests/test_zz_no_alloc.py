"""gdist_query_noalloc (the entry point that allocates no device memory)
against gdist_query, through the C ABI: two calls in a row, the second on a
smaller input, in both modes; the same answer (distance, pair, tie count,
FP32 optimum, points) bit for bit, and the oracle's answer.  A refitted mesh
beyond the path's limit is rejected before anything runs, and the path keeps
working afterwards."""
import numpy as np
import pytest

import meshgen as g
from gpu_common import check_against_oracle, oracle_query
from paper_2411_11244_amd import gdist

pytestmark = pytest.mark.gpu


def _same(r, a):
    assert r["status"] == a["status"] == 0
    assert r["distance"] == a["distance"]
    assert r["distance_fp32"] == a["distance_fp32"]
    assert (r["tri_a"], r["tri_b"]) == (a["tri_a"], a["tri_b"])
    assert r["n_ties"] == a["n_ties"]
    assert r["flags"] == a["flags"]
    assert list(r["point_a"]) == list(a["point_a"]) and list(r["point_b"]) == list(a["point_b"])


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_equals_query(gctx, orc, mode):
    rng = np.random.default_rng(31 + mode)
    big = (g.icosphere(60, 1.0, 1e-3, rng), g.heightfield(120, 0.02, rng))       # 72,000 and 28,800 triangles
    small = (g.torus(40, 20, 1.0, 0.3), g.icosphere(12, 0.7, 1e-3, rng))        # 1,600 and 2,880 triangles
    for A, B in (big, small):
        pa, pb = g.place_with_gap(rng, A, B, 0.05, g.random_rotation(rng), g.random_rotation(rng))
        ha, hb = gdist.gdist_build(gctx, A.verts, A.tris), gdist.gdist_build(gctx, B.verts, B.tris)
        try:
            want = gdist.gdist_query(gctx, ha, hb, pa, pb, mode)
            got = gdist.gdist_query_noalloc(gctx, ha, hb, pa, pb, mode)
            _same(got, want)
            ref = oracle_query(orc, A, pa, B, pb, mode)
            check_against_oracle(orc, got, ref, A, pa, B, pb, mode)
        finally:
            gdist.gdist_release(gctx, ha)
            gdist.gdist_release(gctx, hb)


def test_noalloc_limit_and_reuse(gctx):
    big = g.torus(1024, 1024, 1.0, 0.25)          # 2,097,152 triangles: 2^21 leaves
    h = gdist.gdist_build(gctx, big.verts, big.tris)
    try:
        ident = (np.eye(3), np.zeros(3))
        far = (np.eye(3), np.array([3.0, 0.0, 0.0]))
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_query_noalloc(gctx, h, h, ident, far, 0)
        assert e.value.status == gdist.GDIST_E_INVALID
    finally:
        gdist.gdist_release(gctx, h)
    w = g.tiny(3)
    m, q = w.meshes[0], w.queries[0]
    h = gdist.gdist_build(gctx, m.verts, m.tris)
    try:
        _same(gdist.gdist_query_noalloc(gctx, h, h, q.pose_a, q.pose_b, 0),
              gdist.gdist_query(gctx, h, h, q.pose_a, q.pose_b, 0))
    finally:
        gdist.gdist_release(gctx, h)
