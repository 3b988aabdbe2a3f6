"""The seeded input generators (CPU only): the same seed gives the same
bytes, so the GPU path, the oracle and the stored expected values all see one
workload; the shapes match the workload definitions."""
import numpy as np

import meshgen as g


def _same_mesh(a, b):
    assert np.array_equal(a.verts, b.verts) and np.array_equal(a.tris, b.tris)


def _same_pose(p, q):
    assert np.array_equal(p[0], q[0]) and np.array_equal(p[1], q[1])


def test_generators_are_deterministic():
    _same_mesh(g.tiny(3).meshes[0], g.tiny(3).meshes[0])
    _same_pose(g.tiny(3).queries[0].pose_b, g.tiny(3).queries[0].pose_b)
    a, b = g.batched_pair(1, 17), g.batched_pair(1, 17)
    _same_mesh(a[0], b[0]); _same_mesh(a[1], b[1]); _same_pose(a[3], b[3])
    _same_mesh(g.serving_mesh(2, 5, 1e3, 2e4), g.serving_mesh(2, 5, 1e3, 2e4))
    pool = [g.serving_mesh(2, i, 1e3, 2e4) for i in range(4)]
    s1, s2 = g.serving_stream(pool, 500.0, 20, seed=9), g.serving_stream(pool, 500.0, 20, seed=9)
    for x, y in zip(s1, s2):
        assert (x.a, x.b, x.mode, x.arrival) == (y.a, y.b, y.mode, y.arrival)
        _same_pose(x.pose_b, y.pose_b)
    r1, r2 = g.rings(frames=3, nu=40, nv=20), g.rings(frames=3, nu=40, nv=20)
    _same_mesh(r1.meshes[0], r2.meshes[0])
    for x, y in zip(r1.queries, r2.queries):
        _same_pose(x.pose_b, y.pose_b)


def test_workload_shapes():
    t = g.tiny(0)
    assert t.meshes[0].n_tris == 2 * 32 * 32
    r = g.rings(frames=5, nu=40, nv=20)
    assert r.meshes[0].n_tris == 2 * 40 * 20 and len(r.queries) == 5
    h = g.hard(seed=4, n=10)
    assert [m.n_tris for m in h.meshes] == [20 * 10 * 10] * 2 and [q.mode for q in h.queries] == [0, 1]
    pool = [g.serving_mesh(2, i, 1e4, 2e6) for i in range(3)]
    assert all(1e4 * 0.5 <= m.n_tris <= 2e6 * 1.5 for m in pool)
    qs = g.serving_stream(pool, 1000.0, 200, seed=1)
    assert all(b.arrival >= a.arrival for a, b in zip(qs, qs[1:]))
    assert {q.mode for q in qs} == {0, 1}
