"""Failure handling through the C ABI: a device-memory budget that a build or
a query exceeds, and releasing a mesh while an asynchronous batch that uses
it is still queued.  Every condition is forced from the host; every kernel
still exits normally.

The context's device memory is observed from outside through the caller's
allocator hook (gdist_set_allocator): every byte the library holds was
handed out by the test's allocator, so the sum of live blocks is what the
context holds.
"""
import numpy as np
import pytest

import meshgen as g
from paper_2411_11244_amd import gdist

pytestmark = pytest.mark.gpu


class Tracker:
    def __init__(self):
        import torch
        self.torch = torch
        self.live = {}

    def alloc(self, n, user):
        p = self.torch.cuda.caching_allocator_alloc(int(n))
        self.live[p] = int(n)
        return p

    def free(self, p, user):
        self.live.pop(p)
        self.torch.cuda.caching_allocator_delete(p)

    def held(self):
        return sum(self.live.values())


def _same(r, a):
    assert r["status"] == a["status"] == 0
    assert r["distance"] == a["distance"]
    assert (r["tri_a"], r["tri_b"]) == (a["tri_a"], a["tri_b"])
    assert r["n_ties"] == a["n_ties"]


def test_memory_budget_oom(gctx):
    rng = np.random.default_rng(5)
    A = g.icosphere(30, 1.0, 1e-3, rng)          # 18,000 triangles
    B = g.heightfield(60, 0.02, rng)             # 7,200 triangles
    pa, pb = g.place_with_gap(rng, A, B, 0.01, g.random_rotation(rng), g.random_rotation(rng))
    ha0, hb0 = gdist.gdist_build(gctx, A.verts, A.tris), gdist.gdist_build(gctx, B.verts, B.tris)
    try:
        want = gdist.gdist_query(gctx, ha0, hb0, pa, pb, 0)
    finally:
        gdist.gdist_release(gctx, ha0)
        gdist.gdist_release(gctx, hb0)

    t = Tracker()
    ctx = gdist.gdist_create(0)
    try:
        keep = gdist.gdist_set_allocator(ctx, t.alloc, t.free)
        ha = gdist.gdist_build(ctx, A.verts, A.tris)
        held_a = t.held()
        assert held_a == gdist.gdist_mesh_info(ctx, ha)["device_bytes"]
        # budgets below B's build, failing at the first allocation and after
        # the uploads and the first sort buffer: E_OOM, every temporary returned
        nv, nt = len(B.verts), len(B.tris)
        for extra in (4096, 12 * nv + 12 * nt + 64 + 8 * nt + 1024):
            gdist.gdist_set_option(ctx, "memory_budget", held_a + extra)
            with pytest.raises(gdist.GdistError) as e:
                gdist.gdist_build(ctx, B.verts, B.tris)
            assert e.value.status == gdist.GDIST_E_OOM
            assert t.held() == held_a
        # room for B's tree but not for a query's workspace
        gdist.gdist_set_option(ctx, "memory_budget", 0)
        hb = gdist.gdist_build(ctx, B.verts, B.tris)
        held_ab = t.held()
        gdist.gdist_set_option(ctx, "memory_budget", held_ab + (1 << 20))
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_query(ctx, ha, hb, pa, pb, 0)
        assert e.value.status == gdist.GDIST_E_OOM
        assert t.held() == held_ab               # the workspace cache was released
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_query_batch(ctx, [gdist.make_desc(ha, hb, pa, pb, 0)] * 3)
        assert e.value.status == gdist.GDIST_E_OOM
        assert t.held() == held_ab
        # the context is still usable once the budget allows the query
        gdist.gdist_set_option(ctx, "memory_budget", 0)
        _same(gdist.gdist_query(ctx, ha, hb, pa, pb, 0), want)
        gdist.gdist_release(ctx, hb)
        gdist.gdist_release(ctx, ha)
    finally:
        gdist.gdist_destroy(ctx)
    assert t.held() == 0
    del keep


def test_release_while_async_in_flight(gctx):
    """gdist_release of a mesh that a queued asynchronous batch uses waits for
    that batch: the batch's results are intact, and the handle is gone
    afterwards."""
    rng = np.random.default_rng(9)
    meshes = [g.icosphere(40, 1.0, 1e-3, rng), g.torus(120, 60, 1.0, 0.3), g.heightfield(80, 0.02, rng)]
    hs = [gdist.gdist_build(gctx, m.verts, m.tris) for m in meshes]
    try:
        descs = []
        for i in range(24):
            a, b = i % 3, (i + 1) % 3
            pa, pb = g.place_with_gap(rng, meshes[a], meshes[b], [0.02, 0.3, -0.1][i % 3],
                                      g.random_rotation(rng), g.random_rotation(rng))
            descs.append(gdist.make_desc(hs[a], hs[b], pa, pb, i % 2))
        want = gdist.gdist_query_batch(gctx, descs)
        pend = [gdist.gdist_query_batch_async(gctx, descs) for _ in range(3)]
        gdist.gdist_release(gctx, hs[1])          # used by every batch in flight
        released = hs.pop(1)
        gdist.gdist_sync(gctx)
        for b in pend:
            for r, a in zip(b.results(), want):
                _same(r, a)
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_query_batch_async(gctx, descs[:1])
        assert e.value.status == gdist.GDIST_E_HANDLE
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_release(gctx, released)
        assert e.value.status == gdist.GDIST_E_HANDLE
    finally:
        for h in hs:
            gdist.gdist_release(gctx, h)
