"""Deformable meshes (gdist_update) through the C ABI.

A mesh built with GDIST_BUILD_DEFORMABLE and given new vertex positions keeps
the leaf order of its first build, so its tree differs from a fresh build of
the deformed mesh; the results may not: same FP64 distance bits, same pair,
same tie count, same points, and the FP64 oracle on the deformed mesh agrees.
"""
import numpy as np
import pytest

import meshgen as g
from gpu_common import check_against_oracle, oracle_query
from paper_2411_11244_amd import gdist

pytestmark = pytest.mark.gpu


def _deform(m, t):
    """Radial ripple of the torus tube: each vertex moves along the direction
    from the tube's centre circle, by an amount that changes with t."""
    v = m.verts.astype(np.float64)
    u = np.arctan2(v[:, 1], v[:, 0])
    c = np.stack([np.cos(u), np.sin(u), np.zeros_like(u)], 1)     # centre circle, R = 1
    d = v - c
    s = 1.0 + 0.25 * np.sin(5 * u + t) * np.cos(3 * u - 2 * t)
    return g.Mesh((c + d * s[:, None]).astype(np.float32), m.tris)


def _same(r, a):
    assert r["status"] == a["status"] == 0
    assert r["distance"] == a["distance"]
    assert (r["tri_a"], r["tri_b"]) == (a["tri_a"], a["tri_b"])
    assert r["n_ties"] == a["n_ties"]
    assert np.array_equal(r["point_a"], a["point_a"]) and np.array_equal(r["point_b"], a["point_b"])


@pytest.mark.parametrize("mode", [0, 1])
def test_update_equals_fresh_build(orc, gctx, mode):
    rng = np.random.default_rng(3)
    A = g.torus(96, 32, 1.0, 0.2)
    B = g.icosphere(10, 0.6, 1e-3, rng)
    pa = (g.random_rotation(rng), np.zeros(3))
    pb = (g.random_rotation(rng), np.array([0.4, 2.0, 0.3]))
    ha = gdist.gdist_build(gctx, A.verts, A.tris, gdist.GDIST_BUILD_DEFORMABLE)
    hb = gdist.gdist_build(gctx, B.verts, B.tris)
    try:
        for t in (0.0, 0.7, 2.9):          # a sequence of frames on the same handle
            D = _deform(A, t)
            gdist.gdist_update(gctx, ha, D.verts)
            r = gdist.gdist_query(gctx, ha, hb, pa, pb, mode)
            hf = gdist.gdist_build(gctx, D.verts, D.tris)
            try:
                _same(r, gdist.gdist_query(gctx, hf, hb, pa, pb, mode))
            finally:
                gdist.gdist_release(gctx, hf)
            ref = oracle_query(orc, D, pa, B, pb, mode)
            check_against_oracle(orc, r, ref, D, pa, B, pb, mode)
        # the refitted boxes are tight: the root box is the deformed mesh's box
        info = gdist.gdist_mesh_info(gctx, ha)
        root = np.array(info["root_box"], np.float64)
        assert np.array_equal(root[:3], D.verts.min(0).astype(np.float64))
        assert np.array_equal(root[3:], D.verts.max(0).astype(np.float64))
    finally:
        gdist.gdist_release(gctx, ha)
        gdist.gdist_release(gctx, hb)


def test_update_from_device_tensor(gctx):
    import torch
    A = g.torus(48, 24, 1.0, 0.2)
    B = g.torus(40, 20, 1.0, 0.2)
    pb = (g.quat_to_rot(np.array([1.0, 1.0, 0.0, 0.0])), np.array([1.0, 0.0, 0.0]))
    D = _deform(A, 1.3)
    h1 = gdist.gdist_build(gctx, A.verts, A.tris, gdist.GDIST_BUILD_DEFORMABLE)
    h2 = gdist.gdist_build(gctx, A.verts, A.tris, gdist.GDIST_BUILD_DEFORMABLE)
    hb = gdist.gdist_build(gctx, B.verts, B.tris)
    try:
        gdist.gdist_update(gctx, h1, D.verts)
        gdist.gdist_update(gctx, h2, torch.from_numpy(D.verts).cuda())
        torch.cuda.synchronize()
        for mode in (0, 1):
            _same(gdist.gdist_query(gctx, h1, hb, g.identity_pose(), pb, mode),
                  gdist.gdist_query(gctx, h2, hb, g.identity_pose(), pb, mode))
    finally:
        for h in (h1, h2, hb):
            gdist.gdist_release(gctx, h)


def test_update_errors_leave_the_mesh(gctx):
    A = g.torus(32, 16, 1.0, 0.25)
    pb = (np.eye(3), np.array([3.0, 0.0, 0.0]))
    hr = gdist.gdist_build(gctx, A.verts, A.tris)
    hd = gdist.gdist_build(gctx, A.verts, A.tris, gdist.GDIST_BUILD_DEFORMABLE)
    try:
        before = gdist.gdist_query(gctx, hd, hr, g.identity_pose(), pb, 0)
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_update(gctx, hr, A.verts)          # built rigid
        assert e.value.status == gdist.GDIST_E_INVALID
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_update(gctx, hd, A.verts[:-1])     # vertex count differs
        assert e.value.status == gdist.GDIST_E_INVALID
        bad = _deform(A, 0.5).verts.copy()
        bad[7, 1] = np.nan
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_update(gctx, hd, bad)
        assert e.value.status == gdist.GDIST_E_INVALID
        with pytest.raises(gdist.GdistError) as e:
            gdist.gdist_update(gctx, hd + 1000, A.verts)
        assert e.value.status == gdist.GDIST_E_HANDLE
        _same(gdist.gdist_query(gctx, hd, hr, g.identity_pose(), pb, 0), before)
    finally:
        gdist.gdist_release(gctx, hr)
        gdist.gdist_release(gctx, hd)
