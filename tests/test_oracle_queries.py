"""Pins for the oracle's mesh-pair queries (CPU only).

Closed forms, invariants and the two independent search strategies (brute
force over all triangle pairs, and the oracle's own median-split BVH) checked
against each other.
"""
import math

import numpy as np
import pytest

import meshgen as g


def flat(p):
    return g.pose_to_flat(p)


def run(orc, ma, pa, mb, pb, mode=0, method="brute", **kw):
    return orc.query(ma.verts, ma.tris, flat(pa), mb.verts, mb.tris, flat(pb), mode, method, **kw)


def test_tiny_identity_closed_form(orc):
    """Two 32x32 tori (R=1, r=0.25) translated by dx along x: the outer
    equator vertices face each other, so D_min = dx - 2(R + r) = dx - 2.5,
    attained by the 6 x 6 triangles around those two vertices."""
    for seed in (0, 5):
        w = g.tiny(seed, identity_rotation=True)
        m, q = w.meshes[0], w.queries[0]
        for method in ("brute", "bvh"):
            r = run(orc, m, q.pose_a, m, q.pose_b, 0, method)
            assert abs(r["distance"] - (w.notes["dx"] - 2.5)) <= 1e-15
            assert r["n_ties"] == 36


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_random_rotation(orc, seed):
    """Bounding spheres give D_min >= dx - 2.5; brute force and BVH agree."""
    w = g.tiny(seed)
    m, q = w.meshes[0], w.queries[0]
    rb = run(orc, m, q.pose_a, m, q.pose_b, 0, "brute", threads=8)
    rv = run(orc, m, q.pose_a, m, q.pose_b, 0, "bvh")
    assert rb["distance"] >= w.notes["dx"] - 2.5 - 1e-12
    assert rb["distance"] == rv["distance"]
    assert (rb["tri_a"], rb["tri_b"]) == (rv["tri_a"], rv["tri_b"])
    assert rb["n_ties"] == rv["n_ties"]
    assert rb["pairs_tested"] == 2048 * 2048


def test_parallel_planes(orc):
    """Flat grids at z=0 and z=h overlapping in xy: D_min = h (to rounding;
    every overlapping pair ties); unshifted unit squares: D_max = sqrt(2 + h^2)."""
    A = g.heightfield(6, 0.0)
    h = 0.375
    r = run(orc, A, g.identity_pose(), A, (np.eye(3), np.array([0.3, 0.2, h])), 0, "brute")
    assert abs(r["distance"] - h) <= 2e-16
    assert r["n_ties"] > 20
    rv = run(orc, A, g.identity_pose(), A, (np.eye(3), np.array([0.3, 0.2, h])), 0, "bvh")
    assert rv["distance"] == r["distance"] and rv["n_ties"] == r["n_ties"]
    assert (rv["tri_a"], rv["tri_b"]) == (r["tri_a"], r["tri_b"])
    rm = run(orc, A, g.identity_pose(), A, (np.eye(3), np.array([0, 0, h])), 1, "brute")
    assert rm["distance"] == pytest.approx(math.sqrt(2 + h * h), rel=1e-15)


def test_penetration_gives_zero(orc):
    """A vertical grid through a horizontal one, and two chained tori."""
    A = g.heightfield(5, 0.0)
    Rv = g.rot_axis("x", math.pi / 2)
    r = run(orc, A, g.identity_pose(), A, (Rv, np.array([0.2, 0.5, -0.5])), 0, "brute")
    assert r["distance"] == 0.0
    T = g.torus(24, 12, 1.0, 0.2)
    # B's centre line passes through A's centre line: the tube surfaces cross
    r = run(orc, T, g.identity_pose(), T, (g.rot_axis("x", math.pi / 2), np.array([2.0, 0, 0])), 0, "bvh")
    assert r["distance"] == 0.0


def test_separated_spheres(orc):
    """Geodesic spheres with an icosahedron vertex pointing at each other:
    D_min is squeezed between the circumscribed-ball bound and the distance of
    the two facing vertices."""
    r1, r2, D = 1.0, 0.6, 3.1
    A = g.icosphere(6, r1)
    B = g.icosphere(5, r2)
    def facing_rotation(mesh, target):
        v = mesh.verts.astype(np.float64)
        i = int(np.argmax(v[:, 2]))          # an icosahedron vertex
        u = v[i] / np.linalg.norm(v[i])
        axis = np.cross(u, target)
        s, c = np.linalg.norm(axis), u @ target
        K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]]) / s
        return np.eye(3) + s * K + (1 - c) * K @ K, i
    Ra, ia = facing_rotation(A, np.array([1.0, 0, 0]))
    Rb, ib = facing_rotation(B, np.array([-1.0, 0, 0]))
    pa, pb = (Ra, np.zeros(3)), (Rb, np.array([D, 0, 0]))
    r = run(orc, A, pa, B, pb, 0, "bvh")
    va = Ra @ A.verts[ia].astype(np.float64)
    vb = Rb @ B.verts[ib].astype(np.float64) + pb[1]
    upper = np.linalg.norm(va - vb)
    lower = D - np.linalg.norm(A.verts.astype(np.float64), axis=1).max() \
              - np.linalg.norm(B.verts.astype(np.float64), axis=1).max()
    assert lower - 1e-12 <= r["distance"] <= upper + 1e-12
    assert upper - lower < 1e-6


def test_symmetry_and_rigid_invariance(orc):
    rng = np.random.default_rng(7)
    A = g.ellipsoid(8, 16, (1.0, 0.7, 0.5))
    B = g.heightfield(7, 0.05, rng)
    pa = (g.random_rotation(rng), rng.normal(size=3))
    pb = (g.random_rotation(rng), pa[1] + np.array([1.9, 0.3, -0.2]))
    r1 = run(orc, A, pa, B, pb, 0, "brute")
    r2 = run(orc, B, pb, A, pa, 0, "brute")
    assert r1["distance"] == pytest.approx(r2["distance"], rel=1e-14)
    assert (r1["tri_a"], r1["tri_b"]) == (r2["tri_b"], r2["tri_a"]) or r1["n_ties"] > 1
    M = (g.random_rotation(rng), rng.normal(size=3) * 5)
    r3 = run(orc, A, g.compose(M, pa), B, g.compose(M, pb), 0, "brute")
    assert r3["distance"] == pytest.approx(r1["distance"], rel=1e-12)
    for mode in (0, 1):
        s1 = run(orc, A, pa, B, pb, mode, "bvh")
        s3 = run(orc, A, g.compose(M, pa), B, g.compose(M, pb), mode, "bvh")
        assert s3["distance"] == pytest.approx(s1["distance"], rel=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_max_mode_equals_vertex_pairs(orc, seed):
    """D_max over triangle pairs equals the max over vertex pairs (the plain
    definition restricted to vertices, computed by a separate routine)."""
    rng = np.random.default_rng(seed)
    A = g.random_soup(rng, 300)
    B = g.ellipsoid(6, 12, tuple(rng.uniform(0.5, 1.5, 3)))
    pa = (g.random_rotation(rng), np.zeros(3))
    pb = (g.random_rotation(rng), rng.normal(size=3))
    r = run(orc, A, pa, B, pb, 1, "brute")
    rv = run(orc, A, pa, B, pb, 1, "bvh")
    vm = orc.max_vertex_pairs(A.verts, flat(pa), B.verts, flat(pb))
    assert r["distance"] == vm == rv["distance"]
    assert (r["tri_a"], r["tri_b"]) == (rv["tri_a"], rv["tri_b"])


@pytest.mark.parametrize("seed", range(3))
def test_vertex_row_max_brute(orc, seed):
    """Each row maximum equals the plain maximum over all posed vertex pairs."""
    rng = np.random.default_rng(50 + seed)
    va = rng.normal(size=(97, 3)).astype(np.float32)
    vb = rng.normal(size=(61, 3)).astype(np.float32)
    pa = flat((g.random_rotation(rng), rng.normal(size=3)))
    pb = flat((g.random_rotation(rng), rng.normal(size=3)))
    rm = orc.vertex_row_max(va, pa, vb, pb, threads=3)
    A, B = orc.pose_points(va, pa), orc.pose_points(vb, pb)
    ref = np.sqrt(((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)).max(1)
    assert np.allclose(rm, ref, rtol=1e-15, atol=0)
    assert rm.max() == orc.max_vertex_pairs(va, pa, vb, pb)


@pytest.mark.parametrize("case", ["hard", "soup"])
def test_max_by_vertices_matches_brute(orc, case):
    """The vertex-pair route to D_max (value and tie set) agrees with brute
    force over all triangle pairs, on the concentric-spheres geometry (every
    tied vertex pair ties all its incident triangle pairs) and on a soup."""
    if case == "hard":
        w = g.hard(seed=4, n=6)
        A, B = w.meshes
        q = w.queries[1]
        pa, pb = q.pose_a, q.pose_b
    else:
        rng = np.random.default_rng(9)
        A, B = g.random_soup(rng, 200), g.random_soup(rng, 150)
        pa, pb = (g.random_rotation(rng), np.zeros(3)), (g.random_rotation(rng), rng.normal(size=3))
    r = run(orc, A, pa, B, pb, 1, "brute")
    v = orc.max_by_vertices(A.verts, A.tris, flat(pa), B.verts, B.tris, flat(pb), threads=2)
    assert v["distance"] == pytest.approx(r["distance"], rel=1e-15, abs=0)
    assert v["tau"] == r["tau"]
    assert (v["tri_a"], v["tri_b"]) == (r["tri_a"], r["tri_b"])
    assert v["n_ties"] == r["n_ties"]
    assert sorted(map(tuple, v["ties"].tolist())) == sorted(map(tuple, r["ties"][:r["n_ties"]].tolist()))
    if case == "hard":
        assert r["n_ties"] >= 25


def _random_pair(rng, kind):
    if kind == "soup":
        return g.random_soup(rng, 400, 1.0, 0.15), g.random_soup(rng, 350, 1.0, 0.15)
    if kind == "height":
        return g.heightfield(12, 0.02, rng), g.heightfield(11, 0.02, rng)
    return g.icosphere(4, 1.0, 1e-3, rng), g.ellipsoid(9, 18, (1.2, 0.6, 0.9))


@pytest.mark.parametrize("kind", ["soup", "height", "sphere"])
@pytest.mark.parametrize("mode", [0, 1])
def test_brute_vs_bvh(orc, kind, mode):
    rng = np.random.default_rng(hash((kind, mode)) % 2**32)
    A, B = _random_pair(rng, kind)
    for gap in (0.05, 0.4, -0.2):
        ra, rb = g.random_rotation(rng), g.random_rotation(rng)
        pa, pb = g.place_with_gap(rng, A, B, gap, ra, rb)
        r1 = run(orc, A, pa, B, pb, mode, "brute", threads=8)
        r2 = run(orc, A, pa, B, pb, mode, "bvh")
        assert r1["distance"] == r2["distance"]
        assert r1["n_ties"] == r2["n_ties"]
        assert (r1["tri_a"], r1["tri_b"]) == (r2["tri_a"], r2["tri_b"])
        if mode == 0 and gap > 0:
            assert r1["distance"] >= gap - 1e-12
        if mode == 1:
            assert r2["pairs_tested"] < r1["pairs_tested"]


def test_coarse_rings_gap(orc):
    """Interlocked tori with smooth gap 0.7 - 2r = 0.5 at every frame; the
    tessellation moves the mesh distance by at most a few sagittas."""
    w = g.rings(frames=3, nu=120, nv=40)
    m = w.meshes[0]
    vals = []
    for q in w.queries:
        r = run(orc, m, q.pose_a, m, q.pose_b, 0, "bvh")
        vals.append(r["distance"])
    sag = 1.1 * (1 - math.cos(math.pi / 120)) + 0.1 * (1 - math.cos(math.pi / 40))
    for v in vals:
        assert abs(v - 0.5) <= 2 * sag


def test_rejects_bad_input(orc):
    A = g.heightfield(2, 0.0)
    bad = A.tris.copy()
    bad[0, 0] = 10_000
    with pytest.raises(ValueError):
        orc.query(A.verts, bad, flat(g.identity_pose()), A.verts, A.tris, flat(g.identity_pose()))
    v = A.verts.copy()
    v[0, 0] = np.nan
    with pytest.raises(ValueError):
        orc.query(v, A.tris, flat(g.identity_pose()), A.verts, A.tris, flat(g.identity_pose()))
