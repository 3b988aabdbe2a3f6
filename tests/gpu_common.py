"""Helpers shared by the GPU parity tests (test code only)."""
import numpy as np

import meshgen as g


def world_tri(mesh, pose, t):
    v = mesh.verts[mesh.tris[t]].astype(np.float64)
    return v @ pose[0].T + pose[1]


def on_triangle(x, T, tol):
    a, b, c = T
    n = np.cross(b - a, c - a)
    nn = n @ n
    size = max(np.linalg.norm(b - a), np.linalg.norm(c - a), np.linalg.norm(c - b))
    if nn <= (1e-10 * size * size) ** 2:
        # (numerically) degenerate, e.g. collinear vertices after a rotation:
        # distance to its three edges
        def segd(p, u, v):
            d = v - u
            L = d @ d
            s = 0.0 if L == 0 else np.clip((p - u) @ d / L, 0, 1)
            return np.linalg.norm(p - (u + s * d))
        return min(segd(x, a, b), segd(x, b, c), segd(x, c, a)) <= tol
    if abs((x - a) @ n) / np.sqrt(nn) > tol:
        return False
    l1 = np.cross(c - b, x - b) @ n / nn
    l2 = np.cross(a - c, x - c) @ n / nn
    l3 = np.cross(b - a, x - a) @ n / nn
    scale = max(np.linalg.norm(b - a), np.linalg.norm(c - a), 1e-300)
    return min(l1, l2, l3) * scale >= -tol


def check_against_oracle(orc, r, ref, ma, pa, mb, pb, mode=0, abs_tol=1e-6, rel_tol=1e-5):
    """The parity contract: distance within 1e-6 absolute or 1e-5
    relative; the reported pair is in the oracle's tie set (its own FP64
    distance within tau of the optimum) and equals the oracle's pair when the
    tie set has one element; the points lie on the reported triangles and
    realise the pair's distance."""
    D = ref["distance"]
    d = r["distance"]
    assert r["status"] == 0, r
    assert abs(d - D) <= max(abs_tol, rel_tol * abs(D)), (d, D)
    Pa = world_tri(ma, pa, r["tri_a"])
    Pb = world_tri(mb, pb, r["tri_b"])
    dp = (orc.tri_tri_max if mode else orc.tri_tri_min)(Pa, Pb)[0]
    tau = ref["tau"]
    assert abs(dp - D) <= tau + 1e-14 * max(1.0, abs(D)), ("pair not in tie set", dp, D, tau)
    if ref["n_ties"] == 1:
        assert (r["tri_a"], r["tri_b"]) == (ref["tri_a"], ref["tri_b"])
    tol = 1e-9 * max(1.0, float(np.abs(Pa).max()), float(np.abs(Pb).max()))
    assert on_triangle(np.asarray(r["point_a"]), Pa, tol)
    assert on_triangle(np.asarray(r["point_b"]), Pb, tol)
    assert abs(np.linalg.norm(np.asarray(r["point_a"]) - np.asarray(r["point_b"])) - dp) <= tol


def oracle_query(orc, ma, pa, mb, pb, mode=0, method="auto"):
    return orc.query(ma.verts, ma.tris, g.pose_to_flat(pa), mb.verts, mb.tris, g.pose_to_flat(pb),
                     mode, method)
