"""FP64 CPU oracle for mesh-to-mesh minimum / maximum distance (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library and never imports it.

The C sources (``oracle.c``) restate the paper's definitions plainly:
D_min / D_max (gDist Sec. 3, Eqs. 1-2), the AABB bounds of Sec. 4 (the
conventional ones and the enhanced ones evaluated literally over the 36 face
pairs), and the exact triangle-triangle distance as a minimum over
vertex-triangle and edge-edge feature pairs plus an edge-crossing test for
intersection (distance zero on penetration, Sec. 7).

Reported pair (a reading of the paper, which does not say which pair to
report): the tie set is every triangle pair whose distance lies within
``tau = 1e-12 * max(1, M)`` of the optimum, with M the largest world
coordinate magnitude over the corners of either mesh's local bounding box
under its pose; the canonical pair is the
lexicographically smallest (tri_a, tri_b) of the tie set.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, no contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
               "-shared", "-pthread", "-Wall", "-o", tmp, src, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrcResult(C.Structure):
    _fields_ = [("distance", C.c_double), ("tri_a", C.c_int64), ("tri_b", C.c_int64),
                ("point_a", C.c_double * 3), ("point_b", C.c_double * 3),
                ("pair_distance", C.c_double), ("n_ties", C.c_int64),
                ("pairs_tested", C.c_int64)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build_oracle(force=False)
    lib = C.CDLL(_LIB_PATH)
    dp, fp, up = C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_uint32)
    i64, i64p = C.c_int64, C.POINTER(C.c_int64)
    lib.orc_tri_tri_min.restype = C.c_double
    lib.orc_tri_tri_min.argtypes = [dp, dp, dp, dp]
    lib.orc_tri_tri_max.restype = C.c_double
    lib.orc_tri_tri_max.argtypes = [dp, dp, dp, dp]
    lib.orc_point_triangle.restype = C.c_double
    lib.orc_point_triangle.argtypes = [dp, dp, dp]
    lib.orc_point_segment.restype = C.c_double
    lib.orc_point_segment.argtypes = [dp, dp, dp, dp]
    lib.orc_segment_segment.restype = C.c_double
    lib.orc_segment_segment.argtypes = [dp, dp, dp, dp, dp, dp]
    lib.orc_segment_pierces.restype = C.c_int
    lib.orc_segment_pierces.argtypes = [dp, dp, dp, dp]
    lib.orc_box_bounds.restype = None
    lib.orc_box_bounds.argtypes = [dp, dp, dp]
    lib.orc_pose_points.restype = None
    lib.orc_pose_points.argtypes = [fp, i64, dp, dp]
    q = [fp, i64, up, i64, dp, fp, i64, up, i64, dp, C.c_int, C.c_double]
    lib.orc_brute.restype = C.c_int
    lib.orc_brute.argtypes = q + [C.c_int, C.POINTER(OrcResult), i64p, i64]
    lib.orc_bvh.restype = C.c_int
    lib.orc_bvh.argtypes = q + [C.POINTER(OrcResult), i64p, i64]
    lib.orc_max_vertex_pairs.restype = C.c_double
    lib.orc_max_vertex_pairs.argtypes = [fp, i64, dp, fp, i64, dp, C.c_int]
    lib.orc_vertex_row_max.restype = None
    lib.orc_vertex_row_max.argtypes = [fp, i64, dp, fp, i64, dp, C.c_int, dp]
    _lib = lib
    return lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


# ---------------------------------------------------------------- primitives
def tri_tri_min(P, Q):
    """Exact distance between closed triangles P, Q (3x3 arrays of vertices)."""
    lib = _load()
    P, Q = _d(P).reshape(9), _d(Q).reshape(9)
    cp, cq = np.zeros(3), np.zeros(3)
    d = lib.orc_tri_tri_min(_ptr(P, C.c_double), _ptr(Q, C.c_double),
                            _ptr(cp, C.c_double), _ptr(cq, C.c_double))
    return d, cp, cq


def tri_tri_max(P, Q):
    lib = _load()
    P, Q = _d(P).reshape(9), _d(Q).reshape(9)
    cp, cq = np.zeros(3), np.zeros(3)
    d = lib.orc_tri_tri_max(_ptr(P, C.c_double), _ptr(Q, C.c_double),
                            _ptr(cp, C.c_double), _ptr(cq, C.c_double))
    return d, cp, cq


def point_triangle(p, T):
    lib = _load()
    p, T, q = _d(p).reshape(3), _d(T).reshape(9), np.zeros(3)
    d = lib.orc_point_triangle(_ptr(p, C.c_double), _ptr(T, C.c_double), _ptr(q, C.c_double))
    return d, q


def segment_segment(p0, p1, q0, q1):
    lib = _load()
    a = [_d(x).reshape(3) for x in (p0, p1, q0, q1)]
    cp, cq = np.zeros(3), np.zeros(3)
    d = lib.orc_segment_segment(*[_ptr(x, C.c_double) for x in a],
                                _ptr(cp, C.c_double), _ptr(cq, C.c_double))
    return d, cp, cq


def segment_pierces(p0, p1, T):
    lib = _load()
    p0, p1, T, x = _d(p0).reshape(3), _d(p1).reshape(3), _d(T).reshape(9), np.zeros(3)
    hit = lib.orc_segment_pierces(_ptr(p0, C.c_double), _ptr(p1, C.c_double),
                                  _ptr(T, C.c_double), _ptr(x, C.c_double))
    return bool(hit), x


def box_bounds(a, b):
    """(d_min^L, d_min^U enhanced, d_max^U, d_max^L enhanced) for boxes
    a, b = [minx, miny, minz, maxx, maxy, maxz]."""
    lib = _load()
    a, b, out = _d(a).reshape(6), _d(b).reshape(6), np.zeros(4)
    lib.orc_box_bounds(_ptr(a, C.c_double), _ptr(b, C.c_double), _ptr(out, C.c_double))
    return out


def pose_points(verts, pose12):
    lib = _load()
    v = np.ascontiguousarray(verts, dtype=np.float32)
    p = _d(pose12).reshape(12)
    out = np.zeros((v.shape[0], 3))
    lib.orc_pose_points(_ptr(v, C.c_float), v.shape[0], _ptr(p, C.c_double), _ptr(out, C.c_double))
    return out


# ---------------------------------------------------------------- queries
def tau_for(verts_a, tris_a, pose_a12, verts_b, tris_b, pose_b12) -> float:
    """Tie tolerance 1e-12 * max(1, M).  M is the largest world coordinate
    magnitude over the eight corners of each mesh's local bounding box (the
    box of the vertices its triangles use), posed in FP64."""
    def extent(v, f, p):
        fi = np.asarray(f, dtype=np.int64).ravel()
        if fi.size == 0 or fi.min() < 0 or fi.max() >= v.shape[0]:
            raise ValueError("triangle vertex index out of range (or no triangles)")
        used = np.zeros(v.shape[0], dtype=bool)
        used[fi] = True
        u = v[used].astype(np.float64)
        lo, hi = u.min(axis=0), u.max(axis=0)
        corners = np.array([[hi[k] if (c >> k) & 1 else lo[k] for k in range(3)] for c in range(8)])
        p = np.asarray(p, dtype=np.float64).reshape(12)
        return float(np.abs(corners @ p[:9].reshape(3, 3).T + p[9:]).max())
    m = max(extent(verts_a, tris_a, pose_a12), extent(verts_b, tris_b, pose_b12))
    return 1e-12 * max(1.0, m)


def query(verts_a, tris_a, pose_a12, verts_b, tris_b, pose_b12, mode: int = 0,
          method: str = "auto", threads: Optional[int] = None, tau: Optional[float] = None,
          tie_cap: int = 4096) -> dict:
    """Exact D_min (mode 0) or D_max (mode 1) with the canonical pair.

    method: "brute" (all pairs, multithreaded), "bvh" (the oracle's own tree,
    single thread) or "auto" (brute when the pair count is small).
    """
    lib = _load()
    va = np.ascontiguousarray(verts_a, dtype=np.float32)
    vb = np.ascontiguousarray(verts_b, dtype=np.float32)
    fa = np.ascontiguousarray(tris_a, dtype=np.uint32)
    fb = np.ascontiguousarray(tris_b, dtype=np.uint32)
    pa, pb = _d(pose_a12).reshape(12), _d(pose_b12).reshape(12)
    if tau is None:
        tau = tau_for(va, fa, pa, vb, fb, pb)
    if method == "auto":
        method = "brute" if fa.shape[0] * fb.shape[0] <= 8_000_000 else "bvh"
    if threads is None:
        threads = max(1, min(16, os.cpu_count() or 1))
    res = OrcResult()
    ties = np.zeros((tie_cap, 2), dtype=np.int64)
    common = [_ptr(va, C.c_float), va.shape[0], _ptr(fa, C.c_uint32), fa.shape[0], _ptr(pa, C.c_double),
              _ptr(vb, C.c_float), vb.shape[0], _ptr(fb, C.c_uint32), fb.shape[0], _ptr(pb, C.c_double),
              int(mode), float(tau)]
    if method == "brute":
        rc = lib.orc_brute(*common, int(threads), C.byref(res), _ptr(ties, C.c_int64), tie_cap)
    elif method == "bvh":
        rc = lib.orc_bvh(*common, C.byref(res), _ptr(ties, C.c_int64), tie_cap)
    else:
        raise ValueError(method)
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    n = int(res.n_ties)
    return {
        "distance": float(res.distance),
        "tri_a": int(res.tri_a), "tri_b": int(res.tri_b),
        "point_a": np.array(res.point_a[:]), "point_b": np.array(res.point_b[:]),
        "pair_distance": float(res.pair_distance),
        "n_ties": n, "ties": ties[:min(n, tie_cap)].copy(),
        "pairs_tested": int(res.pairs_tested), "tau": float(tau), "method": method,
    }


def max_vertex_pairs(verts_a, pose_a12, verts_b, pose_b12, threads: int = 8) -> float:
    lib = _load()
    va = np.ascontiguousarray(verts_a, dtype=np.float32)
    vb = np.ascontiguousarray(verts_b, dtype=np.float32)
    pa, pb = _d(pose_a12).reshape(12), _d(pose_b12).reshape(12)
    return float(lib.orc_max_vertex_pairs(_ptr(va, C.c_float), va.shape[0], _ptr(pa, C.c_double),
                                          _ptr(vb, C.c_float), vb.shape[0], _ptr(pb, C.c_double),
                                          int(threads)))


def vertex_row_max(verts_a, pose_a12, verts_b, pose_b12, threads: int = 8) -> np.ndarray:
    """rowmax[i] = max over vertices b of |a_i - b| after the poses (FP64)."""
    lib = _load()
    va = np.ascontiguousarray(verts_a, dtype=np.float32)
    vb = np.ascontiguousarray(verts_b, dtype=np.float32)
    pa, pb = _d(pose_a12).reshape(12), _d(pose_b12).reshape(12)
    out = np.zeros(va.shape[0])
    lib.orc_vertex_row_max(_ptr(va, C.c_float), va.shape[0], _ptr(pa, C.c_double),
                           _ptr(vb, C.c_float), vb.shape[0], _ptr(pb, C.c_double), int(threads),
                           _ptr(out, C.c_double))
    return out


def max_by_vertices(verts_a, tris_a, pose_a12, verts_b, tris_b, pose_b12, threads: int = 8,
                    tau: Optional[float] = None) -> dict:
    """D_max and its tie set from the vertex-pair definition (the maximum over
    two closed triangles is attained at vertices, so the triangle pairs tied
    at D_max are the pairs of triangles incident to the tied vertex pairs).
    Exact for the value; the tie set is complete for pairs within tau."""
    va = np.ascontiguousarray(verts_a, dtype=np.float32)
    vb = np.ascontiguousarray(verts_b, dtype=np.float32)
    fa = np.ascontiguousarray(tris_a, dtype=np.uint32)
    fb = np.ascontiguousarray(tris_b, dtype=np.uint32)
    if tau is None:
        tau = tau_for(va, fa, pose_a12, vb, fb, pose_b12)
    rm = vertex_row_max(va, pose_a12, vb, pose_b12, threads)
    D = float(rm.max())
    A = pose_points(va, pose_a12)
    B = pose_points(vb, pose_b12)
    tied_pairs = []
    for i in np.nonzero(rm >= D - tau)[0]:
        d = np.sqrt(((B - A[i]) ** 2).sum(1))
        for j in np.nonzero(d >= D - tau)[0]:
            tied_pairs.append((int(i), int(j)))
    tri_pairs = set()
    for i, j in tied_pairs:
        ta = np.nonzero((fa == i).any(1))[0]
        tb = np.nonzero((fb == j).any(1))[0]
        for x in ta:
            for y in tb:
                tri_pairs.add((int(x), int(y)))
    ties = sorted(tri_pairs)
    return {"distance": D, "tri_a": ties[0][0], "tri_b": ties[0][1], "n_ties": len(ties),
            "ties": np.array(ties, dtype=np.int64), "tau": float(tau), "method": "vertex-pairs"}
