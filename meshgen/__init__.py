"""Seeded synthetic meshes, poses and workloads for the mesh-distance path.

This module produces inputs only: indexed FP32 triangle meshes, FP64 rigid
poses and request streams.  It contains none of the distance arithmetic, so
both the FP64 CPU oracle and the GPU library can be fed from it without
sharing any of the method's code.

Every generator takes either explicit sizes or a ``numpy.random.Generator``
(PCG64 via ``numpy.random.default_rng(seed)``) so a workload is fully
determined by its seed.

Mesh convention: ``verts`` is ``float32[nv, 3]`` (C-contiguous), ``tris`` is
``uint32[nt, 3]`` (C-contiguous), indices are 0-based.
Pose convention: ``(R, t)`` with ``R`` ``float64[3, 3]`` row-major and ``t``
``float64[3]``; a local point x maps to world ``R @ x + t``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

Pose = Tuple[np.ndarray, np.ndarray]


@dataclass
class Mesh:
    verts: np.ndarray  # float32 [nv, 3]
    tris: np.ndarray   # uint32 [nt, 3]
    name: str = ""

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])


def _finish(v64: np.ndarray, f: np.ndarray, name: str) -> Mesh:
    v = np.ascontiguousarray(v64, dtype=np.float32)
    t = np.ascontiguousarray(f, dtype=np.uint32)
    return Mesh(v, t, name)


# --------------------------------------------------------------------------
# Mesh generators
# --------------------------------------------------------------------------

def torus(nu: int, nv: int, R: float, r: float) -> Mesh:
    """Parametric torus grid with axis z, centred at the origin.

    Vertex (i, j) sits at u = 2*pi*i/nu, v = 2*pi*j/nv:
    ((R + r cos v) cos u, (R + r cos v) sin u, r sin v).
    Quad (i, j) with corners a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1)
    (indices wrap) gives triangles (a, b, c) and (a, c, d).
    nu*nv vertices, 2*nu*nv triangles.
    """
    u = 2.0 * np.pi * np.arange(nu, dtype=np.float64) / nu
    v = 2.0 * np.pi * np.arange(nv, dtype=np.float64) / nv
    uu, vv = np.meshgrid(u, v, indexing="ij")
    x = (R + r * np.cos(vv)) * np.cos(uu)
    y = (R + r * np.cos(vv)) * np.sin(uu)
    z = r * np.sin(vv)
    verts = np.stack([x, y, z], axis=-1).reshape(-1, 3)
    i = np.arange(nu, dtype=np.int64)[:, None]
    j = np.arange(nv, dtype=np.int64)[None, :]
    i1 = (i + 1) % nu
    j1 = (j + 1) % nv
    a = (i * nv + j).ravel()
    b = np.broadcast_to(i1 * nv + j, (nu, nv)).ravel()
    c = (i1 * nv + j1).ravel()
    d = np.broadcast_to(i * nv + j1, (nu, nv)).ravel()
    t1 = np.stack([a, b, c], axis=-1)
    t2 = np.stack([a, c, d], axis=-1)
    tris = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return _finish(verts, tris, f"torus{nu}x{nv}")


def _icosahedron() -> Tuple[np.ndarray, np.ndarray]:
    """12 unit vertices and 20 outward-oriented faces of a regular icosahedron.

    The faces are found rather than tabulated: every vertex triple whose
    three pairwise distances equal the edge length is a face.
    """
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    raw = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            raw.append((0.0, s1, s2 * phi))
            raw.append((s1, s2 * phi, 0.0))
            raw.append((s2 * phi, 0.0, s1))
    V = np.array(raw, dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    d = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=-1)
    edge = np.min(d[d > 1e-9])
    adj = np.abs(d - edge) < 1e-9
    faces = []
    for a in range(12):
        for b in range(a + 1, 12):
            if not adj[a, b]:
                continue
            for c in range(b + 1, 12):
                if adj[a, c] and adj[b, c]:
                    n = np.cross(V[b] - V[a], V[c] - V[a])
                    if np.dot(n, V[a] + V[b] + V[c]) < 0:
                        faces.append((a, c, b))
                    else:
                        faces.append((a, b, c))
    F = np.array(faces, dtype=np.int64)
    assert F.shape == (20, 3)
    return V, F


def icosphere(n: int, radius: float = 1.0, noise: float = 0.0,
              rng: np.random.Generator | None = None) -> Mesh:
    """Geodesic sphere: each icosahedron face split into n*n triangles.

    Grid points of a face (A, B, C) carry integer weights (n-i-j, i, j) on
    its corners; points shared by neighbouring faces are merged through an
    exact integer key of their (corner id, weight) pairs, giving 10 n^2 + 2
    vertices and 20 n^2 triangles.  Each vertex is projected to the sphere and
    its radius is drawn uniformly from [radius - noise, radius + noise].
    """
    V, F = _icosahedron()
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    m = (ii + jj) <= n
    gi, gj = ii[m], jj[m]                      # grid points of one face
    gw = np.stack([n - gi - gj, gi, gj], -1)   # weights on (A, B, C)
    local = -np.ones((n + 1, n + 1), dtype=np.int64)
    local[gi, gj] = np.arange(gi.size)
    # triangles of one face in local grid-point numbering
    ti, tj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    up = (ti + tj) < n
    a_i, a_j = ti[up], tj[up]
    t_up = np.stack([local[a_i, a_j], local[a_i + 1, a_j], local[a_i, a_j + 1]], -1)
    dn = (ti + tj) < n - 1
    b_i, b_j = ti[dn], tj[dn]
    t_dn = np.stack([local[b_i + 1, b_j], local[b_i + 1, b_j + 1], local[b_i, b_j + 1]], -1)
    tloc = np.concatenate([t_up, t_dn], 0)
    P = gi.size
    base = 13 * (n + 1)
    keys = np.empty((20, P), dtype=np.int64)
    pos = np.empty((20, P, 3), dtype=np.float64)
    for f in range(20):
        vid = np.broadcast_to(F[f], gw.shape).copy()
        w = gw.copy()
        vid[w == 0] = 12                       # sentinel sorts last
        order = np.argsort(vid, axis=1, kind="stable")
        vid = np.take_along_axis(vid, order, 1)
        w = np.take_along_axis(w, order, 1)
        code = vid * (n + 1) + w
        keys[f] = (code[:, 0] * base + code[:, 1]) * base + code[:, 2]
        vv = np.where(vid[..., None] < 12, V[np.minimum(vid, 11)], 0.0)
        pos[f] = (w[..., None] * vv).sum(1) / n
    ukeys, first, inv = np.unique(keys.ravel(), return_index=True, return_inverse=True)
    verts = pos.reshape(-1, 3)[first]
    verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    rad = np.full(verts.shape[0], radius, dtype=np.float64)
    if noise > 0.0:
        assert rng is not None
        rad = rad + rng.uniform(-noise, noise, size=verts.shape[0])
    verts *= rad[:, None]
    inv = inv.reshape(20, P)
    tris = np.concatenate([inv[f][tloc] for f in range(20)], 0)
    return _finish(verts, tris, f"icosphere{n}")


def ellipsoid(n_lat: int, n_lon: int, axes: Tuple[float, float, float]) -> Mesh:
    """UV ellipsoid: two poles, n_lat - 1 latitude rings of n_lon vertices.

    Ring k (1..n_lat-1) is at polar angle pi*k/n_lat; 2*n_lon*(n_lat-1)
    triangles (pole fans plus quads split in two).
    """
    a, b, c = axes
    th = np.pi * np.arange(1, n_lat, dtype=np.float64) / n_lat
    ph = 2.0 * np.pi * np.arange(n_lon, dtype=np.float64) / n_lon
    T, Pp = np.meshgrid(th, ph, indexing="ij")
    ring = np.stack([a * np.sin(T) * np.cos(Pp), b * np.sin(T) * np.sin(Pp),
                     c * np.cos(T)], -1).reshape(-1, 3)
    verts = np.concatenate([[[0.0, 0.0, c]], ring, [[0.0, 0.0, -c]]], 0)
    top, bot = 0, verts.shape[0] - 1

    def rid(k, m):
        return 1 + k * n_lon + (m % n_lon)

    m = np.arange(n_lon)
    fans_t = np.stack([np.full(n_lon, top), rid(0, m), rid(0, m + 1)], -1)
    kk, mm = np.meshgrid(np.arange(n_lat - 2), m, indexing="ij")
    kk, mm = kk.ravel(), mm.ravel()
    q1 = np.stack([rid(kk, mm), rid(kk + 1, mm), rid(kk + 1, mm + 1)], -1)
    q2 = np.stack([rid(kk, mm), rid(kk + 1, mm + 1), rid(kk, mm + 1)], -1)
    fans_b = np.stack([rid(n_lat - 2, m), np.full(n_lon, bot), rid(n_lat - 2, m + 1)], -1)
    tris = np.concatenate([fans_t, q1, q2, fans_b], 0)
    return _finish(verts, tris, f"ellipsoid{n_lat}x{n_lon}")


def heightfield(m: int, sigma: float, rng: np.random.Generator | None = None,
                extent: float = 1.0) -> Mesh:
    """(m+1)^2 grid on [0, extent]^2 with z ~ N(0, sigma^2) per vertex; 2 m^2 triangles."""
    xs = np.linspace(0.0, extent, m + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Z = np.zeros_like(X)
    if sigma > 0.0:
        assert rng is not None
        Z = rng.normal(0.0, sigma, size=X.shape)
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    i, j = i.ravel(), j.ravel()
    a = i * (m + 1) + j
    b = (i + 1) * (m + 1) + j
    c = (i + 1) * (m + 1) + j + 1
    d = i * (m + 1) + j + 1
    tris = np.concatenate([np.stack([a, b, c], -1), np.stack([a, c, d], -1)], 0)
    return _finish(verts, tris, f"heightfield{m}")


def random_mesh_of_size(rng: np.random.Generator, target: int) -> Mesh:
    """One mesh from the three families at roughly ``target`` triangles."""
    kind = int(rng.integers(0, 3))
    if kind == 0:
        n = max(1, int(round(math.sqrt(target / 20.0))))
        return icosphere(n, 1.0, 1e-3, rng)
    if kind == 1:
        nl = max(2, int(round(math.sqrt(target / 4.0))))
        ax = tuple(float(x) for x in rng.uniform(0.5, 1.5, size=3))
        return ellipsoid(nl, 2 * nl, ax)
    m = max(1, int(round(math.sqrt(target / 2.0))))
    return heightfield(m, 0.02, rng)


def random_soup(rng: np.random.Generator, n_tris: int, scale: float = 1.0,
                tri_size: float = 0.1) -> Mesh:
    """Unstructured triangle soup: small random triangles in a cube (test input)."""
    c = rng.uniform(-scale, scale, size=(n_tris, 1, 3))
    off = rng.normal(0.0, tri_size, size=(n_tris, 3, 3))
    verts = (c + off).reshape(-1, 3)
    tris = np.arange(3 * n_tris, dtype=np.int64).reshape(-1, 3)
    return _finish(verts, tris, f"soup{n_tris}")


# --------------------------------------------------------------------------
# Poses
# --------------------------------------------------------------------------

def identity_pose() -> Pose:
    return np.eye(3), np.zeros(3)


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform SO(3) sample: a normalised 4-D Gaussian quaternion."""
    return quat_to_rot(rng.normal(size=4))


def rot_axis(axis: str, angle: float) -> np.ndarray:
    c, s = math.cos(angle), math.sin(angle)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)
    if axis == "y":
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def compose(p: Pose, q: Pose) -> Pose:
    """p after q: x -> Rp (Rq x + tq) + tp."""
    return p[0] @ q[0], p[0] @ q[1] + p[1]


def support(mesh: Mesh, pose: Pose, u: np.ndarray) -> float:
    """max over vertices of u . (R x + t) in FP64 (placement only)."""
    w = mesh.verts.astype(np.float64) @ pose[0].T + pose[1]
    return float(np.max(w @ u))


def place_with_gap(rng: np.random.Generator, ma: Mesh, mb: Mesh, gap: float,
                   ra: np.ndarray, rb: np.ndarray) -> Tuple[Pose, Pose]:
    """A at the origin with rotation ra; B with rotation rb translated along a
    random unit direction u so that the supporting planes of A (along u) and
    B (along -u) are ``gap`` apart.  For gap >= 0 the distance is >= gap."""
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    pa = (ra, np.zeros(3))
    hb = support(mb, (rb, np.zeros(3)), -u)
    ha = support(ma, pa, u)
    pb = (rb, u * (ha + hb + gap))
    return pa, pb


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclass
class Query:
    a: int                 # index into the mesh list
    b: int
    pose_a: Pose
    pose_b: Pose
    mode: int = 0          # 0 = min distance, 1 = max distance
    arrival: float = 0.0   # seconds (serving streams only)
    gap: float = float("nan")   # support-function gap of the placement (< 0: overlapping), where drawn


@dataclass
class Workload:
    name: str
    meshes: List[Mesh]
    queries: List[Query] = field(default_factory=list)
    notes: dict = field(default_factory=dict)


TORUS_TINY = dict(nu=32, nv=32, R=1.0, r=0.25)
TORUS_RINGS = dict(nu=2740, nv=1369, R=1.0, r=0.1)


def tiny(seed: int, identity_rotation: bool = False) -> Workload:
    """Two 32x32 tori (2,048 triangles each, R=1, r=0.25), one handle used twice.

    A is at the identity.  B gets a uniform random rotation (or none) and a
    translation dx ~ U[2.6, 3.0] along x.  Draw order: dx, then the quaternion.
    """
    rng = np.random.default_rng(seed)
    m = torus(**TORUS_TINY)
    dx = float(rng.uniform(2.6, 3.0))
    R = np.eye(3) if identity_rotation else random_rotation(rng)
    q = Query(0, 0, identity_pose(), (R, np.array([dx, 0.0, 0.0])), 0)
    return Workload("tiny", [m], [q], {"dx": dx})


def rings_pose_b(frame: int, R: float = 1.0, offset: float = 0.3,
                 deg_per_frame: float = 0.5) -> Pose:
    """B's pose in the Rings sequence: the torus axis turned from z to y, its
    centre moved to (R + offset, 0, 0), then the whole of B rotated about the
    world z axis by deg_per_frame * frame degrees."""
    base = (rot_axis("x", math.pi / 2.0), np.array([R + offset, 0.0, 0.0]))
    spin = (rot_axis("z", math.radians(deg_per_frame * frame)), np.zeros(3))
    return compose(spin, base)


def rings(frames: int = 100, nu: int = TORUS_RINGS["nu"], nv: int = TORUS_RINGS["nv"],
          R: float = 1.0, r: float = 0.1, first_frame: int = 0) -> Workload:
    """Two interlocked, non-touching tori (one handle twice).  A: axis z at the
    origin.  B: axis y, centre (R + 0.3, 0, 0), rotated about world z by
    0.5 degrees per frame.  Smooth-surface gap is 0.7 - 2 r."""
    m = torus(nu, nv, R, r)
    qs = [Query(0, 0, identity_pose(), rings_pose_b(f + first_frame, R), 0)
          for f in range(frames)]
    return Workload("rings", [m], qs, {"gap_smooth": 0.7 - 2 * r})


def batched_pair(seed: int, p: int, t_min: float = 1e3, t_max: float = 5e5, gap_min: float = 1e-3,
                 gap_max: float = 1.0):
    """Pair p of the batched workload, drawn from its own stream
    default_rng([seed, p]) so any pair can be generated alone.
    Returns (mesh_a, mesh_b, pose_a, pose_b, gap)."""
    rng = np.random.default_rng([seed, p])
    ta = math.exp(rng.uniform(math.log(t_min), math.log(t_max)))
    tb = math.exp(rng.uniform(math.log(t_min), math.log(t_max)))
    ma = random_mesh_of_size(rng, ta)
    mb = random_mesh_of_size(rng, tb)
    ra, rb = random_rotation(rng), random_rotation(rng)
    g = math.exp(rng.uniform(math.log(gap_min), math.log(gap_max)))
    pa, pb = place_with_gap(rng, ma, mb, g, ra, rb)
    return ma, mb, pa, pb, g


def batched(seed: int = 1, n_pairs: int = 256, t_min: float = 1e3, t_max: float = 5e5,
            gap_min: float = 1e-3, gap_max: float = 1.0) -> Workload:
    """n_pairs independent mesh pairs with log-uniform sizes, random SO(3)
    poses and a support-function gap g (log-uniform), so each distance >= g."""
    meshes: List[Mesh] = []
    qs: List[Query] = []
    gaps = []
    for p in range(n_pairs):
        ma, mb, pa, pb, g = batched_pair(seed, p, t_min, t_max, gap_min, gap_max)
        meshes += [ma, mb]
        qs.append(Query(2 * p, 2 * p + 1, pa, pb, 0))
        gaps.append(g)
    return Workload("batched", meshes, qs, {"gaps": gaps})


def serving_mesh(seed: int, i: int, t_min: float = 1e4, t_max: float = 2e6) -> Mesh:
    """Mesh i of the serving pool, from its own stream default_rng([seed, i])."""
    rng = np.random.default_rng([seed, i])
    t = math.exp(rng.uniform(math.log(t_min), math.log(t_max)))
    return random_mesh_of_size(rng, t)


def serving_pool(seed: int = 2, n_meshes: int = 64, t_min: float = 1e4,
                 t_max: float = 2e6) -> List[Mesh]:
    return [serving_mesh(seed, i, t_min, t_max) for i in range(n_meshes)]


def serving_stream(pool: List[Mesh], rate: float, n_queries: int, seed: int = 3,
                   overlap_frac: float = 0.1, max_frac: float = 0.5) -> List[Query]:
    """Open-loop Poisson arrivals at ``rate`` queries/s.  Each query: a uniform
    random pair of pool meshes, random SO(3) poses, a support-function gap
    (negative for ``overlap_frac`` of queries, so the meshes overlap), and
    mode max with probability ``max_frac``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    qs = []
    for _ in range(n_queries):
        t += float(rng.exponential(1.0 / rate))
        a, b = (int(x) for x in rng.integers(0, len(pool), size=2))
        ra, rb = random_rotation(rng), random_rotation(rng)
        if rng.uniform() < overlap_frac:
            g = -float(rng.uniform(0.05, 0.3))
        else:
            g = math.exp(rng.uniform(math.log(1e-3), math.log(1.0)))
        pa, pb = place_with_gap(rng, pool[a], pool[b], g, ra, rb)
        mode = 1 if rng.uniform() < max_frac else 0
        qs.append(Query(a, b, pa, pb, mode, t, g))
    return qs


def hard(seed: int = 4, n: int = 316, r_a: float = 1.0, r_b: float = 1.0001,
         noise: float = 2e-5) -> Workload:
    """Two concentric noisy geodesic spheres (20 n^2 triangles each) with
    uniform radial noise U[-noise, noise]; B is randomly rotated about the
    shared centre.  Queries: min and max distance."""
    rng = np.random.default_rng(seed)
    ma = icosphere(n, r_a, noise, rng)
    mb = icosphere(n, r_b, noise, rng)
    rb = random_rotation(rng)
    pa, pb = identity_pose(), (rb, np.zeros(3))
    qs = [Query(0, 1, pa, pb, 0), Query(0, 1, pa, pb, 1)]
    return Workload("hard", [ma, mb], qs, {})


def pose_to_flat(p: Pose) -> np.ndarray:
    """12 doubles: R row-major then t."""
    return np.concatenate([np.asarray(p[0], np.float64).ravel(),
                           np.asarray(p[1], np.float64).ravel()])
