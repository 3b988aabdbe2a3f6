"""GPU parity of the individual device routines and of the tree build."""
import numpy as np
import pytest

import meshgen as g
from paper_2411_11244_amd import gdist

pytestmark = pytest.mark.gpu


def random_boxes(rng, n):
    c = rng.normal(size=(n, 3)) * rng.uniform(0.1, 3, size=(n, 1))
    h = np.abs(rng.normal(size=(n, 3))) * rng.uniform(0.01, 1.5, size=(n, 1))
    flat = rng.uniform(size=(n, 3)) < 0.1          # some flat boxes
    h[flat] = 0.0
    return np.concatenate([c - h, c + h], 1).astype(np.float32)


def test_box_bounds_vs_oracle(orc, gctx):
    rng = np.random.default_rng(11)
    n = 3000
    a = random_boxes(rng, n)
    b = random_boxes(rng, n)
    b[: n // 3] = a[: n // 3] + np.float32(0.05) * rng.normal(size=(n // 3, 6)).astype(np.float32)
    b[: n // 3, 3:] = np.maximum(b[: n // 3, 3:], b[: n // 3, :3])
    got = gdist.gdist_eval_box_bounds(gctx, a, b)
    want = np.array([orc.box_bounds(a[i].astype(np.float64), b[i].astype(np.float64)) for i in range(n)])
    scale = np.maximum(np.abs(a).max(1), np.abs(b).max(1))[:, None]
    err = np.abs(got - want)
    # FP32 evaluation of sums of squares: a few ulps of the coordinate scale
    assert np.all(err <= 16 * 2.0 ** -24 * (scale + want)), err.max()


def tri_cases(rng, n):
    P = rng.normal(size=(n, 3, 3))
    off = rng.normal(size=(n, 1, 3)) * rng.uniform(0, 2.5, size=(n, 1, 1))
    Q = rng.normal(size=(n, 3, 3)) * rng.uniform(0.05, 1.0, size=(n, 1, 1)) + off
    # degenerate triangles and shared-vertex / coplanar configurations
    k = n // 10
    P[:k, 2] = P[:k, 0] + 0.5 * (P[:k, 1] - P[:k, 0])
    Q[k:2 * k] = P[k:2 * k] + np.array([0.3, -0.2, 0.0])
    Q[2 * k:3 * k, 0] = P[2 * k:3 * k, 0]
    return P.astype(np.float32), Q.astype(np.float32)


@pytest.mark.parametrize("mode", [0, 1])
def test_tri_tri_vs_oracle(orc, gctx, mode):
    rng = np.random.default_rng(21 + mode)
    n = 4000
    P, Q = tri_cases(rng, n)
    d32, d64 = gdist.gdist_eval_tri_tri(gctx, P.reshape(n, 9), Q.reshape(n, 9), mode)
    f = orc.tri_tri_max if mode else orc.tri_tri_min
    ref = np.array([f(P[i].astype(np.float64), Q[i].astype(np.float64))[0] for i in range(n)])
    scale = np.maximum(np.abs(P).reshape(n, -1).max(1), np.abs(Q).reshape(n, -1).max(1))
    assert np.all(np.abs(d64 - ref) <= 1e-12 * (1 + scale)), np.abs(d64 - ref).max()
    # FP32 routine: within the inflation window the traversal uses (kappa 64)
    assert np.all(np.abs(d32 - ref) <= 64 * 2.0 ** -24 * (1 + scale)), np.abs(d32 - ref).max()


def morton_bits(n):
    """Bits per axis: 4 more than ceil(floor(log2 n) / 3), at most 21 and at
    most what fits in a 64-bit key beside the index bits of n - 1."""
    b = min(21, (int(np.floor(np.log2(n))) + 2) // 3 + 4)
    index_bits = int(n - 1).bit_length()
    return min(b, (64 - index_bits) // 3)


def numpy_morton_order(mesh):
    """Leaf order from the definition: Morton code of the FP32 centroid in the
    box of all vertices, morton_bits(n) bits per axis, stable sort."""
    v = mesh.verts
    t = mesh.tris
    b = morton_bits(len(t))
    c = (v[t[:, 0]] + v[t[:, 1]] + v[t[:, 2]]) * np.float32(1.0 / 3.0)
    lo, hi = v.min(0), v.max(0)
    ext = hi - lo
    u = np.where(ext > 0, (c - lo) / np.where(ext > 0, ext, 1), 0).astype(np.float32)
    s = u * np.float32(2.0 ** b)
    qmax = 2 ** b - 1
    q = np.where(s <= 0, 0, np.where(s >= np.float32(qmax), qmax, np.floor(s))).astype(np.uint64)
    code = np.zeros(len(t), np.uint64)
    for bit in range(b):
        for k in range(3):
            code |= ((q[:, k] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + (2 - k))
    return np.argsort(code, kind="stable")


def tied_mesh(rng, n_same, n_other):
    """n_same copies of one triangle (equal keys) interleaved with a soup: the
    stable order keeps the copies in index order across tiles and passes."""
    soup = g.random_soup(rng, n_other)
    verts = np.concatenate([np.array([[0.1, 0.2, 0.3], [0.15, 0.2, 0.3], [0.1, 0.25, 0.3]], np.float32),
                            soup.verts])
    other = soup.tris.astype(np.int64) + 3
    tris = np.zeros((n_same + n_other, 3), np.int64)
    pos = np.sort(rng.choice(n_same + n_other, n_other, replace=False))
    mask = np.zeros(n_same + n_other, bool)
    mask[pos] = True
    tris[mask] = other
    tris[~mask] = [0, 1, 2]
    return g.Mesh(verts, tris.astype(np.uint32))


MESHES = {
    "one": lambda: g.Mesh(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), np.array([[0, 1, 2]], np.uint32)),
    "three": lambda: g.random_soup(np.random.default_rng(3), 3),
    "seven": lambda: g.random_soup(np.random.default_rng(7), 7),
    "torus": lambda: g.torus(32, 32, 1.0, 0.25),
    "soup": lambda: g.random_soup(np.random.default_rng(5), 5000),
    "sphere": lambda: g.icosphere(9, 1.0, 1e-3, np.random.default_rng(2)),
    "height": lambda: g.heightfield(40, 0.02, np.random.default_rng(4)),
    # several sort tiles (8,192 keys) and a ragged last tile
    "soup100k": lambda: g.random_soup(np.random.default_rng(8), 100_003),
    # 30,000 equal keys spread over five tiles among 5,000 others
    "ties": lambda: tied_mesh(np.random.default_rng(9), 30_000, 5_000),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_build_invariants(gctx, name):
    m = MESHES[name]()
    h = gdist.gdist_build(gctx, m.verts, m.tris)
    try:
        e = gdist.gdist_mesh_export(gctx, h)
    finally:
        gdist.gdist_release(gctx, h)
    n, L, D = m.n_tris, e["n_leaves"], e["depth"]
    assert L == 1 << int(np.floor(np.log2(n))) and L == 1 << D
    orig = e["orig"].astype(np.int64)
    assert np.array_equal(np.sort(orig), np.arange(n))                # a permutation
    assert np.array_equal(orig, numpy_morton_order(m))               # bit-exact sort order
    assert np.array_equal(e["tris"].reshape(n, 3, 3), m.verts[m.tris[orig]])
    boxes = e["boxes"]
    tris = e["tris"].reshape(n, 3, 3)
    j = np.arange(L, dtype=np.int64)                                 # leaf boxes: tight
    s0, s1 = (j * n) // L, ((j + 1) * n) // L
    assert np.all((s1 - s0 >= 1) & (s1 - s0 <= 2))
    tmin, tmax = tris.min(1), tris.max(1)
    assert np.array_equal(boxes[L:2 * L, :3], np.minimum.reduceat(tmin, s0))
    assert np.array_equal(boxes[L:2 * L, 3:], np.maximum.reduceat(tmax, s0))
    i = np.arange(1, L)                                              # parent = union
    assert np.array_equal(boxes[i, :3], np.minimum(boxes[2 * i, :3], boxes[2 * i + 1, :3]))
    assert np.array_equal(boxes[i, 3:], np.maximum(boxes[2 * i, 3:], boxes[2 * i + 1, 3:]))
    assert np.array_equal(boxes[1, :3], m.verts[m.tris].reshape(-1, 3).min(0))


def test_concurrent_builds_two_contexts():
    """Builds on two contexts from two threads at once (the library takes them
    in turns per device) give the same trees as a build alone."""
    import threading
    m = MESHES["soup100k"]()
    ctxs = [gdist.gdist_create(0) for _ in range(2)]
    out, errs = [None, None], []

    def run(i):
        try:
            orders = []
            for _ in range(3):
                h = gdist.gdist_build(ctxs[i], m.verts, m.tris)
                e = gdist.gdist_mesh_export(ctxs[i], h)
                orders.append((e["orig"].copy(), e["boxes"].copy()))
                gdist.gdist_release(ctxs[i], h)
            out[i] = orders
        except Exception as ex:   # reported below
            errs.append(ex)

    try:
        ts = [threading.Thread(target=run, args=(i,)) for i in range(2)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert not errs, errs
        ref = numpy_morton_order(m)
        for orders in out:
            for orig, boxes in orders:
                assert np.array_equal(orig.astype(np.int64), ref)
                assert np.array_equal(boxes[1:], out[0][0][1][1:])   # entry 0 is unused
    finally:
        for c in ctxs:
            gdist.gdist_destroy(c)
