"""Pins for the oracle's geometric primitives (CPU only).

Each primitive is checked against something other than itself: hand cases with
known closed-form answers, and dense point sampling of the two sets, which
bounds the exact distance from the other side (the sampled minimum can only
exceed the true minimum, by at most the sampling spacing; the sampled maximum
equals the true maximum because the vertices are among the samples).
"""
import numpy as np
import pytest


def tri_samples(T, n):
    """Barycentric grid on triangle T (includes its vertices and edges)."""
    T = np.asarray(T, np.float64).reshape(3, 3)
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    m = (i + j) <= n
    a, b = i[m] / n, j[m] / n
    w = np.stack([1 - a - b, a, b], -1)
    return w @ T


def sampled_minmax(P, Q, n=80):
    X, Y = tri_samples(P, n), tri_samples(Q, n)
    d2 = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    return np.sqrt(d2.min()), np.sqrt(d2.max())


def diam(T):
    T = np.asarray(T).reshape(3, 3)
    return max(np.linalg.norm(T[i] - T[j]) for i in range(3) for j in range(3))


def on_triangle(x, T, tol=1e-9):
    """x lies on closed triangle T (distance to its plane and barycentrics)."""
    T = np.asarray(T).reshape(3, 3)
    a, b, c = T
    n = np.cross(b - a, c - a)
    nn = n @ n
    if nn == 0:
        return True
    if abs((x - a) @ n) / np.sqrt(nn) > tol:
        return False
    l1 = np.cross(c - b, x - b) @ n / nn
    l2 = np.cross(a - c, x - c) @ n / nn
    l3 = np.cross(b - a, x - a) @ n / nn
    return min(l1, l2, l3) >= -tol


# ------------------------------------------------------------------ hand cases
def test_point_segment_hand(orc):
    d = orc.segment_segment([0.5, 2, 0], [0.5, 2, 0], [0, 0, 0], [1, 0, 0])[0]
    assert d == pytest.approx(2.0)
    d, _ = orc.point_triangle([0.2, 0.2, 3.0], [[0, 0, 0], [1, 0, 0], [0, 1, 0]])
    assert d == pytest.approx(3.0, abs=1e-15)


def test_point_triangle_regions(orc):
    T = [[0, 0, 0], [2, 0, 0], [0, 2, 0]]
    # above the face interior: height
    d, q = orc.point_triangle([0.5, 0.5, -1.5], T)
    assert d == pytest.approx(1.5, abs=1e-15) and np.allclose(q, [0.5, 0.5, 0])
    # beyond vertex (2,0,0)
    d, q = orc.point_triangle([3, -1, 0], T)
    assert d == pytest.approx(np.sqrt(2)) and np.allclose(q, [2, 0, 0])
    # beyond the hypotenuse edge: distance to the line x+y=2 at z=1
    d, q = orc.point_triangle([2, 2, 1], T)
    assert d == pytest.approx(np.sqrt(2 + 1)) and np.allclose(q, [1, 1, 0])
    # degenerate triangle (collinear) falls back to its edges
    d, q = orc.point_triangle([0.5, 1, 0], [[0, 0, 0], [1, 0, 0], [2, 0, 0]])
    assert d == pytest.approx(1.0)


def test_segment_segment_hand(orc):
    # crossing skew segments (x axis at z=0, y axis at z=0.7): the gap 0.7
    d, cp, cq = orc.segment_segment([-1, 0, 0], [1, 0, 0], [0, -1, 0.7], [0, 1, 0.7])
    assert d == pytest.approx(0.7, abs=1e-15)
    assert np.allclose(cp, [0, 0, 0]) and np.allclose(cq, [0, 0, 0.7])
    # parallel, overlapping: perpendicular offset
    d, _, _ = orc.segment_segment([0, 0, 0], [2, 0, 0], [1, 0.3, 0], [3, 0.3, 0])
    assert d == pytest.approx(0.3, abs=1e-15)
    # parallel, disjoint along the line: endpoint gap
    d, _, _ = orc.segment_segment([0, 0, 0], [1, 0, 0], [2, 0.0, 0], [3, 0.0, 0])
    assert d == pytest.approx(1.0)
    # a degenerate (point) segment
    d, _, _ = orc.segment_segment([0, 0, 0], [0, 0, 0], [1, -1, 0], [1, 1, 0])
    assert d == pytest.approx(1.0)


def test_tri_tri_hand_cases(orc):
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    # parallel planes, overlapping footprints: the plane gap
    d, cp, cq = orc.tri_tri_min(P, P + [0.2, 0.1, 0.4])
    assert d == pytest.approx(0.4, abs=1e-15)
    # vertex above the face interior
    Q = np.array([[0.25, 0.25, 0.3], [0.3, 0.5, 2.0], [0.6, 0.2, 2.0]])
    d, cp, cq = orc.tri_tri_min(P, Q)
    assert d == pytest.approx(0.3, abs=1e-15) and np.allclose(cq, [0.25, 0.25, 0.3])
    # skew edges: only an edge-edge pair attains the minimum
    A = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, -0.2]])
    B = np.array([[0, -1, 0.5], [0, 1, 0.5], [0.1, 0, 1.5]])
    d, cp, cq = orc.tri_tri_min(A, B)
    assert d == pytest.approx(0.5, abs=1e-15)
    assert np.allclose(cp, [0, 0, 0]) and np.allclose(cq, [0, 0, 0.5])
    # piercing: a long thin triangle through the interior of P
    Pb = np.array([[-1, -1, 0], [3, -1, 0], [-1, 3, 0]], float)
    Qp = np.array([[0.3, 0.3, -1], [0.35, 0.3, 1], [0.3, 0.35, 1]])
    d, cp, cq = orc.tri_tri_min(Pb, Qp)
    assert d == 0.0 and np.allclose(cp, cq)
    # every feature distance is positive in this case: the crossing test decides
    feat = min(orc.point_triangle(Qp[i], Pb)[0] for i in range(3))
    assert feat > 0.5
    # coplanar overlap
    d, _, _ = orc.tri_tri_min(P, P + [0.2, 0.2, 0])
    assert d == 0.0
    # touching at a vertex
    d, _, _ = orc.tri_tri_min(P, -P)
    assert d == 0.0
    # both degenerate (collinear) triangles: segment-segment distance
    S1 = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], float)
    S2 = np.array([[1, -1, 0.25], [1, 0, 0.25], [1, 1, 0.25]], float)
    d, _, _ = orc.tri_tri_min(S1, S2)
    assert d == pytest.approx(0.25)


def test_pierce_hand(orc):
    T = [[-1, -1, 0], [3, -1, 0], [-1, 3, 0]]
    hit, x = orc.segment_pierces([0, 0, -1], [0, 0, 1], T)
    assert hit and np.allclose(x, 0)
    hit, _ = orc.segment_pierces([5, 5, -1], [5, 5, 1], T)
    assert not hit
    hit, _ = orc.segment_pierces([0, 0, 0.5], [0, 0, 1], T)
    assert not hit


# ------------------------------------------------------------- sampling pins
@pytest.mark.parametrize("seed", range(12))
def test_tri_tri_min_vs_sampling(orc, seed):
    rng = np.random.default_rng(seed)
    P = rng.normal(size=(3, 3))
    Q = rng.normal(size=(3, 3)) + rng.normal(size=3) * rng.uniform(0, 3)
    d, cp, cq = orc.tri_tri_min(P, Q)
    n = 80
    smin, smax = sampled_minmax(P, Q, n)
    assert d <= smin + 1e-12
    assert smin <= d + (diam(P) + diam(Q)) / n
    # the reported points lie on their triangles and realise d
    assert on_triangle(cp, P) and on_triangle(cq, Q)
    assert np.linalg.norm(cp - cq) == pytest.approx(d, abs=1e-12)
    dm, pa, pb = orc.tri_tri_max(P, Q)
    assert dm == pytest.approx(smax, rel=1e-15, abs=1e-15)
    assert np.linalg.norm(pa - pb) == pytest.approx(dm)


@pytest.mark.parametrize("seed", range(6))
def test_tri_tri_intersecting_random(orc, seed):
    """Triangles built to share an interior point must give zero."""
    rng = np.random.default_rng(100 + seed)
    X = rng.normal(size=3)
    def through(X):
        w = rng.dirichlet([2, 2, 2])
        E = rng.normal(size=(3, 3))
        E -= w @ E                      # barycentre combination of the corners is 0
        return X + E
    P, Q = through(X), through(X)
    d, cp, cq = orc.tri_tri_min(P, Q)
    assert d <= 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_point_triangle_vs_sampling(orc, seed):
    rng = np.random.default_rng(200 + seed)
    T = rng.normal(size=(3, 3))
    p = rng.normal(size=3) * 2
    d, q = orc.point_triangle(p, T)
    S = tri_samples(T, 300)
    s = np.sqrt(((S - p) ** 2).sum(-1)).min()
    assert d <= s + 1e-12 and s <= d + diam(T) / 300
    assert on_triangle(q, T)


@pytest.mark.parametrize("seed", range(6))
def test_segment_segment_vs_sampling(orc, seed):
    rng = np.random.default_rng(300 + seed)
    p0, p1, q0, q1 = rng.normal(size=(4, 3))
    d, cp, cq = orc.segment_segment(p0, p1, q0, q1)
    s = np.linspace(0, 1, 2001)
    X = p0 + s[:, None] * (p1 - p0)
    Y = q0 + s[:, None] * (q1 - q0)
    smin = np.sqrt(((X[:, None] - Y[None]) ** 2).sum(-1)).min()
    assert d <= smin + 1e-12
    assert smin <= d + (np.linalg.norm(p1 - p0) + np.linalg.norm(q1 - q0)) / 2000
    assert np.linalg.norm(cp - cq) == pytest.approx(d, abs=1e-12)


def test_planted_mistake_is_caught(orc):
    """A plausible oracle mistake -- dropping the edge-edge features -- would
    give a value far above the sampled minimum on the skew-edge case, which
    is what the sampling pin checks."""
    A = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, -0.2]])
    B = np.array([[0, -1, 0.5], [0, 1, 0.5], [0.1, 0, 1.5]])
    vertex_only = min([orc.point_triangle(A[i], B)[0] for i in range(3)] +
                      [orc.point_triangle(B[j], A)[0] for j in range(3)])
    smin, _ = sampled_minmax(A, B, 80)
    assert vertex_only > smin + (diam(A) + diam(B)) / 80
