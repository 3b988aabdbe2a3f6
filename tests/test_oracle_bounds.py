"""Pins for the oracle's AABB distance bounds (gDist Sec. 4), CPU only.

* A hand-derived worked example (unit cubes), stored in tests/golden/.
* Property test on tight boxes (boxes of random point clouds: each face holds
  a point, which is the paper's tightness condition): the four bounds bracket
  the true point-set min / max distance.
* The enhanced upper bound of the minimum re-derived from face corners (the
  farthest points of two rectangles are corners), independent of the per-axis
  formula the oracle uses.
"""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "box_bounds.txt")


def load_golden():
    rows = []
    with open(GOLD) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            vals = [float(eval(x, {"sqrt": np.sqrt})) for x in line.split()]
            rows.append((vals[:6], vals[6:12], vals[12:16]))
    return rows


def test_golden_examples(orc):
    rows = load_golden()
    assert len(rows) >= 3
    for a, b, want in rows:
        got = orc.box_bounds(a, b)
        assert np.allclose(got, want, rtol=1e-15, atol=1e-15), (a, b, got, want)


def face_corners(box, k):
    lo, hi = np.asarray(box[:3], float), np.asarray(box[3:], float)
    ax = k % 3
    v = hi[ax] if k // 3 else lo[ax]
    out = []
    for bits in range(8):
        c = np.where([(bits >> i) & 1 for i in range(3)], hi, lo)
        c[ax] = v
        out.append(c)
    return np.unique(np.array(out), axis=0)


def corner_based_min_upper(a, b):
    best = np.inf
    for i in range(6):
        for j in range(6):
            A, B = face_corners(a, i), face_corners(b, j)
            m = np.sqrt(((A[:, None] - B[None]) ** 2).sum(-1)).max()
            best = min(best, m)
    return best


@pytest.mark.parametrize("seed", range(40))
def test_bounds_bracket_point_sets(orc, seed):
    rng = np.random.default_rng(seed)
    n1, n2 = rng.integers(2, 12, size=2)
    X = rng.normal(size=(n1, 3)) * rng.uniform(0.1, 2, size=3)
    Y = rng.normal(size=(n2, 3)) * rng.uniform(0.1, 2, size=3) + rng.normal(size=3) * rng.uniform(0, 4)
    a = np.concatenate([X.min(0), X.max(0)])
    b = np.concatenate([Y.min(0), Y.max(0)])
    lo_min, up_min, up_max, lo_max = orc.box_bounds(a, b)
    D = np.sqrt(((X[:, None] - Y[None]) ** 2).sum(-1))
    eps = 1e-12
    assert lo_min <= D.min() + eps
    assert D.min() <= up_min + eps          # needs tightness (Sec. 4)
    assert up_min <= up_max + eps           # enhanced is no worse than conventional
    assert lo_max <= D.max() + eps          # needs tightness
    assert D.max() <= up_max + eps
    assert lo_max >= lo_min - eps
    assert up_min == pytest.approx(corner_based_min_upper(a, b), rel=1e-14, abs=1e-14)


def test_enhanced_upper_needs_tightness(orc):
    """A loose box can make d_min^U smaller than the true distance: the
    reason the paper forbids enlarging boxes (Sec. 4)."""
    X = np.array([[-5.0, 0.0, 0.0]])
    Y = np.array([[3.0, 0.0, 0.0]])
    a = np.array([-5, -0.1, -0.1, 0, 0.1, 0.1])   # loose box: no point on its x-max face
    b = np.array([1, -0.1, -0.1, 3, 0.1, 0.1])    # loose box: no point on its x-min face
    up_min = orc.box_bounds(a, b)[1]
    assert up_min < 8.0                           # below the true distance: would cull wrongly
