"""Host-side quality metrics, pinned by brute force."""
import numpy as np
import pytest

from paper_2205_13399_amd import quality


def _grid_area(points, ref):
    """Unit cells [x, x+1) x [y, y+1) below ref dominated by some point (integer data)."""
    area = 0
    for x in range(0, ref[0]):
        for y in range(0, ref[1]):
            if any(px <= x and py <= y for px, py in points):
                area += 1
    return area


@pytest.mark.parametrize("seed", range(8))
def test_hypervolume_equals_dominated_cells(seed):
    rng = np.random.default_rng(seed)
    pts = rng.integers(0, 30, size=(rng.integers(1, 12), 2))
    assert quality.hypervolume_2d(pts, (30, 30)) == _grid_area(pts.tolist(), (30, 30))


def test_hypervolume_special_cases():
    assert quality.hypervolume_2d(np.array([[1.0, 1.0]])) == pytest.approx(1.1 * 1.1)
    assert quality.hypervolume_2d(np.zeros((0, 2))) == 0.0
    assert quality.hypervolume_2d(np.array([[2.2, 1.0]])) == 0.0      # beyond the reference point
    # dominated and duplicate points change nothing
    base = np.array([[1.0, 1.8], [1.5, 1.2]])
    more = np.vstack([base, [[1.6, 1.9], [1.5, 1.2]]])
    assert quality.hypervolume_2d(more) == pytest.approx(quality.hypervolume_2d(base))


def test_nondominated_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(20):
        pts = rng.integers(0, 8, size=(15, 2))
        got = set(map(tuple, pts[quality.nondominated(pts)]))
        want = {tuple(p) for p in pts
                if not any((q[0] <= p[0] and q[1] <= p[1]) and tuple(q) != tuple(p) for q in pts)}
        assert got == want


def test_normalised_range():
    a = np.array([[10, 50], [20, 40]])
    b = np.array([[15, 45], [30, 30]])
    norm = quality.normaliser([a, b])
    allp = np.vstack([norm(a), norm(b)])
    assert allp.min() == 1.0 and allp.max() == 2.0
    res = quality.compare([a, b])
    assert all(0 <= r["hypervolume"] <= 1.21 for r in res)
