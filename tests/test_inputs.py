"""The seeded input generators shared by the oracle tests and the device
tests: the irregular polygons are simple, counter-clockwise and reproducible."""
import numpy as np

from paper_2606_10784_amd import workloads as wl


def _segments_cross(p, q, r, s):
    def orient(a, b, c):
        return np.sign((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
    return orient(p, q, r) * orient(p, q, s) < 0 and orient(r, s, p) * orient(r, s, q) < 0


def test_irregular_polygon_is_simple_and_ccw():
    for seed, n in ((1, 3), (2, 4), (3, 40), (4, 157)):
        xy = wl.irregular_polygon(np.random.default_rng(seed), 1.0, n)
        assert xy.shape == (n, 2)
        x, y = xy[:, 0], xy[:, 1]
        assert 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y) > 0          # CCW
        th = np.unwrap(np.arctan2(y, x))
        assert np.all(np.diff(th) > 0) and th[-1] - th[0] < 2 * np.pi           # star-shaped order
        segs = [(xy[i], xy[(i + 1) % n]) for i in range(n)]
        for i in range(n):
            for j in range(i + 2, n):
                if i == 0 and j == n - 1:
                    continue
                assert not _segments_cross(*segs[i], *segs[j])
        assert np.array_equal(xy, wl.irregular_polygon(np.random.default_rng(seed), 1.0, n))
