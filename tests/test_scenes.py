"""The seeded generators: determinism, counts, geometry and the workload shapes (CPU)."""
import numpy as np

import scenes


def test_box_room_exact():
    s = scenes.box_room()
    assert s.n_points == 6700
    assert s.xyz.dtype == np.float32 and s.normal.dtype == np.float32 and s.label.dtype == np.uint32
    counts = np.bincount(s.label)
    assert list(counts) == [2000, 2000, 600, 600, 750, 750]
    # every point lies on its face, with the inward unit normal of that face
    faces = {0: (2, 0.0, +1), 1: (2, 3.0, -1), 2: (0, 0.0, +1), 3: (0, 10.0, -1), 4: (1, 0.0, +1), 5: (1, 8.0, -1)}
    for lab, (axis, c, sign) in faces.items():
        m = s.label == lab
        assert np.all(s.xyz[m, axis] == c)
        e = np.zeros(3, np.float32)
        e[axis] = sign
        assert np.all(s.normal[m] == e)
    # 20 cm spacing: cell centres
    assert np.allclose(np.unique(s.xyz[s.label == 0, 0]), np.arange(50) * 0.2 + 0.1)


def test_determinism():
    a = scenes.furnished_room(n_points=50_000, seed=3)
    b = scenes.furnished_room(n_points=50_000, seed=3)
    c = scenes.furnished_room(n_points=50_000, seed=4)
    assert np.array_equal(a.xyz, b.xyz) and np.array_equal(a.normal, b.normal) and np.array_equal(a.tx, b.tx)
    assert not np.array_equal(a.xyz[:100], c.xyz[:100]) or a.n_points != c.n_points


def test_furnished_room_shape():
    s = scenes.furnished_room(n_points=200_000)
    assert 200_000 <= s.n_points <= 215_000
    assert set(np.unique(s.label)) <= set(range(20))
    assert len(s.extra["boxes"]) == 30 and len(s.rx) == 16
    n = np.linalg.norm(s.normal.astype(np.float64), axis=1)
    assert np.allclose(n, 1.0, atol=1e-6)
    # TX/RX in free space: inside the room, outside every box by 0.3 m
    for p in np.vstack([s.tx, s.rx]):
        assert np.all(p >= 0.3 - 1e-6) and np.all(p[:2] <= np.array([12.0, 10.0]) - 0.3 + 1e-6)
        for lo, hi in s.extra["boxes"]:
            assert not (np.all(p >= lo - 0.3 + 1e-6) and np.all(p <= hi + 0.3 - 1e-6))
    assert abs(s.surfel_radius - 0.75 * s.spacing) < 1e-12


def test_street_canyon_small():
    s = scenes.street_canyon(n_points=300_000, n_tx=2, n_rx=5, scale=0.25, levels=(2.0, 0.5, 0.1))
    assert 290_000 <= s.n_points <= 330_000
    assert len(s.extra["buildings"]) == 120 and s.tx.shape == (2, 3) and s.rx.shape == (5, 3)
    assert s.label.max() <= 49
    # no ground point inside a footprint
    g = s.label == 0
    for lo, hi in s.extra["buildings"][:20]:
        inside = ((s.xyz[g, 0] > lo[0] + 0.05) & (s.xyz[g, 0] < hi[0] - 0.05) & (s.xyz[g, 1] > lo[1] + 0.05)
                  & (s.xyz[g, 1] < hi[1] - 0.05))
        assert not inside.any()


def test_moving_canyon_frames():
    sc, mover = scenes.moving_canyon(n_points=100_000, extent=(60.0, 60.0), lots=(2, 2), levels=(4.0, 1.0, 0.25))
    ids = sc.extra["moving_idx"]
    assert 0.03 * sc.n_points < len(ids) < 0.08 * sc.n_points
    i0, x0, n0 = mover(0)
    assert np.array_equal(i0, ids) and np.array_equal(x0, sc.xyz[ids])
    i1, x1, n1 = mover(1)
    step = np.linalg.norm(x1 - x0, axis=1)
    moved = step[step < 10.0]          # wrap-around excluded
    assert np.all(moved >= 0.5 - 1e-4) and np.all(moved <= 1.5 + 1e-4)   # 5-15 m/s over 100 ms
    assert np.array_equal(n1, n0)


def test_poisson_queries():
    sc, _ = scenes.moving_canyon(n_points=50_000, extent=(60.0, 60.0), lots=(2, 2))
    q = scenes.poisson_queries(seed=1, rate=200.0, duration=5.0, scene=sc)
    t = np.array([x["t"] for x in q])
    assert np.all(np.diff(t) > 0) and t[-1] <= 5.0
    assert 800 < len(q) < 1200
    rays = np.array([x["n_rays"] for x in q])
    assert rays.min() >= 65_536 - 256 and rays.max() <= 1_000_000 and np.all(rays % 256 == 0)
    assert all(1 <= len(x["rx"]) <= 8 for x in q)


def test_batch_scene_sizes():
    s = scenes.batch_scenes(seeds=[0, 1], point_scale=0.05, ray_scale=0.05)
    assert s[0].name.startswith("batch_0_furnished_room") and s[1].name.startswith("batch_1_street_canyon")
    assert all(x.n_rays % 256 == 0 and 1 <= len(x.rx) <= 32 for x in s)


def test_box_edges_are_convex_edges_of_the_box():
    """Every edge lies on the box's surface along one axis, its two face normals are
    unit, perpendicular to it and to each other and point away from the box; the
    RX of the corner building lies in the building's shadow seen from its TX."""
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([6.0, 6.0, 4.0])
    seg, nrm, lab = scenes.box_edges(lo, hi, 100)
    assert seg.shape == (8, 2, 3) and nrm.shape == (8, 2, 3)
    assert list(lab) == list(range(100, 108))
    centre = 0.5 * (lo + hi)
    for (a, b), (n1, n2) in zip(seg.astype(np.float64), nrm.astype(np.float64)):
        w = b - a
        assert np.count_nonzero(w) == 1 and np.linalg.norm(w) > 0
        mid = 0.5 * (a + b)
        # on two faces of the box: two coordinates at a bound
        at_bound = np.isclose(mid, lo) | np.isclose(mid, hi)
        assert at_bound.sum() == 2
        for n in (n1, n2):
            assert abs(np.linalg.norm(n) - 1.0) < 1e-6 and abs(n @ w) < 1e-9
            assert n @ (mid - centre) > 0
        assert abs(n1 @ n2) < 1e-9
    s = scenes.corner_building()
    t, r = s.tx[0].astype(np.float64), s.rx[0].astype(np.float64)
    # the straight segment TX -> RX passes through the building's footprint below its roof
    u = np.linspace(0.0, 1.0, 1001)[:, None]
    p = t + u * (r - t)
    inside = np.all((p > lo) & (p < hi), axis=1)
    assert inside.any()
