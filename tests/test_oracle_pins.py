"""Pins of the CPU oracle against facts fixed by geometry and the paper.

Each test checks the FP64 brute force against something other than itself:
hand-derived closed forms, the image method (paper, Introduction and
Section 2.3), the reflection law, the Fibonacci-lattice definition, and
brute-force single-surfel cases.  A dropped term, a wrong sign or index or a
transposed operand in oracle.c breaks at least one of them.
"""
import math
import os

import numpy as np
import pytest

import scenes

HERE = os.path.dirname(os.path.abspath(__file__))
SQRT3 = math.sqrt(3.0)


def _golden_box_room():
    out = {}
    with open(os.path.join(HERE, "golden", "box_room_image_paths.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, l2 = line.split()
            seq = () if name == "-" else tuple(int(x) for x in name.split(","))
            out[seq] = float(l2)
    return out


def _box_t_eps():
    return 1e-5 * math.sqrt(10 ** 2 + 8 ** 2 + 3 ** 2)


@pytest.fixture(scope="module")
def box_run(oracle_lib):
    s = scenes.box_room()
    d = oracle_lib.fibonacci(s.n_rays)
    r = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, d, K=2, r_s=s.surfel_radius, t_eps=_box_t_eps())
    return s, d, r


# --------------------------------------------------------------------------- directions

def test_fibonacci_definition(oracle_lib):
    for n in (1, 2, 7, 1000, 12345):
        d = oracle_lib.fibonacci(n).astype(np.float64)
        j = np.arange(n)
        z_expected = (1.0 - (2 * j + 1) / n).astype(np.float32).astype(np.float64)
        assert np.array_equal(d[:, 2], z_expected)
        assert np.max(np.abs(np.linalg.norm(d, axis=1) - 1.0)) < 4e-7
    # consecutive azimuths advance by the golden angle 2 pi (1 - g) = pi (3 - sqrt 5)
    d = oracle_lib.fibonacci(1000).astype(np.float64)
    phi = np.arctan2(d[:, 1], d[:, 0])
    step = np.mod(np.diff(phi), 2 * math.pi)
    golden = math.pi * (3.0 - math.sqrt(5.0))
    assert np.max(np.abs(step - golden)) < 1e-4
    with pytest.raises(ValueError):
        oracle_lib.fibonacci(0)


def test_ray_spacing_closed_form(oracle_lib):
    # hexagonal cells of area (sqrt3/2) a^2 cover 4 pi: a = sqrt(8 pi / (sqrt3 N))
    for n in (10, 10_000, 4_000_000):
        a = oracle_lib.ray_spacing(n)
        assert abs(n * (SQRT3 / 2) * a * a - 4 * math.pi) < 1e-9 * 4 * math.pi


def test_fibonacci_covering_radius(oracle_lib):
    """Every direction on the sphere lies within sigma * alpha / sqrt3 (sigma = 1.25) of a ray."""
    from scipy.spatial import cKDTree
    n = 10_000
    d = oracle_lib.fibonacci(n).astype(np.float64)
    rng = np.random.default_rng(0)
    probe = rng.normal(size=(200_000, 3))
    probe /= np.linalg.norm(probe, axis=1, keepdims=True)
    dist, _ = cKDTree(d).query(probe)
    ang = 2.0 * np.arcsin(np.minimum(dist / 2.0, 1.0))
    alpha = oracle_lib.ray_spacing(n)
    assert ang.max() <= 1.25 * alpha / SQRT3
    # and the lattice is not much finer than ideal either (median NN angle ~ alpha)
    nn, _ = cKDTree(d).query(d, k=2)
    med = np.median(2.0 * np.arcsin(nn[:, 1] / 2.0))
    assert 0.9 * alpha < med < 1.1 * alpha


# --------------------------------------------------------------------------- single surfels

def _one(oracle_lib, pts, nrms, o, d, r_s=0.1, t_eps=1e-6, K=0, rx=None, labels=None, **kw):
    pts = np.asarray(pts, np.float32).reshape(-1, 3)
    nrms = np.asarray(nrms, np.float32).reshape(-1, 3)
    lab = np.arange(pts.shape[0], dtype=np.uint32) if labels is None else np.asarray(labels, np.uint32)
    rx = np.zeros((0, 3), np.float32) if rx is None else np.asarray(rx, np.float32).reshape(-1, 3)
    return oracle_lib.launch(pts, nrms, lab, np.asarray(o, np.float32), rx, np.asarray(d, np.float32).reshape(1, 3),
                             K=K, r_s=r_s, t_eps=t_eps, n_threads=1, **kw)


def test_single_surfel_disk(oracle_lib):
    down = [0, 0, -1]
    # centre hit at t = 1, from either side of the two-sided disk
    r = _one(oracle_lib, [0, 0, 0], [0, 0, 1], [0.05, 0, 1], down)
    assert r["hit_id"][0, 0] == 0 and r["hit_t"][0, 0] == 1.0
    r = _one(oracle_lib, [0, 0, 0], [0, 0, -1], [0.05, 0, 1], down)
    assert r["hit_id"][0, 0] == 0 and r["hit_t"][0, 0] == 1.0
    # inside / outside the radius (both axes, so a transposed component fails)
    assert _one(oracle_lib, [0, 0, 0], [0, 0, 1], [0.0, 0.099, 1], down)["hit_id"][0, 0] == 0
    assert _one(oracle_lib, [0, 0, 0], [0, 0, 1], [0.0, 0.101, 1], down)["hit_id"][0, 0] == -1
    assert _one(oracle_lib, [0, 0, 0], [0, 0, 1], [0.101, 0.0, 1], down)["hit_id"][0, 0] == -1
    # tilted surfel: the hit distance follows the plane, not the centre
    n = np.array([0.0, 0.6, 0.8])
    r = _one(oracle_lib, [0, 0, 0], n, [0, 0.03, 2.0], down)
    assert abs(r["hit_t"][0, 0] - (2.0 + 0.03 * 0.6 / 0.8)) < 1e-7
    # behind the origin, and inside t_eps: no hit
    assert _one(oracle_lib, [0, 0, 0], [0, 0, 1], [0, 0, 1], [0, 0, 1])["hit_id"][0, 0] == -1
    assert _one(oracle_lib, [0, 0, 0], [0, 0, 1], [0, 0, 1e-3], down, t_eps=2e-3)["hit_id"][0, 0] == -1
    assert _one(oracle_lib, [0, 0, 0], [0, 0, 1], [0, 0, 3e-3], down, t_eps=2e-3)["hit_id"][0, 0] == 0
    # parallel ray: no hit
    assert _one(oracle_lib, [0, 0, 0], [0, 0, 1], [-1, 0, 0], [1, 0, 0])["hit_id"][0, 0] == -1


def test_nearest_and_tie_break(oracle_lib):
    down = [0, 0, -1]
    # nearer surfel wins regardless of index order
    r = _one(oracle_lib, [[0, 0, 0], [0, 0, 0.5]], [[0, 0, 1], [0, 0, 1]], [0, 0, 1], down)
    assert r["hit_id"][0, 0] == 1 and r["hit_t"][0, 0] == 0.5
    r = _one(oracle_lib, [[0, 0, 0.5], [0, 0, 0]], [[0, 0, 1], [0, 0, 1]], [0, 0, 1], down)
    assert r["hit_id"][0, 0] == 0
    # exact tie: the smaller index wins
    r = _one(oracle_lib, [[0.02, 0, 0], [0, 0, 0], [0.01, 0, 0]], [[0, 0, 1]] * 3, [0, 0, 1], down)
    assert r["hit_id"][0, 0] == 0


def test_skip_surfel_just_left(oracle_lib):
    # a ray bouncing between two parallel mirrors: the surfel it leaves is not hit again
    pts = [[0, 0, 0], [0, 0, 1]]
    nrm = [[0, 0, 1], [0, 0, -1]]
    r = _one(oracle_lib, pts, nrm, [0, 0, 0.5], [0, 0, -1], K=3, t_eps=0.0)
    assert list(r["hit_id"][0]) == [0, 1, 0, 1]
    assert list(r["seq"][0]) == [0, 1, 0]
    assert np.allclose(r["hit_t"][0], [0.5, 1.0, 1.0, 1.0])


def test_skip_surfel_just_left_tilted_mirrors(oracle_lib):
    # two parallel mirrors tilted off the axes, 1 m apart, t_eps = 0: a reflection point computed
    # in floating point sits a rounding error off its mirror's plane, in front of or behind it;
    # from behind, the plane lies at a tiny positive distance ahead.  Skipping the surfel just
    # left, every ray still alternates between the two mirrors for all six segments.
    n = np.array([0.3, 0.2, 1.0]) / np.linalg.norm([0.3, 0.2, 1.0])
    pts = np.array([[0.0, 0.0, 0.0], n]).astype(np.float32)
    nrm = np.array([n, -n]).astype(np.float32)
    rng = np.random.default_rng(7)
    dirs = -n[None] + 0.05 * rng.normal(size=(400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    o = (0.5 * n).astype(np.float32)[None]
    r = oracle_lib.launch(pts, nrm, np.arange(2, dtype=np.uint32), o, np.zeros((0, 3), np.float32),
                          dirs.astype(np.float32), K=5, r_s=10.0, t_eps=0.0, n_threads=1)
    assert np.array_equal(r["hit_id"], np.tile([0, 1, 0, 1, 0, 1], (400, 1)))
    assert np.all(r["hit_t"] > 0.4)


def test_reception_sphere(oracle_lib):
    # no points; one RX straight ahead at distance 10 and one off-axis
    alpha = 0.01
    rho10 = 1.25 * 10 * alpha / SQRT3
    rx = [[10, 0, 0], [10, 0.99 * rho10, 0], [10, 1.01 * rho10, 0], [-10, 0, 0]]
    r = oracle_lib.launch(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros(0, np.uint32),
                          np.zeros((1, 3), np.float32), np.asarray(rx, np.float32),
                          np.asarray([[1, 0, 0]], np.float32), K=1, r_s=0.1, t_eps=1e-6, alpha=alpha)
    got = sorted(int(x) for x in r["rec_rx"][r["rec_flags"] & 1 == 1])
    assert got == [0, 1]
    q = int(np.where(r["rec_rx"] == 0)[0][0])
    assert r["rec_lpoly"][q] == 10.0 and r["rec_lunf"][q] == 10.0 and r["rec_b"][q] == 0
    q = int(np.where(r["rec_rx"] == 1)[0][0])
    assert abs(r["rec_lunf"][q] - 10.0) < 1e-12
    assert abs(r["rec_lpoly"][q] - math.hypot(10.0, float(np.float32(0.99 * rho10)))) < 1e-12


def test_reception_only_before_hit(oracle_lib):
    # wall at x = 5 blocks the RX at x = 10 on segment 0, the reflection comes back to x = 2
    r = oracle_lib.launch(np.array([[5, 0, 0]], np.float32), np.array([[-1, 0, 0]], np.float32),
                          np.array([7], np.uint32), np.zeros((1, 3), np.float32),
                          np.array([[10, 0, 0], [2, 0, 0]], np.float32), np.array([[1, 0, 0]], np.float32),
                          K=1, r_s=0.1, t_eps=1e-6, alpha=0.01)
    rec = sorted((int(b), int(x), float(lp)) for b, x, lp in zip(r["rec_b"], r["rec_rx"], r["rec_lpoly"]))
    # RX1 at x=2 is passed on segment 0 (s = 2) and again after the bounce (L = 5, s = 3)
    assert rec == [(0, 1, 2.0), (1, 1, 8.0)]
    assert list(r["seq"][0]) == [7]


# --------------------------------------------------------------------------- closed forms on the box room

def test_golden_box_room_hand_values():
    g = _golden_box_room()
    # hand-derived images: TX (2,2,1.5), RX (7,5,1.5)
    assert g[()] == (7 - 2) ** 2 + (5 - 2) ** 2                       # line of sight
    assert g[(0,)] == 5 ** 2 + 3 ** 2 + (1.5 + 1.5) ** 2              # floor image (2,2,-1.5)
    assert g[(2,)] == (7 + 2) ** 2 + 3 ** 2                           # wall x=0 image (-2,2,1.5)
    assert g[(3,)] == (18 - 7) ** 2 + 3 ** 2                          # wall x=10 image (18,2,1.5)
    assert g[(0, 1)] == 5 ** 2 + 3 ** 2 + (7.5 - 1.5) ** 2            # floor then ceiling: (2,2,7.5)
    assert len(g) == 25
    assert sum(1 for s in g if len(s) == 1) == 6 and sum(1 for s in g if len(s) == 2) == 18


def test_golden_matches_image_method(oracle_lib):
    g = _golden_box_room()
    img = oracle_lib.image_method.box_room_paths((2, 2, 1.5), (7, 5, 1.5), (10, 8, 3), 2)
    assert set(img) == set(g)
    for seq, (L, _) in img.items():
        assert abs(L * L - g[seq]) < 1e-6


def test_los_closed_form(box_run, oracle_lib):
    """P1: the line-of-sight path length is the TX-RX distance."""
    s, d, r = box_run
    los = (r["rec_b"] == 0) & (r["rec_flags"] & 1 == 1)
    assert los.sum() >= 1
    L = math.sqrt(34.0)
    assert np.all(np.abs(r["rec_lpoly"][los] - L) <= 1e-12 * L)
    rho = 1.25 * L * oracle_lib.ray_spacing(s.n_rays) / SQRT3
    assert np.all(r["rec_lunf"][los] <= L * (1 + 1e-12))
    assert np.all(r["rec_lunf"][los] >= L - rho * rho / L)


def test_single_plane_image_source(oracle_lib):
    """P2: a ray aimed at the floor image point is received with L = |TX - RX'|."""
    s = scenes.box_room()
    d = np.array([5.0, 3.0, -3.0]) / math.sqrt(43.0)
    r = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, d.astype(np.float32).reshape(1, 3), K=1,
                          r_s=s.surfel_radius, t_eps=_box_t_eps(), alpha=oracle_lib.ray_spacing(s.n_rays))
    assert r["seq"][0, 0] == 0
    assert np.allclose(r["pts"][0, 0], [4.5, 3.5, 0.0], atol=1e-6)
    ok = (r["rec_b"] == 1) & (r["rec_flags"] & 1 == 1)
    assert ok.sum() == 1
    L = math.sqrt(43.0)
    assert abs(r["rec_lpoly"][ok][0] - L) <= 1e-12 * L
    assert abs(r["rec_lunf"][ok][0] - L) <= 1e-12 * L
    # the hit is the surfel centred on the image point (unique: neighbours are 0.2 m > r_s away)
    hid = int(r["hit_id"][0, 0])
    assert np.allclose(s.xyz[hid], [4.5, 3.5, 0.0])


def test_box_room_paths_equal_image_method(box_run, oracle_lib):
    """P4: with <= 2 reflections the coarse paths are exactly the 25 image-method sequences."""
    s, d, r = box_run
    paths, keys, _ = oracle_lib.dedup(r, 2)
    g = _golden_box_room()
    assert set(k[3] for k in keys) == set(g)
    assert all(k[0] == 0 and k[1] == 0 and k[2] == len(k[3]) for k in keys)
    img = oracle_lib.image_method.box_room_paths(s.tx[0], s.rx[0], (10, 8, 3), 2)
    c = 1.25 * oracle_lib.ray_spacing(s.n_rays) / SQRT3
    for k in keys:
        seq = k[3]
        L_img = math.sqrt(g[seq])
        lp = paths[k]["rows"][0][0]
        if seq:
            s_last = float(np.linalg.norm(img[seq][1][-1] - s.rx[0].astype(np.float64)))
        else:
            s_last = L_img
        assert L_img * (1 - 1e-12) <= lp <= L_img * (1 + c * c * L_img / s_last) + 1e-12


def test_reflection_law(oracle_lib):
    """P3: angle of incidence equals angle of reflection, in the plane of incidence."""
    s = scenes.random_scene(5, tilt_sigma=0.2, n_rays=1500, K=3)
    d = oracle_lib.fibonacci(s.n_rays)
    r = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, d, K=3, r_s=s.surfel_radius, t_eps=1e-6,
                          want_segments=True)
    nrm = s.normal.astype(np.float64)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    checked = 0
    for ray in range(r["hit_id"].shape[0]):
        for b in range(1, 4):
            m = r["hit_id"][ray, b - 1]
            if m < 0 or np.isnan(r["seg_d"][ray, b, 0]):
                break
            d0, d1, n = r["seg_d"][ray, b - 1], r["seg_d"][ray, b], nrm[m]
            assert abs(d1 @ n + d0 @ n) <= 1e-12
            assert abs(np.cross(d0, n) @ d1) <= 1e-12
            assert abs(np.linalg.norm(d1) - 1.0) <= 1e-12
            # the new origin lies on the surfel's plane, inside its disk
            o1 = r["seg_o"][ray, b]
            assert abs((o1 - s.xyz[m]) @ n) <= 1e-9
            assert np.linalg.norm(o1 - s.xyz[m]) <= s.surfel_radius * (1 + 1e-9)
            checked += 1
    assert checked > 100


def test_reciprocity(oracle_lib):
    """Swapping TX and RX reverses every coarse path of the box room."""
    s = scenes.box_room()
    d = oracle_lib.fibonacci(s.n_rays)
    a = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, d, K=2, r_s=s.surfel_radius, t_eps=_box_t_eps())
    b = oracle_lib.launch(s.xyz, s.normal, s.label, s.rx, s.tx, d, K=2, r_s=s.surfel_radius, t_eps=_box_t_eps())
    ka = set(k[3] for k in oracle_lib.dedup(a, 2)[1])
    kb = set(k[3][::-1] for k in oracle_lib.dedup(b, 2)[1])
    assert ka == kb


def test_monotone_in_k(box_run, oracle_lib):
    s, d, r2 = box_run
    r1 = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, d, K=1, r_s=s.surfel_radius, t_eps=_box_t_eps())
    k1 = set(oracle_lib.dedup(r1, 1)[1])
    k2 = set(oracle_lib.dedup(r2, 2)[1])
    assert k1 < k2
    assert k1 == {k for k in k2 if k[2] <= 1}


def test_empty_cloud_and_no_rx(oracle_lib):
    d = oracle_lib.fibonacci(2000)
    z = np.zeros((0, 3), np.float32)
    r = oracle_lib.launch(z, z, np.zeros(0, np.uint32), [[0, 0, 0]], [[3, 0, 0]], d, K=2, r_s=0.1, t_eps=1e-6)
    assert np.all(r["hit_id"][:, 0] == -1)
    assert r["n_rec"] >= 1 and np.all(r["rec_b"] == 0)
    assert np.allclose(r["rec_lpoly"], 3.0)
    s = scenes.box_room()
    r = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, np.zeros((0, 3), np.float32), d, K=2,
                          r_s=s.surfel_radius, t_eps=_box_t_eps())
    assert r["n_rec"] == 0


# --------------------------------------------------------------------------- dedup semantics

def test_dedup_kappa_and_order(oracle_lib):
    # hand-made records: three rays share key (0,0,1,(4,)), one differs
    res = {
        "n_rec": 5,
        "rec_sel": np.array([0, 1, 2, 3, 1]), "rec_g": np.array([10, 11, 12, 13, 11]),
        "rec_tx": np.array([0, 0, 0, 0, 0]), "rec_rx": np.array([0, 0, 0, 0, 1]),
        "rec_b": np.array([1, 1, 1, 1, 1]),
        "rec_lpoly": np.array([5.0, 4.0, 4.0, 6.0, 9.0]), "rec_lunf": np.array([5.0, 4.0, 4.0, 6.0, 9.0]),
        "rec_flags": np.array([1, 1, 1, 1, 1]),
        "seq": np.array([[4], [4], [4], [2]]),
    }
    paths, keys, _ = oracle_lib.dedup(res, 1, kappa=2)
    assert keys == [(0, 0, 1, (2,)), (0, 0, 1, (4,)), (0, 1, 1, (4,))]
    p = paths[(0, 0, 1, (4,))]
    assert p["count"] == 3
    assert [row[2] for row in p["rows"]] == [11, 12]        # equal L_poly: smaller ray id first
    paths, keys, _ = oracle_lib.dedup(res, 1, kappa=1)
    assert [row[2] for row in paths[(0, 0, 1, (4,))]["rows"]] == [11]


def test_parity_sets_contain_exact_answer(oracle_lib):
    s = scenes.random_scene(2, tilt_sigma=0.05, pos_sigma=0.01, n_rays=300)
    d = oracle_lib.fibonacci(s.n_rays)
    r = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, d, K=3, r_s=s.surfel_radius, t_eps=1e-5,
                          parity=True, err_abs=1e-6, err_dir=1e-6)
    traced = r["hit_id"] > -2
    for ray, b in zip(*np.nonzero(traced)):
        n = r["acc_n"][ray, b]
        assert n >= 1
        acc = r["acc_id"][ray, b, :min(n, 16)]
        assert r["hit_id"][ray, b] in acc
    # the bands are narrow: most segments have a single admissible answer
    assert np.mean(r["acc_n"][traced] == 1) > 0.8


def test_acceptable_set_beyond_the_stored_array(oracle_lib):
    """A ray that grazes a row of 200 coplanar surfels at |d.n| = 1e-9: every surfel lies at the
    same t and inside the projected error band, so every one of them, and "no hit" (no clear hit
    exists), is acceptable: 201 members, more than the stored array holds.  oracle.accepts decides
    the members that were not stored."""
    n = 200
    xyz = np.zeros((n, 3), np.float32)
    xyz[:, 0] = 0.1 * np.arange(n, dtype=np.float32)
    nrm = np.tile(np.array([0, 0, 1], np.float32), (n, 1))
    lab = np.zeros(n, np.uint32)
    d = np.array([[1.0, 0.0, -1e-9]], np.float32)
    tx = np.array([[-1.0, 0.0, 1e-8]], np.float32)
    r = oracle_lib.launch(xyz, nrm, lab, tx, np.zeros((0, 3), np.float32), d, K=0, r_s=0.075, t_eps=1e-5,
                          parity=True, err_abs=1e-6, err_dir=1e-6)
    assert r["acc_n"][0, 0] == n + 1
    assert r["acc_id"][0, 0, 0] == -1
    assert all(oracle_lib.accepts(r, 0, 0, m) for m in range(-1, n))
    # a steep ray over the same row: one clear hit, nothing else acceptable
    d2 = np.array([[0.6, 0.0, -0.8]], np.float32)
    tx2 = np.array([[5.0, 0.0, 4.0]], np.float32)        # hits x = 8, the centre of surfel 80
    r2 = oracle_lib.launch(xyz, nrm, lab, tx2, np.zeros((0, 3), np.float32), d2, K=0, r_s=0.075, t_eps=1e-5,
                           parity=True, err_abs=1e-6, err_dir=1e-6)
    assert r2["hit_id"][0, 0] == 80 and r2["acc_n"][0, 0] == 1
    assert [m for m in range(-1, n) if oracle_lib.accepts(r2, 0, 0, m)] == [80]


def test_accepts_equals_the_stored_sets(oracle_lib):
    """Where a set fits the array, oracle.accepts agrees with it for every point and for "no hit"."""
    s = scenes.random_scene(5, tilt_sigma=0.0, pos_sigma=0.0, n_rays=60)
    d = oracle_lib.fibonacci(s.n_rays)
    r = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, d, K=2, r_s=s.surfel_radius, t_eps=1e-4,
                          parity=True, err_abs=1e-5, err_dir=1e-5)
    checked = 0
    for ray, b in zip(*np.nonzero(r["hit_id"] > -2)):
        na = int(r["acc_n"][ray, b])
        if na > oracle_lib.MAXACC:
            continue
        stored = set(int(x) for x in r["acc_id"][ray, b, :na])
        got = {m for m in range(-1, s.n_points) if oracle_lib.accepts(r, ray, b, m)}
        assert got == stored, (ray, b)
        checked += 1
    assert checked > 50


# --------------------------------------------------------------------------- acceleration exactness

def _axis_and_diagonal_dirs():
    d = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (1, -1, 0), (0, 1, 1), (1, 0, -1), (1, 1, 1), (-1, 1, -1), (1e-9, 1, 0), (1, 1e-12, 1e-12)]
    d = np.asarray(d, np.float64)
    return (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("cell_over_rs", [0.3, 1.0, 2.5])
def test_grid_dda_equals_brute_force(oracle_lib, seed, cell_over_rs):
    # the acceleration logic (every point listed in each cell its disk can be hit
    # in, cells in ray order, stop once the best hit precedes the cell's exit)
    # must reproduce the brute force bit for bit: same hit ids, same distances
    s = scenes.random_scene(seed, n_rays=2000, n_rx=3, pos_sigma=0.01, tilt_sigma=0.05)
    r_s = float(np.float32(s.surfel_radius))
    t_eps = 1e-4
    grid = oracle_lib.Grid(s.xyz, r_s, cell_over_rs * r_s)
    for dirs in (oracle_lib.fibonacci(s.n_rays), _axis_and_diagonal_dirs()):
        a = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, dirs, 3, r_s, t_eps)
        b = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, dirs, 3, r_s, t_eps, grid=grid)
        assert np.array_equal(a["hit_id"], b["hit_id"])
        assert np.array_equal(a["hit_t"], b["hit_t"], equal_nan=True)
        assert a["n_rec"] == b["n_rec"] and np.array_equal(a["rec_lpoly"], b["rec_lpoly"])


def test_grid_dda_on_the_box_room(box_run, oracle_lib):
    # axis-aligned walls on cell boundaries (0.25 m cells, walls at 0, 3, 8, 10 m)
    s, d, r = box_run
    grid = oracle_lib.Grid(s.xyz, s.surfel_radius, 0.25)
    g = oracle_lib.launch(s.xyz, s.normal, s.label, s.tx, s.rx, d, K=2, r_s=s.surfel_radius, t_eps=_box_t_eps(),
                          grid=grid)
    assert np.array_equal(r["hit_id"], g["hit_id"])
    assert np.array_equal(r["hit_t"], g["hit_t"], equal_nan=True)
