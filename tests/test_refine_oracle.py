"""Pins of the oracle's path refinement (Section 2.3, Eq. 2) and refined-path dedup.

The refinement is pinned against closed forms that do not use the oracle's
own arithmetic:
  * the image method: in the empty box room every coarse path refines to the
    image-source path of its reflection sequence, whose squared lengths are
    the fixtures of tests/golden/box_room_image_paths.txt, and the dedup
    leaves exactly those 25 sequences;
  * a single tilted plane: the exact reflection point is where the line from
    the mirrored TX to the RX crosses the plane;
  * outcomes that geometry decides: a straight crossing of a free plate is
    not a reflection, a plate over the last segment blocks it, a specular
    point off a finite plate makes the re-traced ray miss.
The dedup is pinned on hand-made paths with the first Fresnel zone radius
sqrt(lambda d1 d2 / (d1 + d2)) worked out by hand at 60 GHz.

Diffraction points (D_k = c_k + t_k w_k on an edge) are pinned at the
corner building's vertical edge at (0, 0): TX and RX lie sqrt(34) from the
edge on either side, so unfolding the two half-planes about the edge makes
the diffracted path a straight line of horizontal extent 2 sqrt(34); with a
ground reflection the RX is mirrored in z = 0 first.  The outcomes a point
off the finite edge, a neighbour inside the wedge and a segment through the
ground are decided by the geometry.  A face surfel tilted across the
segments leaving the diffraction point, within r_s of it, changes nothing
(rays leave a diffraction point r_s along).

Each of these mistakes planted in the oracle's diffraction code fails one of
the pins: the step along the edge with the wrong sign, no clearance for
segments arriving at a diffraction point, the wedge test's "or" made "and",
and no clearance for rays leaving it (in the iteration or in the final
check).
"""
import math
import os

import numpy as np
import pytest

import oracle
import scenes
from oracle import image_method

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "box_room_image_paths.txt")):
        if line.startswith("#"):
            continue
        name, l2 = line.split()
        seq = () if name == "-" else tuple(int(x) for x in name.split(","))
        out[seq] = float(l2)
    return out


def _scene(faces, h):
    xyz, nrm, lab = scenes._sample_faces(faces, h)
    return xyz.astype(np.float32), nrm.astype(np.float32), lab.astype(np.uint32)


def _refine_one(xyz, nrm, lab, r_s, tx, rx, pts, **kw):
    pts = np.asarray(pts, np.float64).reshape(1, -1, 3)
    n_refl = np.array([pts.shape[1]], np.int32)
    return oracle.refine(xyz, nrm, lab, r_s, 1e-5, np.asarray(tx, np.float64)[None], np.asarray(rx, np.float64)[None],
                         n_refl, pts, **kw)


@pytest.fixture(scope="module")
def box_refined():
    s = scenes.box_room()
    K = 2
    t_eps = 1e-5 * math.sqrt(10 ** 2 + 8 ** 2 + 3 ** 2)
    res = oracle.launch(s.xyz, s.normal, s.label, s.tx, s.rx, oracle.fibonacci(s.n_rays), K, s.surfel_radius, t_eps)
    paths, keys, _ = oracle.dedup(res, K, kappa=5)
    rows = [(key, r) for key in keys for r in paths[key]["rows"]]
    n = len(rows)
    pts = np.full((n, K, 3), np.nan)
    for i, (key, r) in enumerate(rows):
        pts[i, :key[2]] = res["pts"][r[3], :key[2]].astype(np.float32)  # the coarse points, as FP32 records hold them
    txp = np.repeat(s.tx.astype(np.float64), n, 0)
    rxp = np.repeat(s.rx.astype(np.float64), n, 0)
    nr = np.array([key[2] for key, _ in rows], np.int32)
    out = oracle.refine(s.xyz, s.normal, s.label, s.surfel_radius, t_eps, txp, rxp, nr, pts, step=0.75)
    return s, rows, nr, txp, out


def test_box_room_refines_to_image_paths(box_refined):
    s, rows, nr, _, out = box_refined
    gold = _golden()
    assert (out["status"] == oracle.REF_VALID).all()
    assert (out["grad"] < oracle.REF_GRAD_TOL).all()
    img = image_method.box_room_paths(s.tx[0], s.rx[0], (10.0, 8.0, 3.0), 2)
    for i, (key, _) in enumerate(rows):
        seq = tuple(int(x) for x in out["labels"][i, :nr[i]])
        assert seq == key[3], (i, seq, key)        # refinement keeps the walls of the coarse path
        L_img = math.sqrt(gold[seq])
        # the image path is the shortest path through its planes: f >= L_img, and at
        # a gradient below 1e-4 the excess is second order (below 1e-7 relative)
        assert L_img * (1 - 1e-12) <= out["length"][i] <= L_img * (1 + 1e-7), (seq, out["length"][i], L_img)
        # the points converge only to within |g| / (smallest tangent curvature of f),
        # a few mm where a segment grazes its wall
        for k, q in enumerate(img[seq][1]):
            assert np.linalg.norm(out["points"][i, k] - q) < 1e-2, (seq, k)


def test_box_room_dedup_leaves_the_image_sequences(box_refined):
    s, rows, nr, txp, out = box_refined
    kept = oracle.refine_dedup(np.zeros(len(rows)), nr, out["labels"], out["points"], out["length"], out["status"],
                               txp)
    got = sorted(tuple(int(x) for x in out["labels"][i, :nr[i]]) for i in np.nonzero(kept)[0])
    assert got == sorted(_golden())
    assert len(got) == 25


def _mirror(p, c, n):
    p = np.asarray(p, np.float64)
    return p - 2.0 * np.dot(p - c, n) * n


def test_tilted_plane_reflection_point():
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    u, v, n = q[:, 0] * 4.0, q[:, 1] * 4.0, q[:, 2]
    c = np.array([1.0, 2.0, 0.5])
    xyz, nrm, lab = _scene([(c - 0.5 * u - 0.5 * v, u, v, n, 7)], 0.05)
    r_s = 0.75 * 0.05
    tx = c + 1.5 * n + 0.4 * q[:, 0]
    rx = c + 1.0 * n - 0.5 * q[:, 1]
    img = _mirror(tx, c, n)
    lam = np.dot(c - img, n) / np.dot(rx - img, n)
    spec = img + lam * (rx - img)
    coarse = spec + 0.3 * q[:, 0] - 0.2 * q[:, 1]     # a point of the plane, 36 cm off
    out = _refine_one(xyz, nrm, lab, r_s, tx, rx, [coarse])
    assert out["status"][0] == oracle.REF_VALID and out["labels"][0, 0] == 7
    L = np.linalg.norm(rx - img)
    # the surfels hold the plane rounded to FP32 (a few 1e-7 m off the exact plane)
    assert abs(out["length"][0] - L) <= 1e-6 * L
    assert np.linalg.norm(out["points"][0, 0] - spec) < 2e-3
    assert 0 < out["iters"][0] < 200


def test_crossing_a_free_plate_is_not_a_reflection():
    # TX above, RX below a horizontal plate: the length is smallest where the
    # straight line crosses the plate, which is a stationary point but no reflection
    xyz, nrm, lab = _scene([((-1.0, -1.0, 0.0), (2.0, 0, 0), (0, 2.0, 0), (0, 0, 1.0), 1)], 0.05)
    out = _refine_one(xyz, nrm, lab, 0.0375, (0.0, 0.0, 1.0), (0.4, 0.2, -1.0), [(0.5, -0.3, 0.0)])
    assert out["status"][0] == oracle.REF_WRONG_SIDE
    assert np.linalg.norm(out["points"][0, 0] - (0.2, 0.1, 0.0)) < 2e-3


def test_plate_over_last_segment_occludes():
    floor = ((-3.0, -3.0, 0.0), (10.0, 0, 0), (0, 6.0, 0), (0, 0, 1.0), 0)
    plate = ((2.8, -0.2, 1.0), (0.4, 0, 0), (0, 0.4, 0), (0, 0, 1.0), 1)   # over (3, 0, 1)
    xyz, nrm, lab = _scene([floor, plate], 0.05)
    tx, rx = (0.0, 0.0, 2.0), (4.0, 0.0, 2.0)
    out = _refine_one(xyz, nrm, lab, 0.0375, tx, rx, [(1.7, 0.3, 0.0)])
    assert out["status"][0] == oracle.REF_OCCLUDED
    assert np.linalg.norm(out["points"][0, 0] - (2.0, 0.0, 0.0)) < 2e-3
    # without the plate the same path is valid, of length |TX' - RX|
    xyz, nrm, lab = _scene([floor], 0.05)
    out = _refine_one(xyz, nrm, lab, 0.0375, tx, rx, [(1.7, 0.3, 0.0)])
    assert out["status"][0] == oracle.REF_VALID
    assert abs(out["length"][0] - math.sqrt(4 ** 2 + 4 ** 2)) < 1e-6


def test_specular_point_off_the_plate_misses():
    xyz, nrm, lab = _scene([((-0.5, -0.5, 0.0), (1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0), 2)], 0.05)
    out = _refine_one(xyz, nrm, lab, 0.0375, (3.0, 0.0, 1.0), (5.0, 0.0, 1.0), [(0.4, 0.0, 0.0)])
    assert out["status"][0] == oracle.REF_MISS
    assert np.isnan(out["length"][0]) and out["ids"][0, 0] == -1


def test_iteration_limit():
    xyz, nrm, lab = _scene([((-3.0, -3.0, 0.0), (6.0, 0, 0), (0, 6.0, 0), (0, 0, 1.0), 0)], 0.05)
    out = _refine_one(xyz, nrm, lab, 0.0375, (0.0, 0.0, 1.0), (2.0, 0.0, 1.0), [(-1.0, 1.0, 0.0)], max_iters=3)
    assert out["status"][0] == oracle.REF_NOT_CONVERGED and out["iters"][0] == 3
    assert out["grad"][0] >= oracle.REF_GRAD_TOL
    full = _refine_one(xyz, nrm, lab, 0.0375, (0.0, 0.0, 1.0), (2.0, 0.0, 1.0), [(-1.0, 1.0, 0.0)])
    assert full["status"][0] == oracle.REF_VALID and full["iters"][0] > 3
    assert np.linalg.norm(full["points"][0, 0] - (1.0, 0.0, 0.0)) < 2e-3


def test_line_of_sight_paths_need_no_iteration():
    xyz, nrm, lab = _scene([((-3.0, -3.0, 0.0), (6.0, 0, 0), (0, 6.0, 0), (0, 0, 1.0), 0)], 0.05)
    out = oracle.refine(xyz, nrm, lab, 0.0375, 1e-5, np.array([[0.0, 0.0, 1.0]]), np.array([[3.0, 4.0, 1.0]]),
                        np.array([0], np.int32), np.zeros((1, 2, 3)))
    assert out["status"][0] == oracle.REF_VALID and out["iters"][0] == 0
    assert out["length"][0] == 5.0 and (out["ids"][0] == -1).all()


def test_smoothing_keeps_the_box_room_image_paths(box_refined):
    # flat walls: the averaged normal is the wall's own wherever the exact points lie
    # (>= 0.35 m from every edge, beyond the 0.24 m radius)
    s, rows, nr, txp, out = box_refined
    t_eps = 1e-5 * math.sqrt(10 ** 2 + 8 ** 2 + 3 ** 2)
    pts = np.full((len(rows), 2, 3), np.nan)
    for i, (key, r) in enumerate(rows):
        pts[i, :key[2]] = out["points"][i, :key[2]]
    sm = oracle.refine(s.xyz, s.normal, s.label, s.surfel_radius, t_eps, txp, np.repeat(s.rx.astype(np.float64),
                       len(rows), 0), nr, pts, smooth_radius=0.24)
    gold = _golden()
    assert (sm["status"] == oracle.REF_VALID).all()
    for i in range(len(rows)):
        seq = tuple(int(x) for x in sm["labels"][i, :nr[i]])
        L = math.sqrt(gold[seq])
        assert L * (1 - 1e-12) <= sm["length"][i] <= L * (1 + 1e-7)


def test_smoothing_finds_the_specular_point_of_a_noisy_plane():
    # a plane sampled exactly, normals tilted by N(0, 0.02 rad): with each surfel's
    # own normal the refinement stops wherever a surfel's tilted mirror condition
    # holds (centimetres off); the averaged normal recovers the plane's specular point
    h = 0.05
    xyz, nrm, lab = scenes._sample_faces([((-3.0, -3.0, 0.0), (6.0, 0, 0), (0, 6.0, 0), (0, 0, 1.0), 0)], h)
    rng = np.random.default_rng(3)
    _, nrm = scenes._jitter(rng, xyz, nrm, 0.0, 0.02)
    xyz, nrm, lab = xyz.astype(np.float32), nrm.astype(np.float32), lab.astype(np.uint32)
    tx, rx = np.array([0.0, 0.0, 1.0]), np.array([2.0, 0.5, 1.5])
    img = np.array([0.0, 0.0, -1.0])
    spec = img + (rx - img) / 2.5
    starts = spec + rng.uniform(-0.3, 0.3, size=(40, 3)) * [1, 1, 0]
    n = len(starts)
    args = (xyz, nrm, lab, 0.75 * h, 1e-5, np.tile(tx, (n, 1)), np.tile(rx, (n, 1)), np.ones(n, np.int32),
            starts[:, None, :])
    own = oracle.refine(*args)
    avg = oracle.refine(*args, smooth_radius=0.09)
    assert (own["status"] == oracle.REF_VALID).all() and (avg["status"] == oracle.REF_VALID).all()
    assert np.linalg.norm(own["points"][:, 0] - spec, axis=1).max() > 0.01
    assert np.linalg.norm(avg["points"][:, 0] - spec, axis=1).max() < 0.005
    # the disks are tilted, so a hit lies up to r_s * 0.02 off the plane
    L = np.linalg.norm(rx - img)
    assert np.abs(avg["length"] - L).max() < 1e-3 * L


# ---------------------------------------------------------------------------
# dedup of refined paths
# ---------------------------------------------------------------------------

LAM = oracle.LIGHT_SPEED / 60e9   # 4.9965 mm


def _one_bounce_paths(points, lengths, labels, groups=None):
    n = len(points)
    pts = np.asarray(points, np.float64).reshape(n, 1, 3)
    tx = np.tile([0.0, 0.0, 3.0], (n, 1))
    return dict(group=np.zeros(n) if groups is None else np.asarray(groups), n_refl=np.ones(n, np.int32),
                labels=np.asarray(labels).reshape(n, 1), points=pts, length=np.asarray(lengths, np.float64),
                status=np.zeros(n, np.int32), tx=tx)


def _dedup(d, carrier_hz=oracle.CARRIER_HZ):
    return oracle.refine_dedup(d["group"], d["n_refl"], d["labels"], d["points"], d["length"], d["status"], d["tx"],
                               carrier_hz=carrier_hz)


def test_fresnel_radius_by_hand():
    # lambda = c / 60 GHz; at d1 = d2 = 3 m the first zone has radius sqrt(lambda * 1.5)
    assert abs(LAM - 0.0049965409) < 1e-9
    assert abs(oracle.fresnel_radius(3.0, 3.0, LAM) - 0.0865726) < 1e-6


def test_shortest_per_label_sequence():
    # same labels, points far apart (no Fresnel overlap): only the shorter stays
    d = _one_bounce_paths([(0, 0, 0), (2, 0, 0)], [6.2, 6.0], [4, 4])
    assert _dedup(d).tolist() == [False, True]
    d = _one_bounce_paths([(0, 0, 0), (2, 0, 0)], [6.2, 6.0], [4, 5])
    assert _dedup(d).tolist() == [True, True]


def test_fresnel_zone_merges_nearby_paths():
    # TX (0,0,3), point (0,0,0), path length 6: d1 = 3, d2 = 3, radius 8.657 cm
    d = _one_bounce_paths([(0, 0, 0), (0.05, 0, 0)], [6.0, 6.001], [1, 2])
    assert _dedup(d).tolist() == [True, False]
    d = _one_bounce_paths([(0, 0, 0), (0.09, 0, 0)], [6.0, 6.001], [1, 2])
    assert _dedup(d).tolist() == [True, True]
    assert _dedup(_one_bounce_paths([(0, 0, 0), (0.05, 0, 0)], [6.0, 6.001], [1, 2]), carrier_hz=-1).tolist() == \
        [True, True]
    # other (TX, RX) pairs never merge
    d = _one_bounce_paths([(0, 0, 0), (0.05, 0, 0)], [6.0, 6.001], [1, 2], groups=[0, 1])
    assert _dedup(d).tolist() == [True, True]


def test_fresnel_sweep_is_greedy_in_length_order():
    # b lies in a's zone, c in b's but not in a's: b goes, c stays (only kept paths absorb)
    d = _one_bounce_paths([(0, 0, 0), (0.06, 0, 0), (0.12, 0, 0)], [6.0, 6.001, 6.002], [1, 2, 3])
    assert _dedup(d).tolist() == [True, False, True]


def test_invalid_paths_never_kept():
    d = _one_bounce_paths([(0, 0, 0), (2, 0, 0)], [6.0, 6.1], [1, 2])
    d["status"][0] = oracle.REF_NOT_CONVERGED
    assert _dedup(d).tolist() == [False, True]


# --------------------------------------------------------------------------- diffraction (Section 2.3)

def _corner(tx, rx, pts, edge_of):
    s = scenes.corner_building(tx=tx, rx=rx)
    pts = np.asarray(pts, np.float64).reshape(1, -1, 3)
    eo = np.asarray(edge_of, np.int32).reshape(1, -1)
    return oracle.refine(s.xyz, s.normal, s.label, s.surfel_radius, 1e-5, np.asarray(tx, np.float64)[None],
                         np.asarray(rx, np.float64)[None], np.array([pts.shape[1]], np.int32), pts,
                         edges=s.extra["edges"], edge_of=eo)


def _keller(a, d, b, w):
    """cosines of the incoming and outgoing directions with the edge"""
    u, v = (d - a) / np.linalg.norm(d - a), (b - d) / np.linalg.norm(b - d)
    return float(u @ w), float(v @ w)


@pytest.mark.parametrize("z_tx,z_rx", [(1.5, 1.5), (1.0, 2.0), (0.5, 3.5)])
def test_corner_diffraction_point(z_tx, z_rx):
    """Unfolded about the edge the path is straight: length sqrt((2 sqrt 34)^2 + dz^2), the point at the
    height where the straight line crosses the edge, Keller's law at it."""
    tx, rx = np.array([-3.0, 5.0, z_tx]), np.array([5.0, -3.0, z_rx])
    r = _corner(tx, rx, [(0.0, 0.0, 2.9)], [0])
    L = math.sqrt(136.0 + (z_rx - z_tx) ** 2)
    assert r["status"][0] == oracle.REF_VALID
    assert L <= r["length"][0] <= L * (1 + 1e-8)
    d = r["points"][0, 0]
    assert abs(d[2] - 0.5 * (z_tx + z_rx)) <= 1e-3 and abs(d[0]) + abs(d[1]) == 0.0
    ci, co = _keller(tx, d, rx, np.array([0.0, 0.0, 1.0]))
    assert abs(ci - co) <= 1e-4
    assert r["labels"][0, 0] == 100 and r["ids"][0, 0] == -2


@pytest.mark.parametrize("case", ["to the RX", "to a ground reflection"])
def test_rays_leave_a_diffraction_point_clear_of_its_faces(case):
    """A face surfel at the corner edge tilted by 30 degrees (normal (0.5, -0.866, 0), centre 5 cm
    along the face y = 0, at the diffraction point's height) meets the segment leaving the
    diffraction point about 3 cm from it, inside the disk.  A ray leaving a diffraction point starts
    r_s = 7.5 cm along, so the path keeps its status and points: the last segment to the RX, or the
    re-trace towards the ground reflection that follows the diffraction (the closed forms of the
    tests around this one)."""
    if case == "to the RX":
        tx, rx = np.array([-3.0, 5.0, 1.5]), np.array([5.0, -3.0, 1.5])
        D, nxt = np.array([0.0, 0.0, 1.5]), rx
        pts, eo, L = np.array([[[0.0, 0.0, 2.9]]]), np.array([[0]], np.int32), 2.0 * math.sqrt(34.0)
    else:
        tx, rx = np.array([-3.0, 5.0, 3.0]), np.array([5.0, -3.0, 1.5])
        D, nxt = np.array([0.0, 0.0, 0.75]), np.array([5.0 / 3.0, -1.0, 0.0])
        pts, eo, L = np.array([[[0.0, 0.0, 1.0], [1.5, -1.2, 0.0]]]), np.array([[0, -1]], np.int32), 12.5
    s = scenes.corner_building(tx=tx, rx=rx)
    u = np.array([0.5, -math.sqrt(0.75), 0.0])
    c = np.array([0.05, 0.0, D[2]])
    d = (nxt - D) / np.linalg.norm(nxt - D)
    t = float(u @ (c - D)) / float(u @ d)         # where the leaving ray meets the tilted disk
    assert 1e-3 < t < 0.75 * s.surfel_radius and np.linalg.norm(D + t * d - c) < 0.5 * s.surfel_radius
    xyz = np.vstack([s.xyz, c[None]]).astype(np.float32)
    nrm = np.vstack([s.normal, u[None]]).astype(np.float32)
    lab = np.concatenate([s.label, np.array([4], s.label.dtype)])
    args = (s.surfel_radius, 1e-5, tx[None], rx[None], np.array([pts.shape[1]], np.int32), pts)
    plain = oracle.refine(s.xyz, s.normal, s.label, *args, edges=s.extra["edges"], edge_of=eo)
    tilted = oracle.refine(xyz, nrm, lab, *args, edges=s.extra["edges"], edge_of=eo)
    assert plain["status"][0] == tilted["status"][0] == oracle.REF_VALID
    assert L <= tilted["length"][0] <= L * (1 + 1e-7)
    assert np.array_equal(plain["points"], tilted["points"])


def test_corner_diffraction_then_ground_reflection():
    """TX at 3 m, RX at 1.5 m: mirrored in the ground the RX is at -1.5 m; the straight unfolded line
    has horizontal extent 2 sqrt(34) and drop 4.5: length 12.5, crossing the edge at 0.75 m and the
    ground a third of the way from the edge to the RX, at (5/3, -1, 0)."""
    tx, rx = np.array([-3.0, 5.0, 3.0]), np.array([5.0, -3.0, 1.5])
    r = _corner(tx, rx, [(0.0, 0.0, 1.0), (1.5, -1.2, 0.0)], [0, -1])
    assert r["status"][0] == oracle.REF_VALID
    assert 12.5 <= r["length"][0] <= 12.5 * (1 + 1e-7)
    assert abs(r["points"][0, 0, 2] - 0.75) <= 2e-3
    assert np.abs(r["points"][0, 1] - np.array([5.0 / 3.0, -1.0, 0.0])).max() <= 5e-3
    assert list(r["labels"][0]) == [100, 0]
    ci, co = _keller(tx, r["points"][0, 0], r["points"][0, 1], np.array([0.0, 0.0, 1.0]))
    assert abs(ci - co) <= 1e-4


def test_diffraction_point_off_the_edge():
    """TX and RX at 8 m: the stationary point (8 m) lies above the 4 m edge."""
    r = _corner((-3.0, 5.0, 8.0), (5.0, -3.0, 8.0), [(0.0, 0.0, 3.0)], [0])
    assert r["status"][0] == oracle.REF_OFF_EDGE


def test_diffraction_neighbour_inside_the_wedge():
    """An RX inside the building: the stationary point exists, but the path enters the wedge."""
    r = _corner((-3.0, 5.0, 1.5), (3.0, 3.0, 1.5), [(0.0, 0.0, 1.0)], [0])
    assert r["status"][0] == oracle.REF_WRONG_SIDE


@pytest.mark.parametrize("tx_z,rx_z", [(1.5, -1.0), (-1.0, 1.5)])
def test_diffraction_segment_through_the_ground(tx_z, rx_z):
    """An antenna 1 m below the ground: the stationary point is at 0.25 m and the segment to the
    buried antenna crosses the ground's surfels (the last segment, or one arriving at the edge)."""
    r = _corner((-3.0, 5.0, tx_z), (5.0, -3.0, rx_z), [(0.0, 0.0, 1.0)], [0])
    assert r["status"][0] == oracle.REF_OCCLUDED
    assert abs(r["points"][0, 0, 2] - 0.25) <= 1e-3
