"""Pins of the cone-tracer oracle (oracle/cone.py) against closed forms.

* SplitMix64: the published first output for state 0 (the generator's
  reference value);
* IEs of the empty box room: the count per wall from the sampling grid and
  the subvoxel grid (integer arithmetic by hand), reception points on the
  wall planes, normals equal to the wall normals;
* cone-sphere distances in the four regimes (inside, lateral, apex, behind);
* block margins of a segment against voxel blocks;
* transmission phase in the convex empty room: every IE and the RX are
  visible from the TX (a convex room hides nothing);
* propagation in the box room: the line-of-sight path has length |TX - RX|,
  every single reflection of the image method is found with a polyline no
  shorter than the image path, no partial path interacts twice with one
  planar wall in a row (the separation plane), with two reflections the
  25 image-method label sequences are all found, and similar partial paths
  are merged (one certain node per TX, labels and IE in every generation);
* transmission behind a partition wall: IEs whose sight line crosses the
  wall's rectangle are hidden, the TX's convex half is all visible;
* diffraction: Keller's law and the sector partition, the sector count
  N = ceil(pi sin(beta) / theta) (each sector 360 / N degrees wide between its
  planes) and the exterior sectors of a 90 degree wedge counted by hand, every
  diffraction child of the corner building inside one of its node's kept
  sectors, edge pieces tiling their edges, edges inert at a diffraction limit
  of 0, and the corner diffraction's closed form 2 sqrt(34).

Each of these mistakes planted in the oracle fails one of the pins: the
sector count rounded down, a sector plane's sign, the exterior test's "or"
made "and", the cone-sphere distance with sine and cosine swapped, the
reflected separation plane's sign, a SplitMix64 constant, the Keller cone
reversed along the edge, a sector's upper plane left out of the target
test, the visibility ray's box exit taken for its entry, hits counted up to
the target point, the slab test without its swap, an IE's reception point
taken as its first point, subvoxels by rounding, and no merge.
"""
import math

import numpy as np
import pytest

import scenes
from oracle import cone, image_method

ORIGIN = np.array([-0.55, -0.45, -0.6], np.float32)
VOXEL, DV, DIMS = 0.5, 2, (23, 19, 9)


def test_splitmix64_reference_value():
    # first output of SplitMix64 seeded with 0
    assert cone.splitmix64(0) == 0xE220A8397B1DCDAF


def _wall_counts():
    """Subvoxels holding points, per wall, by hand: points sit at cell centres
    0.1, 0.3, ... of a 0.2 m grid; subvoxels are 0.25 m from the origin."""
    sv = 0.25

    def cells(lo, n, o):     # subvoxel indices of n points lo, lo + 0.2, ...
        return len({int(math.floor((lo + 0.2 * k - o) / sv)) for k in range(n)})
    x, y, z = cells(0.1, 50, -0.55), cells(0.1, 40, -0.45), cells(0.1, 15, -0.6)
    return {0: x * y, 1: x * y, 2: y * z, 3: y * z, 4: x * z, 5: x * z}


def test_box_room_ies_closed_form():
    s = scenes.box_room()
    ies = cone.ie_build(s.xyz, s.normal, s.label, ORIGIN, VOXEL, DV, DIMS)
    want = _wall_counts()
    got = {lab: int(np.sum(ies["label"] == lab)) for lab in range(6)}
    assert got == want
    assert int(ies["count"].sum()) == s.n_points
    planes = {0: (2, 0.0), 1: (2, 3.0), 2: (0, 0.0), 3: (0, 10.0), 4: (1, 0.0), 5: (1, 8.0)}
    for lab, (ax, c) in planes.items():
        m = ies["label"] == lab
        assert np.allclose(ies["pos"][m][:, ax], c, atol=1e-6)
        n = np.zeros(3)
        n[ax] = 1.0
        assert np.allclose(np.abs(ies["nrm"][m] @ n), 1.0, atol=1e-12)
    assert np.all(np.diff(ies["key"]) > 0)


def test_cone_sphere_regimes():
    o = np.zeros(3)
    d = np.array([1.0, 0.0, 0.0])
    t = math.radians(10.0)
    ct, st = math.cos(t), math.sin(t)
    # on the axis: inside, distance 0
    assert cone.cone_sphere_margin(o, d, ct, st, np.array([5.0, 0, 0]), 0.1) == pytest.approx(0.1)
    # lateral: centre at (5, h): distance to the surface line h cos t - 5 sin t
    h = 2.0
    assert cone.cone_sphere_margin(o, d, ct, st, np.array([5.0, h, 0]), 0.3) == pytest.approx(
        0.3 - (h * ct - 5.0 * st))
    # behind the apex, off axis: nearest point is the apex
    c = np.array([-1.0, 0.5, 0.0])
    assert cone.cone_sphere_margin(o, d, ct, st, c, 0.2) == pytest.approx(0.2 - math.hypot(1.0, 0.5))
    # beside the apex within the polar region boundary: a cos t + rho sin t = 0 -> apex distance
    rho = 1.0
    a = -rho * st / ct
    c = np.array([a, rho, 0.0])
    assert cone.cone_sphere_margin(o, d, ct, st, c, 0.0) == pytest.approx(-math.hypot(a, rho), rel=1e-9)


def test_block_margins():
    o = np.array([0.25, 0.25, 0.25])
    d = np.array([1.0, 0.0, 0.0])
    cells = np.array([[0, 0, 0], [5, 0, 0], [3, 2, 0], [3, 3, 0]])
    m = cone.block_margins(o, d, 2.0, cells, np.zeros(3), 0.5)
    # block of (0,0,0) is [-0.5, 1.0)^3: the segment covers x in [0.25, 1.0] -> 0.75
    assert m[0] == pytest.approx(0.75)
    # (5,0,0): block x in [2.0, 3.5): the segment ends at 2.25 -> overlap 0.25
    assert m[1] == pytest.approx(0.25)
    # (3,2,0): block y in [0.5, 2.0): the ray at y = 0.25 misses by 0.25
    assert m[2] == pytest.approx(-0.25)
    assert m[3] == pytest.approx(-0.75)


@pytest.fixture(scope="module")
def room_k1():
    s = scenes.box_room()
    ies = cone.ie_build(s.xyz, s.normal, s.label, ORIGIN, VOXEL, DV, DIMS)
    sc = cone.Scene(s.xyz, s.normal, s.label, s.surfel_radius, 1e-4)
    res = cone.trace(sc, ies, s.tx, s.rx, ORIGIN, VOXEL, DV, DIMS, K=1, kappa=0, half_angle=math.radians(2.5))
    return s, ies, res


def test_transmission_sees_every_ie_in_a_convex_room(room_k1):
    s, ies, res = room_k1
    assert len(res["nodes"][0]) == len(ies["label"])
    los = [r for r in res["records"] if r["chain"] == ()]
    assert len(los) == 1
    assert los[0]["length"] == pytest.approx(math.sqrt(34.0), rel=1e-12)


def test_single_reflections_and_separation_plane(room_k1):
    s, ies, res = room_k1
    img = image_method.box_room_paths(s.tx[0].astype(float), s.rx[0].astype(float), max_reflections=1)
    found = {k[3]: g for k, g in res["paths"].items()}
    for seq, (L, _) in img.items():
        assert seq in found, seq
        if seq:
            for r in found[seq]["rows"]:
                assert r["length"] >= L * (1 - 1e-12)        # a polyline via the wall is no shorter
                assert r["length"] <= L * 1.01
    for r in res["records"]:
        labs = r["labels"]
        assert all(a != b for a, b in zip(labs, labs[1:]))


@pytest.mark.timeout(600)
def test_two_reflections_find_the_image_sequences():
    s = scenes.box_room()
    ies = cone.ie_build(s.xyz, s.normal, s.label, ORIGIN, VOXEL, DV, DIMS)
    sc = cone.Scene(s.xyz, s.normal, s.label, s.surfel_radius, 1e-4)
    res = cone.trace(sc, ies, s.tx, s.rx, ORIGIN, VOXEL, DV, DIMS, K=2, kappa=100, half_angle=math.radians(2.5))
    img = image_method.box_room_paths(s.tx[0].astype(float), s.rx[0].astype(float), max_reflections=2)
    found = {k[3] for k in res["paths"]}
    assert set(img) <= found, sorted(set(img) - found)
    for k, g in res["paths"].items():
        assert len(g["rows"]) <= 100 and g["count"] >= len(g["rows"])
        labs = k[3]
        assert all(a != b for a, b in zip(labs, labs[1:]))
    # similar partial paths (same TX, labels in the same order, same IE) are merged into one:
    # every generation holds at most one certain node per (TX, labels, IE), and the second
    # generation reaches IEs through several first-generation nodes of one wall
    for gen in res["nodes"]:
        sure = [(c["tx"], c["labels"], c["chain"][-1]) for c in gen if c["exact"] and not c["excused"]]
        assert len(sure) == len(set(sure))
    reached = {}
    for c in res["nodes"][1]:
        reached.setdefault((c["labels"], c["chain"][-1]), set()).add(c["chain"][0])
    assert max(len(v) for v in reached.values()) == 1      # the kept node of each group only


# --------------------------------------------------------------------------- diffraction (Section 2.2.4)

def test_keller_sectors_law_and_exterior():
    """Every diffracted axis keeps the incoming angle with the edge (Keller's
    law), only axes that leave the wedge are kept, and the sectors' planes
    give every exterior target exactly one sector."""
    rng = np.random.default_rng(1)
    w = np.array([0.0, 0.0, 1.0])
    n1, n2 = np.array([-1.0, 0.0, 0.0]), np.array([0.0, -1.0, 0.0])   # the solid is x > 0, y > 0
    o = np.array([0.0, 0.0, 1.0])
    for _ in range(20):
        prev = np.array([-rng.uniform(1, 5), rng.uniform(-5, 5), rng.uniform(-2, 4)])
        din = (o - prev) / np.linalg.norm(o - prev)
        secs, _ = cone.keller_sectors(o, prev, w, n1, n2, math.radians(2.5))
        assert secs
        for axis, n_lo, n_hi, ext in secs:
            assert abs(float(axis @ w) - float(din @ w)) <= 1e-12
            v = axis - float(axis @ w) * w
            assert float(v @ n1) >= -1e-12 or float(v @ n2) >= -1e-12
        for _ in range(50):
            ang = rng.uniform(0, 2 * math.pi)
            p = o + np.array([math.cos(ang), math.sin(ang), rng.uniform(-1, 1)]) * rng.uniform(0.5, 5)
            inside = [float((p - o) @ a) >= 0 and float((p - o) @ b) < 0 for _, a, b, _ in secs]
            exterior = math.cos(ang) < 0 or math.sin(ang) < 0
            assert sum(inside) <= 1
            # directions well inside the exterior quadrants sit in some kept sector
            if math.cos(ang) < -0.1 or math.sin(ang) < -0.1:
                assert sum(inside) == 1
            if not exterior:
                assert sum(inside) == 0 or min(abs(math.cos(ang)), abs(math.sin(ang))) < 0.05


def test_edge_ies_cover_the_edges():
    """Edge IEs: the pieces of every edge tile it (midpoints on the edge, one piece per subvoxel crossed)."""
    s = scenes.corner_building()
    E = s.extra["edges"]
    origin = np.array([-10.292, -10.292, -0.292], np.float32)
    eies = cone.edge_ies(E["seg"], E["normals"], E["label"], origin, 0.4, 2, (53, 53, 13))
    for j in range(len(E["seg"])):
        m = eies["edge"] == j
        a, b = E["seg"][j].astype(np.float64)
        # an axis-aligned edge has one piece per subvoxel layer it spans along its axis
        ax = int(np.argmax(np.abs(b - a)))
        u = (np.array([a[ax], b[ax]]) - float(origin[ax])) / 0.2
        assert int(m.sum()) == int(math.floor(u.max()) - math.floor(u.min()) + 1)
        d = (b - a) / np.linalg.norm(b - a)
        r = eies["pos"][m] - a
        assert np.allclose(r - (r @ d)[:, None] * d, 0.0, atol=1e-5)
        assert len({tuple(x) for x in eies["sub"][m]}) == int(m.sum())
    assert np.all(np.diff(eies["key"]) >= 0)


@pytest.mark.timeout(600)
def test_corner_diffraction_closed_form():
    """The RX behind the building's corner: no line of sight, no reflection;
    with one diffraction the only coarse path goes through the vertical edge at
    (0, 0), no shorter than the exact diffraction path 2 sqrt(34) (equal heights:
    the diffraction point is at z = 1.5) and within a subvoxel of it."""
    s = scenes.corner_building()
    E = s.extra["edges"]
    origin = np.array([-10.292, -10.292, -0.292], np.float32)
    dims = (53, 53, 13)
    ies = cone.ie_build(s.xyz, s.normal, s.label, origin, 0.4, 2, dims)
    eies = cone.edge_ies(E["seg"], E["normals"], E["label"], origin, 0.4, 2, dims)
    sc = cone.Scene(s.xyz, s.normal, s.label, s.surfel_radius, s.t_eps_value)
    L_star = 2.0 * math.sqrt(34.0)
    res = cone.trace(sc, ies, s.tx, s.rx, origin, 0.4, 2, dims, K=1, kappa=100, half_angle=math.radians(2.5),
                     edges=eies, max_diff=1)
    assert set(res["paths"]) == {(0, 0, 1, (100,))}
    for r in res["paths"][(0, 0, 1, (100,))]["rows"]:
        assert L_star * (1 - 1e-12) <= r["length"] <= L_star + 0.01
        e = r["chain"][0] - len(ies["label"])
        assert abs(eies["pos"][e][2] - 1.5) <= 0.2
    res0 = cone.trace(sc, ies, s.tx, s.rx, origin, 0.4, 2, dims, K=1, kappa=100, half_angle=math.radians(2.5),
                      edges=eies, max_diff=0)
    assert not res0["paths"]


def test_edges_are_inert_without_diffraction():
    """With a diffraction limit of 0 the edge pieces are never targets: the
    partial paths, their priorities and the receptions equal those of the
    table without edges (point IEs keep their indices ahead of the pieces)."""
    s = scenes.corner_building(tx=(-3.0, 5.0, 1.5), rx=(-2.0, -3.0, 1.5))
    E = s.extra["edges"]
    origin = np.array([-10.292, -10.292, -0.292], np.float32)
    dims = (53, 53, 13)
    ies = cone.ie_build(s.xyz, s.normal, s.label, origin, 0.4, 2, dims)
    eies = cone.edge_ies(E["seg"], E["normals"], E["label"], origin, 0.4, 2, dims)
    sc = cone.Scene(s.xyz, s.normal, s.label, s.surfel_radius, s.t_eps_value)
    kw = dict(K=1, kappa=100, half_angle=math.radians(2.5))
    a = cone.trace(sc, ies, s.tx, s.rx, origin, 0.4, 2, dims, **kw)
    b = cone.trace(sc, ies, s.tx, s.rx, origin, 0.4, 2, dims, edges=eies, max_diff=0, **kw)
    key = lambda c: (c["tx"], c["chain"], c["prio"], round(c["length"], 12))  # noqa: E731
    assert [key(c) for c in a["nodes"][0]] == [key(c) for c in b["nodes"][0]]
    rec = lambda r: (r["tx"], r["rx"], r["chain"], r["labels"], round(r["length"], 12))  # noqa: E731
    assert sorted(map(rec, a["records"])) == sorted(map(rec, b["records"]))
    assert a["records"], "the RX in front of the building is reached"


def test_keller_sector_count_closed_form():
    """Incidence perpendicular to the edge (beta = 90 degrees) with a 2.5 degree
    half-angle: N = ceil(pi sin(beta) / theta) = 72 sectors of 5 degrees; a 90 degree
    convex wedge leaves 270 degrees of exterior, which hold the centres of 54 of
    them.  At beta = 41 degrees N = ceil(47.24) = 48 (no sector centre on a face),
    of which the centres in the exterior are counted directly; along the edge N = 1."""
    w = np.array([0.0, 0.0, 1.0])
    n1, n2 = np.array([-1.0, 0.0, 0.0]), np.array([0.0, -1.0, 0.0])
    o = np.zeros(3)
    th = math.radians(2.5)
    secs, _ = cone.keller_sectors(o, np.array([-4.0, 1.0, 0.0]), w, n1, n2, th)
    assert len(secs) == 54
    for axis, n_lo, n_hi, _ in secs:
        assert abs(axis[2]) < 1e-12                      # Keller: the cone degenerates to the plane
        # a sector spans 360 / N degrees between its planes (pins N itself)
        assert math.degrees(math.acos(float(np.clip(n_lo @ n_hi, -1, 1)))) == pytest.approx(5.0, abs=1e-9)
    # beta = 41 degrees: the incoming direction makes 41 degrees with the edge; the sector
    # centres (k + 1/2) 360 / N degrees from the first face's normal lie outside the wedge
    # when in [0, 180] or [270, 360] (cos >= 0 against face 1, sin >= 0 against face 2)
    b = math.radians(41.0)
    prev = -np.array([math.sin(b), 0.0, math.cos(b)])
    N = math.ceil(math.pi * math.sin(b) / th)
    assert N == 48
    ext = sum(1 for k in range(N) if (k + 0.5) * 360.0 / N <= 180.0 or (k + 0.5) * 360.0 / N >= 270.0)
    secs, _ = cone.keller_sectors(o, prev, w, n1, n2, th)
    assert len(secs) == ext
    for axis, n_lo, n_hi, _ in secs:
        assert axis[2] == pytest.approx(math.cos(b), abs=1e-12)
        assert math.degrees(math.acos(float(np.clip(n_lo @ n_hi, -1, 1)))) == pytest.approx(7.5, abs=1e-9)
    secs, _ = cone.keller_sectors(o, np.array([0.0, 0.0, -3.0]), w, n1, n2, th)
    assert len(secs) == 1 and secs[0][1] is None


def test_diffraction_children_lie_in_kept_sectors():
    """Corner building, two interactions, one diffraction: every certain child
    of a node at an edge piece lies between the two separation planes of one
    of the exterior sectors that node casts (Keller sectors of the incoming
    direction from the TX).  A sector is cast whole, so a child may lie up to
    half a sector inside the wedge; none lies beyond the kept sectors."""
    s = scenes.corner_building()
    E = s.extra["edges"]
    origin = np.array([-10.292, -10.292, -0.292], np.float32)
    dims = (53, 53, 13)
    ies = cone.ie_build(s.xyz, s.normal, s.label, origin, 0.4, 2, dims)
    eies = cone.edge_ies(E["seg"], E["normals"], E["label"], origin, 0.4, 2, dims)
    sc = cone.Scene(s.xyz, s.normal, s.label, s.surfel_radius, s.t_eps_value)
    th = math.radians(2.5)
    res = cone.trace(sc, ies, s.tx, s.rx, origin, 0.4, 2, dims, K=2, kappa=100, half_angle=th, edges=eies,
                     max_diff=1)
    npt = len(ies["label"])

    def pos(i):
        return np.asarray(ies["pos"][i] if i < npt else eies["pos"][i - npt], np.float64)

    tx = np.asarray(s.tx[0], np.float64)
    n_children = 0
    for c in res["nodes"][1]:
        a, b = c["chain"]
        if a < npt or not c["exact"] or c["excused"]:
            continue
        e = int(eies["edge"][a - npt])
        seg = np.asarray(E["seg"][e], np.float64)
        w = (seg[1] - seg[0]) / np.linalg.norm(seg[1] - seg[0])
        secs, _ = cone.keller_sectors(pos(a), tx, w, np.asarray(E["normals"][e][0], np.float64),
                                      np.asarray(E["normals"][e][1], np.float64), th)
        v = pos(b) - pos(a)
        assert any(lo is None or (v @ lo >= 0 and v @ hi < 0) for _, lo, hi, _ in secs), (a, b)
        n_children += 1
    assert n_children > 10_000


def test_transmission_behind_a_partition():
    """Transmission phase in a non-convex room: the box room with a partition
    wall in the plane x = 5 (y in [0, 6], full height; a 2 m gap at y > 6).  From
    the TX at (2, 3, 1.5), an IE whose segment from the TX crosses the wall's
    rectangle at least 0.3 m inside its border is hidden; every IE with x < 4.7
    (the convex half of the room the TX stands in) is visible."""
    s = scenes.box_room()
    wall = [(np.array([5.0, 0.0, 0.0]), np.array([0.0, 6.0, 0.0]), np.array([0.0, 0.0, 3.0]),
             np.array([-1.0, 0.0, 0.0]), 6)]
    wx, wn, wl = scenes._sample_faces(wall, 0.2)
    xyz = np.vstack([s.xyz, wx.astype(np.float32)]).astype(np.float32)
    nrm = np.vstack([s.normal, wn.astype(np.float32)]).astype(np.float32)
    lab = np.concatenate([s.label, wl.astype(np.uint32)]).astype(np.uint32)
    tx = np.array([[2.0, 3.0, 1.5]], np.float32)
    ies = cone.ie_build(xyz, nrm, lab, ORIGIN, VOXEL, DV, DIMS)
    sc = cone.Scene(xyz, nrm, lab, s.surfel_radius, 1e-4)
    res = cone.trace(sc, ies, tx, np.zeros((0, 3), np.float32), ORIGIN, VOXEL, DV, DIMS, K=1, kappa=0,
                     half_angle=math.radians(2.5))
    seen = {c["chain"][0] for c in res["nodes"][0]}
    t = tx[0].astype(np.float64)
    hidden, front = [], []
    for e, p in enumerate(ies["pos"]):
        if p[0] < 4.7:
            front.append(e)
        if p[0] > 5.3:
            u = (5.0 - t[0]) / (p[0] - t[0])
            q = t + u * (p - t)
            if 0.3 <= q[1] <= 5.7 and 0.3 <= q[2] <= 2.7:
                hidden.append(e)
    assert len(hidden) > 100 and len(front) > 1000
    assert not (set(hidden) & seen)
    assert set(front) <= seen
