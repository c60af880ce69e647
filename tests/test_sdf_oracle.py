"""Pins of the oracle's intersection with the implicit surface of Eq. 1
(Section 2.2.1) against closed forms, hand-computed marches and invariances.

The cases use flat clouds on exact FP32 grids, where the weighted averages of
Eq. 1 reduce to known planes: f(x) is the signed height above the plane, so
the march, the segment placement and the sign-change rule can be followed by
hand.
"""
import math

import numpy as np
import pytest

import oracle

LEAF = 0.1
ORG = np.array([-1.2, -1.2, -0.55], np.float32)  # the plane z = 0 lies mid-leaf


def plane(spacing=0.02, half=1.0, z=0.0, up=True, offset=0.01):
    g = np.arange(-half + offset, half, spacing)
    X, Y = np.meshgrid(g, g)
    xyz = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], 1).astype(np.float32)
    nrm = np.zeros_like(xyz)
    nrm[:, 2] = 1.0 if up else -1.0
    return xyz, nrm


def run(xyz, nrm, o, d, **kw):
    return oracle.sdf_intersect(xyz, nrm, ORG, LEAF, np.asarray(o, np.float32), np.asarray(d, np.float32), **kw)


def test_plane_from_above_and_below_closed_form():
    """f is the height above the plane: a ray approaching from either side stops
    within eps of it (the march never crosses a plane), normal +z."""
    rng = np.random.default_rng(3)
    xyz, nrm = plane()
    n = 200
    land = rng.uniform(-0.6, 0.6, size=(n, 2))
    d = rng.normal(size=(n, 3))
    d[:, 2] = -np.abs(d[:, 2]) - 0.5
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    side = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)  # odd rays come from below
    d[:, 2] *= side
    h0 = rng.uniform(0.15, 0.45, size=n)
    # place the origin h0 away from the plane along -d so the ray lands at `land`
    t_true = h0 / np.abs(d[:, 2])
    o = np.column_stack([land, np.zeros(n)]) - t_true[:, None] * d
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    r = run(xyz, nrm, o32, d32)
    eps = oracle.SDF_EPS_SCALE * float(np.float32(LEAF))
    o64, d64 = o32.astype(np.float64), d32.astype(np.float64)
    d64 /= np.linalg.norm(d64, axis=1, keepdims=True)
    t_ex = -o64[:, 2] / d64[:, 2]
    assert np.all(np.isfinite(r["t"]))
    # the march approaches from the ray's side: |z| <= eps, t short of the plane
    z = r["point"][:, 2]
    assert np.all(np.abs(z) <= eps + 1e-12)
    assert np.all(np.sign(z) * np.sign(o64[:, 2]) >= 0)
    assert np.all(r["t"] <= t_ex + 1e-12)
    assert np.all(r["t"] >= t_ex - eps / np.abs(d64[:, 2]) - 1e-12)
    np.testing.assert_allclose(r["normal"], np.tile([0.0, 0.0, 1.0], (n, 1)), atol=1e-12)


def test_parallel_and_receding_rays_miss():
    xyz, nrm = plane()
    o = [[-0.5, 0.05, 0.04], [0.1, 0.2, 0.04], [0.0, 0.0, 0.2], [0.0, 0.0, -0.04]]
    d = [[1.0, 0.0, 0.0], [0.3, 0.4, 0.5], [1.0, 0.0, 0.0], [0.1, 0.0, -1.0]]
    r = run(xyz, nrm, o, d)
    assert np.all(np.isinf(r["t"]))
    assert np.all(r["leaf_cell"] == -1)
    assert np.all(np.isnan(r["point"]))


def test_normal_incidence_step_count():
    """A vertical ray meets one occupied leaf; its segment starts half a
    diagonal above the plane (inside h), one step of |f| lands on the plane:
    two evaluations."""
    xyz, nrm = plane()
    o, d = [[0.05, 0.05, 0.3]], [[0.0, 0.0, -1.0]]
    assert np.isinf(run(xyz, nrm, o, d, max_steps=1)["t"][0])
    r = run(xyz, nrm, o, d, max_steps=2)
    oz = float(np.float32(0.3))
    assert r["t"][0] == pytest.approx(oz, abs=1e-12)
    assert abs(r["point"][0, 2]) <= 1e-12
    # h below half a diagonal: the first samples have no point within h and
    # advance by h / 2 (0.0866 -> 0.0616 -> 0.0366, then |f| to the plane)
    h = 0.05
    assert np.isinf(run(xyz, nrm, o, d, max_steps=3, h=h)["t"][0])
    r = run(xyz, nrm, o, d, max_steps=4, h=h)
    assert r["t"][0] == pytest.approx(oz, abs=1e-12)


def test_sign_change_interpolates_between_samples():
    """Normals +z for x < 0 and -z for x > 0: above the plane f = +z while x < 0
    and f = -z once n(x) flips at x = 0.  A slowly rising ray steps by the
    height z, so the two samples around x = 0 have different |f| and the zero
    of their linear interpolation is not their midpoint.  With t_lo the
    samples of the two leaves around x = 0 are fixed by hand; the nearer
    intersection wins."""
    xyz, nrm = plane()
    nrm[xyz[:, 0] > 0, 2] = -1.0
    o32 = np.array([[-0.5, 0.05, 0.01]], np.float32)
    d32 = np.array([[1.0, 0.0, 0.05]], np.float32)
    t_lo = float(np.float32(0.407))
    r = run(xyz, nrm, o32, d32, trange=[[t_lo, np.inf]])
    o = o32[0].astype(np.float64)
    d = d32[0].astype(np.float64)
    d /= np.linalg.norm(d)
    eps = oracle.SDF_EPS_SCALE * float(np.float32(LEAF))
    half = 0.5 * math.sqrt(3.0) * float(np.float32(LEAF))

    def hand(start, end):
        # f = z on the x < 0 side, -z beyond; steps of |f|
        t, prev = start, None
        while t <= end:
            x = o + t * d
            f = x[2] if x[0] < 0 else -x[2]
            if abs(f) <= eps:
                return t
            if prev is not None and (f < 0) != (prev[1] < 0):
                return prev[0] + (t - prev[0]) * prev[1] / (prev[1] - f)
            prev = (t, f)
            t += abs(f)
        return math.inf

    def leaf_segment(cx):
        # box centre of the leaf's own points: (cx, 0.05, 0)
        tc = float(np.dot(np.array([cx, float(np.float32(0.05)), 0.0]) - o, d))
        return max(tc - half, t_lo), tc + half

    f32 = lambda v: float(np.float32(v))  # noqa: E731
    t_a = hand(*leaf_segment(0.5 * (f32(-0.09) + f32(-0.01))))
    t_b = hand(*leaf_segment(0.5 * (f32(0.01) + f32(0.09))))
    t_exp = min(t_a, t_b)
    assert math.isfinite(t_exp)
    assert r["t"][0] == pytest.approx(t_exp, abs=1e-12)
    np.testing.assert_allclose(r["point"][0], o + t_exp * d, atol=1e-12)
    np.testing.assert_allclose(r["normal"][0], [0.0, 0.0, -1.0], atol=1e-12)
    assert abs(r["point"][0, 0]) < 0.04  # within one step (the height, ~0.035) of x = 0


def test_two_planes_nearest_and_ranges():
    xyz1, n1 = plane(z=0.0)
    xyz2, n2 = plane(z=-0.3)
    xyz, nrm = np.vstack([xyz1, xyz2]), np.vstack([n1, n2])
    o, d = [[0.05, 0.05, 0.3]], [[0.0, 0.0, -1.0]]
    eps = oracle.SDF_EPS_SCALE * float(np.float32(LEAF))
    r = run(xyz, nrm, o, d)
    assert -1e-12 <= r["point"][0, 2] <= eps
    # the range ends before the upper plane: no intersection, also when the
    # plane's leaf is entered (at t = 0.25) but the segment is clipped short
    # of the plane (t = 0.3)
    assert np.isinf(run(xyz, nrm, o, d, trange=[[0.0, 0.2]])["t"][0])
    assert np.isinf(run(xyz, nrm, o, d, trange=[[0.0, 0.27]])["t"][0])
    # the range starts below the upper plane: the lower one
    r = run(xyz, nrm, o, d, trange=[[0.35, np.inf]])
    z2 = float(np.float32(-0.3))
    assert z2 - 1e-12 <= r["point"][0, 2] <= z2 + eps


def test_weighted_average_fixed_point():
    """Two half-planes at different heights within h of the ray, the second
    with tilted normals: the surface is the zero of f(z) = (x - p) . n with p
    and n the weighted averages of the definition, found here by bisection
    over a brute-force sum (no cells, leaves or segments); the march stops
    within eps (along n) above it, with n(x) as its normal."""
    xyz1, n1 = plane(z=0.0)
    xyz2, n2 = plane(z=0.02)
    phi = 0.3
    n2[:] = [math.sin(phi), 0.0, math.cos(phi)]
    keep1, keep2 = xyz1[:, 0] < 0, xyz2[:, 0] >= 0
    xyz = np.vstack([xyz1[keep1], xyz2[keep2]])
    nrm = np.vstack([n1[keep1], n2[keep2]]).astype(np.float32)
    x0, y0 = 0.013, 0.047
    o, d = [[x0, y0, 0.3]], [[0.0, 0.0, -1.0]]
    h = oracle.SDF_H_SCALE * float(np.float32(LEAF))
    P = xyz.astype(np.float64)
    N = nrm.astype(np.float64)
    N /= np.linalg.norm(N, axis=1, keepdims=True)

    def f_and_n(z):
        x = np.array([float(np.float32(x0)), float(np.float32(y0)), z])
        d2 = ((P - x) ** 2).sum(1)
        w = np.where(d2 < h * h, (1 - d2 / (h * h)) ** 4, 0.0)
        p = (w[:, None] * P).sum(0) / w.sum()
        n = (w[:, None] * N).sum(0)
        n /= np.linalg.norm(n)
        return float(np.dot(x - p, n)), n

    lo, hi = 0.0, 0.02
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f_and_n(mid)[0] > 0:
            hi = mid
        else:
            lo = mid
    z_star = 0.5 * (lo + hi)
    assert 0.002 < z_star < 0.018  # both half-planes matter
    r = run(xyz, nrm, o, d, max_steps=10_000)
    eps = oracle.SDF_EPS_SCALE * float(np.float32(LEAF))
    z_hit = r["point"][0, 2]
    assert z_star - 1e-9 <= z_hit <= z_star + 2 * eps
    f_hit, n_hit = f_and_n(z_hit)
    assert abs(f_hit) <= eps + 1e-12
    np.testing.assert_allclose(r["normal"][0], n_hit, atol=1e-9)
    assert n_hit[0] > 0.05  # the tilted normals carry weight


def test_origin_leaf_counts():
    """A ray starting inside the plane's leaf finds the plane through that
    leaf's own segment (the leaf the ray starts in is crossed)."""
    xyz, nrm = plane()
    o, d = [[0.05, 0.05, 0.03]], [[0.0, 0.0, -1.0]]
    r = run(xyz, nrm, o, d)
    eps = oracle.SDF_EPS_SCALE * float(np.float32(LEAF))
    assert -1e-12 <= r["point"][0, 2] <= eps
    np.testing.assert_array_equal(r["leaf_cell"][0], [12, 12, 5])


def _dyadic_scene(rng):
    # coordinates on a 1/64 grid and a leaf of 1/8 are exact in FP32, so a
    # translation by whole metres changes no rounding of the leaf assignment
    xyz, nrm = plane(spacing=1 / 64, half=1.0, offset=1 / 128)
    bump = (np.abs(xyz[:, 0] - 0.25) < 0.2) & (np.abs(xyz[:, 1] + 0.1) < 0.3)
    xyz[bump, 2] = 1 / 32
    nrm = nrm + rng.normal(0, 0.05, size=nrm.shape).astype(np.float32)
    o = np.column_stack([np.round(rng.uniform(-0.5, 0.5, (64, 2)) * 1024) / 1024,
                         np.full(64, 0.375)]).astype(np.float32)
    d = np.column_stack([rng.normal(0, 0.4, (64, 2)), -np.ones(64)]).astype(np.float32)
    return xyz, nrm.astype(np.float32), o, d


def test_translation_permutation_and_mirror_invariance():
    rng = np.random.default_rng(11)
    xyz, nrm, o, d = _dyadic_scene(rng)
    org = np.array([-1.25, -1.25, -0.625], np.float32)
    base = oracle.sdf_intersect(xyz, nrm, org, 0.125, o, d)
    assert np.isfinite(base["t"]).sum() > 40
    sh = np.array([2.0, -1.0, 4.0], np.float32)
    tr = oracle.sdf_intersect(xyz + sh, nrm, org + sh, 0.125, o + sh, d)
    np.testing.assert_allclose(tr["t"], base["t"], rtol=0, atol=1e-9)
    np.testing.assert_array_equal(tr["leaf_cell"], base["leaf_cell"])
    perm = rng.permutation(len(xyz))
    pm = oracle.sdf_intersect(xyz[perm], nrm[perm], org, 0.125, o, d)
    np.testing.assert_allclose(pm["t"], base["t"], rtol=0, atol=1e-12)
    # mirror x -> -x: the grid mirrors onto itself when the origin is mirrored
    # to the far corner's image (cells 0..19 on x)
    M = np.array([-1.0, 1.0, 1.0], np.float32)
    org_m = org.copy()
    org_m[0] = -(org[0] + 20 * 0.125)
    mr = oracle.sdf_intersect(xyz * M, nrm * M, org_m, 0.125, o * M, d * M)
    fin = np.isfinite(base["t"])
    np.testing.assert_array_equal(np.isfinite(mr["t"]), fin)
    np.testing.assert_allclose(mr["t"][fin], base["t"][fin], rtol=0, atol=1e-9)


def test_empty_cloud_and_bad_arguments():
    xyz = np.zeros((0, 3), np.float32)
    r = oracle.sdf_intersect(xyz, xyz, ORG, LEAF, [[0, 0, 1]], [[0, 0, -1]])
    assert np.isinf(r["t"][0])
    with pytest.raises(ValueError):
        oracle.sdf_intersect(xyz, xyz, ORG, LEAF, [[0, 0, 1]], [[0, 0, -1]], h=-1.0)


def test_sdf_launch_box_room_paths_are_image_paths():
    """In the empty box room every wall's implicit surface is its plane, so the
    oracle's SDF launch reflects on the walls: each interaction lies within
    eps of a wall plane, and every received label sequence is one of the
    image-method paths of tests/golden/ (line of sight included)."""
    import os
    import scenes
    s = scenes.box_room()
    golden = set()
    here = os.path.dirname(os.path.abspath(__file__))
    for line in open(os.path.join(here, "golden", "box_room_image_paths.txt")):
        if line.startswith("#"):
            continue
        name = line.split()[0]
        golden.add(() if name == "-" else tuple(int(x) for x in name.split(",")))
    org = np.array([-0.5, -0.5, -0.5], np.float32)
    leaf = 0.25
    r = oracle.sdf_launch(s.xyz, s.normal, s.label, org, leaf, s.tx, s.rx, oracle.fibonacci(4000), K=2)
    eps = oracle.SDF_EPS_SCALE * leaf
    got = r["rec_got"] & ~r["rec_band"]
    assert got.sum() > 10
    seqs = set()
    for g, b in zip(r["rec_g"][got], r["rec_b"][got]):
        seqs.add(tuple(int(x) for x in r["label"][g, :b]))
    assert () in seqs and seqs <= golden and len(seqs) >= 4
    # first hits away from the room's edges (where the implicit surface rounds
    # the corner) lie within eps of a wall plane: there f is the height above it
    tx = np.asarray(s.tx[0], np.float64)
    d = oracle.fibonacci(4000).astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p = tx + r["t"][:, 0:1] * d
    planes = np.sort(np.stack([np.abs(p[:, 0]), np.abs(p[:, 0] - 10), np.abs(p[:, 1]), np.abs(p[:, 1] - 8),
                               np.abs(p[:, 2]), np.abs(p[:, 2] - 3)], 1), axis=1)
    face = planes[:, 1] > oracle.SDF_H_SCALE * leaf + 0.1
    assert face.sum() > 3000
    assert np.all(planes[face, 0] <= eps + 1e-9)
