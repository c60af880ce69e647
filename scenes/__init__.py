"""Seeded synthetic inputs: labeled point clouds, antenna positions and query streams.

This module is the single source of input data for both the CPU oracle and the
HIP path.  It holds no part of the ray-launching arithmetic (no ray directions,
no intersection, no reception radius): it only samples surfaces into points
with a position, a unit normal and a label, which is the input format of the
method (Section 2: every point carries at least a position, a normal vector and
a label; labels stand for segmented surfaces).

Every generator is deterministic for a given seed (``numpy.random.default_rng``)
and returns float32 positions/normals and uint32 labels, the layout the C ABI
takes.  Surfaces are sampled at the centres of a regular grid on each face with
``ceil(side / h)`` cells per side, so the spacing never exceeds ``h``.

Scenes
------
* ``box_room``        empty 10 x 8 x 3 m room, 20 cm grid, 6 labels, no noise
                      (6,700 points exactly)
* ``furnished_room``  12 x 10 x 3 m room with 30 axis-aligned boxes, position
                      noise N(0, 2 mm), normal tilt N(0, 0.02 rad), 20 labels
* ``street_canyon``   400 x 400 m ground with 120 extruded buildings, position
                      noise N(0, 5 mm), 50 labels
* ``random_scene``    tiny random planes/boxes for property tests
* ``batch_scenes``    256 scenes of uneven size (rooms and canyons)
* ``moving_canyon``   canyon with moving vehicle boxes (serving workload)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "box_room", "furnished_room", "street_canyon", "random_scene",
    "batch_scenes", "moving_canyon", "poisson_queries", "face_grid",
]


@dataclass
class Scene:
    """A labeled point cloud plus the antennas and launch settings of a workload."""
    name: str
    xyz: np.ndarray            # [N, 3] float32
    normal: np.ndarray         # [N, 3] float32 (unit up to noise/rounding)
    label: np.ndarray          # [N] uint32
    tx: np.ndarray             # [n_tx, 3] float32
    rx: np.ndarray             # [n_rx, 3] float32
    spacing: float             # sampling step h of the face grids (m)
    surfel_radius: float       # r_s used for this scene (m)
    levels: tuple              # voxel level edge lengths, coarse -> fine (m)
    n_rays: int                # rays per TX
    max_reflections: int       # K
    t_eps: float = 0.0         # self-intersection distance (<= 0: library default)
    extra: dict = field(default_factory=dict)

    @property
    def n_points(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def t_eps_value(self) -> float:
        """The self-intersection distance a launch on this scene uses: the
        scene's own, else 1e-5 x the diagonal of the points' bounding box."""
        if self.t_eps > 0:
            return float(self.t_eps)
        if self.xyz.size == 0:
            return 1e-6
        lo, hi = self.xyz.min(0).astype(np.float64), self.xyz.max(0).astype(np.float64)
        return max(1e-5 * math.sqrt(float(((hi - lo) ** 2).sum())), 1e-6)


# ----------------------------------------------------------------------------
# face sampling
# ----------------------------------------------------------------------------

def face_grid(corner, u, v, normal, h, label):
    """Sample the rectangle ``corner + a*u + b*v`` (a, b in [0, 1]) at cell centres.

    ``u`` and ``v`` are edge vectors (their lengths are the side lengths).  The
    grid has ``ceil(|u|/h) x ceil(|v|/h)`` cells.  Returns float64 arrays
    (xyz [n,3], normal [n,3]) and a uint32 label array.
    """
    corner = np.asarray(corner, np.float64)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    nu = max(1, int(math.ceil(np.linalg.norm(u) / h - 1e-9)))
    nv = max(1, int(math.ceil(np.linalg.norm(v) / h - 1e-9)))
    a = (np.arange(nu, dtype=np.float64) + 0.5) / nu
    b = (np.arange(nv, dtype=np.float64) + 0.5) / nv
    A, B = np.meshgrid(a, b, indexing="ij")
    pts = corner[None, :] + A.reshape(-1, 1) * u[None, :] + B.reshape(-1, 1) * v[None, :]
    nrm = np.broadcast_to(np.asarray(normal, np.float64), pts.shape).copy()
    lab = np.full(pts.shape[0], label, dtype=np.uint32)
    return pts, nrm, lab


def _face_count(u_len, v_len, h):
    return max(1, int(math.ceil(u_len / h - 1e-9))) * max(1, int(math.ceil(v_len / h - 1e-9)))


def _box_faces(lo, hi, label, inward, bottom=True):
    """Six (or five, without the bottom) faces of an axis-aligned box.

    Returns a list of (corner, u, v, normal, label).  ``inward`` points the
    normals into the box (a room seen from inside) instead of out of it.
    """
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d = hi - lo
    s = -1.0 if inward else 1.0
    ex, ey, ez = np.eye(3)
    faces = []
    if bottom:
        faces.append((lo, ex * d[0], ey * d[1], -s * ez, label[0]))            # z = lo
    faces.append((np.array([lo[0], lo[1], hi[2]]), ex * d[0], ey * d[1], s * ez, label[1]))  # z = hi
    faces.append((lo, ey * d[1], ez * d[2], -s * ex, label[2]))                # x = lo
    faces.append((np.array([hi[0], lo[1], lo[2]]), ey * d[1], ez * d[2], s * ex, label[3]))  # x = hi
    faces.append((lo, ex * d[0], ez * d[2], -s * ey, label[4]))                # y = lo
    faces.append((np.array([lo[0], hi[1], lo[2]]), ex * d[0], ez * d[2], s * ey, label[5]))  # y = hi
    return faces


def _sample_faces(faces, h):
    xs, ns, ls = [], [], []
    for corner, u, v, n, lab in faces:
        p, q, l = face_grid(corner, u, v, n, h, lab)
        xs.append(p)
        ns.append(q)
        ls.append(l)
    if not xs:
        return (np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, np.uint32))
    return np.concatenate(xs), np.concatenate(ns), np.concatenate(ls)


def _area_count(faces, h):
    return sum(_face_count(np.linalg.norm(u), np.linalg.norm(v), h) for _, u, v, _, _ in faces)


def _spacing_for(faces_fn, n_target):
    """Largest grid step h whose face sampling gives at least ``n_target`` points."""
    faces = faces_fn()
    area = sum(np.linalg.norm(np.cross(u, v)) for _, u, v, _, _ in faces)
    h = math.sqrt(area / max(n_target, 1))
    # ceil() per side adds points; shrink h slightly only if we fell short
    for _ in range(50):
        if _area_count(faces, h) >= n_target:
            break
        h *= 0.995
    return h


def _jitter(rng, xyz, nrm, pos_sigma, tilt_sigma):
    if pos_sigma > 0:
        xyz = xyz + rng.normal(0.0, pos_sigma, size=xyz.shape)
    if tilt_sigma > 0:
        # two tangent directions per normal, then a small rotation about each
        helper = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
        t1 = np.cross(nrm, helper)
        t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
        t2 = np.cross(nrm, t1)
        a = rng.normal(0.0, tilt_sigma, size=(nrm.shape[0], 1))
        b = rng.normal(0.0, tilt_sigma, size=(nrm.shape[0], 1))
        nrm = nrm + np.tan(a) * t1 + np.tan(b) * t2
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return xyz, nrm


def _pack(name, xyz, nrm, lab, tx, rx, h, levels, n_rays, K, rs_factor=0.75, t_eps=0.0, **extra):
    return Scene(
        name=name,
        xyz=np.ascontiguousarray(xyz, dtype=np.float32),
        normal=np.ascontiguousarray(nrm, dtype=np.float32),
        label=np.ascontiguousarray(lab, dtype=np.uint32),
        tx=np.ascontiguousarray(np.asarray(tx, np.float64).reshape(-1, 3), dtype=np.float32),
        rx=np.ascontiguousarray(np.asarray(rx, np.float64).reshape(-1, 3), dtype=np.float32),
        spacing=float(h),
        surfel_radius=float(rs_factor * h),
        levels=tuple(float(x) for x in levels),
        n_rays=int(n_rays),
        max_reflections=int(K),
        t_eps=float(t_eps),
        extra=dict(extra),
    )


# ----------------------------------------------------------------------------
# C1: empty box room
# ----------------------------------------------------------------------------

BOX_ROOM_LABELS = {"floor": 0, "ceiling": 1, "x0": 2, "x10": 3, "y0": 4, "y8": 5}


def box_room(h=0.2, size=(10.0, 8.0, 3.0), tx=(2.0, 2.0, 1.5), rx=(7.0, 5.0, 1.5),
             n_rays=10_000, K=2, levels=(0.5, 0.25)):
    """Empty axis-aligned room [0,10]x[0,8]x[0,3] with inward unit normals.

    Labels: 0 floor (z=0), 1 ceiling (z=3), 2 wall x=0, 3 wall x=10,
    4 wall y=0, 5 wall y=8.  At h = 0.2 m this gives exactly 6,700 points.
    Levels (0.5, 0.25) read Table 1's voxel size 0.5 with division factor 2.
    """
    faces = _box_faces((0, 0, 0), size, label=(0, 1, 2, 3, 4, 5), inward=True)
    xyz, nrm, lab = _sample_faces(faces, h)
    return _pack("box_room", xyz, nrm, lab, tx, rx, h, levels, n_rays, K)


# ----------------------------------------------------------------------------
# C2: furnished room
# ----------------------------------------------------------------------------

def _room_boxes(rng, size, n_boxes, lo=0.3, hi=2.0):
    boxes = []
    for _ in range(n_boxes):
        d = rng.uniform(lo, hi, size=3)
        d[2] = min(d[2], size[2] - 0.05)
        x0 = rng.uniform(0.0, size[0] - d[0])
        y0 = rng.uniform(0.0, size[1] - d[1])
        boxes.append((np.array([x0, y0, 0.0]), np.array([x0 + d[0], y0 + d[1], d[2]])))
    return boxes


def _furnished_faces(size, boxes):
    faces = _box_faces((0, 0, 0), size, label=(0, 1, 2, 3, 4, 5), inward=True)
    for b, (lo, hi) in enumerate(boxes):
        lab = 6 + (b % 14)
        faces += _box_faces(lo, hi, label=(lab,) * 6, inward=False, bottom=False)
    return faces


def _free_point(rng, size, boxes, margin, zlo, zhi):
    for _ in range(100_000):
        p = np.array([rng.uniform(margin, size[0] - margin),
                      rng.uniform(margin, size[1] - margin),
                      rng.uniform(zlo, zhi)])
        ok = True
        for lo, hi in boxes:
            if np.all(p >= lo - margin) and np.all(p <= hi + margin):
                ok = False
                break
        if ok:
            return p
    raise RuntimeError("no free point found")


def furnished_room(n_points=1_000_000, seed=0, antenna_seed=1, n_rx=16, n_rays=1_000_000, K=3,
                   levels=(0.5, 0.05), n_boxes=30, size=(12.0, 10.0, 3.0), h=None,
                   pos_sigma=0.002, tilt_sigma=0.02):
    """Room 12x10x3 m plus ``n_boxes`` random axis-aligned boxes standing on the floor.

    Box sides are U[0.3, 2] m, overlaps allowed, bottom faces not sampled.
    The grid step is derived from the point budget (``h = sqrt(area / N)``)
    unless ``h`` is given.  Labels: room faces 0..5, box b -> 6 + (b mod 14).
    One TX and ``n_rx`` RX lie in free space (0.3 m from walls and boxes,
    z in [0.5, 2.5]).
    """
    rng = np.random.default_rng(seed)
    boxes = _room_boxes(rng, size, n_boxes)
    if h is None:
        h = _spacing_for(lambda: _furnished_faces(size, boxes), n_points)
    xyz, nrm, lab = _sample_faces(_furnished_faces(size, boxes), h)
    xyz, nrm = _jitter(rng, xyz, nrm, pos_sigma, tilt_sigma)
    arng = np.random.default_rng(antenna_seed)
    tx = _free_point(arng, size, boxes, 0.3, 0.5, 2.5)
    rx = np.stack([_free_point(arng, size, boxes, 0.3, 0.5, 2.5) for _ in range(n_rx)])
    rs = 0.75 * h
    return _pack("furnished_room", xyz, nrm, lab, tx, rx, h, levels, n_rays, K,
                 t_eps=rs, boxes=boxes, size=size)


# ----------------------------------------------------------------------------
# C3: street canyon
# ----------------------------------------------------------------------------

def _canyon_buildings(rng, extent, lots, side=(10.0, 30.0), height=(8.0, 40.0)):
    lx = extent[0] / lots[0]
    ly = extent[1] / lots[1]
    blds = []
    for i in range(lots[0]):
        for j in range(lots[1]):
            sx = min(rng.uniform(*side), lx - 2.0)
            sy = min(rng.uniform(*side), ly - 2.0)
            hz = rng.uniform(*height)
            cx = (i + 0.5) * lx
            cy = (j + 0.5) * ly
            blds.append((np.array([cx - sx / 2, cy - sy / 2, 0.0]), np.array([cx + sx / 2, cy + sy / 2, hz])))
    return blds


def _canyon_faces(extent, blds, n_labels):
    faces = []
    for b, (lo, hi) in enumerate(blds):
        lab = 1 + (b % (n_labels - 1))
        faces += _box_faces(lo, hi, label=(lab,) * 6, inward=False, bottom=False)
    return faces


def _ground(extent, blds, h, lots=None):
    """Ground grid minus building footprints.

    With ``lots`` (one building per lot, inside its lot, in lot-major order)
    each point is tested against its own lot's footprint only; the result is
    the same as testing every footprint.
    """
    p, n, l = face_grid((0, 0, 0), (extent[0], 0, 0), (0, extent[1], 0), (0, 0, 1), h, 0)
    if lots is None:
        keep = np.ones(p.shape[0], bool)
        for lo, hi in blds:
            keep &= ~((p[:, 0] > lo[0]) & (p[:, 0] < hi[0]) & (p[:, 1] > lo[1]) & (p[:, 1] < hi[1]))
        return p[keep], n[keep], l[keep]
    lx = extent[0] / lots[0]
    ly = extent[1] / lots[1]
    i = np.minimum((p[:, 0] / lx).astype(np.int64), lots[0] - 1)
    j = np.minimum((p[:, 1] / ly).astype(np.int64), lots[1] - 1)
    lo = np.array([b[0] for b in blds])
    hi = np.array([b[1] for b in blds])
    k = i * lots[1] + j
    inside = (p[:, 0] > lo[k, 0]) & (p[:, 0] < hi[k, 0]) & (p[:, 1] > lo[k, 1]) & (p[:, 1] < hi[k, 1])
    keep = ~inside
    return p[keep], n[keep], l[keep]


def _street_point(rng, extent, blds, margin, z):
    for _ in range(100_000):
        p = np.array([rng.uniform(margin, extent[0] - margin), rng.uniform(margin, extent[1] - margin), z])
        if all(not (lo[0] - margin < p[0] < hi[0] + margin and lo[1] - margin < p[1] < hi[1] + margin)
               for lo, hi in blds):
            return p
    raise RuntimeError("no street point found")


def street_canyon(n_points=20_000_000, seed=0, antenna_seed=1, n_tx=4, n_rx=64, n_rays=4_000_000, K=4,
                  levels=(8.0, 1.0, 0.1), extent=(400.0, 400.0), lots=(12, 10), n_labels=50,
                  scale=1.0, h=None, pos_sigma=0.005):
    """Ground plane plus extruded-box buildings on a lot grid (facades and roofs sampled).

    Footprint sides U[10, 30] m (capped to leave a 2 m street), heights
    U[8, 40] m, all multiplied by ``scale``.  Labels: ground 0, building b ->
    1 + (b mod 49).  TX at z = 10 m and RX at z = 1.5 m (times ``scale``) lie in
    streets at least 2 m from any footprint.
    """
    rng = np.random.default_rng(seed)
    extent = (extent[0] * scale, extent[1] * scale)
    blds = _canyon_buildings(rng, extent, lots, side=(10.0 * scale, 30.0 * scale),
                             height=(8.0 * scale, 40.0 * scale))
    ground_area = extent[0] * extent[1] - sum((hi[0] - lo[0]) * (hi[1] - lo[1]) for lo, hi in blds)
    if h is None:
        faces = _canyon_faces(extent, blds, n_labels)
        area = ground_area + sum(np.linalg.norm(np.cross(u, v)) for _, u, v, _, _ in faces)
        h = math.sqrt(area / max(n_points, 1))
    g = _ground(extent, blds, h, lots)
    b = _sample_faces(_canyon_faces(extent, blds, n_labels), h)
    xyz = np.concatenate([g[0], b[0]])
    nrm = np.concatenate([g[1], b[1]])
    lab = np.concatenate([g[2], b[2]])
    xyz, nrm = _jitter(rng, xyz, nrm, pos_sigma, 0.0)
    arng = np.random.default_rng(antenna_seed)
    margin = 2.0 * scale
    tx = np.stack([_street_point(arng, extent, blds, margin, 10.0 * scale) for _ in range(n_tx)])
    rx = np.stack([_street_point(arng, extent, blds, margin, 1.5 * scale) for _ in range(n_rx)])
    rs = 0.75 * h
    return _pack("street_canyon", xyz, nrm, lab, tx, rx, h, levels, n_rays, K,
                 t_eps=rs, buildings=blds, extent=extent)


# ----------------------------------------------------------------------------
# tiny random scenes for property tests
# ----------------------------------------------------------------------------

def box_edges(lo, hi, label, top=True, vertical=True):
    """Convex edges of an axis-aligned box standing on the ground: the four
    vertical edges and the four roof edges (its bottom edges meet the ground
    and are not convex).  Returns segments [n, 2, 3], the outward normals of
    the two faces meeting at each edge [n, 2, 3] and labels [n] (label, label
    + 1, ...)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    seg, nrm = [], []
    if vertical:
        for x, nx in ((lo[0], -1.0), (hi[0], 1.0)):
            for y, ny in ((lo[1], -1.0), (hi[1], 1.0)):
                seg.append(((x, y, lo[2]), (x, y, hi[2])))
                nrm.append(((nx, 0.0, 0.0), (0.0, ny, 0.0)))
    if top:
        z = hi[2]
        for y, ny in ((lo[1], -1.0), (hi[1], 1.0)):
            seg.append(((lo[0], y, z), (hi[0], y, z)))
            nrm.append(((0.0, ny, 0.0), (0.0, 0.0, 1.0)))
        for x, nx in ((lo[0], -1.0), (hi[0], 1.0)):
            seg.append(((x, lo[1], z), (x, hi[1], z)))
            nrm.append(((nx, 0.0, 0.0), (0.0, 0.0, 1.0)))
    n = len(seg)
    return (np.asarray(seg, np.float32).reshape(n, 2, 3), np.asarray(nrm, np.float32).reshape(n, 2, 3),
            (label + np.arange(n)).astype(np.uint32))


def corner_building(h=0.1, tx=(-3.0, 5.0, 1.5), rx=(5.0, -3.0, 1.5), n_rays=20_000, K=2, levels=(0.4, 0.2, 0.1),
                    ground=10.0):
    """A ground of 2 ``ground`` x 2 ``ground`` m (label 0) and one building [0,6] x [0,6] x [0,4]
    (roof 1, faces x=0: 2, x=6: 3, y=0: 4, y=6: 5; outward normals) with its
    eight convex edges (labels 100..107) in ``extra['edges']``.  The default RX
    lies in the building's shadow seen from the TX: no line of sight and no
    reflection reaches it; the vertical edge at (0, 0) diffracts towards it."""
    faces = [(np.array([-ground, -ground, 0.0]), np.array([2 * ground, 0.0, 0.0]), np.array([0.0, 2 * ground, 0.0]),
              np.array([0.0, 0.0, 1.0]), 0)]
    faces += _box_faces((0.0, 0.0, 0.0), (6.0, 6.0, 4.0), label=(0, 1, 2, 3, 4, 5), inward=False, bottom=False)
    xyz, nrm, lab = _sample_faces(faces, h)
    # ground points under the building are not sampled
    keep = ~((lab == 0) & (xyz[:, 0] > 0) & (xyz[:, 0] < 6) & (xyz[:, 1] > 0) & (xyz[:, 1] < 6))
    seg, enrm, elab = box_edges((0.0, 0.0, 0.0), (6.0, 6.0, 4.0), 100)
    return _pack("corner_building", xyz[keep], nrm[keep], lab[keep], tx, rx, h, levels, n_rays, K,
                 edges=dict(seg=seg, normals=enrm, label=elab))


def random_scene(seed, n_planes=4, n_boxes=2, extent=4.0, h=0.25, n_rays=512, n_tx=1, n_rx=3, K=3,
                 pos_sigma=0.0, tilt_sigma=0.0, levels=None):
    """A few random rectangles and boxes inside a cube of side ``extent``.

    Rectangles have random orientation (not axis-aligned), so surfel disks
    straddle leaf borders in every direction.  Used at 10^2 - 10^4 points.
    """
    rng = np.random.default_rng(seed)
    faces = []
    lab = 0
    for _ in range(n_planes):
        c = rng.uniform(0.1 * extent, 0.9 * extent, size=3)
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        a, b = rng.uniform(0.3 * extent, 0.8 * extent, size=2)
        u = q[:, 0] * a
        v = q[:, 1] * b
        faces.append((c - 0.5 * u - 0.5 * v, u, v, q[:, 2], lab))
        lab += 1
    for _ in range(n_boxes):
        lo = rng.uniform(0.1 * extent, 0.6 * extent, size=3)
        hi = lo + rng.uniform(0.1 * extent, 0.35 * extent, size=3)
        faces += _box_faces(lo, hi, label=(lab,) * 6, inward=False)
        lab += 1
    xyz, nrm, labs = _sample_faces(faces, h)
    xyz, nrm = _jitter(rng, xyz, nrm, pos_sigma, tilt_sigma)
    tx = rng.uniform(0.0, extent, size=(n_tx, 3))
    rx = rng.uniform(0.0, extent, size=(n_rx, 3))
    if levels is None:
        levels = (4 * h, 2 * h, h)
    return _pack(f"random_{seed}", xyz, nrm, labs, tx, rx, h, levels, n_rays, K)


# ----------------------------------------------------------------------------
# C4: batch of uneven scenes
# ----------------------------------------------------------------------------

def batch_scenes(n_scenes=256, seeds=None, n_min=50_000, n_max=2_000_000, rays_min=65_536,
                 rays_max=1_000_000, K=3, max_rx=32, point_scale=1.0, ray_scale=1.0):
    """Scenes of uneven size: seed s is a furnished room if even, a canyon if odd.

    Point counts are log-uniform in [n_min, n_max]; rooms take their grid
    step from the count, canyons keep the street-canyon density and scale
    their extent by sqrt(N / 20M).  Each scene gets one TX, U{1..32} RX and a
    ray count log-uniform in [64k, 1M] rounded to a multiple of 256.
    ``point_scale`` / ``ray_scale`` shrink the workload for tests.
    """
    seeds = list(range(n_scenes)) if seeds is None else list(seeds)
    out = []
    for s in seeds:
        rng = np.random.default_rng(10_000 + s)
        n = int(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) * point_scale)
        n = max(n, 2_000)
        rays = int(math.exp(rng.uniform(math.log(rays_min), math.log(rays_max))) * ray_scale)
        rays = max(256, (rays // 256) * 256)
        n_rx = int(rng.integers(1, max_rx + 1))
        if s % 2 == 0:
            sc = furnished_room(n_points=n, seed=s, antenna_seed=100_000 + s, n_rx=n_rx, n_rays=rays, K=K)
        else:
            f = math.sqrt(n / 20_000_000)
            sc = street_canyon(n_points=n, seed=s, antenna_seed=100_000 + s, n_tx=1, n_rx=n_rx,
                               n_rays=rays, K=K, scale=f, levels=(8.0 * f, 1.0 * f, 0.1 * f)
                               if f > 0.2 else (max(2.0 * f, 0.4), max(0.5 * f, 0.1), 0.05))
        sc.name = f"batch_{s}_{sc.name}"
        out.append(sc)
    return out


# ----------------------------------------------------------------------------
# C5: canyon with moving vehicles, and the query stream
# ----------------------------------------------------------------------------

def moving_canyon(n_points=5_000_000, seed=0, moving_fraction=0.05, vehicle=(4.5, 1.8, 1.5),
                  extent=(200.0, 200.0), lots=(6, 5), speed=(5.0, 15.0), frame_dt=0.1,
                  levels=(8.0, 1.0, 0.1)):
    """Street canyon whose ``moving_fraction`` of points belong to vehicle boxes.

    Returns (scene, mover) where ``mover(frame)`` gives the (indices, xyz, normal)
    of the moving points at that frame: every vehicle drives along its street
    at a fixed speed U[5, 15] m/s and wraps around the scene; frames are
    ``frame_dt`` seconds apart.  Vehicle bottoms are not sampled.
    """
    rng = np.random.default_rng(seed)
    blds = _canyon_buildings(rng, extent, lots)
    ground_area = extent[0] * extent[1] - sum((hi[0] - lo[0]) * (hi[1] - lo[1]) for lo, hi in blds)
    faces = _canyon_faces(extent, blds, 50)
    area = ground_area + sum(np.linalg.norm(np.cross(u, v)) for _, u, v, _, _ in faces)
    static_n = int(n_points * (1.0 - moving_fraction))
    h = math.sqrt(area / static_n)
    g = _ground(extent, blds, h, lots)
    b = _sample_faces(faces, h)
    vx, vy, vz = vehicle
    vfaces = _box_faces((0, 0, 0), (vx, vy, vz), label=(49,) * 6, inward=False, bottom=False)
    per_vehicle = _area_count(vfaces, h)
    n_veh = max(1, int(round(n_points * moving_fraction / per_vehicle)))
    vp, vn, vl = _sample_faces(vfaces, h)
    # streets run along x between lot rows and along y between lot columns
    lx = extent[0] / lots[0]
    ly = extent[1] / lots[1]
    starts, vel = [], []
    for _ in range(n_veh):
        if rng.uniform() < 0.5:
            row = rng.integers(0, lots[1] + 1)
            y = min(max(row * ly, 1.0), extent[1] - 1.0 - vy)
            starts.append([rng.uniform(0, extent[0] - vx), y, 0.0])
            vel.append([rng.uniform(*speed) * rng.choice([-1, 1]), 0.0, 0.0])
        else:
            col = rng.integers(0, lots[0] + 1)
            x = min(max(col * lx, 1.0), extent[0] - 1.0 - vx)
            starts.append([x, rng.uniform(0, extent[1] - vx), 0.0])
            vel.append([0.0, rng.uniform(*speed) * rng.choice([-1, 1]), 0.0])
    starts = np.array(starts)
    vel = np.array(vel)
    xyz_s = np.concatenate([g[0], b[0]])
    nrm_s = np.concatenate([g[1], b[1]])
    lab_s = np.concatenate([g[2], b[2]])
    xyz_s, nrm_s = _jitter(rng, xyz_s, nrm_s, 0.005, 0.0)
    n_static = xyz_s.shape[0]
    nv = vp.shape[0]
    moving_idx = np.arange(n_static, n_static + n_veh * nv, dtype=np.int64)
    span = np.array([extent[0] - vx, extent[1] - vx, 1.0])

    def positions(frame):
        off = starts + vel * (frame * frame_dt)
        off[:, 0] = np.mod(off[:, 0], span[0])
        off[:, 1] = np.mod(off[:, 1], span[1])
        return (off[:, None, :] + vp[None, :, :]).reshape(-1, 3)

    xyz = np.concatenate([xyz_s, positions(0)])
    nrm = np.concatenate([nrm_s, np.tile(vn, (n_veh, 1))])
    lab = np.concatenate([lab_s, np.tile(vl, n_veh)])
    arng = np.random.default_rng(seed + 1)
    tx = _street_point(arng, extent, blds, 2.0, 10.0)
    rx = np.stack([_street_point(arng, extent, blds, 2.0, 1.5) for _ in range(8)])
    sc = _pack("moving_canyon", xyz, nrm, lab, tx, rx, h, levels, 65_536, 3, t_eps=0.75 * h,
               buildings=blds, extent=extent, n_vehicles=n_veh, moving_idx=moving_idx)
    vnrm32 = np.ascontiguousarray(np.tile(vn, (n_veh, 1)), dtype=np.float32)

    def mover(frame):
        return (moving_idx, np.ascontiguousarray(positions(frame), dtype=np.float32), vnrm32)

    return sc, mover


def poisson_queries(seed=1, rate=200.0, duration=30.0, rays=(65_536, 1_000_000), max_rx=8, scene=None,
                    K=3):
    """Poisson arrival stream of TX/RX queries for the serving workload.

    Each query: arrival time (s), a TX in a street at z = 10 m, U{1..max_rx}
    RX at z = 1.5 m and a ray count log-uniform in ``rays`` rounded to 256.
    ``scene`` must carry ``extra['buildings']`` and ``extra['extent']``.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    blds = scene.extra["buildings"]
    extent = scene.extra["extent"]
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        n = int(math.exp(rng.uniform(math.log(rays[0]), math.log(rays[1]))))
        n = max(256, (n // 256) * 256)
        n_rx = int(rng.integers(1, max_rx + 1))
        tx = _street_point(rng, extent, blds, 2.0, 10.0).astype(np.float32)
        rx = np.stack([_street_point(rng, extent, blds, 2.0, 1.5) for _ in range(n_rx)]).astype(np.float32)
        out.append({"t": t, "tx": tx.reshape(1, 3), "rx": rx, "n_rays": n, "K": K})
    return out
