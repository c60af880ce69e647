"""Oracle of the environment-driven coarse tracer (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may use this module.  It is a plain FP64 definition of
what the HIP cone tracer computes and shares no code with it.

The paper's own coarse path tracing, in its order:

* Section 2.1: low-resolution voxels of edge V, each divided into D_v^3
  subvoxels.  An intersectable entity (IE) is the set of points of one label
  whose position lies in one subvoxel; it carries that label, a reception
  point (the mean of its points) and a normal (the normalised mean of their
  unit normals).  Every RX is an IE too: its reception point is the RX
  itself, in the subvoxel that holds it.  ``ie_build``.
* Section 2.2.2, transmission phase: from each TX a ray is cast towards the
  reception point of every IE; a visible RX is a line-of-sight path, a
  visible point IE is a first interaction.  ``visible``.
* Section 2.2.3, propagation phase: from each interaction a reflected
  conical ray (apex at the reception point, axis the mirror image of the
  incoming direction about the IE's normal, constant half-angle) is traced;
  every IE it reaches is the next interaction, up to the interaction limit;
  every RX it reaches ends a coarse path.  At most kappa paths share the same
  labels in the same order.
* Section 2.2.4, voxel cone tracing: the axis is marched through the voxel
  grid; at every voxel the neighbouring voxels are evaluated (the march
  distance only skips voxels with no IE within one voxel, so the evaluated
  voxels are those within Chebyshev distance 1 of a voxel the axis
  crosses); an IE is reached when the cone meets the bounding sphere of its
  subvoxel (the voxel's bounding sphere contains it, so its test adds
  nothing), its reception point lies in front of the separation plane at
  the apex, and a visibility ray from the apex reaches its subvoxel.

Readings where the paper is silent (each listed in the design notes):
  * IE reception point = mean of its points, normal = normalised mean of
    their unit normals; the subvoxel of a point is taken in FP32 as
    floor((p - origin) * (1 / subvoxel)) with FP32 operations (an integer
    decided by floating point, taken in the kernel's precision);
  * visibility: the surfel disks of the launcher (radius r_s, t > t_eps) are
    the geometry; the target is visible iff no disk is hit before the ray
    enters the target's subvoxel;
  * the march of a cone ends at the voxel of the first disk its axis hits
    (beyond it everything is behind that surface), or at the grid's exit;
  * separation plane of a reflected cone: through the apex, with the IE's
    normal turned towards the reflected side as its normal; a target is in
    front iff (p - apex) . n > tau, tau = 1e-3 subvoxel edges (a target on
    the reflecting plane itself is never in front);
  * similar partial paths (Section 2.2.3: the same labels in the same
    order, here also reaching the same IE) are merged: one node is kept,
    the one of smallest priority (SplitMix64 of the parent's priority plus
    the IE index + 1; the TX's priority is SplitMix64(tx)), ties by parent;
    kappa then bounds the rows of each coarse path (TX, RX, labels), chosen
    by the same priority, with the count of all;
  * coarse path length = polyline TX -> reception points -> RX.

Diffraction (Sections 2, 2.2.4 and 3): caller-given convex edges with the
outward normals of their two faces are cut at the subvoxel faces they cross;
each piece is an IE in the subvoxel of its midpoint (reception point the
midpoint, the edge's label).  A node at an edge piece casts the Keller cone
of the directions keeping the incoming angle with the edge, cut into
N = max(1, ceil(pi sin(beta) / half_angle)) sectors measured from the first
face's normal across the edge; a sector is cast when its axis leaves the
wedge (v . n1 >= 0 or v . n2 >= 0), and its two separation planes contain
the edge at its bounding azimuths (a target lies in the sector iff
(p - o) . n_lo >= 0 and (p - o) . n_hi < 0).  A node's own edge is never its
target, and edge pieces are targets only while the path has fewer than
max_diff diffractions.

Parity: every decision that compares floating-point values (cone-sphere,
separation planes, visibility, the candidate block of a voxel, the axis's
first hit, a sector's exterior test, the sector count) is reported with its
margin.  An admission (a conjunction of such tests) is undecided when one
term lies inside the FP32 error band and none is outside it on the false
side; a sector whose exterior margin is inside the band is kept or dropped
by rounding, so its targets are undecided; a sector count within 1e-3 of an
integer step makes every sector's decisions undecided.  A node reached
through an undecided decision is excused together with its subtree, and a
target reached by two cones of one node is one candidate.

Parity unpinned: the cone half-angle, the separation-plane clearance tau,
the merge priorities (SplitMix64 of the parent's priority and the IE) and
the FP32 error band are conventions the paper does not fix; they are pinned
only by the shared definition.  The pins fix the method around them.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (Steele, Lea and Flood, OOPSLA 2014):
    z = x + 0x9E3779B97F4A7C15; then two xor-shift-multiply rounds and a final
    xor-shift (the finaliser of the published generator)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def child_priority(parent_prio: int, ie_index: int) -> int:
    return splitmix64((parent_prio + ie_index + 1) & MASK64)


# --------------------------------------------------------------------------- IEs (Section 2.1)

def subvoxel_of(xyz, origin, voxel, dv):
    """Subvoxel cell of each position, decided in FP32."""
    sv = np.float32(voxel) / np.float32(dv)
    inv = np.float32(1.0) / sv
    rel = np.asarray(xyz, np.float32) - np.asarray(origin, np.float32)[None, :]
    return np.floor(rel * inv).astype(np.int64)


def ie_build(xyz, normal, label, origin, voxel, dv, dims):
    """Point IEs: points grouped by (subvoxel, label), sorted by (voxel, subvoxel within voxel, label).

    Returns a dict of arrays, one entry per IE: ``sub`` [n,3] subvoxel cell,
    ``voxel`` [n] linear voxel index, ``label``, ``count``, ``pos`` [n,3] mean
    position, ``nrm`` [n,3] normalised mean unit normal, ``key`` (the sort key)
    and ``members`` (point indices per IE)."""
    dims = np.asarray(dims, np.int64)
    s = subvoxel_of(xyz, origin, voxel, dv)
    if len(s) and (s.min() < 0 or np.any(s >= dims[None, :] * dv)):
        raise ValueError("points outside the IE grid")
    vox = s // dv
    loc = s - vox * dv
    vlin = vox[:, 0] + dims[0] * (vox[:, 1] + dims[1] * vox[:, 2])
    llin = loc[:, 0] + dv * (loc[:, 1] + dv * loc[:, 2])
    lab = np.asarray(label, np.int64)
    key = ((vlin * dv ** 3 + llin) << 32) | lab
    order = np.argsort(key, kind="stable")
    ks = key[order]
    starts = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]]) if len(ks) else np.zeros(0, np.int64)
    ends = np.r_[starts[1:], len(ks)]
    x64 = np.asarray(xyz, np.float64)
    n64 = np.asarray(normal, np.float64)
    n64 = n64 / np.linalg.norm(n64, axis=1, keepdims=True)
    n_ie = len(starts)
    out = {"key": ks[starts] if n_ie else np.zeros(0, np.int64), "sub": np.zeros((n_ie, 3), np.int64),
           "voxel": np.zeros(n_ie, np.int64), "label": np.zeros(n_ie, np.int64), "count": np.zeros(n_ie, np.int64),
           "pos": np.zeros((n_ie, 3)), "nrm": np.zeros((n_ie, 3)), "members": []}
    for i, (a, b) in enumerate(zip(starts, ends)):
        idx = order[a:b]
        out["sub"][i] = s[idx[0]]
        out["voxel"][i] = vlin[idx[0]]
        out["label"][i] = lab[idx[0]]
        out["count"][i] = b - a
        out["pos"][i] = x64[idx].mean(axis=0)
        m = n64[idx].mean(axis=0)
        out["nrm"][i] = m / np.linalg.norm(m)
        out["members"].append(idx)
    return out


def subvoxel_box(sub, origin, voxel, dv):
    sv = float(np.float32(voxel) / np.float32(dv))
    lo = np.asarray(origin, np.float64) + np.asarray(sub, np.float64) * sv
    return lo, lo + sv


def edge_ies(seg, normals, labels, origin, voxel, dv, dims):
    """Diffraction IEs of caller-given convex edges (Section 2.1: a subvoxel may
    hold diffraction edge segments): every edge a -> b is cut at the subvoxel
    faces it crosses; each piece is one IE in the subvoxel of its midpoint,
    reception point = the midpoint, with the edge's label, unit direction and
    the outward normals of its two faces.  The cut parameters, midpoints and
    cells are computed in FP32 (t = ((origin + k sv) - a) / (b - a) per face
    plane k; midpoint a + ((t0 + t1) / 2) (b - a)): integers decided by
    floating point, in the kernel's precision.  IEs are ordered by (voxel,
    subvoxel within the voxel, label, edge)."""
    f = np.float32
    sv = f(voxel) / f(dv)
    inv = f(1.0) / sv
    org = np.asarray(origin, np.float32)
    dims = np.asarray(dims, np.int64)
    rows = []
    for j in range(len(seg)):
        a = np.asarray(seg[j][0], np.float32)
        b = np.asarray(seg[j][1], np.float32)
        d = (b - a).astype(np.float32)
        ts = {f(0.0), f(1.0)}
        for ax in range(3):
            if d[ax] == 0:
                continue
            u0 = (a[ax] - org[ax]) * inv
            u1 = (b[ax] - org[ax]) * inv
            for k in range(int(math.floor(min(u0, u1))) + 1, int(math.floor(max(u0, u1))) + 1):
                t = ((org[ax] + f(k) * sv) - a[ax]) / d[ax]
                if f(0.0) < t < f(1.0):
                    ts.add(f(t))
        ts = sorted(ts)
        wd = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64))
        for t0, t1 in zip(ts[:-1], ts[1:]):
            tm = (t0 + t1) * f(0.5)
            m = (a + tm * d).astype(np.float32)
            sub = np.floor((m - org) * inv).astype(np.int64)
            if sub.min() < 0 or np.any(sub >= dims * dv):
                raise ValueError("edge outside the IE grid")
            vox = sub // dv
            loc = sub - vox * dv
            vlin = int(vox[0] + dims[0] * (vox[1] + dims[1] * vox[2]))
            llin = int(loc[0] + dv * (loc[1] + dv * loc[2]))
            key = ((vlin * dv ** 3 + llin) << 32) | int(labels[j])
            rows.append((key, j, sub, m.astype(np.float64), wd, normals[j]))
    rows.sort(key=lambda r: (r[0], r[1]))
    n = len(rows)
    return {"key": np.array([r[0] for r in rows], np.int64), "edge": np.array([r[1] for r in rows], np.int64),
            "sub": np.array([r[2] for r in rows], np.int64).reshape(n, 3),
            "label": np.array([int(labels[r[1]]) for r in rows], np.int64),
            "pos": np.array([r[3] for r in rows]).reshape(n, 3), "w": np.array([r[4] for r in rows]).reshape(n, 3),
            "n1": np.array([np.asarray(r[5][0], np.float64) for r in rows]).reshape(n, 3),
            "n2": np.array([np.asarray(r[5][1], np.float64) for r in rows]).reshape(n, 3)}


def combine(point_ies, edges=None):
    """One IE index space: point IEs first, then edge IEs."""
    n_p = len(point_ies["label"])
    n_e = 0 if edges is None else len(edges["label"])
    out = {"label": np.concatenate([point_ies["label"], edges["label"] if n_e else np.zeros(0, np.int64)]),
           "sub": np.concatenate([point_ies["sub"], edges["sub"] if n_e else np.zeros((0, 3), np.int64)]),
           "pos": np.concatenate([point_ies["pos"], edges["pos"] if n_e else np.zeros((0, 3))]),
           "nrm": np.concatenate([point_ies["nrm"], np.zeros((n_e, 3))]),
           "type": np.r_[np.zeros(n_p, np.int64), np.ones(n_e, np.int64)],
           "edge": np.r_[np.full(n_p, -1, np.int64), edges["edge"] if n_e else np.zeros(0, np.int64)]}
    for f in ("w", "n1", "n2"):
        out[f] = np.concatenate([np.zeros((n_p, 3)), edges[f] if n_e else np.zeros((0, 3))])
    return out


def keller_sectors(o, prev, w, n1, n2, half_angle, slack=0.0):
    """Diffracted conical rays of an edge point o hit from prev (Section 2.2.4):
    the Keller cone of the directions d with d . w = d_in . w, cut into N
    sectors of azimuth dphi = 2 pi / N around the edge, N = max(1, ceil(2 pi
    sin(beta) / (2 half_angle))) (neighbouring axes 2 half_angle apart);
    sector i (azimuths [i, i + 1) dphi from the face-1 normal, turning towards
    w x n1) keeps its axis when that axis leaves the wedge (exterior edges:
    v . n1 >= 0 or v . n2 >= 0 for its direction v across the edge).  Each
    sector's two separation planes contain the edge at its bounding azimuths;
    a target lies in the sector iff (p - o) . n_lo >= 0 and (p - o) . n_hi < 0
    (no planes when N = 1).  Returns (list of (axis, n_lo, n_hi, exterior
    margin), N's distance to the nearest integer step); with ``slack`` > 0 the
    list also holds the sectors whose margin is in [-slack, 0) (an axis that
    grazes a face, kept or dropped by rounding)."""
    din = o - prev
    din = din / np.linalg.norm(din)
    cb = float(din @ w)
    sb = math.sqrt(max(0.0, 1.0 - cb * cb))
    e1 = n1 - float(n1 @ w) * w
    e1 = e1 / np.linalg.norm(e1)
    e2 = np.cross(w, e1)
    arg = 2.0 * math.pi * sb / (2.0 * half_angle)
    N = max(1, int(math.ceil(arg)))
    step_margin = abs(arg - round(arg)) if arg > 0.5 else 1.0
    dphi = 2.0 * math.pi / N
    plane = lambda j: math.cos(j * dphi) * e2 - math.sin(j * dphi) * e1  # noqa: E731
    out = []
    for i in range(N):
        phi = (i + 0.5) * dphi
        v = math.cos(phi) * e1 + math.sin(phi) * e2
        ext = max(float(v @ n1), float(v @ n2))
        if ext < -slack:
            continue
        axis = cb * w + sb * v
        axis = axis / np.linalg.norm(axis)
        out.append((axis, plane(i) if N > 1 else None, plane(i + 1) if N > 1 else None, ext))
    return out, step_margin


# --------------------------------------------------------------------------- cone geometry (Section 2.2.4)

def cone_sphere_margin(o, d, cos_t, sin_t, c, R):
    """R minus the distance from c to the solid cone {apex o, unit axis d,
    half-angle t}: the cone meets the sphere (c, R) iff the margin is >= 0.
    With v = c - o, a = v.d and rho = |v - a d|: c inside the cone when
    rho cos t <= a sin t; nearest to the apex when a cos t + rho sin t < 0;
    else at distance rho cos t - a sin t from the cone's surface."""
    v = np.asarray(c, np.float64) - np.asarray(o, np.float64)
    a = float(v @ d)
    rho = float(np.linalg.norm(v - a * d))
    lateral = rho * cos_t - a * sin_t
    if lateral <= 0.0:
        dist = 0.0
    elif a * cos_t + rho * sin_t < 0.0:
        dist = float(np.linalg.norm(v))
    else:
        dist = lateral
    return R - dist


def block_margins(o, d, t_end, cells, origin, voxel):
    """For each voxel cell w (rows of ``cells``): the signed overlap length of
    the segment o + t d, 0 <= t <= t_end, with the 3x3x3 voxel block
    [w - 1, w + 2) V around w (>= 0 iff they meet; minus the gap along the
    ray, or across it, when they do not).  The voxels within Chebyshev
    distance 1 of a voxel the segment crosses are the w whose block it meets."""
    V = float(voxel)
    lo = np.asarray(origin, np.float64)[None, :] + (np.asarray(cells, np.float64) - 1.0) * V
    hi = lo + 3.0 * V
    t0 = np.zeros(len(lo))
    t1 = np.full(len(lo), float(t_end))
    gap = np.full(len(lo), -np.inf)
    for ax in range(3):
        if d[ax] != 0.0:
            ta = (lo[:, ax] - o[ax]) / d[ax]
            tb = (hi[:, ax] - o[ax]) / d[ax]
            t0 = np.maximum(t0, np.minimum(ta, tb))
            t1 = np.minimum(t1, np.maximum(ta, tb))
        else:
            gap = np.maximum(gap, np.maximum(lo[:, ax] - o[ax], o[ax] - hi[:, ax]))
    m = t1 - t0
    return np.where(gap > 0, -gap, m)


def near_cells(o, d, t_far, origin, voxel, dims):
    """Voxel cells of the grid within two voxels of the segment's bounding box."""
    origin = np.asarray(origin, np.float64)
    dims = np.asarray(dims, np.int64)
    end = o + (t_far if np.isfinite(t_far) else 1e6) * d
    lo_c = np.maximum(np.floor((np.minimum(o, end) - origin) / voxel).astype(np.int64) - 2, 0)
    hi_c = np.minimum(np.floor((np.maximum(o, end) - origin) / voxel).astype(np.int64) + 2, dims - 1)
    if np.any(hi_c < lo_c):
        return np.zeros((0, 3), np.int64)
    g = np.stack(np.meshgrid(*[np.arange(lo_c[a], hi_c[a] + 1) for a in range(3)], indexing="ij"), axis=-1)
    return g.reshape(-1, 3)


def grid_exit(o, d, origin, voxel, dims):
    lo = np.asarray(origin, np.float64)
    hi = lo + np.asarray(dims, np.float64) * float(voxel)
    t1 = math.inf
    for ax in range(3):
        if d[ax] > 0:
            t1 = min(t1, (hi[ax] - o[ax]) / d[ax])
        elif d[ax] < 0:
            t1 = min(t1, (lo[ax] - o[ax]) / d[ax])
    return max(t1, 0.0)


# --------------------------------------------------------------------------- visibility and axis hits

def visible(lib_args, o, p, box_lo, box_hi):
    """States per ray (1 visible, 0 blocked, 2 ambiguous in parity mode) and t_in."""
    from . import OracleArgs, _load, _p  # noqa: F401
    lib = _load()
    n = len(o)
    o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
    p = np.ascontiguousarray(p, np.float64).reshape(-1, 3)
    box = np.ascontiguousarray(np.concatenate([np.asarray(box_lo, np.float64).reshape(-1, 3),
                                               np.asarray(box_hi, np.float64).reshape(-1, 3)], axis=1))
    state = np.zeros(n, np.int32)
    t_in = np.zeros(n, np.float64)
    if n == 0:
        return state, t_in
    rc = lib.oracle_visibility(C.byref(lib_args), n, _p(o), _p(p), _p(box), _p(state), _p(t_in))
    if rc != 0:
        raise RuntimeError(f"oracle_visibility failed with status {rc}")
    return state, t_in


class Scene:
    """The point cloud and the bands of one oracle run."""

    def __init__(self, xyz, normal, label, r_s, t_eps, parity=False, err_abs=0.0, err_dir=0.0, tie_rel=1e-4,
                 edge_rel=1e-4, den_amb=1e-6, n_threads=None):
        from . import OracleArgs, _p, default_threads
        self.xyz = np.ascontiguousarray(xyz, np.float32)
        self.normal = np.ascontiguousarray(normal, np.float32)
        self.label = np.ascontiguousarray(label, np.uint32)
        self.r_s, self.t_eps = float(r_s), float(t_eps)
        self.parity = parity
        self.err_abs, self.err_dir, self.tie_rel, self.edge_rel, self.den_amb = err_abs, err_dir, tie_rel, edge_rel, den_amb
        a = OracleArgs()
        a.xyz, a.nrm, a.label, a.n_pts = _p(self.xyz), _p(self.normal), _p(self.label), self.xyz.shape[0]
        a.r_s, a.t_eps = self.r_s, self.t_eps
        a.parity, a.tie_rel, a.err_abs, a.err_dir = int(bool(parity)), tie_rel, err_abs, err_dir
        a.edge_rel, a.den_amb = edge_rel, den_amb
        a.n_threads = int(n_threads or default_threads())
        self.args = a

    def axis_hits(self, o, d):
        """Nearest disk hit of each axis ray (t > t_eps): t (inf if none) and, in
        parity mode, the extent [t_lo, t_hi] of the acceptable answers."""
        from . import launch
        n = len(o)
        if n == 0:
            return np.zeros(0), np.zeros(0), np.zeros(0)
        idx = np.arange(n, dtype=np.int64)
        res = launch(self.xyz, self.normal, self.label, np.asarray(o, np.float32), np.zeros((0, 3), np.float32),
                     np.asarray(d, np.float32), K=0, r_s=self.r_s, t_eps=self.t_eps, sel=idx * n + idx,
                     parity=self.parity, tie_rel=self.tie_rel, err_abs=self.err_abs, err_dir=self.err_dir,
                     edge_rel=self.edge_rel, den_amb=self.den_amb)
        t = np.where(res["hit_id"][:, 0] >= 0, res["hit_t"][:, 0], np.inf)
        if not self.parity:
            return t, t, t
        lo, hi = t.copy(), t.copy()
        so, sd = res["seg_o"][:, 0], res["seg_d"][:, 0]
        for r in range(n):
            na = int(res["acc_n"][r, 0])
            for m in res["acc_id"][r, 0, :min(na, res["acc_id"].shape[2])]:
                if m < 0:
                    hi[r] = np.inf
                    continue
                nm = self.normal[m].astype(np.float64)
                nm /= np.linalg.norm(nm)
                tm = float((self.xyz[m].astype(np.float64) - so[r]) @ nm / (sd[r] @ nm))
                lo[r], hi[r] = min(lo[r], tm), max(hi[r], tm)
            if na > res["acc_id"].shape[2]:
                lo[r], hi[r] = 0.0, np.inf      # the stored set is partial: any end is acceptable
        return t, lo, hi


# --------------------------------------------------------------------------- the tracer (Sections 2.2.2-2.2.4)

def _merge_similar(kids):
    """Partial paths that reach the same IE with the same labels in the same
    order are similar paths: per (tx, labels, IE) one node is kept, the one of
    smallest (priority, parent).  The definition keeps the smallest exact
    node.  A node admitted only through a banded decision may or may not
    exist in an FP32 implementation, so every such node ordered before the
    group's first certain node (exact, no banded decision on its chain) is
    kept too, and all of them are excused: any of them can be the one kept."""
    kids.sort(key=lambda c: (c["tx"], c["labels"], c["ie"], c["prio"], c["parent"]))
    out = []
    i = 0
    while i < len(kids):
        j = i
        key = (kids[i]["tx"], kids[i]["labels"], kids[i]["ie"])
        while j < len(kids) and (kids[j]["tx"], kids[j]["labels"], kids[j]["ie"]) == key:
            j += 1
        group = kids[i:j]
        head = []
        for c in group:
            head.append(c)
            if c["exact"] and not c["excused"]:
                break
        if len(head) > 1 or not (head[0]["exact"] and not head[0]["excused"]):
            for c in head:
                c["excused"] = True
        # the definition's own choice: the smallest exact node
        best_exact = next((c for c in group if c["exact"]), None)
        if best_exact is not None and not any(c is best_exact for c in head):
            best_exact["excused"] = True
            head.append(best_exact)
        for c in head:
            c["exact"] = c["exact"] and c is best_exact
        out += head
        i = j
    out.sort(key=lambda c: (c["tx"], c["labels"], c["ie"], c["prio"]))
    return out


def trace(scene: Scene, ies, tx, rx, origin, voxel, dv, dims, K, kappa, half_angle, edges=None, max_diff=0):
    """Environment-driven coarse tracing with conical rays (Sections 2.2.2-2.2.4).

    A node is a partial path TX -> IE chain.  Per node: ``exact`` (every
    decision of the chain admits it by the definition) and ``excused`` (some
    decision on the chain lies inside the error band: the node, or its
    absence, cannot be held against an FP32 implementation).  Returns a dict
    with ``nodes`` (per depth 1..K, after the kappa limit), ``records`` (every
    reception: tx, rx, chain, labels, length, prio, exact, excused) and
    ``paths`` ((tx, rx, n, labels) -> {"count", "rows", "excused"}; rows are
    the kappa exact records of smallest (priority, chain))."""
    tx = np.asarray(tx, np.float64).reshape(-1, 3)
    rx = np.asarray(rx, np.float64).reshape(-1, 3)
    ies = combine(ies, edges)
    sv = float(np.float32(voxel) / np.float32(dv))
    R = sv * math.sqrt(3.0) / 2.0
    tau = float(np.float32(1e-3) * np.float32(sv))   # a reflected target must clear the plane by this much
    cos_t, sin_t = math.cos(half_angle), math.sin(half_angle)
    ext = float(max(np.abs(scene.xyz).max() if len(scene.xyz) else 1.0, np.abs(tx).max(), 1.0))
    band = 64 * (2.0 ** -24) * ext if scene.parity else 0.0
    n_ie = len(ies["label"])
    dims = np.asarray(dims, np.int64)
    rx_sub = subvoxel_of(rx.astype(np.float32), origin, voxel, dv) if len(rx) else np.zeros((0, 3), np.int64)
    ie_lo = np.asarray(origin, np.float64)[None, :] + ies["sub"] * sv
    rx_lo = np.asarray(origin, np.float64)[None, :] + rx_sub * sv
    ie_cell = ies["sub"] // dv
    rx_cell = rx_sub // dv
    by_voxel = {}
    for i in range(n_ie):
        by_voxel.setdefault(tuple(int(x) for x in ie_cell[i]), []).append(i)
    rx_by_voxel = {}
    for j in range(len(rx)):
        rx_by_voxel.setdefault(tuple(int(x) for x in rx_cell[j]), []).append(j)

    records = []

    def record(c, j, length, exact, excused):
        records.append(dict(tx=c["tx"], rx=j, chain=c["chain"], labels=c["labels"], length=length, prio=c["prio"],
                            exact=exact, excused=excused))

    # ---- transmission phase: from every TX a ray towards every IE and RX
    roots = [dict(tx=i, chain=(), labels=(), prio=splitmix64(i), length=0.0, o=tx[i], prev=None, ie=-1,
                  ndiff=0, exact=True, excused=False) for i in range(len(tx))]
    q = []   # (parent index, kind, target, exact, excused)
    for i in range(len(tx)):
        q += [(i, "ie", e, True, False) for e in range(n_ie) if ies["type"][e] == 0 or max_diff > 0]
        q += [(i, "rx", j, True, False) for j in range(len(rx))]
    parents = roots
    nodes_by_depth = []
    for k in range(0, K + 1):
        # ---- visibility of this generation's candidates
        o = np.array([parents[pi]["o"] for pi, _, _, _, _ in q]).reshape(-1, 3)
        p = np.array([ies["pos"][t] if kind == "ie" else rx[t] for _, kind, t, _, _ in q]).reshape(-1, 3)
        lo = np.array([ie_lo[t] if kind == "ie" else rx_lo[t] for _, kind, t, _, _ in q]).reshape(-1, 3)
        st, _ = visible(scene.args, o, p, lo, lo + sv)
        kids = []
        for (pi, kind, t, ex, exc), s in zip(q, st):
            if s == 0:
                continue
            P = parents[pi]
            exact = ex and s == 1
            excused = exc or s == 2 or P["excused"]
            if kind == "rx":
                record(P, t, P["length"] + float(np.linalg.norm(rx[t] - P["o"])), exact and P["exact"], excused)
            elif k < K:
                kids.append(dict(tx=P["tx"], chain=P["chain"] + (t,), labels=P["labels"] + (int(ies["label"][t]),),
                                 prio=child_priority(P["prio"], t), parent=pi,
                                 length=P["length"] + float(np.linalg.norm(ies["pos"][t] - P["o"])),
                                 o=ies["pos"][t], prev=P["o"], ie=t, ndiff=P["ndiff"] + int(ies["type"][t]),
                                 exact=exact and P["exact"], excused=excused))
        if k == K:
            break
        kept = _merge_similar(kids)
        nodes_by_depth.append(kept)
        # ---- propagation: the reflected cone of every node of depth k + 1
        q = []
        if not kept:
            break
        # cones of every node: the reflected cone of a point IE, the exterior
        # Keller sectors of an edge IE; (node, axis, plane normals, ambiguous)
        cones = []
        for ci, c in enumerate(kept):
            e = c["ie"]
            if ies["type"][e] == 0:
                din = c["o"] - c["prev"]
                din = din / np.linalg.norm(din)
                n_e = ies["nrm"][e]
                dout = din - 2.0 * float(din @ n_e) * n_e
                dout = dout / np.linalg.norm(dout)
                cones.append((ci, dout, ("refl", n_e if float(n_e @ dout) > 0 else -n_e), False, False))
            else:
                secs, step_margin = keller_sectors(c["o"], c["prev"], ies["w"][e], ies["n1"][e], ies["n2"][e],
                                                   half_angle, slack=band if scene.parity else 0.0)
                amb_n = scene.parity and step_margin <= 1e-3
                for axis, n_lo, n_hi, ext in secs:
                    # a sector whose axis grazes a face (|margin| within the band) is kept or
                    # dropped by rounding: its targets are ambiguous, exact only when kept
                    cones.append((ci, axis, ("diff", n_lo, n_hi, ext >= 0), amb_n, abs(ext) <= band))
        if not cones:
            break
        apex = np.array([kept[ci]["o"] for ci, _, _, _, _ in cones])
        axes = np.array([ax for _, ax, _, _, _ in cones])
        t_hit, t_lo, t_hi = scene.axis_hits(apex.astype(np.float32), axes.astype(np.float32))
        for qi, (ci, d1, sep, amb_n, graze) in enumerate(cones):
            c = kept[ci]
            o1 = apex[qi]
            t_exit = grid_exit(o1, d1, origin, voxel, dims)
            t_end, t_near, t_far = min(t_hit[qi], t_exit), min(t_lo[qi], t_exit), min(t_hi[qi], t_exit)
            cells = near_cells(o1, d1, t_far, origin, voxel, dims)
            if len(cells) == 0:
                continue
            m_end = block_margins(o1, d1, t_end, cells, origin, voxel)
            m_near = block_margins(o1, d1, t_near, cells, origin, voxel) if t_near < t_end else m_end
            m_far = block_margins(o1, d1, t_far, cells, origin, voxel) if t_far > t_end else m_end
            own_edge = ies["edge"][c["ie"]]
            for w, me, mn, mf in zip(cells, m_end, m_near, m_far):
                if mf < -band:
                    continue                      # no end of the axis reaches this block
                w_in = me >= 0
                w_amb = scene.parity and mn <= band   # some acceptable end, or rounding, leaves it out
                wt = (int(w[0]), int(w[1]), int(w[2]))
                # the last generation's cones only end paths: no IE targets; no diffraction beyond
                # the limit; never a point of the node's own IE or edge
                targets = []
                if k + 1 < K:
                    for e in by_voxel.get(wt, []):
                        if e == c["ie"] or (ies["type"][e] == 1 and (c["ndiff"] >= max_diff or
                                                                      (own_edge >= 0 and ies["edge"][e] == own_edge))):
                            continue
                        targets.append(("ie", e))
                targets += [("rx", j) for j in rx_by_voxel.get(wt, [])]
                for kind, t in targets:
                    pc = ie_lo[t] + 0.5 * sv if kind == "ie" else rx_lo[t] + 0.5 * sv
                    pr = ies["pos"][t] if kind == "ie" else rx[t]
                    m_cone = cone_sphere_margin(o1, d1, cos_t, sin_t, pc, R)
                    if sep[0] == "refl":
                        m_sep = float((pr - o1) @ sep[1]) - tau
                        sep_in = m_sep > 0
                        sep_amb = abs(m_sep) <= band
                        sep_out = m_sep < -band
                    elif sep[1] is None:
                        sep_in, sep_amb, sep_out = sep[3], False, False
                    else:
                        m_lo, m_hi = float((pr - o1) @ sep[1]), float((pr - o1) @ sep[2])
                        sep_in = sep[3] and m_lo >= 0 and m_hi < 0
                        sep_amb = abs(m_lo) <= band or abs(m_hi) <= band
                        sep_out = m_lo < -band or m_hi > band
                    exact = w_in and m_cone >= 0 and sep_in
                    # a conjunction is undecided when one of its terms is within the band and
                    # none is outside it on the false side; a sector count N within the band
                    # of an integer step moves every sector: all its decisions are undecided
                    out = m_cone < -band or sep_out
                    amb = scene.parity and (amb_n or (not out and (graze or w_amb or abs(m_cone) <= band or sep_amb)))
                    if exact or amb:
                        q.append((ci, kind, t, exact, amb))
        # one candidate per (node, target): a target reached by two cones of one node
        # (banded at the plane two sectors share) is admitted once
        merged = {}
        for ci, kind, t, ex, amb in q:
            e0, a0 = merged.get((ci, kind, t), (False, False))
            merged[(ci, kind, t)] = (e0 or ex, a0 or amb)
        q = [(ci, kind, t, ex, amb) for (ci, kind, t), (ex, amb) in merged.items()]
        parents = kept
    # ---- coarse paths: per (tx, rx, labels) the count and the kappa exact rows of smallest priority
    paths = {}
    for r in sorted(records, key=lambda r: (r["tx"], r["rx"], len(r["labels"]), r["labels"], r["prio"], r["chain"])):
        key = (r["tx"], r["rx"], len(r["labels"]), r["labels"])
        g = paths.setdefault(key, {"count": 0, "rows": [], "excused": True, "exact": False})
        g["excused"] = g["excused"] and r["excused"]
        if not r["exact"]:
            continue
        g["exact"] = True
        g["count"] += 1
        if kappa <= 0 or len(g["rows"]) < kappa:
            g["rows"].append(r)
    return {"nodes": nodes_by_depth, "records": records, "paths": paths}
