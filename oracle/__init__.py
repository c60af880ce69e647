"""CPU oracle for coarse-path ray launching (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import this package.  It is a plain, slow FP64
definition of what the HIP path computes and shares no code with it.

* ``fibonacci(n)``       uniformly spaced launch directions (Fibonacci lattice)
* ``ray_spacing(n)``     ideal angular spacing alpha of n directions
* ``launch(...)``        brute force: every ray against every point
                         (``oracle.c``), with parity bands on request; or,
                         given a ``Grid``, a CPU uniform-grid DDA that must
                         give the same hits bit for bit
* ``dedup(...)``         coarse paths = records grouped by (tx, rx, b, labels)
                         with the kappa shortest kept (Section 2.2.3)
* ``image_method``       closed-form image-source paths in a box room
                         (the refinement reference of Section 2.3)
* ``refine(...)``        path refinement (Section 2.3, Eq. 2): gradient
                         descent on the path length with re-tracing, brute
                         force (``oracle.c``)
* ``refine_dedup(...)``  refined-path dedup: shortest per label sequence,
                         then first-Fresnel-zone uniqueness (Section 2.3)
* ``sdf_intersect(...)`` ray intersection with the implicit surface of Eq. 1
                         by marching line segments through occupied leaves
                         (``sdf.c``)
* ``sdf_launch(...)``    a coarse launch whose segments end at that surface
                         (FP64 ray state, nearest-point labels, reception as
                         in ``launch``)

Parity unpinned: sigma (reception sphere scale), r_s (surfel radius) and
t_eps (self-intersection distance) are conventions the paper does not fix;
they are pinned only by the shared definition.  Likewise the implicit surface's kernel
weights, h, eps, max_steps and the restart offset after a reflection.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from collections import defaultdict

import numpy as np

from . import image_method  # noqa: F401  (closed forms)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "sdf.c")]
MAXACC = 64


def _stale() -> bool:
    return not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(f) for f in _SRCS)


def build(force: bool = True) -> str:
    """Compile oracle.c and sdf.c with gcc (plain FP64, no FMA contraction)."""
    if force or _stale():
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-pthread", *_SRCS, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class OracleArgs(C.Structure):
    _fields_ = [
        ("xyz", C.c_void_p), ("nrm", C.c_void_p), ("label", C.c_void_p), ("n_pts", C.c_int64),
        ("tx", C.c_void_p), ("n_tx", C.c_int32), ("rx", C.c_void_p), ("n_rx", C.c_int32),
        ("dirs", C.c_void_p), ("n_rays", C.c_int64), ("sel", C.c_void_p), ("n_sel", C.c_int64),
        ("K", C.c_int32), ("r_s", C.c_double), ("t_eps", C.c_double), ("sigma", C.c_double),
        ("alpha", C.c_double),
        ("parity", C.c_int32), ("tie_rel", C.c_double), ("err_abs", C.c_double), ("err_dir", C.c_double),
        ("edge_rel", C.c_double), ("den_amb", C.c_double), ("n_threads", C.c_int32),
        ("hit_id", C.c_void_p), ("hit_t", C.c_void_p), ("acc_n", C.c_void_p), ("acc_id", C.c_void_p),
        ("acc_tc", C.c_void_p), ("seg_o", C.c_void_p), ("seg_d", C.c_void_p),
        ("seq", C.c_void_p), ("pts", C.c_void_p),
        ("rec_cap", C.c_int64), ("n_rec", C.c_int64),
        ("rec_sel", C.c_void_p), ("rec_g", C.c_void_p), ("rec_tx", C.c_void_p), ("rec_rx", C.c_void_p),
        ("rec_b", C.c_void_p), ("rec_lpoly", C.c_void_p), ("rec_lunf", C.c_void_p), ("rec_flags", C.c_void_p),
        ("grid", C.c_void_p),
    ]


class OracleRefineArgs(C.Structure):
    _fields_ = [
        ("xyz", C.c_void_p), ("nrm", C.c_void_p), ("label", C.c_void_p), ("n_pts", C.c_int64),
        ("r_s", C.c_double), ("t_eps", C.c_double), ("n_paths", C.c_int64), ("K", C.c_int32),
        ("tx", C.c_void_p), ("rx", C.c_void_p), ("n_refl", C.c_void_p), ("pts", C.c_void_p),
        ("max_iters", C.c_int32), ("grad_tol", C.c_double), ("step", C.c_double), ("smooth_h", C.c_double),
        ("n_threads", C.c_int32),
        ("status", C.c_void_p), ("iters", C.c_void_p), ("grad", C.c_void_p), ("length", C.c_void_p),
        ("out_pts", C.c_void_p), ("out_id", C.c_void_p), ("out_label", C.c_void_p),
        ("edge_of", C.c_void_p), ("n_edges", C.c_int32), ("edge_seg", C.c_void_p), ("edge_nrm", C.c_void_p),
        ("edge_label", C.c_void_p),
    ]


class OracleSdfArgs(C.Structure):
    _fields_ = [
        ("xyz", C.c_void_p), ("nrm", C.c_void_p), ("n_pts", C.c_int64),
        ("origin", C.c_float * 3), ("leaf", C.c_float),
        ("o", C.c_void_p), ("d", C.c_void_p), ("trange", C.c_void_p), ("n_rays", C.c_int64),
        ("h", C.c_double), ("eps", C.c_double), ("max_steps", C.c_int32), ("n_threads", C.c_int32),
        ("diam_scale", C.c_double), ("cross_margin", C.c_double),
        ("t", C.c_void_p), ("point", C.c_void_p), ("normal", C.c_void_p), ("leaf_cell", C.c_void_p),
        ("o64", C.c_void_p), ("d64", C.c_void_p), ("trange64", C.c_void_p),
    ]


# SDF intersection (Eq. 1) conventions the paper does not fix: neighbourhood
# radius h and near-zero threshold eps as fractions of the finest edge, and
# the evaluations a leaf's march may take
SDF_H_SCALE = 0.95
SDF_EPS_SCALE = 1e-3
SDF_MAX_STEPS = 64

# refinement outcome of a path
REF_VALID, REF_NOT_CONVERGED, REF_MISS, REF_WRONG_SIDE, REF_OCCLUDED, REF_DEGENERATE, REF_OFF_EDGE = range(7)
# Table 1: convergence threshold delta and refinement iterations rho; carrier 60 GHz
REF_GRAD_TOL = 1e-4
REF_MAX_ITERS = 2000
# step scale eta (the paper gives no step size)
REF_STEP = 0.75
CARRIER_HZ = 60e9
LIGHT_SPEED = 299_792_458.0

_lib = None


def _load():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        lib = C.CDLL(_SO)
        lib.oracle_fibonacci.argtypes = [C.c_int64, C.c_void_p]
        lib.oracle_fibonacci.restype = C.c_int
        lib.oracle_ray_spacing.argtypes = [C.c_int64]
        lib.oracle_ray_spacing.restype = C.c_double
        lib.oracle_launch.argtypes = [C.POINTER(OracleArgs)]
        lib.oracle_launch.restype = C.c_int
        lib.oracle_accepts.argtypes = [C.POINTER(OracleArgs), C.c_void_p, C.c_void_p, C.c_int32, C.c_int64,
                                       C.c_double, C.c_int64]
        lib.oracle_accepts.restype = C.c_int
        lib.oracle_visibility.argtypes = [C.POINTER(OracleArgs), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p]
        lib.oracle_visibility.restype = C.c_int
        lib.oracle_refine.argtypes = [C.POINTER(OracleRefineArgs)]
        lib.oracle_refine.restype = C.c_int
        lib.oracle_sdf_intersect.argtypes = [C.POINTER(OracleSdfArgs)]
        lib.oracle_sdf_intersect.restype = C.c_int
        lib.oracle_grid_build.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_double]
        lib.oracle_grid_build.restype = C.c_void_p
        lib.oracle_grid_free.argtypes = [C.c_void_p]
        lib.oracle_grid_free.restype = None
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def fibonacci(n: int) -> np.ndarray:
    """[n, 3] float32 unit directions on the Fibonacci lattice (FP64, then rounded)."""
    out = np.empty((n, 3), np.float32)
    if _load().oracle_fibonacci(int(n), _p(out)) != 0:
        raise ValueError("n must be positive")
    return out


def ray_spacing(n: int) -> float:
    return float(_load().oracle_ray_spacing(int(n)))


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


class Grid:
    """Uniform grid of cubic cells listing every point whose disk's bounding
    sphere meets the cell (``oracle_grid_build``); pass it to ``launch`` to
    trace by DDA instead of brute force (same results, bit for bit)."""

    def __init__(self, xyz, r_s, cell):
        self._xyz = np.ascontiguousarray(xyz, np.float32)
        self._h = _load().oracle_grid_build(_p(self._xyz), self._xyz.shape[0], float(r_s), float(cell))
        if not self._h:
            raise MemoryError("oracle_grid_build failed")

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None):
            _load().oracle_grid_free(self._h)
            self._h = None


def launch(xyz, normal, label, tx, rx, dirs, K, r_s, t_eps, sigma=1.25, alpha=0.0, sel=None,
           parity=False, tie_rel=1e-4, err_abs=0.0, err_dir=0.0, edge_rel=1e-4, den_amb=1e-6,
           n_threads=None, want_segments=False, rec_cap=None, grid=None):
    """Brute-force launch of ``len(dirs)`` rays from every TX (FP64).

    Returns a dict of numpy arrays.  Per traced ray r and segment b (index
    ``[r, b]``): ``hit_id`` (-1 none), ``hit_t``; in parity mode ``acc_n`` and
    ``acc_id`` (the acceptable answers, -1 = no hit).  Per reflection:
    ``seq`` labels and ``pts`` points.  Records: ``rec_*`` arrays in traced-ray
    order (``rec_flags`` bit0 received, bit1 ambiguous).  With ``grid`` (a
    ``Grid`` over the same points) the nearest hits come from its DDA; parity
    mode always uses the brute force.
    """
    lib = _load()
    xyz = np.ascontiguousarray(xyz, np.float32)
    normal = np.ascontiguousarray(normal, np.float32)
    label = np.ascontiguousarray(label, np.uint32)
    tx = np.ascontiguousarray(np.asarray(tx, np.float32).reshape(-1, 3))
    rx = np.ascontiguousarray(np.asarray(rx, np.float32).reshape(-1, 3))
    dirs = np.ascontiguousarray(np.asarray(dirs, np.float32).reshape(-1, 3))
    n_rays = dirs.shape[0]
    if sel is not None:
        sel = np.ascontiguousarray(sel, np.int64)
        n_trace = sel.shape[0]
    else:
        n_trace = tx.shape[0] * n_rays
    S = K + 1
    out = {
        "hit_id": np.empty((n_trace, S), np.int64),
        "hit_t": np.empty((n_trace, S), np.float64),
        "seq": np.empty((n_trace, max(K, 1)), np.int64),
        "pts": np.empty((n_trace, max(K, 1), 3), np.float64),
    }
    if parity:
        out["acc_n"] = np.zeros((n_trace, S), np.int32)
        out["acc_id"] = np.full((n_trace, S, MAXACC), -3, np.int64)
        out["acc_tc"] = np.full((n_trace, S), np.nan)
    if want_segments or parity:
        out["seg_o"] = np.full((n_trace, S, 3), np.nan)
        out["seg_d"] = np.full((n_trace, S, 3), np.nan)
    cap = rec_cap if rec_cap is not None else max(1024, 4 * n_trace)
    for _ in range(2):
        recs = {
            "rec_sel": np.empty(cap, np.int64), "rec_g": np.empty(cap, np.int64),
            "rec_tx": np.empty(cap, np.int32), "rec_rx": np.empty(cap, np.int32),
            "rec_b": np.empty(cap, np.int32), "rec_lpoly": np.empty(cap, np.float64),
            "rec_lunf": np.empty(cap, np.float64), "rec_flags": np.empty(cap, np.int32),
        }
        a = OracleArgs()
        a.xyz, a.nrm, a.label, a.n_pts = _p(xyz), _p(normal), _p(label), xyz.shape[0]
        a.tx, a.n_tx, a.rx, a.n_rx = _p(tx), tx.shape[0], _p(rx), rx.shape[0]
        a.dirs, a.n_rays = _p(dirs), n_rays
        a.sel, a.n_sel = (_p(sel), sel.shape[0]) if sel is not None else (None, 0)
        a.K, a.r_s, a.t_eps, a.sigma, a.alpha = K, r_s, t_eps, sigma, alpha
        a.parity, a.tie_rel, a.err_abs, a.err_dir = int(bool(parity)), tie_rel, err_abs, err_dir
        a.edge_rel, a.den_amb = edge_rel, den_amb
        a.n_threads = int(n_threads or default_threads())
        a.hit_id, a.hit_t = _p(out["hit_id"]), _p(out["hit_t"])
        a.acc_n = _p(out.get("acc_n"))
        a.acc_id = _p(out.get("acc_id"))
        a.acc_tc = _p(out.get("acc_tc"))
        a.seg_o, a.seg_d = _p(out.get("seg_o")), _p(out.get("seg_d"))
        a.seq = _p(out["seq"]) if K > 0 else None
        a.pts = _p(out["pts"]) if K > 0 else None
        a.rec_cap = cap
        a.grid = grid.handle if grid is not None else None
        for k, v in recs.items():
            setattr(a, k, _p(v))
        rc = lib.oracle_launch(C.byref(a))
        if rc == -3:
            cap = int(a.n_rec)
            continue
        if rc != 0:
            raise RuntimeError(f"oracle_launch failed with status {rc}")
        n = int(a.n_rec)
        for k, v in recs.items():
            out[k] = v[:n]
        out["n_rec"] = n
        out["alpha"] = alpha if alpha > 0 else ray_spacing(n_rays)
        out["sel"] = sel if sel is not None else np.arange(n_trace, dtype=np.int64)
        if parity:
            out["_bands"] = dict(xyz=xyz, normal=normal, n_pts=xyz.shape[0], r_s=r_s, t_eps=t_eps,
                                 tie_rel=tie_rel, err_abs=err_abs, err_dir=err_dir, edge_rel=edge_rel,
                                 den_amb=den_amb)
        return out
    raise RuntimeError("record capacity retry failed")


def accepts(res, r, b, m):
    """Whether point m (or -1, no hit) is in the acceptable set of segment b
    of traced ray r of a parity-mode ``launch`` result.  The result stores
    only the first MAXACC members of each set; this decides membership for
    any point with the same band test."""
    lib = _load()
    bd = res["_bands"]
    a = OracleArgs()
    a.xyz, a.nrm, a.n_pts = _p(bd["xyz"]), _p(bd["normal"]), bd["n_pts"]
    a.r_s, a.t_eps = bd["r_s"], bd["t_eps"]
    a.tie_rel, a.err_abs, a.err_dir = bd["tie_rel"], bd["err_abs"], bd["err_dir"]
    a.edge_rel, a.den_amb = bd["edge_rel"], bd["den_amb"]
    o = np.ascontiguousarray(res["seg_o"][r, b], np.float64)
    d = np.ascontiguousarray(res["seg_d"][r, b], np.float64)
    last = int(res["hit_id"][r, b - 1]) if b > 0 else -1
    rc = lib.oracle_accepts(C.byref(a), _p(o), _p(d), int(b), last, float(res["acc_tc"][r, b]), int(m))
    if rc < 0:
        raise ValueError("oracle_accepts: bad arguments")
    return bool(rc)


def dedup(res, K, kappa=1, include_ambiguous=False):
    """Coarse paths: group reception records by (tx, rx, b, labels[0:b]).

    Section 2.2.3 limits the number of paths with the same labels in the same
    order to kappa; here the kappa records with the smallest (L_poly, ray id)
    are kept per key, together with the total count.  Returns a dict
    key -> {"count", "rows": [(L_poly, L_unf, g, sel_index), ...]} and the
    list of keys in sorted order.  Only received records count unless
    ``include_ambiguous``; ambiguous-only receptions are returned separately
    in "ambiguous_keys".
    """
    groups = defaultdict(list)
    amb_keys = set()
    flags = res["rec_flags"]
    for q in range(res["n_rec"]):
        r = int(res["rec_sel"][q])
        b = int(res["rec_b"][q])
        labels = tuple(int(x) for x in res["seq"][r, :b]) if b > 0 else ()
        key = (int(res["rec_tx"][q]), int(res["rec_rx"][q]), b, labels)
        if flags[q] & 2:
            amb_keys.add(key)
        if not (flags[q] & 1) and not include_ambiguous:
            continue
        groups[key].append((float(res["rec_lpoly"][q]), float(res["rec_lunf"][q]), int(res["rec_g"][q]), r,
                            int(flags[q])))
    paths = {}
    for key, rows in groups.items():
        rows.sort(key=lambda x: (x[0], x[2]))
        paths[key] = {"count": len(rows), "rows": rows[:kappa], "all": rows}
    return paths, sorted(paths.keys()), amb_keys


def refine(xyz, normal, label, r_s, t_eps, tx, rx, n_refl, pts, max_iters=REF_MAX_ITERS, grad_tol=REF_GRAD_TOL,
           step=REF_STEP, smooth_radius=0.0, n_threads=None, edges=None, edge_of=None):
    """Refine coarse paths into exact paths (Section 2.3, Eq. 2), FP64 brute force.

    Per path p: ``tx[p]``, ``rx[p]`` (positions), ``n_refl[p]`` = N and the
    coarse interaction points ``pts[p, :N]`` ([n, K, 3]).  ``smooth_radius`` > 0
    takes the surface normal at each point as the weighted average of the
    normals within that radius (Eq. 1's n(x)) instead of the hit surfel's.
    ``edges`` = dict(seg [E, 2, 3], normals [E, 2, 3], label [E]) and
    ``edge_of`` [n, K] (edge of interaction k, -1 for a reflection) make the
    interactions with an edge diffractions, D_k = c_k + t_k w_k on the edge.
    Returns a dict:
    ``status`` (REF_*), ``iters`` (gradient steps), ``grad`` (final norm of
    the gradient), ``length`` (f of Eq. 2), ``points`` [n, K, 3] (NaN past
    N), ``ids`` (surfel; -2 - edge for a diffraction) and ``labels`` [n, K]
    (-1 past N).
    """
    lib = _load()
    xyz = np.ascontiguousarray(xyz, np.float32)
    normal = np.ascontiguousarray(normal, np.float32)
    label = np.ascontiguousarray(label, np.uint32)
    tx = np.ascontiguousarray(np.asarray(tx, np.float64).reshape(-1, 3))
    rx = np.ascontiguousarray(np.asarray(rx, np.float64).reshape(-1, 3))
    n_refl = np.ascontiguousarray(n_refl, np.int32)
    pts = np.ascontiguousarray(pts, np.float64)
    n = n_refl.shape[0]
    K = pts.shape[1] if pts.ndim == 3 else 0
    out = {"status": np.empty(n, np.int32), "iters": np.empty(n, np.int32), "grad": np.empty(n),
           "length": np.empty(n), "points": np.empty((n, max(K, 1), 3)), "ids": np.empty((n, max(K, 1)), np.int64),
           "labels": np.empty((n, max(K, 1)), np.int64)}
    a = OracleRefineArgs()
    a.xyz, a.nrm, a.label, a.n_pts = _p(xyz), _p(normal), _p(label), xyz.shape[0]
    a.r_s, a.t_eps, a.n_paths, a.K = float(r_s), float(t_eps), n, K
    a.tx, a.rx, a.n_refl, a.pts = _p(tx), _p(rx), _p(n_refl), _p(pts)
    a.max_iters, a.grad_tol, a.step, a.smooth_h = int(max_iters), float(grad_tol), float(step), float(smooth_radius)
    a.n_threads = int(n_threads or default_threads())
    a.status, a.iters, a.grad, a.length = _p(out["status"]), _p(out["iters"]), _p(out["grad"]), _p(out["length"])
    a.out_pts, a.out_id, a.out_label = _p(out["points"]), _p(out["ids"]), _p(out["labels"])
    if edge_of is not None:
        edge_of = np.ascontiguousarray(np.asarray(edge_of, np.int32).reshape(n, K))
        eseg = np.ascontiguousarray(np.asarray(edges["seg"], np.float64).reshape(-1, 6))
        enrm = np.ascontiguousarray(np.asarray(edges["normals"], np.float64).reshape(-1, 6))
        elab = np.ascontiguousarray(np.asarray(edges["label"], np.int64).reshape(-1))
        a.edge_of, a.n_edges = _p(edge_of), eseg.shape[0]
        a.edge_seg, a.edge_nrm, a.edge_label = _p(eseg), _p(enrm), _p(elab)
    rc = lib.oracle_refine(C.byref(a))
    if rc != 0:
        raise RuntimeError(f"oracle_refine failed with status {rc}")
    out["points"] = out["points"][:, :K]
    out["ids"] = out["ids"][:, :K]
    out["labels"] = out["labels"][:, :K]
    return out


def fresnel_radius(d1, d2, wavelength):
    """Radius of the first Fresnel zone at distances d1, d2 from the two ends."""
    return float(np.sqrt(wavelength * d1 * d2 / (d1 + d2)))


def refine_dedup(group, n_refl, labels, points, length, status, tx, carrier_hz=CARRIER_HZ):
    """Unique exact paths among refined ones (Section 2.3, last paragraph).

    ``group[p]`` identifies the (TX, RX) pair of path p; ``tx[p]`` is its TX
    position.  Paths are compared only within one (TX, RX) pair and one
    number of interactions (reflections only: the chain of interactions is
    their number).  In order of increasing length (ties: smaller index):
      1. a valid path whose label sequence already occurred is dropped (the
         shortest path of every label sequence is kept);
      2. a path is dropped if every interaction point lies within the first
         Fresnel zone of the corresponding point of an already kept path
         (radius sqrt(lambda d1 d2 / (d1 + d2)), d1 and d2 the kept path's
         lengths from the TX to the point and from the point to the RX).
    ``carrier_hz <= 0`` skips step 2.  Returns a bool array ``kept``.
    """
    n = len(n_refl)
    kept = np.zeros(n, bool)
    lam = LIGHT_SPEED / carrier_hz if carrier_hz > 0 else 0.0
    by_group = defaultdict(list)
    for p in range(n):
        if status[p] == REF_VALID:
            by_group[(int(group[p]), int(n_refl[p]))].append(p)
    for (_, N), rows in by_group.items():
        rows.sort(key=lambda p: (float(length[p]), p))
        seen = set()
        kept_rows = []
        for p in rows:
            lab = tuple(int(x) for x in labels[p][:N])
            if lab in seen:
                continue
            seen.add(lab)
            dup = False
            if lam > 0:
                for q in kept_rows:
                    d1 = 0.0
                    prev = np.asarray(tx[q], np.float64)
                    close = True
                    for k in range(N):
                        cq = np.asarray(points[q][k], np.float64)
                        d1 += float(np.linalg.norm(cq - prev))
                        prev = cq
                        r_f = fresnel_radius(d1, float(length[q]) - d1, lam)
                        if np.linalg.norm(np.asarray(points[p][k], np.float64) - cq) > r_f:
                            close = False
                            break
                    if close:
                        dup = True
                        break
            if not dup:
                kept_rows.append(p)
                kept[p] = True
    return kept


def sdf_intersect(xyz, normal, origin, leaf, o, d, trange=None, h=None, eps=None, max_steps=SDF_MAX_STEPS,
                  diam_scale=1.0, cross_margin=0.0, n_threads=None):
    """First intersection of each ray with the implicit surface of Eq. 1
    (``sdf.c``, FP64, brute force over leaves).

    ``origin``/``leaf`` are the scene's FP32 grid origin and finest edge (the
    leaves' point sets are taken in FP32 like the kernels').  ``h`` and
    ``eps`` default to SDF_H_SCALE and SDF_EPS_SCALE times ``leaf``.
    ``diam_scale`` and ``cross_margin`` perturb the segment length and the
    leaf-crossing test (1 and 0 give the definition).  Returns a dict of
    ``t`` (+inf for none), ``point``, ``normal`` and ``leaf_cell`` (-1 none).
    """
    xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    normal = np.ascontiguousarray(normal, np.float32).reshape(-1, 3)
    # float64 rays are taken as they are (reflected rays carry FP64 state)
    wide = isinstance(o, np.ndarray) and o.dtype == np.float64
    ft = np.float64 if wide else np.float32
    o = np.ascontiguousarray(np.asarray(o, ft).reshape(-1, 3))
    d = np.ascontiguousarray(np.asarray(d, ft).reshape(-1, 3))
    if o.shape != d.shape:
        raise ValueError("o and d must have the same shape")
    n = o.shape[0]
    tr = None if trange is None else np.ascontiguousarray(np.asarray(trange, ft).reshape(n, 2))
    leaf = float(np.float32(leaf))
    h = SDF_H_SCALE * leaf if h is None else float(h)
    eps = SDF_EPS_SCALE * leaf if eps is None else float(eps)
    out = dict(t=np.empty(n), point=np.empty((n, 3)), normal=np.empty((n, 3)),
               leaf_cell=np.empty((n, 3), np.int32))
    a = OracleSdfArgs()
    a.xyz, a.nrm, a.n_pts = _p(xyz), _p(normal), xyz.shape[0]
    a.origin[:] = [float(v) for v in np.asarray(origin, np.float32).reshape(3)]
    a.leaf = leaf
    if wide:
        a.o64, a.d64, a.trange64 = _p(o), _p(d), (_p(tr) if tr is not None else None)
    else:
        a.o, a.d, a.trange = _p(o), _p(d), (_p(tr) if tr is not None else None)
    a.n_rays = n
    a.h, a.eps, a.max_steps = h, eps, int(max_steps)
    a.n_threads = default_threads() if n_threads is None else int(n_threads)
    a.diam_scale, a.cross_margin = float(diam_scale), float(cross_margin)
    a.t, a.point, a.normal, a.leaf_cell = (_p(out["t"]), _p(out["point"]), _p(out["normal"]),
                                           _p(out["leaf_cell"]))
    rc = _load().oracle_sdf_intersect(C.byref(a))
    if rc != 0:
        raise ValueError(f"oracle_sdf_intersect failed ({rc})")
    return out


def sdf_launch(xyz, normal, label, origin, leaf, tx, rx, dirs, K, sigma=1.25, alpha=0.0, h=None, eps=None,
               max_steps=SDF_MAX_STEPS, diam_scale=1.0, cross_margin=0.0, band=1e-5, n_threads=None):
    """Coarse launch whose segments end at the implicit surface of Eq. 1 (FP64;
    the definition behind PCRL_LAUNCH_SDF).

    Every ray (global id g = tx index * n_rays + direction index) runs
    segments b = 0..K: the first intersection of ``sdf_intersect`` from
    t_lo (0 from the TX; after a reflection 4 eps / max(|d.n|, 0.05), just
    outside the |f| <= eps band the ray leaves); the interaction's label and
    id are those of the nearest point (a miss if none lies within h); every
    RX sphere is tested on [0, t] as in ``launch`` (reading R8); the ray
    reflects about n(x).  Returns per ray and segment ``t`` (+inf miss, NaN
    not traced), ``pid``, ``label`` and ``label_margin`` (distance to the
    second-nearest point minus the nearest), ``cos`` = |d.n| at the hit, and
    the records ``rec_*`` with
    ``rec_band`` set where the reception test lies within ``band`` of its
    threshold.
    """
    from scipy.spatial import cKDTree
    xyz32 = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    lab = np.asarray(label, np.uint32).reshape(-1)
    tx = np.asarray(tx, np.float32).reshape(-1, 3).astype(np.float64)
    rx = np.asarray(rx, np.float32).reshape(-1, 3).astype(np.float64)
    dirs = np.asarray(dirs, np.float32).reshape(-1, 3).astype(np.float64)
    n_rays = dirs.shape[0]
    n = tx.shape[0] * n_rays
    leaf32 = float(np.float32(leaf))
    h = SDF_H_SCALE * leaf32 if h is None else float(h)
    eps = SDF_EPS_SCALE * leaf32 if eps is None else float(eps)
    if alpha <= 0.0:
        alpha = math.sqrt(8.0 * math.pi / (math.sqrt(3.0) * n_rays))
    sig_c = sigma * alpha / math.sqrt(3.0)
    tree = cKDTree(xyz32.astype(np.float64)) if len(xyz32) else None
    o = np.repeat(tx, n_rays, axis=0)
    d = np.tile(dirs, (tx.shape[0], 1))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    L = np.zeros(n)
    t_lo = np.zeros(n)
    alive = np.ones(n, bool)
    T = np.full((n, K + 1), np.nan)
    PID = np.full((n, K + 1), -1, np.int64)
    LAB = np.full((n, K + 1), -1, np.int64)
    MARG = np.full((n, K + 1), np.inf)
    COS = np.full((n, K + 1), np.nan)
    recs = []
    for b in range(K + 1):
        idx = np.nonzero(alive)[0]
        if len(idx) == 0:
            break
        tr = np.column_stack([t_lo[idx], np.full(len(idx), np.inf)])
        r = sdf_intersect(xyz32, normal, origin, leaf, o[idx], d[idx], trange=tr, h=h, eps=eps,
                          max_steps=max_steps, diam_scale=diam_scale, cross_margin=cross_margin,
                          n_threads=n_threads)
        t = r["t"].copy()
        hit = np.isfinite(t)
        q = o[idx] + np.where(hit, t, 0.0)[:, None] * d[idx]
        if tree is not None and hit.any():
            dist, nn = tree.query(q[hit], k=2 if len(xyz32) > 1 else 1)
            dist = dist.reshape(len(nn), -1)
            nn = nn.reshape(len(nn), -1)
            first = nn[:, 0].copy()
            if dist.shape[1] > 1:
                tie = dist[:, 1] == dist[:, 0]
                first[tie] = np.minimum(nn[tie, 0], nn[tie, 1])
                marg = dist[:, 1] - dist[:, 0]
            else:
                marg = np.full(len(first), np.inf)
            near = dist[:, 0] < h
            hi_idx = np.nonzero(hit)[0]
            PID[idx[hi_idx[near]], b] = first[near]
            LAB[idx[hi_idx[near]], b] = lab[first[near]]
            MARG[idx[hi_idx], b] = np.where(near, marg, np.inf)
            hit[hi_idx[~near]] = False
        t[~hit] = np.inf
        T[idx, b] = t
        COS[idx, b] = np.abs((d[idx] * r["normal"]).sum(1))
        # reception on [0, t] (reading R8)
        for ri in range(rx.shape[0]):
            v = rx[ri] - o[idx]
            s_ = (v * d[idx]).sum(1)
            c = v - s_[:, None] * d[idx]
            dist2 = (c * c).sum(1)
            rho = sig_c * (L[idx] + s_)
            inside = (s_ > 0) & (s_ <= t)
            got = inside & (dist2 <= rho * rho)
            near_thr = (np.abs(dist2 - rho * rho) <= band * np.maximum(rho * rho, 1e-30)) | \
                (np.abs(s_) <= band * (1 + np.abs(s_))) | (np.isfinite(t) & (np.abs(s_ - t) <= band * (1 + t)))
            for k in np.nonzero(got | (near_thr & (dist2 <= rho * rho * (1 + 2 * band))))[0]:
                recs.append((idx[k], ri, b, L[idx[k]] + math.sqrt((v[k] ** 2).sum()), L[idx[k]] + s_[k],
                             bool(got[k]), bool(near_thr[k])))
        surv = hit & (b < K)
        alive[idx[~surv]] = False
        si = idx[surv]
        if len(si):
            n_ = r["normal"][surv]
            dn = (d[si] * n_).sum(1)
            dd = d[si] - 2.0 * dn[:, None] * n_
            dd /= np.linalg.norm(dd, axis=1, keepdims=True)
            L[si] += t[surv]
            o[si] = q[surv]
            d[si] = dd
            t_lo[si] = 4.0 * eps / np.maximum(np.abs(dn), 0.05)
    rec = np.array([x[:5] for x in recs], dtype=np.float64).reshape(-1, 5)
    return dict(t=T, pid=PID, label=LAB, label_margin=MARG, cos=COS,
                rec_g=rec[:, 0].astype(np.int64), rec_rx=rec[:, 1].astype(np.int64), rec_b=rec[:, 2].astype(np.int64),
                rec_lpoly=rec[:, 3], rec_lunf=rec[:, 4],
                rec_got=np.array([x[5] for x in recs], bool), rec_band=np.array([x[6] for x in recs], bool))
