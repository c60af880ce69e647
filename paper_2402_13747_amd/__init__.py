"""MI355X-native coarse-path ray launching over voxelised labeled point clouds.

Python face of libpcrl.so (include/pcrl.h), same names as the C ABI:

    scene  = build_voxels(xyz, normal, label, levels=(0.5, 0.25), surfel_radius=0.15)
    launch = launch_rays(scene, tx, rx, n_rays=10_000, max_reflections=2)
    paths  = collect_paths(launch, kappa=1)

Inputs are torch tensors (or numpy arrays, copied to ``device``); the
library enqueues all work on torch's current stream.  Every computation runs
in HIP kernels; this module only marshals arguments.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import math

import numpy as np
import torch

from . import _lib
from ._lib import (KEY_LABELS, KEY_LEAVES, LAUNCH_COHERENT, LAUNCH_SDF, LAUNCH_STATS, LAUNCH_TIMING, PCRL_EOVERFLOW,
                   REFINE_DEGENERATE, REFINE_MISS, REFINE_NOT_CONVERGED, REFINE_OCCLUDED, REFINE_OFF_EDGE,
                   REFINE_VALID, REFINE_WRONG_SIDE, PcrlError, check, lib)

__all__ = ["ie_build", "cone_launch", "cone_collect", "IeTable", "ConeLaunch", "build_voxels", "launch_rays", "launch_batch", "batch_autotune", "launch_directions", "collect_paths",
           "refine_paths", "refine_cone_paths", "sdf_intersect", "use_torch_allocator", "Scene", "Launch", "Server",
           "serve_query_bytes", "PcrlError", "KEY_LABELS",
           "KEY_LEAVES", "REFINE_VALID", "REFINE_NOT_CONVERGED", "REFINE_MISS", "REFINE_WRONG_SIDE",
           "REFINE_OCCLUDED", "REFINE_DEGENERATE", "REFINE_OFF_EDGE", "version", "library_path"]


# Every installed allocator's ctypes callbacks, kept for the life of the
# process: the library frees each block through the allocator that made it,
# also after a switch back, so the callbacks must outlive every such block.
_allocators = []


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's device allocations through torch's caching allocator
    (set_allocator); ``enable=False`` returns to the library's own."""
    if not enable:
        check("set_allocator", lib.set_allocator(None))
        return

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
        except Exception:  # reported by the library as PCRL_ENOMEM
            return None

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = _lib.PcrlAllocator(_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free), None)
    _allocators.append(a)
    check("set_allocator", lib.set_allocator(C.byref(a)))


def version() -> str:
    return lib.pcrl_version().decode()


def library_path() -> str:
    return _lib.LIB_PATH


def _dev(device):
    if device is None:
        return torch.device("cuda", torch.cuda.current_device())
    return torch.device(device)


def _as_tensor(x, dtype, device, shape_last=None):
    if isinstance(x, torch.Tensor):
        t = x
    else:
        t = torch.from_numpy(np.ascontiguousarray(x))
    if t.dtype != dtype:
        t = t.to(dtype)
    t = t.to(device).contiguous()
    if shape_last is not None:
        t = t.reshape(-1, shape_last)
    return t


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


_NO_SWITCH = contextlib.nullcontext()


def _on(device):
    """Make `device` current for a library call (no switch when it already is)."""
    if device.index is None or device.index == torch.cuda.current_device():
        return _NO_SWITCH
    return torch.cuda.device(device)


class Scene:
    """A device-resident voxel hierarchy (owns a PcrlScene handle)."""

    def __init__(self, handle, device, inputs):
        self._h = handle
        self.device = device
        self._inputs = inputs

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _lib.PcrlSceneInfo()
        check("scene_info", lib.scene_info(self._h, C.byref(inf)))
        out = {}
        for name, _ in inf._fields_:
            v = getattr(inf, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        out["n_nodes"] = out["n_nodes"][: out["n_levels"]]
        return out

    def leaf_table(self):
        inf = self.info()
        nl, m = inf["n_leaves"], inf["n_entries"]
        key = torch.empty(max(nl, 1), dtype=torch.int64, device=self.device)
        begin = torch.empty(max(nl, 1), dtype=torch.int32, device=self.device)
        count = torch.empty(max(nl, 1), dtype=torch.int32, device=self.device)
        ids = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        check("scene_leaf_table", lib.scene_leaf_table(self._h, _ptr(key), _ptr(begin), _ptr(count), _ptr(ids),
                                                       _stream(self.device)))
        return key[:nl], begin[:nl], count[:nl], ids[:m]

    def update_points(self, ids, xyz, normal, label):
        """Replace the dynamic points (global ids distinct from the static ones) -- a new epoch."""
        ids = _as_tensor(np.asarray(ids, np.int64).astype(np.uint32).view(np.int32)
                         if isinstance(ids, np.ndarray) else ids, torch.int32, self.device)
        xyz = _as_tensor(xyz, torch.float32, self.device, 3)
        normal = _as_tensor(normal, torch.float32, self.device, 3)
        if isinstance(label, np.ndarray):
            label = torch.from_numpy(np.ascontiguousarray(label.astype(np.uint32)).view(np.int32))
        label = _as_tensor(label, torch.int32, self.device)
        n = xyz.shape[0]
        if ids.shape[0] != n or normal.shape[0] != n or label.shape[0] != n:
            raise ValueError("ids, xyz, normal and label must have the same length")
        with torch.cuda.device(self.device):
            check("update_points", lib.update_points(self._h, _ptr(ids) if n else None, _ptr(xyz) if n else None,
                                                     _ptr(normal) if n else None, _ptr(label) if n else None, n,
                                                     _stream(self.device)))
        self._dyn = (ids, xyz, normal, label)

    def release(self):
        if self._h:
            lib.release_scene(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def build_voxels(xyz, normal, label, levels, surfel_radius, t_eps=0.0, device=None, compact=False) -> Scene:
    """Voxelise a labeled point cloud (positions [N,3], normals [N,3], labels [N]).

    ``compact`` keeps no dense cell table of the leaves' parent bricks (less
    device memory, slower traversal)."""
    device = _dev(device)
    xyz = _as_tensor(xyz, torch.float32, device, 3)
    normal = _as_tensor(normal, torch.float32, device, 3)
    if isinstance(label, np.ndarray):
        label = torch.from_numpy(np.ascontiguousarray(label.astype(np.uint32)).view(np.int32))
    label = _as_tensor(label, torch.int32, device)
    n = xyz.shape[0]
    if normal.shape[0] != n or label.shape[0] != n:
        raise ValueError("xyz, normal and label must have the same length")
    levels = list(levels)
    if not 1 <= len(levels) <= _lib.MAX_LEVELS:
        raise ValueError("1..4 levels")
    p = _lib.PcrlVoxelParams()
    p.n_levels = len(levels)
    for i, s in enumerate(levels):
        p.level_size[i] = float(s)
    p.surfel_radius = float(surfel_radius)
    p.t_eps = float(t_eps)
    p.flags = _lib.VOXEL_COMPACT if compact else 0
    h = C.c_void_p()
    with _on(device):
        check("build_voxels", lib.build_voxels(_ptr(xyz) if n else None, _ptr(normal) if n else None,
                                               _ptr(label) if n else None, n, C.byref(p), _stream(device),
                                               C.byref(h)))
    return Scene(h, device, (xyz, normal, label))


class Launch:
    """Rays launched into a scene (owns a PcrlLaunch handle)."""

    def __init__(self, handle, scene, device, n_rays, K, n_tx, n_rx, hit_log, args):
        self._h = handle
        self.scene = scene
        self.device = device
        self.n_rays = n_rays
        self.K = K
        self.n_tx = n_tx
        self.n_rx = n_rx
        self.hit_log = hit_log
        self._args = args

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        st = _lib.PcrlLaunchStats()
        check("launch_stats", lib.launch_stats(self._h, C.byref(st)))
        out = {}
        for name, _ in st._fields_:
            v = getattr(st, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        out["active"] = out["active"][: self.K + 1]
        out["kernel_ms"] = out["kernel_ms"][: self.K + 1]
        for k in ("algo_bytes_bounce", "dda_steps_bounce", "surfel_tests_bounce", "wave_dda_bounce"):
            out[k] = out[k][: self.K + 1]
        return out

    def records(self) -> dict:
        n = C.c_int64()
        st = self.stats()
        cap = max(int(st["records"]), 1)
        ray = torch.empty(cap, dtype=torch.int64, device=self.device)
        rx = torch.empty(cap, dtype=torch.int32, device=self.device)
        nb = torch.empty(cap, dtype=torch.int32, device=self.device)
        lp = torch.empty(cap, dtype=torch.float32, device=self.device)
        lu = torch.empty(cap, dtype=torch.float32, device=self.device)
        check("launch_records", lib.launch_records(self._h, cap, _ptr(ray), _ptr(rx), _ptr(nb), _ptr(lp), _ptr(lu),
                                                   C.byref(n)))
        k = int(n.value)
        return {"ray": ray[:k], "rx": rx[:k], "n_refl": nb[:k], "len_poly": lp[:k], "len_unf": lu[:k]}

    def release(self):
        if self._h:
            lib.release_launch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:  # pragma: no cover
            pass


def launch_rays(scene: Scene, tx, rx, n_rays, max_reflections, directions=None, rx_radius_scale=1.25,
                ray_spacing=0.0, record_capacity=0, stats=False, timing=False, coherent=True, hit_log=False,
                sdf=False) -> Launch:
    """Launch ``n_rays`` rays from every TX (Fibonacci lattice unless ``directions``).

    ``coherent`` traces the first bounce in a direction-sorted ray order (same
    results, better locality).  ``sdf`` ends the segments at the implicit
    surface of Eq. 1 instead of the surfels (PCRL_LAUNCH_SDF)."""
    q = _query(scene, tx, rx, n_rays, max_reflections, directions, rx_radius_scale, ray_spacing, record_capacity,
               stats, timing, coherent, hit_log, sdf)
    h = C.c_void_p()
    device = scene.device
    with _on(device):
        check("launch_rays", lib.launch_rays(scene.handle, _ptr(q["tx"]), q["tx"].shape[0],
                                             _ptr(q["rx"]) if q["rx"].shape[0] else None, q["rx"].shape[0],
                                             C.byref(q["params"]), _stream(device), C.byref(h)))
    return _make_launch(h, q)


def _query(scene, tx, rx, n_rays, max_reflections, directions=None, rx_radius_scale=1.25, ray_spacing=0.0,
           record_capacity=0, stats=False, timing=False, coherent=True, hit_log=False, sdf=False):
    """Marshal one query: device tensors, PcrlLaunchParams and the optional hit log."""
    device = scene.device
    tx = _as_tensor(tx, torch.float32, device, 3)
    rx = _as_tensor(rx, torch.float32, device, 3) if rx is not None else torch.zeros((0, 3), device=device)
    dirs = _as_tensor(directions, torch.float32, device, 3) if directions is not None else None
    if dirs is not None and dirs.shape[0] != n_rays:
        raise ValueError("directions must have n_rays rows")
    K = int(max_reflections)
    p = _lib.PcrlLaunchParams()
    p.n_rays = int(n_rays)
    p.directions = _ptr(dirs).value if dirs is not None else None
    p.max_reflections = K
    p.rx_radius_scale = float(rx_radius_scale)
    p.ray_spacing = float(ray_spacing)
    p.record_capacity = int(record_capacity)
    p.flags = ((LAUNCH_STATS if stats else 0) | (LAUNCH_TIMING if timing else 0) | (LAUNCH_COHERENT if coherent else 0)
               | (LAUNCH_SDF if sdf else 0))
    log = None
    if hit_log:
        n = tx.shape[0] * int(n_rays) * (K + 1)
        log = (torch.empty(n, dtype=torch.int32, device=device), torch.empty(n, dtype=torch.float32, device=device))
        p.hit_log_id = log[0].data_ptr()
        p.hit_log_t = log[1].data_ptr()
    args = dict(tx=tx, rx=rx, n_rays=n_rays, max_reflections=max_reflections, directions=dirs,
                rx_radius_scale=rx_radius_scale, ray_spacing=ray_spacing, stats=stats, timing=timing,
                coherent=coherent, hit_log=hit_log, sdf=sdf)
    return {"scene": scene, "tx": tx, "rx": rx, "dirs": dirs, "params": p, "log": log, "args": args, "K": K,
            "n_rays": int(n_rays)}


def _make_launch(h, q):
    log = q["log"]
    n_tx = q["tx"].shape[0]
    if log is not None:
        log = (log[0].view(n_tx * q["n_rays"], q["K"] + 1), log[1].view(n_tx * q["n_rays"], q["K"] + 1))
    return Launch(h, q["scene"], q["scene"].device, q["n_rays"], q["K"], n_tx, q["rx"].shape[0], log, q["args"])


def launch_batch(queries, tile_rays=0, compact_threshold=-1.0, waves_per_cu=0, use_graph=False, autotune=False):
    """Trace many queries together (one persistent kernel per bounce for all of them).

    ``queries``: list of dicts with the keyword arguments of ``launch_rays``
    (``scene``, ``tx``, ``rx``, ``n_rays``, ``max_reflections``, ...).  Returns
    one Launch per query; each is bitwise the same as its solo launch_rays.
    """
    qs = [_query(**q) for q in queries]
    if not qs:
        return []
    device = qs[0]["scene"].device
    arr = (_lib.PcrlQuery * len(qs))()
    for i, q in enumerate(qs):
        arr[i].scene = q["scene"].handle
        arr[i].tx = q["tx"].data_ptr()
        arr[i].n_tx = q["tx"].shape[0]
        arr[i].rx = q["rx"].data_ptr() if q["rx"].shape[0] else None
        arr[i].n_rx = q["rx"].shape[0]
        arr[i].params = q["params"]
    bp = _batch_params(tile_rays, compact_threshold, waves_per_cu, use_graph, autotune)
    out = (C.c_void_p * len(qs))()
    with _on(device):
        check("launch_batch", lib.launch_batch(arr, len(qs), C.byref(bp), _stream(device), out))
    return [_make_launch(C.c_void_p(out[i]), q) for i, q in enumerate(qs)]


def _batch_params(tile_rays=0, compact_threshold=-1.0, waves_per_cu=0, use_graph=False, autotune=False):
    bp = _lib.PcrlBatchParams()
    bp.tile_rays = int(tile_rays)
    bp.compact_threshold = float(compact_threshold)
    bp.waves_per_cu = int(waves_per_cu)
    bp.use_graph = int(bool(use_graph))
    bp.autotune = int(bool(autotune))
    bp.flags = 0
    return bp


def batch_autotune(queries, use_graph=False) -> dict:
    """Tune (tile_rays, compact_threshold, waves_per_cu) on these queries; returns the winner."""
    qs = [_query(**q) for q in queries]
    device = qs[0]["scene"].device
    arr = (_lib.PcrlQuery * len(qs))()
    for i, q in enumerate(qs):
        arr[i].scene = q["scene"].handle
        arr[i].tx = q["tx"].data_ptr()
        arr[i].n_tx = q["tx"].shape[0]
        arr[i].rx = q["rx"].data_ptr() if q["rx"].shape[0] else None
        arr[i].n_rx = q["rx"].shape[0]
        arr[i].params = q["params"]
    bp = _batch_params(use_graph=use_graph)
    with _on(device):
        check("batch_autotune", lib.batch_autotune(arr, len(qs), _stream(device), C.byref(bp)))
    return {"tile_rays": bp.tile_rays, "compact_threshold": bp.compact_threshold, "waves_per_cu": bp.waves_per_cu}


def launch_directions(n_rays, device=None):
    """[n_rays, 3] float32 Fibonacci-lattice directions computed by the library."""
    device = _dev(device)
    out = torch.empty((int(n_rays), 3), dtype=torch.float32, device=device)
    with _on(device):
        check("launch_directions", lib.launch_directions(int(n_rays), _ptr(out), _stream(device)))
    return out


def collect_paths(launch: Launch, kappa=1, key_mode=KEY_LABELS, capacity=None) -> dict:
    """Deduplicated coarse paths; rows sorted by (key, len_poly, ray), at most kappa per key.

    If the launch dropped reception records (capacity exceeded), the launch
    is repeated once with the needed capacity (``launch`` is updated in place).
    """
    device = launch.device
    K = launch.K
    for attempt in range(3):
        cap = int(capacity) if capacity is not None else 4096
        bufs = {
            "tx": torch.empty(cap, dtype=torch.int32, device=device),
            "rx": torch.empty(cap, dtype=torch.int32, device=device),
            "n_refl": torch.empty(cap, dtype=torch.int32, device=device),
            "key": torch.empty(max(cap * K, 1), dtype=torch.int64, device=device),
            "count": torch.empty(cap, dtype=torch.int64, device=device),
            "rank": torch.empty(cap, dtype=torch.int32, device=device),
            "ray": torch.empty(cap, dtype=torch.int64, device=device),
            "len_poly": torch.empty(cap, dtype=torch.float32, device=device),
            "len_unf": torch.empty(cap, dtype=torch.float32, device=device),
            "points": torch.empty(max(cap * K * 3, 1), dtype=torch.float32, device=device),
        }
        out = _lib.PcrlPaths()
        out.capacity = cap
        for k, t in bufs.items():
            setattr(out, k, t.data_ptr() if not (K == 0 and k in ("key", "points")) else None)
        with _on(device):
            st = lib.collect_paths(launch.handle, int(kappa), int(key_mode), C.byref(out), _stream(device))
        if st == PCRL_EOVERFLOW and out.n_rows == -1:
            need = launch.stats()["records"]
            _relaunch(launch, int(need * 1.25) + 1024)
            continue
        if st == PCRL_EOVERFLOW:
            capacity = int(out.n_rows)
            continue
        check("collect_paths", st)
        n = int(out.n_rows)
        res = {k: (t[: n * K].view(n, K) if k == "key" else t[: n * K * 3].view(n, K, 3) if k == "points"
                   else t[:n]) for k, t in bufs.items()}
        res["n_rows"] = n
        res["n_keys"] = int(out.n_keys)
        return res
    raise PcrlError("collect_paths", PCRL_EOVERFLOW, "capacity retries exhausted")


def _refine_outputs(n, K, device):
    res = {
        "status": torch.empty(n, dtype=torch.int32, device=device),
        "iters": torch.empty(n, dtype=torch.int32, device=device),
        "grad": torch.empty(n, dtype=torch.float32, device=device),
        "length": torch.empty(n, dtype=torch.float32, device=device),
        "points": torch.empty((n, K, 3), dtype=torch.float32, device=device),
        "point_id": torch.empty((n, K), dtype=torch.int32, device=device),
        "key": torch.empty((n, K), dtype=torch.int64, device=device),
        "kept": torch.empty(n, dtype=torch.int32, device=device),
    }
    out = _lib.PcrlRefined()
    for k, t in res.items():
        setattr(out, k, t.data_ptr() if t.numel() else None)
    return res, out


def _refine_rows(paths: dict, n, device, fields):
    pp = _lib.PcrlPaths()
    pp.capacity = n
    pp.n_rows = n
    for k in fields:
        t = paths[k]
        assert t.is_contiguous() and t.device == device, k
        setattr(pp, k, t.data_ptr() if t.numel() else None)
    return pp


def _refine_params(max_iters, grad_tol, step, carrier_hz, smooth_radius):
    smooth = _lib.REFINE_SMOOTH if smooth_radius > 0 else 0
    return _lib.PcrlRefineParams(int(max_iters), float(grad_tol), float(step), float(carrier_hz), smooth,
                                 float(smooth_radius))


def refine_paths(scene: Scene, tx, rx, paths: dict, max_iters=2000, grad_tol=1e-4, step=0.75,
                 carrier_hz=60e9, smooth_radius=0.0, edges=None, edge_of=None) -> dict:
    """Exact paths from coarse ones (Section 2.3): gradient descent on the path
    length with re-tracing, then the dedup of refined paths.

    ``paths`` is a ``collect_paths`` result of a launch with these ``tx`` and
    ``rx`` in ``scene``.  Returns per input row: ``status`` (REFINE_*),
    ``iters``, ``grad``, ``length``, ``points`` [n, K, 3], ``point_id`` and
    ``key`` [n, K], ``kept`` (the unique exact paths), plus ``n_kept``.
    ``carrier_hz < 0`` skips the Fresnel-zone step.  ``smooth_radius > 0``
    takes the surface normal at each point as the weighted average of the
    normals within that radius (between the surfel radius and the leaf edge).
    ``edges`` = dict(seg [E, 2, 3], normals [E, 2, 3], label [E]) with
    ``edge_of`` [n, K] (edge of each interaction, -1 for a reflection) makes
    the interactions at edges diffractions (D_k = c_k + t_k w_k).
    """
    device = scene.device
    txt = _as_tensor(tx, torch.float32, device, 3)
    rxt = _as_tensor(rx, torch.float32, device, 3)
    n = int(paths["n_rows"])
    K = int(paths["points"].shape[1]) if paths["points"].dim() == 3 else 0
    res, out = _refine_outputs(n, K, device)
    pp = _refine_rows(paths, n, device, ("tx", "rx", "n_refl", "points"))
    prm = _refine_params(max_iters, grad_tol, step, carrier_hz, smooth_radius)
    keep = []
    if edge_of is not None:
        eo = _as_tensor(np.asarray(edge_of, np.int32).reshape(n, K) if isinstance(edge_of, np.ndarray) else edge_of,
                        torch.int32, device).reshape(-1).contiguous()
        seg = _as_tensor(edges["seg"], torch.float32, device).reshape(-1, 6).contiguous()
        nrm = _as_tensor(edges["normals"], torch.float32, device).reshape(-1, 6).contiguous()
        lab = edges["label"]
        if isinstance(lab, np.ndarray):
            lab = torch.from_numpy(np.ascontiguousarray(lab.astype(np.uint32)).view(np.int32))
        lab = _as_tensor(lab, torch.int32, device).contiguous()
        keep = [eo, seg, nrm, lab]
        prm.edge_of = eo.data_ptr() if eo.numel() else None
        prm.n_edges = int(seg.shape[0])
        prm.edge_seg, prm.edge_normals, prm.edge_label = seg.data_ptr(), nrm.data_ptr(), lab.data_ptr()
    with _on(device):
        check("refine_paths", lib.refine_paths(scene.handle, _ptr(txt), txt.shape[0], _ptr(rxt), rxt.shape[0],
                                               C.byref(pp), K, C.byref(prm), C.byref(out), _stream(device)))
    del keep
    res["n_kept"] = int(out.n_kept)
    return res


def refine_cone_paths(launch: "ConeLaunch", paths: dict, max_iters=2000, grad_tol=1e-4, step=0.75,
                      carrier_hz=60e9, smooth_radius=0.0) -> dict:
    """Refine the rows of a ``cone_collect`` result of ``launch`` (Section 2.3):
    interactions at edge pieces are diffractions on their edges.  Returns as
    ``refine_paths``."""
    device = launch.device
    n = int(paths["n_rows"])
    K = launch.K
    res, out = _refine_outputs(n, K, device)
    pp = _refine_rows(paths, n, device, ("tx", "rx", "n_refl", "ray", "points"))
    prm = _refine_params(max_iters, grad_tol, step, carrier_hz, smooth_radius)
    with _on(device):
        check("refine_cone_paths", lib.refine_cone_paths(launch.handle, C.byref(pp), C.byref(prm), C.byref(out),
                                                         _stream(device)))
    res["n_kept"] = int(out.n_kept)
    return res


def sdf_intersect(scene: Scene, o, d, t_range=None, h=0.0, eps=0.0, max_steps=0, with_stats=False) -> dict:
    """First intersection of each ray with the implicit surface of Eq. 1
    (Section 2.2.1): signed distances f(x) = (x - p(x)) . n(x) of weighted
    neighbourhood averages, marched along line segments through the occupied
    leaves the ray crosses.

    ``o`` and ``d`` are [n, 3] origins and directions, ``t_range`` an optional
    [n, 2] (t_lo, t_hi).  ``h`` (neighbourhood radius), ``eps`` (near-zero
    threshold) and ``max_steps`` (evaluations per leaf) select the defaults
    0.95 and 1e-3 leaf edges and 64 when not positive.  Returns ``t`` (+inf
    for none), ``point``, ``normal`` and ``leaf_cell`` (-1 for none); with
    ``with_stats`` also ``evals`` and ``reads`` (evaluations of f and leaf
    entries read, summed over the rays).
    """
    device = scene.device
    ot = _as_tensor(o, torch.float32, device, 3)
    dt = _as_tensor(d, torch.float32, device, 3)
    if ot.shape != dt.shape:
        raise ValueError("o and d must have the same shape")
    n = ot.shape[0]
    tr = None if t_range is None else _as_tensor(t_range, torch.float32, device, 2)
    if tr is not None and tr.shape[0] != n:
        raise ValueError("t_range must have one row per ray")
    res = {
        "t": torch.empty(n, dtype=torch.float32, device=device),
        "point": torch.empty((n, 3), dtype=torch.float32, device=device),
        "normal": torch.empty((n, 3), dtype=torch.float32, device=device),
        "leaf_cell": torch.empty((n, 3), dtype=torch.int32, device=device),
    }
    stats = torch.zeros(2, dtype=torch.int64, device=device) if with_stats else None
    prm = _lib.PcrlSdfParams(float(h), float(eps), int(max_steps), 0, _ptr(stats) if with_stats else None)
    with _on(device):
        check("sdf_intersect", lib.sdf_intersect(scene.handle, _ptr(ot), _ptr(dt), _ptr(tr) if tr is not None
                                                 else None, n, C.byref(prm), _ptr(res["t"]), _ptr(res["point"]),
                                                 _ptr(res["normal"]), _ptr(res["leaf_cell"]), _stream(device)))
    if with_stats:
        st = stats.cpu()
        res["evals"], res["reads"] = int(st[0]), int(st[1])
    return res


class IeTable:
    """The intersectable entities of a scene on a voxel grid (owns a PcrlIes handle)."""

    def __init__(self, handle, scene, grid):
        self._h = handle
        self.scene = scene
        self.device = scene.device
        self.grid = grid

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _lib.PcrlIeInfo()
        check("ie_info", lib.ie_info(self._h, C.byref(inf)))
        return {name: getattr(inf, name) for name, _ in inf._fields_}

    def table(self) -> dict:
        n = self.info()["n_ies"]
        dev = self.device
        out = {"key": torch.empty(max(n, 1), dtype=torch.int64, device=dev),
               "sub": torch.empty((max(n, 1), 3), dtype=torch.int32, device=dev),
               "label": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
               "count": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
               "pos": torch.empty((max(n, 1), 3), dtype=torch.float32, device=dev),
               "nrm": torch.empty((max(n, 1), 3), dtype=torch.float32, device=dev)}
        with _on(dev):
            check("ie_table", lib.ie_table(self._h, *[_ptr(out[k]) for k in ("key", "sub", "label", "count", "pos",
                                                                               "nrm")], _stream(dev)))
        return {k: v[:n] for k, v in out.items()}

    def add_edges(self, seg, normals, label):
        """Diffraction edges: segments [n, 2, 3], the outward normals of their two
        faces [n, 2, 3] and labels [n] (ie_add_edges)."""
        dev = self.device
        segt = _as_tensor(seg, torch.float32, dev).reshape(-1, 6).contiguous()
        nrmt = _as_tensor(normals, torch.float32, dev).reshape(-1, 6).contiguous()
        if isinstance(label, np.ndarray):
            label = torch.from_numpy(np.ascontiguousarray(label.astype(np.uint32)).view(np.int32))
        labt = _as_tensor(label, torch.int32, dev)
        n = segt.shape[0]
        if nrmt.shape[0] != n or labt.shape[0] != n:
            raise ValueError("seg, normals and label must have the same length")
        with _on(dev):
            check("ie_add_edges", lib.ie_add_edges(self._h, _ptr(segt) if n else None, _ptr(nrmt) if n else None,
                                                   _ptr(labt) if n else None, n, _stream(dev)))
        self._edges = (segt, nrmt, labt)

    def release(self):
        if self._h:
            lib.release_ies(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def ie_build(scene: Scene, origin, voxel, dv, dims) -> IeTable:
    """Intersectable entities (Section 2.1): the scene's static points grouped
    by (subvoxel, label) on the grid of ``dims`` voxels of edge ``voxel`` from
    ``origin``, each voxel divided into ``dv``^3 subvoxels."""
    g = _lib.PcrlIeGrid()
    for a in range(3):
        g.origin[a] = float(origin[a])
        g.dims[a] = int(dims[a])
    g.voxel = float(voxel)
    g.dv = int(dv)
    h = C.c_void_p()
    with _on(scene.device):
        check("ie_build", lib.ie_build(scene.handle, C.byref(g), _stream(scene.device), C.byref(h)))
    return IeTable(h, scene, dict(origin=tuple(float(x) for x in origin), voxel=float(voxel), dv=int(dv),
                                  dims=tuple(int(x) for x in dims)))


class ConeLaunch:
    """One query of the environment-driven cone tracer (owns a PcrlConeLaunch handle)."""

    def __init__(self, handle, ies, K, inputs):
        self._h = handle
        self.ies = ies
        self.device = ies.device
        self.K = K
        self._inputs = inputs

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        st = _lib.PcrlConeStats()
        check("cone_stats", lib.cone_stats(self._h, C.byref(st)))
        out = {}
        for name, _ in st._fields_:
            v = getattr(st, name)
            out[name] = list(v)[: self.K + 1] if hasattr(v, "__len__") else v
        return out

    def nodes(self, k) -> dict:
        n = self.stats()["nodes"][k]
        dev = self.device
        out = {"ie": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
               "parent": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
               "tx": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
               "prio": torch.empty(max(n, 1), dtype=torch.int64, device=dev),
               "length": torch.empty(max(n, 1), dtype=torch.float32, device=dev)}
        if n:
            with _on(dev):
                check("cone_nodes", lib.cone_nodes(self._h, int(k), *[_ptr(out[f]) for f in ("ie", "parent", "tx",
                                                                                             "prio", "length")],
                                                   _stream(dev)))
        return {f: v[:n] for f, v in out.items()}

    def release(self):
        if self._h:
            lib.release_cone(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def cone_launch(ies: IeTable, tx, rx, max_interactions, half_angle=0.0, max_diffractions=0) -> ConeLaunch:
    """Environment-driven coarse tracing with conical rays (Sections 2.2.2-2.2.4);
    with ``max_diffractions`` > 0 the table's edge pieces diffract (Keller-cone sectors)."""
    dev = ies.device
    txt = _as_tensor(tx, torch.float32, dev, 3)
    rxt = _as_tensor(np.zeros((0, 3), np.float32) if rx is None else rx, torch.float32, dev, 3)
    p = _lib.PcrlConeParams(int(max_interactions), float(half_angle), 0, int(max_diffractions))
    h = C.c_void_p()
    with _on(dev):
        check("cone_launch", lib.cone_launch(ies.handle, _ptr(txt), txt.shape[0],
                                             _ptr(rxt) if rxt.shape[0] else None, rxt.shape[0], C.byref(p),
                                             _stream(dev), C.byref(h)))
    return ConeLaunch(h, ies, int(max_interactions), (txt, rxt))


def cone_collect(launch: ConeLaunch, kappa=100, capacity=None) -> dict:
    """Coarse paths of a cone launch: per (tx, rx, n, labels) the count and the
    kappa rows of smallest priority (Section 2.2.3)."""
    dev = launch.device
    K = max(launch.K, 1)
    cap = int(capacity) if capacity is not None else 4096
    for _ in range(2):
        bufs = {
            "tx": torch.empty(cap, dtype=torch.int32, device=dev),
            "rx": torch.empty(cap, dtype=torch.int32, device=dev),
            "n_refl": torch.empty(cap, dtype=torch.int32, device=dev),
            "key": torch.empty(max(cap * K, 1), dtype=torch.int64, device=dev),
            "count": torch.empty(cap, dtype=torch.int64, device=dev),
            "rank": torch.empty(cap, dtype=torch.int32, device=dev),
            "ray": torch.empty(cap, dtype=torch.int64, device=dev),
            "len_poly": torch.empty(cap, dtype=torch.float32, device=dev),
            "len_unf": torch.empty(cap, dtype=torch.float32, device=dev),
            "points": torch.empty(max(cap * K * 3, 1), dtype=torch.float32, device=dev),
        }
        out = _lib.PcrlPaths()
        out.capacity = cap
        for k, t in bufs.items():
            setattr(out, k, t.data_ptr())
        with _on(dev):
            st = lib.cone_collect(launch.handle, int(kappa), C.byref(out), _stream(dev))
        if st == PCRL_EOVERFLOW:
            cap = int(out.n_rows)
            continue
        check("cone_collect", st)
        n = int(out.n_rows)
        res = {k: (t[: n * K].view(n, K) if k == "key" else t[: n * K * 3].view(n, K, 3) if k == "points"
                   else t[:n]) for k, t in bufs.items()}
        res["n_rows"] = n
        res["n_keys"] = int(out.n_keys)
        return res
    raise PcrlError("cone_collect", PCRL_EOVERFLOW, "capacity retry failed")


def _relaunch(launch: Launch, record_capacity: int):
    a = dict(launch._args)
    a["record_capacity"] = record_capacity
    new = launch_rays(launch.scene, a.pop("tx"), a.pop("rx"), **a)
    launch.release()
    launch._h, new._h = new._h, None
    launch.hit_log = new.hit_log
    launch._args = new._args


def _served_params(n_rays, max_reflections, record_capacity=0, coherent=True):
    p = _lib.PcrlLaunchParams()
    p.n_rays = int(n_rays)
    p.max_reflections = int(max_reflections)
    p.record_capacity = int(record_capacity)
    p.flags = LAUNCH_COHERENT if coherent else 0
    return p


def serve_query_bytes(n_tx, n_rx, n_rays, max_reflections, record_capacity=0, coherent=True) -> int:
    """Device bytes a Server charges a query of these arguments (as Server.submit
    takes them) against its memory budget (serve_query_bytes of the C ABI; no
    device call)."""
    p = _served_params(n_rays, max_reflections, record_capacity, coherent)
    b = C.c_int64()
    check("serve_query_bytes", lib.serve_query_bytes(int(n_tx), int(n_rx), C.byref(p), C.byref(b)))
    return b.value


class Server:
    """Request loop over one device-resident, incrementally re-voxelised scene (serve_* of the C ABI).

    ``submit`` queues a TX/RX query (host arrays) and returns a ticket at once;
    a native worker thread admits queries by memory budget and free slots,
    packs them into batched launches on several streams (continuous batching)
    and copies each result to host memory.  ``update`` replaces the dynamic
    points (a new scene epoch).
    """

    def __init__(self, scene: Scene, max_inflight=256, n_streams=4, hbm_budget_bytes=0, max_batch=64, kappa=1,
                 key_mode=KEY_LABELS, tile_rays=0, compact_threshold=-1.0, waves_per_cu=0, use_graph=False,
                 autotune=False):
        self.scene = scene
        self.device = scene.device
        p = _lib.PcrlServeParams()
        p.max_inflight = int(max_inflight)
        p.n_streams = int(n_streams)
        p.hbm_budget_bytes = int(hbm_budget_bytes)
        p.max_batch = int(max_batch)
        p.kappa = int(kappa)
        p.key_mode = int(key_mode)
        p.batch = _batch_params(tile_rays, compact_threshold, waves_per_cu, use_graph, autotune)
        self._h = C.c_void_p()
        self._K = {}
        with torch.cuda.device(self.device):
            check("serve_create", lib.serve_create(scene.handle, C.byref(p), C.byref(self._h)))

    def submit(self, tx, rx, n_rays, max_reflections, record_capacity=0, coherent=True) -> int:
        tx = np.ascontiguousarray(np.asarray(tx, np.float32).reshape(-1, 3))
        rx = np.ascontiguousarray(np.asarray(rx, np.float32).reshape(-1, 3)) if rx is not None else \
            np.zeros((0, 3), np.float32)
        p = _served_params(n_rays, max_reflections, record_capacity, coherent)
        t = C.c_int64()
        check("serve_submit", lib.serve_submit(self._h, tx.ctypes.data, tx.shape[0],
                                               rx.ctypes.data if rx.shape[0] else None, rx.shape[0], C.byref(p),
                                               C.byref(t)))
        self._K[t.value] = int(max_reflections)
        return t.value

    def update(self, ids, xyz, normal, label):
        """Frame update: replace the dynamic points (device tensors or numpy arrays)."""
        ids = _as_tensor(np.asarray(ids, np.int64).astype(np.uint32).view(np.int32)
                         if isinstance(ids, np.ndarray) else ids, torch.int32, self.device)
        xyz = _as_tensor(xyz, torch.float32, self.device, 3)
        normal = _as_tensor(normal, torch.float32, self.device, 3)
        if isinstance(label, np.ndarray):
            label = torch.from_numpy(np.ascontiguousarray(label.astype(np.uint32)).view(np.int32))
        label = _as_tensor(label, torch.int32, self.device)
        torch.cuda.current_stream(self.device).synchronize()
        n = xyz.shape[0]
        with torch.cuda.device(self.device):
            check("serve_update", lib.serve_update(self._h, _ptr(ids) if n else None, _ptr(xyz) if n else None,
                                                   _ptr(normal) if n else None, _ptr(label) if n else None, n))

    def poll(self, ticket, timeout=0.0) -> dict:
        r = _lib.PcrlServeResult()
        check("serve_poll", lib.serve_poll(self._h, int(ticket), float(timeout), C.byref(r)))
        return {name: getattr(r, name) for name, _ in r._fields_ if name != "reserved"}

    def result(self, ticket) -> dict:
        info = self.poll(ticket)
        if info["status"] != 2:
            raise PcrlError("serve_result", -1, f"ticket {ticket} is not finished (status {info['status']})")
        n, K = info["n_rows"], self._K[int(ticket)]
        out = {"tx": np.empty(n, np.int32), "rx": np.empty(n, np.int32), "n_refl": np.empty(n, np.int32),
               "key": np.empty((n, K), np.int64), "count": np.empty(n, np.int64), "rank": np.empty(n, np.int32),
               "ray": np.empty(n, np.int64), "len_poly": np.empty(n, np.float32), "len_unf": np.empty(n, np.float32),
               "points": np.empty((n, K, 3), np.float32)}
        P = _lib.PcrlPaths()
        P.capacity = n
        for k, a in out.items():
            setattr(P, k, a.ctypes.data if a.size else None)
        check("serve_result", lib.serve_result(self._h, int(ticket), C.byref(P)))
        out["n_rows"] = n
        out["n_keys"] = info["n_keys"]
        out["epoch"] = info["epoch"]
        return out

    def cancel(self, ticket):
        """Cancel a pending or running query (its poll then reports PCRL_ECANCELED)."""
        check("serve_cancel", lib.serve_cancel(self._h, int(ticket)))

    def release(self, ticket):
        check("serve_release", lib.serve_release(self._h, int(ticket)))
        self._K.pop(int(ticket), None)

    def stats(self) -> dict:
        s = _lib.PcrlServeStats()
        check("serve_stats", lib.serve_stats(self._h, C.byref(s)))
        return {name: getattr(s, name) for name, _ in s._fields_ if name != "reserved"}

    def close(self):
        if self._h:
            lib.serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass
