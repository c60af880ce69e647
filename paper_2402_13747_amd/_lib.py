"""ctypes binding of libpcrl.so (include/pcrl.h).

Argument marshalling only: every step of the path runs in the HIP library.
torch is imported first so that the library binds to the HIP runtime torch
already loaded (both carry the soname libamdhip64.so.7); torch supplies
device memory and the stream.  There is no CPU fallback: importing this
module without a built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (must precede the library load)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcrl.so")

PCRL_OK = 0
PCRL_EINVAL = -1
PCRL_ENOMEM = -2
PCRL_EOVERFLOW = -3
PCRL_EHIP = -4
PCRL_EBUSY = -5
PCRL_ECANCELED = -6
MAX_LEVELS = 4
MAX_REFLECTIONS = 8

LAUNCH_STATS = 1
LAUNCH_TIMING = 2
LAUNCH_COHERENT = 4
LAUNCH_SDF = 8
VOXEL_COMPACT = 1
KEY_LABELS = 0
KEY_LEAVES = 1
REFINE_VALID = 0
REFINE_NOT_CONVERGED = 1
REFINE_MISS = 2
REFINE_WRONG_SIDE = 3
REFINE_OCCLUDED = 4
REFINE_DEGENERATE = 5
REFINE_OFF_EDGE = 6
REFINE_SMOOTH = 1

STATUS_NAMES = {0: "PCRL_OK", -1: "PCRL_EINVAL", -2: "PCRL_ENOMEM", -3: "PCRL_EOVERFLOW", -4: "PCRL_EHIP",
                -5: "PCRL_EBUSY", -6: "PCRL_ECANCELED"}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class PcrlAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class PcrlVoxelParams(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("level_size", C.c_float * MAX_LEVELS), ("surfel_radius", C.c_float),
                ("t_eps", C.c_float), ("flags", C.c_int32)]


class PcrlSceneInfo(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("n_entries", C.c_int64), ("n_leaves", C.c_int64),
                ("n_nodes", C.c_int64 * MAX_LEVELS), ("max_label", C.c_int32), ("n_levels", C.c_int32),
                ("dims", C.c_int32 * 3), ("dims0", C.c_int32 * 3), ("origin", C.c_float * 3),
                ("leaf_size", C.c_float), ("surfel_radius", C.c_float), ("t_eps", C.c_float),
                ("aabb", C.c_float * 6), ("device_bytes", C.c_int64), ("key_bits", C.c_int32),
                ("reserved", C.c_int32), ("n_dynamic", C.c_int64), ("epoch", C.c_int64)]


class PcrlLaunchParams(C.Structure):
    _fields_ = [("n_rays", C.c_int64), ("directions", C.c_void_p), ("max_reflections", C.c_int32),
                ("rx_radius_scale", C.c_float), ("ray_spacing", C.c_float), ("record_capacity", C.c_int64),
                ("flags", C.c_int32), ("reserved", C.c_int32), ("hit_log_id", C.c_void_p),
                ("hit_log_t", C.c_void_p)]


class PcrlLaunchStats(C.Structure):
    _fields_ = [("rays", C.c_int64), ("segments", C.c_int64), ("active", C.c_int64 * (MAX_REFLECTIONS + 1)),
                ("records", C.c_int64), ("record_capacity", C.c_int64), ("dda_steps", C.c_int64),
                ("leaves_visited", C.c_int64), ("node_lookups", C.c_int64), ("surfel_tests", C.c_int64),
                ("hits", C.c_int64), ("algo_bytes", C.c_int64), ("empty_leaf_steps", C.c_int64),
                ("uniform_leaf_visits", C.c_int64), ("wave_dda_iters", C.c_int64), ("wave_test_iters", C.c_int64),
                ("algo_bytes_bounce", C.c_int64 * (MAX_REFLECTIONS + 1)),
                ("dda_steps_bounce", C.c_int64 * (MAX_REFLECTIONS + 1)),
                ("surfel_tests_bounce", C.c_int64 * (MAX_REFLECTIONS + 1)),
                ("wave_dda_bounce", C.c_int64 * (MAX_REFLECTIONS + 1)),
                ("kernel_ms", C.c_float * (MAX_REFLECTIONS + 1)),
                ("total_ms", C.c_float)]


class PcrlPaths(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("n_rows", C.c_int64), ("n_keys", C.c_int64), ("tx", C.c_void_p),
                ("rx", C.c_void_p), ("n_refl", C.c_void_p), ("key", C.c_void_p), ("count", C.c_void_p),
                ("rank", C.c_void_p), ("ray", C.c_void_p), ("len_poly", C.c_void_p), ("len_unf", C.c_void_p),
                ("points", C.c_void_p)]


class PcrlRefineParams(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("grad_tol", C.c_float), ("step", C.c_float), ("carrier_hz", C.c_float),
                ("flags", C.c_int32), ("smooth_radius", C.c_float), ("edge_of", C.c_void_p), ("n_edges", C.c_int32),
                ("edge_seg", C.c_void_p), ("edge_normals", C.c_void_p), ("edge_label", C.c_void_p)]


class PcrlRefined(C.Structure):
    _fields_ = [("n_kept", C.c_int64), ("status", C.c_void_p), ("iters", C.c_void_p), ("grad", C.c_void_p),
                ("length", C.c_void_p), ("points", C.c_void_p), ("point_id", C.c_void_p), ("key", C.c_void_p),
                ("kept", C.c_void_p)]


class PcrlSdfParams(C.Structure):
    _fields_ = [("h", C.c_float), ("eps", C.c_float), ("max_steps", C.c_int32), ("flags", C.c_int32),
                ("stats", C.c_void_p)]


class PcrlQuery(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("tx", C.c_void_p), ("n_tx", C.c_int32), ("n_rx", C.c_int32),
                ("rx", C.c_void_p), ("params", PcrlLaunchParams)]


class PcrlBatchParams(C.Structure):
    _fields_ = [("tile_rays", C.c_int32), ("compact_threshold", C.c_float), ("waves_per_cu", C.c_int32),
                ("use_graph", C.c_int32), ("autotune", C.c_int32), ("flags", C.c_int32)]


class PcrlServeParams(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("n_streams", C.c_int32), ("hbm_budget_bytes", C.c_int64),
                ("max_batch", C.c_int32), ("kappa", C.c_int32), ("key_mode", C.c_int32), ("reserved", C.c_int32),
                ("batch", PcrlBatchParams)]


class PcrlServeResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("epoch", C.c_int64), ("n_rows", C.c_int64),
                ("n_keys", C.c_int64), ("queue_ms", C.c_double), ("latency_ms", C.c_double)]


class PcrlServeStats(C.Structure):
    _fields_ = [("completed", C.c_int64), ("pending", C.c_int64), ("inflight", C.c_int32), ("reserved", C.c_int32),
                ("rounds", C.c_int64), ("mean_batch", C.c_double), ("rays", C.c_int64), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("max_ms", C.c_double), ("mean_ms", C.c_double), ("rays_per_s", C.c_double),
                ("used_bytes", C.c_int64)]


class PcrlIeGrid(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("voxel", C.c_float), ("dv", C.c_int32), ("dims", C.c_int32 * 3)]


class PcrlIeInfo(C.Structure):
    _fields_ = [("n_ies", C.c_int64), ("n_edge_ies", C.c_int64), ("n_voxels", C.c_int64), ("n_occupied", C.c_int64),
                ("device_bytes", C.c_int64)]


class PcrlConeParams(C.Structure):
    _fields_ = [("max_interactions", C.c_int32), ("half_angle", C.c_float), ("flags", C.c_int32),
                ("max_diffractions", C.c_int32)]


class PcrlConeStats(C.Structure):
    _fields_ = [("nodes", C.c_int64 * (MAX_REFLECTIONS + 1)), ("cones", C.c_int64 * (MAX_REFLECTIONS + 1)),
                ("candidates", C.c_int64 * (MAX_REFLECTIONS + 1)),
                ("visible", C.c_int64 * (MAX_REFLECTIONS + 1)), ("records", C.c_int64),
                ("ms_transmission", C.c_double), ("ms_propagation", C.c_double)]


# name -> (restype, argtypes); every symbol declared in include/pcrl.h
SIGNATURES = {
    "set_allocator": (C.c_int, [C.POINTER(PcrlAllocator)]),
    "build_voxels": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(PcrlVoxelParams),
                               C.c_void_p, C.POINTER(C.c_void_p)]),
    "scene_info": (C.c_int, [C.c_void_p, C.POINTER(PcrlSceneInfo)]),
    "update_points": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "scene_leaf_table": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "release_scene": (C.c_int, [C.c_void_p]),
    "launch_rays": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                              C.POINTER(PcrlLaunchParams), C.c_void_p, C.POINTER(C.c_void_p)]),
    "launch_directions": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p]),
    "launch_stats": (C.c_int, [C.c_void_p, C.POINTER(PcrlLaunchStats)]),
    "launch_records": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.POINTER(C.c_int64)]),
    "release_launch": (C.c_int, [C.c_void_p]),
    "collect_paths": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(PcrlPaths), C.c_void_p]),
    "collect_paths_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(PcrlPaths), C.c_void_p]),
    "refine_paths": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(PcrlPaths),
                               C.c_int32, C.POINTER(PcrlRefineParams), C.POINTER(PcrlRefined), C.c_void_p]),
    "sdf_intersect": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                C.POINTER(PcrlSdfParams), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p]),
    "launch_batch": (C.c_int, [C.POINTER(PcrlQuery), C.c_int32, C.POINTER(PcrlBatchParams), C.c_void_p,
                               C.POINTER(C.c_void_p)]),
    "batch_autotune": (C.c_int, [C.POINTER(PcrlQuery), C.c_int32, C.c_void_p, C.POINTER(PcrlBatchParams)]),
    "ie_build": (C.c_int, [C.c_void_p, C.POINTER(PcrlIeGrid), C.c_void_p, C.POINTER(C.c_void_p)]),
    "ie_add_edges": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "ie_info": (C.c_int, [C.c_void_p, C.POINTER(PcrlIeInfo)]),
    "ie_table": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_void_p]),
    "release_ies": (C.c_int, [C.c_void_p]),
    "cone_launch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(PcrlConeParams),
                              C.c_void_p, C.POINTER(C.c_void_p)]),
    "cone_stats": (C.c_int, [C.c_void_p, C.POINTER(PcrlConeStats)]),
    "cone_nodes": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p]),
    "cone_collect": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(PcrlPaths), C.c_void_p]),
    "refine_cone_paths": (C.c_int, [C.c_void_p, C.POINTER(PcrlPaths), C.POINTER(PcrlRefineParams),
                                    C.POINTER(PcrlRefined), C.c_void_p]),
    "release_cone": (C.c_int, [C.c_void_p]),
    "serve_create": (C.c_int, [C.c_void_p, C.POINTER(PcrlServeParams), C.POINTER(C.c_void_p)]),
    "serve_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(PcrlLaunchParams),
                               C.POINTER(C.c_int64)]),
    "serve_query_bytes": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(PcrlLaunchParams), C.POINTER(C.c_int64)]),
    "serve_update": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "serve_poll": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.POINTER(PcrlServeResult)]),
    "serve_result": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(PcrlPaths)]),
    "serve_cancel": (C.c_int, [C.c_void_p, C.c_int64]),
    "serve_release": (C.c_int, [C.c_void_p, C.c_int64]),
    "serve_stats": (C.c_int, [C.c_void_p, C.POINTER(PcrlServeStats)]),
    "serve_destroy": (C.c_int, [C.c_void_p]),
    "last_error": (C.c_char_p, []),
    "pcrl_version": (C.c_char_p, []),
}


class PcrlError(RuntimeError):
    def __init__(self, fn, status, message):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2402_13747_amd.build.build() "
                          "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(fn, status):
    if status != PCRL_OK:
        msg = lib.last_error()
        raise PcrlError(fn, status, msg.decode() if msg else "")
    return status
