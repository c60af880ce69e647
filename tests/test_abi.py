"""The C-ABI library loads and exports every function include/pcrl.h declares (CPU only).

No compute call is made here: without a GPU the tests only check symbols,
struct layouts and argument validation paths that fail before any HIP call.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def _declared_functions():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([a-z_][a-z0-9_]*)\s*\(", src, re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def pcrl():
    import torch  # noqa: F401
    import paper_2402_13747_amd as p
    return p


def test_header_parses():
    names = _declared_functions()
    for must in ("build_voxels", "launch_rays", "collect_paths", "release_scene", "release_launch", "last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(pcrl):
    lib = C.CDLL(pcrl.library_path())
    missing = [n for n in sorted(_declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_header_constants_match_binding(pcrl):
    from paper_2402_13747_amd import _lib
    src = "".join(open(h).read() for h in HEADERS)
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(PCRL_[A-Z_]+)\s+(-?\d+)", src)}
    assert defs["PCRL_VOXEL_COMPACT"] == _lib.VOXEL_COMPACT
    assert defs["PCRL_LAUNCH_STATS"] == _lib.LAUNCH_STATS and defs["PCRL_LAUNCH_TIMING"] == _lib.LAUNCH_TIMING
    assert defs["PCRL_LAUNCH_COHERENT"] == _lib.LAUNCH_COHERENT
    assert defs["PCRL_KEY_LABELS"] == _lib.KEY_LABELS and defs["PCRL_KEY_LEAVES"] == _lib.KEY_LEAVES
    assert defs["PCRL_MAX_LEVELS"] == _lib.MAX_LEVELS and defs["PCRL_MAX_REFLECTIONS"] == _lib.MAX_REFLECTIONS
    for name in ("OK", "EINVAL", "ENOMEM", "EOVERFLOW", "EHIP", "EBUSY", "ECANCELED"):
        assert defs["PCRL_" + name] == getattr(_lib, "PCRL_" + name)
    for name in ("VALID", "NOT_CONVERGED", "MISS", "WRONG_SIDE", "OCCLUDED", "DEGENERATE", "SMOOTH"):
        assert defs["PCRL_REFINE_" + name] == getattr(_lib, "REFINE_" + name)


def test_binding_covers_header(pcrl):
    from paper_2402_13747_amd import _lib
    assert set(_lib.SIGNATURES) == _declared_functions()


def test_struct_sizes(pcrl):
    from paper_2402_13747_amd import _lib
    # sizes fixed by the header's field lists (natural alignment)
    assert C.sizeof(_lib.PcrlVoxelParams) == 32
    assert C.sizeof(_lib.PcrlLaunchParams) == 64
    assert C.sizeof(_lib.PcrlSceneInfo) == 168
    assert C.sizeof(_lib.PcrlPaths) == 13 * 8
    assert C.sizeof(_lib.PcrlRefineParams) == 64
    assert C.sizeof(_lib.PcrlRefined) == 9 * 8
    assert C.sizeof(_lib.PcrlSdfParams) == 24


def test_version_and_validation_without_gpu(pcrl):
    from paper_2402_13747_amd import _lib
    assert "gfx950" in pcrl.version()
    lib = _lib.lib
    out = C.c_void_p(123)
    # NULL params -> EINVAL before any device call
    assert lib.build_voxels(None, None, None, 0, None, None, C.byref(out)) == _lib.PCRL_EINVAL
    assert out.value is None
    assert b"params" in lib.last_error()
    p = _lib.PcrlVoxelParams()
    p.n_levels = 2
    p.level_size[0] = 0.5
    p.level_size[1] = 0.3          # 0.5 / 0.3 is not an integer
    p.surfel_radius = 0.1
    assert lib.build_voxels(None, None, None, 0, C.byref(p), None, C.byref(out)) == _lib.PCRL_EINVAL
    assert b"integer multiple" in lib.last_error()
    p.n_levels = 5
    assert lib.build_voxels(None, None, None, 0, C.byref(p), None, C.byref(out)) == _lib.PCRL_EINVAL
    p.n_levels = 1
    p.flags = 2                     # unknown flag
    assert lib.build_voxels(None, None, None, 0, C.byref(p), None, C.byref(out)) == _lib.PCRL_EINVAL
    assert b"flags" in lib.last_error()
    lp = _lib.PcrlLaunchParams()
    lp.n_rays = 10
    lp.max_reflections = 9          # K > 8
    assert lib.launch_rays(C.c_void_p(1), C.c_void_p(1), 1, None, 0, C.byref(lp), None, C.byref(out)) == \
        _lib.PCRL_EINVAL
    assert lib.collect_paths(None, 1, 0, None, None) == _lib.PCRL_EINVAL
    ro = _lib.PcrlRefined()
    assert lib.refine_paths(None, None, 0, None, 0, None, 0, None, C.byref(ro), None) == _lib.PCRL_EINVAL
    assert b"refine_paths" in lib.last_error()
    assert lib.sdf_intersect(None, None, None, None, 1, None, None, None, None, None, None) == _lib.PCRL_EINVAL
    assert b"sdf_intersect" in lib.last_error()
    # the implicit-surface launch is launch_rays' only: batches refuse it before touching a scene
    q = _lib.PcrlQuery()
    q.scene = 1
    q.params.flags = _lib.LAUNCH_SDF
    outs = (C.c_void_p * 1)()
    assert lib.launch_batch(C.byref(q), 1, None, None, outs) == _lib.PCRL_EINVAL
    assert b"PCRL_LAUNCH_SDF" in lib.last_error()
    assert lib.release_scene(None) == 0 and lib.release_launch(None) == 0
    # the library's own allocator is the default and can always be restored
    assert lib.set_allocator(None) == _lib.PCRL_OK
    half = _lib.PcrlAllocator()
    half.alloc = _lib.ALLOC_FN(lambda n, s, c: None)
    assert lib.set_allocator(C.byref(half)) == _lib.PCRL_EINVAL
    assert b"alloc and free" in lib.last_error()


def test_every_entry_point_refuses_null_handles_without_a_device(pcrl):
    """NULL handles and arrays are refused with PCRL_EINVAL and a message naming
    the entry point, before any device call; releasing NULL is a no-op."""
    from paper_2402_13747_amd import _lib
    L, N = _lib.lib, None
    calls = {
        "update_points": lambda: L.update_points(N, N, N, N, N, 1, N),
        "scene_info": lambda: L.scene_info(N, N),
        "scene_leaf_table": lambda: L.scene_leaf_table(N, N, N, N, N, N),
        "launch_stats": lambda: L.launch_stats(N, N),
        "launch_records": lambda: L.launch_records(N, 0, N, N, N, N, N, N),
        "launch_batch": lambda: L.launch_batch(N, 0, N, N, N),
        "batch_autotune": lambda: L.batch_autotune(N, 0, N, N),
        "launch_directions": lambda: L.launch_directions(0, N, N),
        "collect_paths_noalloc": lambda: L.collect_paths_noalloc(N, 1, 0, N, N),
        "ie_build": lambda: L.ie_build(N, N, N, N),
        "ie_add_edges": lambda: L.ie_add_edges(N, N, N, N, 1, N),
        "ie_info": lambda: L.ie_info(N, N),
        "ie_table": lambda: L.ie_table(N, N, N, N, N, N, N, N),
        "cone_launch": lambda: L.cone_launch(N, N, 1, N, 0, N, N, N),
        "cone_stats": lambda: L.cone_stats(N, N),
        "cone_nodes": lambda: L.cone_nodes(N, 0, N, N, N, N, N, N),
        "cone_collect": lambda: L.cone_collect(N, 1, N, N),
        "refine_cone_paths": lambda: L.refine_cone_paths(N, N, N, N, N),
        "serve_create": lambda: L.serve_create(N, N, N),
        "serve_submit": lambda: L.serve_submit(N, N, 1, N, 0, N, N),
        "serve_update": lambda: L.serve_update(N, N, N, N, N, 1),
        "serve_poll": lambda: L.serve_poll(N, 1, 0.0, N),
        "serve_result": lambda: L.serve_result(N, 1, N),
        "serve_cancel": lambda: L.serve_cancel(N, 1),
        "serve_release": lambda: L.serve_release(N, 1),
        "serve_stats": lambda: L.serve_stats(N, N),
    }
    for name, call in calls.items():
        assert call() == _lib.PCRL_EINVAL, name
        assert L.last_error().decode().startswith(name + ":"), (name, L.last_error())
    for name in ("release_scene", "release_launch", "release_ies", "release_cone", "serve_destroy"):
        assert getattr(L, name)(N) == _lib.PCRL_OK, name


def test_no_cpu_fallback(tmp_path, monkeypatch):
    """Without the built library the binding refuses to import."""
    import importlib
    import sys
    from paper_2402_13747_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib._load()
    assert "paper_2402_13747_amd" in sys.modules
    importlib.invalidate_caches()


STRUCTS = ["PcrlAllocator", "PcrlVoxelParams", "PcrlSceneInfo", "PcrlLaunchParams", "PcrlLaunchStats", "PcrlQuery",
           "PcrlBatchParams", "PcrlPaths", "PcrlRefineParams", "PcrlRefined", "PcrlSdfParams", "PcrlIeGrid",
           "PcrlIeInfo", "PcrlConeParams", "PcrlConeStats", "PcrlServeParams", "PcrlServeResult", "PcrlServeStats"]


def test_binding_structs_match_the_header(pcrl, tmp_path):
    """Every struct of include/pcrl.h, compiled by the host C compiler, has the
    size and field offsets of its ctypes twin."""
    import shutil
    import subprocess
    from paper_2402_13747_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pcrl.h"', "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for f in getattr(_lib, name)._fields_:
            lines.append(f'    printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        name, field, value = line.split()
        cls = getattr(_lib, name)
        want = C.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(value) == want, (name, field, int(value), want)
