"""set_allocator: the library's device memory from torch's caching allocator.

The same build + launch + collect + refine gives bitwise the same results
with either allocator, torch's allocator holds the scene's memory while the
scene lives, and objects made under one allocator are released correctly
after switching back.
"""
import numpy as np
import pytest

import scenes
from tests import parity

pytestmark = pytest.mark.gpu


def _run(pcrl, s):
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, float(np.float32(s.surfel_radius)),
                              t_eps=float(np.float32(parity.t_eps_of(s))))
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=20_000, max_reflections=2)
    P = pcrl.collect_paths(launch, kappa=3)
    R = pcrl.refine_paths(scene, s.tx, s.rx, P)
    return scene, launch, parity.to_numpy(P), parity.to_numpy(R)


def test_torch_allocator_gives_the_same_results():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2402_13747_amd as pcrl
    s = scenes.box_room()
    print("[alloc] library allocator", flush=True)
    sc0, l0, p0, r0 = _run(pcrl, s)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    try:
        pcrl.use_torch_allocator(True)
        print("[alloc] torch allocator", flush=True)
        sc1, l1, p1, r1 = _run(pcrl, s)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - before
        # the scene and the launch live in torch's pool (at least the surfel streams: 32 B per entry)
        assert held >= 32 * sc1.info()["n_entries"], held
    finally:
        pcrl.use_torch_allocator(False)
    for k in ("tx", "rx", "n_refl", "key", "count", "rank", "ray", "len_poly", "len_unf"):
        assert np.array_equal(p0[k], p1[k]), k
    assert np.array_equal(p0["points"], p1["points"], equal_nan=True)
    for k in ("status", "iters", "point_id", "key", "kept"):
        assert np.array_equal(r0[k], r1[k]), k
    # blocks made by torch's allocator go back to it after the switch
    l1.release()
    sc1.release()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + (1 << 20)
    l0.release()
    sc0.release()
