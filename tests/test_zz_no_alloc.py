"""collect_paths_noalloc: the rows of collect_paths without any allocation.

Through the C ABI: the same launch is collected by collect_paths and by
collect_paths_noalloc into separate caller buffers, and every output array
must be bitwise equal.  Two calls in a row, the second on a smaller launch,
so that the fixed scratch array holds the first call's data when the second
starts.  A counting allocator installed with set_allocator must see no
allocation during the no-allocation calls.
"""
import ctypes as C

import numpy as np
import pytest

import scenes
from tests import parity

pytestmark = pytest.mark.gpu

FIELDS = ("tx", "rx", "n_refl", "key", "count", "rank", "ray", "len_poly", "len_unf", "points")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2402_13747_amd as pcrl
    from paper_2402_13747_amd import _lib
    return torch, pcrl, _lib


def _buffers(torch, cap, K):
    dev = torch.device("cuda", torch.cuda.current_device())
    return {
        "tx": torch.full((cap,), -7, dtype=torch.int32, device=dev),
        "rx": torch.full((cap,), -7, dtype=torch.int32, device=dev),
        "n_refl": torch.full((cap,), -7, dtype=torch.int32, device=dev),
        "key": torch.full((max(cap * K, 1),), -7, dtype=torch.int64, device=dev),
        "count": torch.full((cap,), -7, dtype=torch.int64, device=dev),
        "rank": torch.full((cap,), -7, dtype=torch.int32, device=dev),
        "ray": torch.full((cap,), -7, dtype=torch.int64, device=dev),
        "len_poly": torch.full((cap,), -7.0, dtype=torch.float32, device=dev),
        "len_unf": torch.full((cap,), -7.0, dtype=torch.float32, device=dev),
        "points": torch.full((max(cap * K * 3, 1),), -7.0, dtype=torch.float32, device=dev),
    }


def _collect(torch, _lib, fn, launch, kappa, cap):
    K = launch.K
    bufs = _buffers(torch, cap, K)
    out = _lib.PcrlPaths()
    out.capacity = cap
    for k, t in bufs.items():
        setattr(out, k, t.data_ptr())
    torch.cuda.synchronize()
    st = fn(launch.handle, int(kappa), 0, C.byref(out), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, (st, _lib.lib.last_error().decode())
    torch.cuda.synchronize()
    n = int(out.n_rows)
    res = {k: t.cpu().numpy() for k, t in bufs.items()}
    return n, int(out.n_keys), res


class _Counting:
    """set_allocator callbacks that count calls and delegate to torch."""

    def __init__(self, torch, _lib):
        self.n = 0
        self.torch = torch

        def _alloc(nbytes, stream, ctx):
            self.n += 1
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))

        def _free(ptr, stream, ctx):
            self.n += 1
            torch.cuda.caching_allocator_delete(int(ptr))

        self.a = _lib.PcrlAllocator(_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free), None)


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_collect_equals_collect(env, order):
    torch, pcrl, _lib = env
    lib = _lib.lib
    s = scenes.box_room()
    t_eps = float(np.float32(parity.t_eps_of(s)))
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, float(np.float32(s.surfel_radius)), t_eps=t_eps)
    rng = np.random.default_rng(7)
    rx = (rng.uniform((0.5, 0.5, 0.5), (9.5, 7.5, 2.5), (8, 3))).astype(np.float32)
    # first a launch with well over 2048 records (the sorting path: wide
    # reception spheres, 8 RX), then one with fewer (the one-workgroup path),
    # then a mid-sized one
    cases = [(200_000, 2, 4, 6.0), (3_000, 2, 1, 1.25), (60_000, 3, 2, 3.0)]
    for n_rays, K, kappa, sigma in cases:
        print(f"[noalloc] box room, 8 RX, {n_rays} rays, K={K}, kappa={kappa}, sigma={sigma}", flush=True)
        launch = pcrl.launch_rays(scene, s.tx, rx, n_rays=n_rays, max_reflections=K, rx_radius_scale=sigma)
        n_rec = launch.stats()["records"]
        cap = max(int(n_rec), 16)
        n0, k0, r0 = _collect(torch, _lib, lib.collect_paths, launch, kappa, cap)
        counter = _Counting(torch, _lib)
        assert lib.set_allocator(C.byref(counter.a)) == 0
        try:
            n1, k1, r1 = _collect(torch, _lib, lib.collect_paths_noalloc, launch, kappa, cap)
        finally:
            assert lib.set_allocator(None) == 0
        assert counter.n == 0, f"{counter.n} allocator calls during collect_paths_noalloc"
        print(f"[noalloc] records={n_rec} rows={n0} keys={k0}", flush=True)
        assert (n0, k0) == (n1, k1)
        for f in FIELDS:
            a, b = r0[f], r1[f]
            assert np.array_equal(a, b, equal_nan=True), f
        launch.release()
    scene.release()


def test_noalloc_refuses_more_records_than_its_scratch(env):
    """A launch whose records need more than the fixed array is refused before any work."""
    torch, pcrl, _lib = env
    lib = _lib.lib
    s = scenes.box_room()
    t_eps = float(np.float32(parity.t_eps_of(s)))
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, float(np.float32(s.surfel_radius)), t_eps=t_eps)
    # 64 RX with reception spheres 32x the default radius: about 3M records,
    # beyond the 64 MiB array
    rng = np.random.default_rng(8)
    rx = (rng.uniform((0.5, 0.5, 0.5), (9.5, 7.5, 2.5), (64, 3))).astype(np.float32)
    launch = pcrl.launch_rays(scene, s.tx, rx, n_rays=100_000, max_reflections=2, rx_radius_scale=40.0,
                              record_capacity=8_000_000)
    n_rec = int(launch.stats()["records"])
    print(f"[noalloc] refusal case: {n_rec} records", flush=True)
    assert n_rec > 1_300_000
    out = _lib.PcrlPaths()
    out.capacity = 0
    st = lib.collect_paths_noalloc(launch.handle, 1, 0, C.byref(out),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.PCRL_EINVAL
    assert b"scratch" in lib.last_error()
    launch.release()
    scene.release()
