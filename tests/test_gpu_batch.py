"""Batched launching: every query's result equals its solo launch, bitwise.

Queries differ in scene (room, canyon, random planes; 1-3 voxel levels), ray
count (ragged, not multiples of the tile), K, TX and RX counts.  The batch is
run under several tile sizes, compaction thresholds (always in place, mixed,
always compacted), occupancies, in graph mode (replayed several times with
eager work in between) and with the autotuner.
"""
import numpy as np
import pytest

import scenes
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2402_13747_amd as pcrl
    return torch, pcrl


@pytest.fixture(scope="module")
def workload(env):
    torch, pcrl = env
    specs = [
        scenes.furnished_room(n_points=60_000, seed=2, n_rx=5, n_rays=20_000, K=3),
        scenes.street_canyon(n_points=80_000, seed=3, n_tx=2, n_rx=7, n_rays=9_999, K=2, scale=0.06,
                             levels=(0.48, 0.06, 0.03)),
        scenes.random_scene(21, tilt_sigma=0.05, n_rays=3_001, n_tx=1, n_rx=3, K=4),
        scenes.box_room(n_rays=5_000, K=2),
        scenes.random_scene(22, pos_sigma=0.004, n_rays=777, n_tx=3, n_rx=1, K=1, levels=(0.25,)),
        scenes.furnished_room(n_points=30_000, seed=4, n_rx=2, n_rays=12_345, K=0),
    ]
    built = []
    for s in specs:
        print(f"[batch] scene {s.name}: {s.n_points} pts, {s.n_rays} rays x {len(s.tx)} tx, K={s.max_reflections}",
              flush=True)
        sc = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, float(np.float32(s.surfel_radius)),
                               t_eps=float(np.float32(parity.t_eps_of(s))))
        built.append((s, sc))
    queries = [dict(scene=sc, tx=s.tx, rx=s.rx, n_rays=s.n_rays, max_reflections=s.max_reflections, hit_log=True)
               for s, sc in built]
    solo = []
    for q in queries:
        L = pcrl.launch_rays(**q)
        solo.append(_result(pcrl, L))
    return queries, solo


def _result(pcrl, L):
    p = parity.to_numpy(pcrl.collect_paths(L, kappa=1 << 30))
    return {"paths": p, "hits": L.hit_log[0].cpu().numpy(), "t": L.hit_log[1].cpu().numpy(),
            "active": L.stats()["active"]}


def _same(a, b):
    for k, v in a["paths"].items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, b["paths"][k], equal_nan=True), k
        else:
            assert v == b["paths"][k], k
    assert np.array_equal(a["hits"], b["hits"])
    assert np.array_equal(a["t"], b["t"], equal_nan=True)
    assert a["active"] == b["active"]


@pytest.mark.parametrize("tile,theta,waves", [(64, 0.0, 4), (256, 0.6, 16), (1024, 2.0, 8), (4096, 0.9, 32),
                                              (192, 0.6, 1)])
def test_batch_equals_solo(env, workload, tile, theta, waves):
    torch, pcrl = env
    queries, solo = workload
    print(f"[batch] tile={tile} theta={theta} waves={waves}", flush=True)
    launches = pcrl.launch_batch(queries, tile_rays=tile, compact_threshold=theta, waves_per_cu=waves)
    for L, ref in zip(launches, solo):
        _same(_result(pcrl, L), ref)


def test_batch_graph_replays(env, workload):
    torch, pcrl = env
    queries, solo = workload
    for rep in range(3):
        print(f"[batch] graph replay {rep}", flush=True)
        launches = pcrl.launch_batch(queries, tile_rays=512, compact_threshold=0.6, waves_per_cu=16, use_graph=True)
        for L, ref in zip(launches, solo):
            _same(_result(pcrl, L), ref)
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert float((x * 0).sum()) == 0.0
        eager = pcrl.launch_rays(**queries[2])
        _same(_result(pcrl, eager), solo[2])


def test_batch_autotune(env, workload):
    torch, pcrl = env
    queries, solo = workload
    best = pcrl.batch_autotune(queries[:3])
    assert best["tile_rays"] in (256, 1024, 4096) and best["waves_per_cu"] in (8, 16, 32)
    launches = pcrl.launch_batch(queries, autotune=True)
    for L, ref in zip(launches, solo):
        _same(_result(pcrl, L), ref)


def test_batch_timing_and_stats(env, workload):
    torch, pcrl = env
    queries, solo = workload
    qs = [dict(q, timing=True, stats=True) for q in queries]
    launches = pcrl.launch_batch(qs, tile_rays=256)
    st = [L.stats() for L in launches]
    assert all(s["kernel_ms"][0] > 0 for s in st)
    assert all(s["segments"] == sum(s["active"]) for s in st)
    assert all(s["algo_bytes"] > 0 and sum(s["algo_bytes_bounce"]) == s["algo_bytes"] for s in st)
    for L, ref in zip(launches, solo):
        _same(_result(pcrl, L), ref)


def test_batch_errors(env, workload):
    torch, pcrl = env
    queries, _ = workload
    bad = dict(queries[0], max_reflections=9)
    with pytest.raises(pcrl.PcrlError) as e:
        pcrl.launch_batch([queries[1], bad])
    assert "query 1" in str(e.value)
