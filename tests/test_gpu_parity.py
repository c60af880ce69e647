"""GPU parity: the HIP path against the FP64 CPU oracle, through the C ABI.

Scenes: the empty box room (full size), random tilted planes and boxes with
noise (several seeds, 1-3 voxel levels, ragged ray counts), and the furnished
room at full size with a sampled set of rays.  The comparison rule is in
tests/parity.py.
"""
import math

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
    import oracle
    import paper_2402_13747_amd as pcrl
    oracle.build(force=False)
    return torch, pcrl, oracle


def _f32(x):
    return float(np.float32(x))


def _run(env, s, n_rays, K, sel=None, levels=None, hit_log=True, directions=None, kappa=1 << 30, n_threads=None,
         coherent=True):
    torch, pcrl, oracle = env
    t_eps = _f32(parity.t_eps_of(s))
    r_s = _f32(s.surfel_radius)
    print(f"[parity] {s.name}: {s.n_points} pts, {n_rays} rays x {len(s.tx)} tx, K={K}, levels={levels or s.levels}",
          flush=True)
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, levels or s.levels, r_s, t_eps=t_eps)
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=n_rays, max_reflections=K, hit_log=hit_log,
                              directions=directions, coherent=coherent)
    paths = parity.to_numpy(pcrl.collect_paths(launch, kappa=kappa))
    rec = parity.to_numpy(launch.records())
    ids = launch.hit_log[0].cpu().numpy() if hit_log else None
    dirs = oracle.fibonacci(n_rays) if directions is None else np.asarray(directions, np.float32)
    orc = oracle.launch(s.xyz, s.normal, s.label, s.tx, s.rx, dirs, K=K, r_s=r_s, t_eps=t_eps, sel=sel, parity=True,
                        n_threads=n_threads, **parity.fp32_bands(s.xyz, s.tx, s.rx))
    return scene, launch, paths, rec, ids, orc


def _reception_rich_sample(oracle, s, n_rays, n_rx, radius, n_random, planes=None):
    """Ray ids aimed (within radius * alpha) at the first n_rx RX and at their mirror
    images in the room's six walls, plus n_random random rays.  Pure geometry:
    independent of both the oracle's and the device's tracing."""
    d = oracle.fibonacci(n_rays).astype(np.float64)
    alpha = oracle.ray_spacing(n_rays)
    tx = s.tx[0].astype(np.float64)
    size = s.extra.get("size", (12.0, 10.0, 3.0))
    targets = []
    for r in s.rx[:n_rx].astype(np.float64):
        targets.append(r)
        for axis in range(3):
            for c in (0.0, size[axis]):
                m = r.copy()
                m[axis] = 2 * c - m[axis]
                targets.append(m)
    pick = set()
    for t in targets:
        u = (t - tx) / np.linalg.norm(t - tx)
        pick.update(np.nonzero(d @ u > math.cos(radius * alpha))[0].tolist())
    rng = np.random.default_rng(3)
    pick.update(rng.choice(n_rays, size=n_random, replace=False).tolist())
    return np.array(sorted(pick), np.int64)


def test_street_canyon_full_size_sampled(env):
    """Street canyon at full size (20M points, 4 x 4M rays, K = 4, 64 RX, three levels); ~80 sampled rays of
    the first TX (aimed at 8 RX and at their ground images, plus random ones) against the oracle."""
    torch, pcrl, oracle = env
    s = scenes.street_canyon()
    n_rays, K = s.n_rays, s.max_reflections
    d = oracle.fibonacci(n_rays).astype(np.float64)
    alpha = oracle.ray_spacing(n_rays)
    tx = s.tx[0].astype(np.float64)
    pick = set()
    for r in s.rx[:8].astype(np.float64):
        for tgt in (r, r * np.array([1.0, 1.0, -1.0])):
            u = (tgt - tx) / np.linalg.norm(tgt - tx)
            pick.update(np.nonzero(d @ u > math.cos(1.0 * alpha))[0].tolist())
    pick.update(np.random.default_rng(5).choice(n_rays, size=16, replace=False).tolist())
    sel = np.array(sorted(pick), np.int64)
    scene, launch, paths, rec, ids, orc = _run(env, s, n_rays, K, sel=sel)
    rep = parity.compare(orc, ids, rec, s.xyz, s.normal, s.label, K)
    print(rep.summary())
    assert rep.ok(), (rep.mismatch[:5], rep.record_missing[:5], rep.record_extra[:5], rep.length_bad[:5])
    assert rep.exact + rep.equivalent >= 0.95 * rep.segments
    assert rep.records_checked >= 3        # most RX are hidden from this TX by buildings
    st = launch.stats()
    assert st["records"] <= st["record_capacity"] and st["rays"] == 4 * n_rays


def test_directions_match_oracle(env):
    torch, pcrl, oracle = env
    for n in (1, 7, 10_000, 1_000_003):
        d = pcrl.launch_directions(n).cpu().numpy()
        ref = oracle.fibonacci(n)
        assert parity.fp32_direction_ulps(d, ref) <= 1.0
        assert np.mean(np.all(d == ref, axis=1)) > 0.999


@pytest.mark.parametrize("levels", [(1.0, 0.1), (0.5,), (2.5, 0.1)])
def test_axis_aligned_directions(env, levels):
    """Caller directions with zero components (axes, face and body diagonals) and near-axis ones, traced
    through the cell table, a single-level grid and the brick masks, match the brute-force oracle."""
    torch, pcrl, oracle = env
    s = scenes.random_scene(31, tilt_sigma=0.0, pos_sigma=0.0, n_tx=2, n_rx=4)
    dirs = []
    for x in (-1, 0, 1):
        for y in (-1, 0, 1):
            for z in (-1, 0, 1):
                if (x, y, z) != (0, 0, 0):
                    dirs.append((x, y, z))
    rng = np.random.default_rng(3)
    d = np.asarray(dirs, np.float64)
    near = d[rng.integers(0, len(d), 200)] + rng.normal(0, 1e-6, (200, 3))  # tiny instead of zero components
    d = np.concatenate([d, near, rng.normal(size=(300, 3))])
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    scene, launch, paths, rec, ids, orc = _run(env, s, len(d), 3, levels=levels, directions=d)
    rep = parity.compare(orc, ids, rec, s.xyz, s.normal, s.label, 3)
    print(rep.summary())
    assert rep.ok(), (rep.mismatch[:5], rep.record_missing[:5], rep.record_extra[:5], rep.length_bad[:5])
    assert rep.exact + rep.equivalent >= 0.97 * rep.segments


def test_leaf_table_properties(env):
    """Every entry's leaf lies in its disk's box; every leaf holding a point of a disk lists it; order is stable."""
    torch, pcrl, oracle = env
    s = scenes.random_scene(11, tilt_sigma=0.1, pos_sigma=0.01, h=0.2)
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, (0.8, 0.4, 0.2), s.surfel_radius)
    inf = scene.info()
    key, begin, count, ids = (t.cpu().numpy() for t in scene.leaf_table())
    assert inf["n_leaves"] == len(key) and inf["n_entries"] == len(ids)
    assert np.all(np.diff(key.astype(np.uint64)) > 0)                 # sorted, unique
    assert begin[0] == 0 and np.all(begin[1:] == begin[:-1] + count[:-1]) and begin[-1] + count[-1] == len(ids)
    assert np.all(count > 0)
    # decode the hierarchical key back to leaf coordinates
    dims0 = inf["dims0"]
    ratios = [2, 2]
    bits = [max(1, int(np.ceil(np.log2(max(r ** 3, 2))))) for r in ratios]
    h = inf["leaf_size"]
    org = np.array(inf["origin"], np.float64)
    leaf_xyz = np.zeros((len(key), 3), np.int64)
    k = key.astype(np.uint64)
    spans = [4, 2, 1]
    loc2 = (k & np.uint64((1 << bits[1]) - 1)).astype(np.int64)
    loc1 = ((k >> np.uint64(bits[1])) & np.uint64((1 << bits[0]) - 1)).astype(np.int64)
    lin0 = (k >> np.uint64(bits[0] + bits[1])).astype(np.int64)
    c0 = np.stack([lin0 % dims0[0], (lin0 // dims0[0]) % dims0[1], lin0 // (dims0[0] * dims0[1])], 1)
    l1 = np.stack([loc1 % 2, (loc1 // 2) % 2, loc1 // 4], 1)
    l2 = np.stack([loc2 % 2, (loc2 // 2) % 2, loc2 // 4], 1)
    leaf_xyz = c0 * spans[0] + l1 * spans[1] + l2
    p = s.xyz.astype(np.float64)
    n = s.normal.astype(np.float64)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    ext = s.surfel_radius * np.sqrt(np.maximum(0.0, 1.0 - n * n))
    lo = np.floor((p - ext - org) / h).astype(np.int64)
    hi = np.floor((p + ext - org) / h).astype(np.int64)
    entry_leaf = np.repeat(np.arange(len(key)), count)
    # soundness: the leaf of every entry lies within the point's disk box (+-1 for the rounding pad)
    lc = leaf_xyz[entry_leaf]
    assert np.all(lc >= lo[ids] - 1) and np.all(lc <= hi[ids] + 1)
    # completeness: every leaf that holds a point of the disk lists the point (the disk is sampled on
    # rings out to its rim; samples within 1e-5 h of a leaf face are skipped as ambiguous)
    listed = set(zip(ids.tolist(), map(tuple, lc.tolist())))
    r_s = float(np.float32(s.surfel_radius))
    ang = np.linspace(0, 2 * np.pi, 24, endpoint=False)
    n_checked = 0
    for i in range(0, len(p), 7):
        a = np.cross(n[i], [1.0, 0.0, 0.0] if abs(n[i, 0]) < 0.9 else [0.0, 1.0, 0.0])
        a /= np.linalg.norm(a)
        b = np.cross(n[i], a)
        for rr in (0.0, 0.4, 0.8, 0.999):
            q = p[i] + rr * r_s * (np.cos(ang)[:, None] * a + np.sin(ang)[:, None] * b)
            f = (q - org) / h
            ok = np.all(np.abs(f - np.round(f)) > 1e-5, axis=1)
            for cell in np.floor(f[ok]).astype(np.int64):
                assert (i, tuple(cell.tolist())) in listed
                n_checked += 1
    assert n_checked > 1000
    # stability: point ids ascend within each leaf
    for a, c in zip(begin[:200], count[:200]):
        assert np.all(np.diff(ids[a:a + c]) > 0)


def test_box_room_full_parity(env):
    """Empty box room, 10k Fibonacci rays, K = 2: hits, records, lengths and the 25 coarse paths."""
    torch, pcrl, oracle = env
    s = scenes.box_room()
    scene, launch, paths, rec, ids, orc = _run(env, s, s.n_rays, 2)
    rep = parity.compare(orc, ids, rec, s.xyz, s.normal, s.label, 2)
    print(rep.summary())
    assert rep.ok(), (rep.mismatch[:5], rep.record_missing[:5], rep.record_extra[:5], rep.length_bad[:5])
    assert rep.exact + rep.equivalent >= 0.99 * rep.segments
    dev = parity.device_paths(paths)
    _, keys, amb = oracle.dedup(orc, 2)
    assert set(k[3] for k in dev) == set(k[3] for k in keys)
    assert len(dev) == 25
    # LOS closed form
    los = dev[(0, 0, 0, ())]
    assert all(abs(r["len_poly"] - math.sqrt(34.0)) <= 1e-6 * math.sqrt(34.0) for r in los)


@pytest.mark.parametrize("seed,levels,n_rays,K,coherent", [
    (1, None, 3000, 3, True), (2, (0.25,), 2500, 2, False), (3, (1.0, 0.25), 4099, 3, True),
    (4, None, 1531, 4, False), (5, (0.5, 0.25), 777, 1, True), (6, (1.25, 0.25), 2048, 3, True),
    (8, (2.0, 1.0, 0.5, 0.25), 3001, 2, True),
])
def test_random_scene_parity(env, seed, levels, n_rays, K, coherent):
    torch, pcrl, oracle = env
    s = scenes.random_scene(seed, tilt_sigma=0.05 * (seed % 3), pos_sigma=0.003 * (seed % 2), n_tx=2, n_rx=4)
    scene, launch, paths, rec, ids, orc = _run(env, s, n_rays, K, levels=levels, coherent=coherent)
    rep = parity.compare(orc, ids, rec, s.xyz, s.normal, s.label, K)
    print(rep.summary())
    assert rep.ok(), (rep.mismatch[:5], rep.record_missing[:5], rep.record_extra[:5], rep.length_bad[:5])
    assert rep.exact + rep.equivalent >= 0.97 * rep.segments
    # coarse-path keys: every oracle key carried by a live unambiguous record is found
    dev = parity.device_paths(paths)
    _, keys, _ = oracle.dedup(orc, K)
    sel = orc["sel"]
    for q in range(orc["n_rec"]):
        g = int(orc["rec_g"][q])
        b = int(orc["rec_b"][q])
        if orc["rec_flags"][q] != 1 or (g in rep.diverged and b >= rep.diverged[g]):
            continue
        r = int(orc["rec_sel"][q])
        key = (int(orc["rec_tx"][q]), int(orc["rec_rx"][q]), b, tuple(int(x) for x in orc["seq"][r, :b]))
        assert key in dev


@pytest.mark.parametrize("seed", [11, 12])
def test_traversal_variants_agree(env, seed):
    """The dense cell table with octant skips, the compact brick masks with isotropic skip radii and a
    parent ratio above 16 (masks only) give bitwise the same hits and paths, and match the oracle."""
    torch, pcrl, oracle = env
    s = scenes.random_scene(seed, tilt_sigma=0.03, pos_sigma=0.002, n_tx=2, n_rx=4)
    t_eps, r_s = _f32(parity.t_eps_of(s)), _f32(s.surfel_radius)
    runs = []
    for levels, compact in (((1.0, 0.1), False), ((1.0, 0.1), True), ((2.5, 0.1), False), ((0.5,), False)):
        scene = pcrl.build_voxels(s.xyz, s.normal, s.label, levels, r_s, t_eps=t_eps, compact=compact)
        L = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=4000, max_reflections=3, hit_log=True)
        runs.append((L.hit_log[0].cpu().numpy(), L.hit_log[1].cpu().numpy(),
                     parity.to_numpy(pcrl.collect_paths(L, kappa=1 << 30))))
    h0, t0, p0 = runs[0]
    for h, t, p in runs[1:]:
        assert np.array_equal(h, h0) and np.array_equal(t, t0, equal_nan=True)
        for k in ("tx", "rx", "n_refl", "key", "count", "rank", "ray", "len_poly", "len_unf"):
            assert np.array_equal(np.asarray(p[k]), np.asarray(p0[k])), k
    scene, launch, paths, rec, ids, orc = _run(env, s, 4000, 3, levels=(1.0, 0.1))
    rep = parity.compare(orc, ids, rec, s.xyz, s.normal, s.label, 3)
    print(rep.summary())
    assert rep.ok()


def test_kappa_and_counts(env):
    torch, pcrl, oracle = env
    s = scenes.box_room()
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, _f32(s.surfel_radius), t_eps=_f32(parity.t_eps_of(s)))
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=s.n_rays, max_reflections=2)
    full = parity.device_paths(parity.to_numpy(pcrl.collect_paths(launch, kappa=1 << 30)))
    for kappa in (1, 2, 3):
        got = parity.device_paths(parity.to_numpy(pcrl.collect_paths(launch, kappa=kappa)))
        assert set(got) == set(full)
        for key, rows in got.items():
            allr = full[key]
            assert len(rows) == min(kappa, len(allr))
            assert [r["ray"] for r in rows] == [r["ray"] for r in allr[:kappa]]
            assert all(r["count"] == len(allr) for r in rows)
            assert [r["rank"] for r in rows] == list(range(len(rows)))
            lp = [(r["len_poly"], r["ray"]) for r in allr]
            assert lp == sorted(lp)


def test_stats_per_bounce(env):
    """The statistics pass reports the same paths as a plain launch and splits its counters by bounce."""
    torch, pcrl, oracle = env
    s = scenes.box_room()
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, _f32(s.surfel_radius), t_eps=_f32(parity.t_eps_of(s)))
    plain = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=s.n_rays, max_reflections=3)
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=s.n_rays, max_reflections=3, stats=True, timing=True)
    st = launch.stats()
    a = parity.device_paths(parity.to_numpy(pcrl.collect_paths(plain)))
    b = parity.device_paths(parity.to_numpy(pcrl.collect_paths(launch)))
    assert set(a) == set(b)
    assert len(st["algo_bytes_bounce"]) == 4 and sum(st["algo_bytes_bounce"]) == st["algo_bytes"]
    for k in range(4):
        assert (st["algo_bytes_bounce"][k] > 0) == (st["active"][k] > 0)
        assert st["kernel_ms"][k] > 0
    # every segment reads at least the level-0 map cell it starts in
    assert st["algo_bytes"] >= 4 * st["segments"]
    assert st["hits"] <= st["segments"] and st["leaves_visited"] <= st["dda_steps"]


def test_coherence_order_invariance(env):
    """Large launches trace their bounces in re-sorted coherent orders; results equal the plain order's."""
    torch, pcrl, oracle = env
    s = scenes.furnished_room(n_points=200_000, seed=7, n_rx=6, n_rays=150_000, K=3)
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, _f32(s.surfel_radius), t_eps=_f32(parity.t_eps_of(s)))
    runs = []
    for coherent in (True, False):
        L = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=s.n_rays, max_reflections=3, coherent=coherent, hit_log=True)
        p = parity.to_numpy(pcrl.collect_paths(L, kappa=1 << 30))
        runs.append((L.hit_log[0].cpu().numpy(), L.hit_log[1].cpu().numpy(), p, L.stats()["active"]))
    (h1, t1, p1, a1), (h2, t2, p2, a2) = runs
    assert a1 == a2 and a1[3] > 0
    assert np.array_equal(h1, h2) and np.array_equal(t1, t2, equal_nan=True)
    for k in ("tx", "rx", "n_refl", "key", "count", "rank", "ray", "len_poly", "len_unf", "points"):
        assert np.array_equal(np.asarray(p1[k]), np.asarray(p2[k]), equal_nan=True), k


def test_determinism_and_permutation(env):
    torch, pcrl, oracle = env
    s = scenes.random_scene(7, tilt_sigma=0.05, n_rays=4000)
    args = (s.levels, _f32(s.surfel_radius))
    outs = []
    for _ in range(2):
        scene = pcrl.build_voxels(s.xyz, s.normal, s.label, *args)
        launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=4000, max_reflections=3)
        outs.append(parity.to_numpy(pcrl.collect_paths(launch, kappa=4)))
    for k in outs[0]:
        if isinstance(outs[0][k], np.ndarray):
            assert np.array_equal(outs[0][k], outs[1][k], equal_nan=True), k
    perm = np.random.default_rng(0).permutation(s.n_points)
    scene = pcrl.build_voxels(s.xyz[perm], s.normal[perm], s.label[perm], *args)
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=4000, max_reflections=3)
    p2 = parity.device_paths(parity.to_numpy(pcrl.collect_paths(launch, kappa=4)))
    p1 = parity.device_paths(outs[0])
    # label paths are invariant to point order up to tie breaks between coincident surfels
    common = set(p1) & set(p2)
    assert len(common) >= 0.95 * max(len(p1), len(p2))


def test_translation_invariance(env):
    # a box room on a dyadic grid (0.25 m cells, centres at 0.125 + 0.25 k) moved by an
    # exactly representable offset: the same coarse paths with the same counts, and
    # lengths equal up to FP32 rounding of the larger coordinates
    torch, pcrl, oracle = env
    off = np.array([16.0, 32.0, 8.0], np.float32)
    res = []
    for shift in (np.zeros(3, np.float32), off):
        s = scenes.box_room(h=0.25, tx=tuple(np.array([2.0, 2.0, 1.5]) + shift),
                            rx=tuple(np.array([7.0, 5.0, 1.5]) + shift))
        xyz = (s.xyz + shift).astype(np.float32)
        assert np.array_equal(xyz - shift, s.xyz)       # the move is exact
        scene = pcrl.build_voxels(xyz, s.normal, s.label, s.levels, _f32(s.surfel_radius), t_eps=1e-4)
        launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=10_000, max_reflections=2)
        res.append(parity.device_paths(parity.to_numpy(pcrl.collect_paths(launch, kappa=1))))
    a, b = res
    assert set(a) == set(b) and len(a) == 25
    for key in a:
        assert a[key][0]["count"] == b[key][0]["count"], key
        assert abs(a[key][0]["len_poly"] - b[key][0]["len_poly"]) <= 1e-5 * a[key][0]["len_poly"], key


def test_edge_cases(env):
    torch, pcrl, oracle = env
    z = np.zeros((0, 3), np.float32)
    scene = pcrl.build_voxels(z, z, np.zeros(0, np.uint32), (0.5, 0.25), 0.1, t_eps=1e-5)
    launch = pcrl.launch_rays(scene, [[0, 0, 0]], [[3, 0, 0]], n_rays=2000, max_reflections=2)
    p = parity.to_numpy(pcrl.collect_paths(launch))
    assert p["n_keys"] == 1 and p["n_refl"][0] == 0 and abs(p["len_poly"][0] - 3.0) < 1e-6
    st = launch.stats()
    assert st["active"][1] == 0
    s = scenes.box_room()
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, 0.15)
    launch = pcrl.launch_rays(scene, s.tx, np.zeros((0, 3), np.float32), n_rays=1000, max_reflections=2)
    assert pcrl.collect_paths(launch)["n_rows"] == 0
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=1000, max_reflections=0)
    p = parity.to_numpy(pcrl.collect_paths(launch))
    assert set(p["n_refl"].tolist()) <= {0}
    bad = s.xyz.copy()
    bad[5, 1] = np.nan
    with pytest.raises(pcrl.PcrlError) as e:
        pcrl.build_voxels(bad, s.normal, s.label, s.levels, 0.15)
    assert e.value.status == -1
    nb = s.normal.copy()
    nb[9] = 0
    with pytest.raises(pcrl.PcrlError):
        pcrl.build_voxels(s.xyz, nb, s.label, s.levels, 0.15)
    # record overflow is reported and the binding relaunches with the needed capacity
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=s.n_rays, max_reflections=2, record_capacity=3)
    with pytest.raises(pcrl.PcrlError):
        launch.records()
    p = parity.to_numpy(pcrl.collect_paths(launch))
    assert p["n_keys"] == 25


def test_furnished_room_full_size_sampled(env):
    """Furnished room at full size (1M points, 1M rays, K = 3, 16 RX); ~650 sampled rays against the oracle."""
    torch, pcrl, oracle = env
    s = scenes.furnished_room()
    n_rays, K = s.n_rays, s.max_reflections
    sel = _reception_rich_sample(oracle, s, n_rays, n_rx=16, radius=1.2, n_random=64)
    scene, launch, paths, rec, ids, orc = _run(env, s, n_rays, K, sel=sel)
    rep = parity.compare(orc, ids, rec, s.xyz, s.normal, s.label, K)
    print(rep.summary())
    assert rep.ok(), (rep.mismatch[:5], rep.record_missing[:5], rep.record_extra[:5], rep.length_bad[:5])
    assert rep.exact + rep.equivalent >= 0.95 * rep.segments
    assert rep.records_checked >= 15
    st = launch.stats()
    assert st["records"] <= st["record_capacity"]
