"""GPU intersection with the implicit surface of Eq. 1 (sdf_intersect) against
the FP64 oracle, through the C ABI.

Both sides march the same segments (the leaves' point sets are taken in FP32
on both), so a ray's intersection is the oracle's up to the rounding of the
march.  Bar, per ray whose oracle answer is stable (unchanged, within the
tolerance below, when h, eps, the segment length and the leaf-crossing test
are perturbed by a few units of rounding, and max_steps by one):
  * hit or miss as the oracle;
  * |t - t_ref| <= 2 eps / max(|d . n|, 0.05) + 4e-6 (1 + |o| + t): both stop
    once |f| <= eps, i.e. within eps / |d . n| before the zero along the
    ray, so they may stop one step apart; FP32 positions add ~1e-6
    relative;
  * the normal within 0.05 (n(x) at points that far apart differs by about
    |dx| / h); the leaf cell is one whose segment reaches the hit (the
    segments of neighbouring leaves overlap, and where several marches meet
    the same zero any of them may be named: the cell is not unique).
Unstable rays are excused (their count is bounded).  Scenes: the empty box
room (rays from the TX), random tilted planes and boxes with noise, the
furnished room and the street canyon at full size (samples of rays), plus
edge cases.
"""
import math

import numpy as np
import pytest

import scenes

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


def _build(env, s, levels=None):
    _, pcrl, _ = env
    lv = levels or s.levels
    print(f"[sdf] {s.name}: {s.n_points} pts, levels={lv}", flush=True)
    return pcrl.build_voxels(s.xyz, s.normal, s.label, lv, float(np.float32(s.surfel_radius)))


def _oracle(env, s, info, o, d, tr=None, **kw):
    _, _, oracle = env
    return oracle.sdf_intersect(s.xyz, s.normal, np.asarray(info["origin"], np.float32), info["leaf_size"], o, d,
                                trange=tr, **kw)


def _compare(env, s, scene, o, d, tr=None, h=None, eps=None, max_steps=None, max_excused=0.05):
    _, pcrl, oracle = env
    info = scene.info()
    leaf = float(info["leaf_size"])
    h = oracle.SDF_H_SCALE * leaf if h is None else h
    eps = oracle.SDF_EPS_SCALE * leaf if eps is None else eps
    ms = oracle.SDF_MAX_STEPS if max_steps is None else max_steps
    g = pcrl.sdf_intersect(scene, o, d, t_range=tr, h=h, eps=eps, max_steps=ms)
    gt = g["t"].cpu().numpy().astype(np.float64)
    gp = g["point"].cpu().numpy().astype(np.float64)
    gn = g["normal"].cpu().numpy().astype(np.float64)
    gc = g["leaf_cell"].cpu().numpy()
    ref = _oracle(env, s, info, o, d, tr, h=h, eps=eps, max_steps=ms)
    pa = _oracle(env, s, info, o, d, tr, h=h * (1 + 1e-4), eps=eps * (1 + 1e-2), max_steps=ms + 1,
                 diam_scale=1 + 1e-5, cross_margin=1e-5 * leaf)
    pb = _oracle(env, s, info, o, d, tr, h=h * (1 - 1e-4), eps=eps * (1 - 1e-2), max_steps=max(ms - 1, 1),
                 diam_scale=1 - 1e-5, cross_margin=-1e-5 * leaf)
    dd = np.asarray(d, np.float64)
    dd = dd / np.linalg.norm(dd, axis=1, keepdims=True)
    on = np.linalg.norm(np.asarray(o, np.float64), axis=1)
    rt = ref["t"]
    cos = np.abs((dd * ref["normal"]).sum(1))
    fin = np.isfinite(rt)
    tol = 2 * eps / np.maximum(cos, 0.05) + 4e-6 * (1 + on + np.where(fin, rt, 0.0))

    def agree(a, b):
        fa, fb = np.isfinite(a), np.isfinite(b)
        return (fa == fb) & (~fa | (np.abs(np.where(fa, a, 0) - np.where(fb, b, 0)) <= tol))

    stable = agree(pa["t"], rt) & agree(pb["t"], rt)
    ok = agree(gt, rt)
    bad = stable & ~ok
    n = len(rt)
    excused = int((~stable).sum())
    hits = stable & fin & np.isfinite(gt)
    n_err = np.linalg.norm(gn[hits] - ref["normal"][hits], axis=1)
    p_err = np.linalg.norm(gp[hits] - ref["point"][hits], axis=1)
    same_cell = (gc[hits] == ref["leaf_cell"][hits]).all(1)
    print(f"  rays={n} hits={int(fin.sum())} stable={int(stable.sum())} excused={excused} mismatch={int(bad.sum())} "
          f"max|dn|={n_err.max(initial=0):.2e} max|dp|={p_err.max(initial=0):.2e} "
          f"cell_agree={same_cell.mean() if len(same_cell) else 1:.4f}", flush=True)
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"ray {i}: gpu t={gt[i]!r} oracle t={rt[i]!r} tol={tol[i]:.3g} o={o[i]} d={d[i]}")
    assert excused <= max_excused * n + 2
    assert np.all(n_err <= 0.05)
    assert np.all(p_err <= tol[hits] + 1e-5 * (1 + on[hits]))
    if len(same_cell):
        # where two leaves' marches reach the same zero, either may be named:
        # the cell must at least be one whose segment reaches the hit
        lo = np.asarray(info["origin"], np.float64) + gc[hits] * leaf
        gap = np.linalg.norm(np.maximum(np.maximum(lo - gp[hits], gp[hits] - (lo + leaf)), 0.0), axis=1)
        assert np.all(gap <= 1.5 * math.sqrt(3.0) * leaf + 1e-6)
    # misses carry the documented empty outputs
    miss = ~np.isfinite(gt)
    assert np.all(np.isnan(gp[miss])) and np.all(gn[miss] == 0) and np.all(gc[miss] == -1)
    return fin, stable


def test_box_room_rays_from_tx(env):
    _, _, oracle = env
    s = scenes.box_room()
    scene = _build(env, s)
    d = oracle.fibonacci(3000)
    o = np.repeat(s.tx.astype(np.float32), len(d), axis=0)
    fin, _ = _compare(env, s, scene, o, d)
    assert fin.mean() > 0.99  # a closed room: every ray meets a wall


RANDOM_LEVELS = {1: (0.4, 0.2, 0.1), 2: (0.1,), 3: (0.4, 0.2, 0.1), 7: (0.8, 0.4, 0.2, 0.1)}


@pytest.mark.parametrize("seed", [1, 2, 3, 7])
def test_random_scenes(env, seed):
    """Hierarchies of 3, 1, 3 and 4 levels."""
    rng = np.random.default_rng(100 + seed)
    s = scenes.random_scene(seed, extent=2.0, h=0.05, levels=RANDOM_LEVELS[seed], pos_sigma=0.002, tilt_sigma=0.03)
    scene = _build(env, s)
    n = 2000
    o = rng.uniform(0.0, 2.0, size=(n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    fin, _ = _compare(env, s, scene, o, d)
    assert fin.sum() > 200


def test_ranges_and_parameters(env):
    rng = np.random.default_rng(7)
    s = scenes.random_scene(4, extent=2.0, h=0.05, levels=(0.4, 0.2), pos_sigma=0.002, tilt_sigma=0.03)
    scene = _build(env, s)
    n = 1500
    o = rng.uniform(0.0, 2.0, size=(n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    t_lo = rng.uniform(0.0, 0.5, size=n)
    tr = np.column_stack([t_lo, t_lo + rng.uniform(0.0, 1.5, size=n)]).astype(np.float32)
    _compare(env, s, scene, o, d, tr=tr)
    # a smaller neighbourhood, a tighter threshold and a short budget
    _compare(env, s, scene, o, d, h=0.12, eps=2e-5, max_steps=12, max_excused=0.08)


def test_furnished_room_full_size_sampled(env):
    torch, pcrl, oracle = env
    s = scenes.furnished_room()
    scene = _build(env, s)
    rng = np.random.default_rng(5)
    d = oracle.fibonacci(1_000_000)[rng.choice(1_000_000, 400, replace=False)]
    o = np.repeat(s.tx[:1].astype(np.float32), len(d), axis=0)
    fin, _ = _compare(env, s, scene, o, d)
    assert fin.mean() > 0.95
    # the full launch-sized batch runs and reports its work
    dd = torch.from_numpy(oracle.fibonacci(1_000_000)).cuda()
    oo = torch.from_numpy(s.tx[:1].astype(np.float32)).cuda().expand(1_000_000, 3).contiguous()
    r = pcrl.sdf_intersect(scene, oo, dd, with_stats=True)
    torch.cuda.synchronize()
    sel = torch.from_numpy(rng.choice(1_000_000, 400, replace=False)).cuda()
    assert torch.equal(r["t"][sel].cpu(), pcrl.sdf_intersect(scene, oo[sel], dd[sel])["t"].cpu())
    assert r["evals"] > 1_000_000 and r["reads"] > r["evals"]


def test_street_canyon_full_size_sampled(env):
    """Three-level hierarchy over 20 M points (no dense cell table): 200
    directions from the four TXs against the oracle."""
    _, _, oracle = env
    s = scenes.street_canyon()
    scene = _build(env, s)
    rng = np.random.default_rng(9)
    d = oracle.fibonacci(s.n_rays)[rng.choice(s.n_rays, 200, replace=False)]
    o = np.repeat(s.tx.astype(np.float32), 50, axis=0)
    fin, _ = _compare(env, s, scene, o, d)
    assert fin.mean() > 0.4


def test_concurrent_first_calls(env):
    """The own-point index is built once, under the scene's lock, when two
    threads on two streams make the first calls on a fresh scene together;
    both get the single-call results."""
    import threading
    torch, pcrl, oracle = env
    s = scenes.random_scene(5, extent=2.0, h=0.05, levels=(0.4, 0.2), pos_sigma=0.002, tilt_sigma=0.03)
    rng = np.random.default_rng(13)
    n = 70_000  # above the coherent-order threshold
    o = torch.from_numpy(rng.uniform(0.0, 2.0, size=(n, 3)).astype(np.float32)).cuda()
    d = torch.from_numpy(rng.normal(size=(n, 3)).astype(np.float32)).cuda()
    ref = pcrl.sdf_intersect(_build(env, s), o, d)["t"].cpu()
    scene = _build(env, s)
    torch.cuda.synchronize()  # the inputs and the scene are complete before the side streams start
    out, errs = [None, None], []
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    barrier = threading.Barrier(2)

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                barrier.wait()
                r = pcrl.sdf_intersect(scene, o, d)
                streams[i].synchronize()
                out[i] = r["t"].cpu()
        except Exception as e:  # pragma: no cover - reported below
            errs.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    assert torch.equal(out[0], ref) and torch.equal(out[1], ref)


def _launch_case(case):
    # (scene, rays per TX, K, reception sphere scale sigma)
    if case == "box_room":
        return scenes.box_room(), 3000, 2, 1.25
    if case == "box_room_one_level":
        s = scenes.box_room()
        s.levels = (0.25,)
        return s, 3000, 3, 1.25
    if case == "furnished_room_full":
        s = scenes.furnished_room()
        return s, s.n_rays, s.max_reflections, 1.25
    # seed 8: four of the six RX see the TX directly
    s = scenes.random_scene(8, extent=2.0, h=0.05, levels=(0.4, 0.2), pos_sigma=0.002, tilt_sigma=0.03, n_rx=6)
    return s, 6000, 3, 4.0


def _aimed_sample(oracle, s, n_rays, n_random, seed=7):
    """Direction indices aimed (within 1.2 ray spacings) at every RX and at its
    mirror images in the floor and ceiling, plus random ones: rays that the
    launch is likely to receive, chosen by geometry alone."""
    d = oracle.fibonacci(n_rays).astype(np.float64)
    alpha = oracle.ray_spacing(n_rays)
    tx = s.tx[0].astype(np.float64)
    height = s.extra.get("size", (12.0, 10.0, 3.0))[2]
    pick = set()
    for r in s.rx.astype(np.float64):
        for z in (r[2], -r[2], 2 * height - r[2]):
            u = np.array([r[0], r[1], z]) - tx
            u /= np.linalg.norm(u)
            pick.update(np.nonzero(d @ u > math.cos(1.2 * alpha))[0].tolist())
    pick.update(np.random.default_rng(seed).choice(n_rays, size=n_random, replace=False).tolist())
    return np.array(sorted(pick), np.int64)


EXCUSED_MAX = {"box_room": 0.06, "box_room_one_level": 0.06, "random": 0.06, "furnished_room_full": 0.35}


@pytest.mark.parametrize("case", ["box_room", "box_room_one_level", "random", "furnished_room_full"])
def test_sdf_launch_parity(env, case):
    """launch_rays with PCRL_LAUNCH_SDF against oracle.sdf_launch: per ray,
    segment by segment while the oracle's answer is stable (as in _compare,
    plus a nearest-point label decided by more than 1e-6 h), the hit
    distance within the march's band (widened by 1e-5 of the path so far,
    the FP32 state's drift) and the label equal; no ray may differ.  Rays
    whose every segment matched have the oracle's receptions (outside the
    reception test's rounding band) with lengths to 1e-5 relative.  The
    furnished room runs at full size (1M points, 1M rays, K = 3, 16 RX) and is
    compared on a sample of rays aimed at the RX and their floor and ceiling
    images (the oracle traces those directions with the 1M-ray spacing)."""
    torch, pcrl, oracle = env
    s, n_rays, K, sigma = _launch_case(case)
    scene = _build(env, s)
    info = scene.info()
    leaf = float(info["leaf_size"])
    h = oracle.SDF_H_SCALE * leaf
    eps = oracle.SDF_EPS_SCALE * leaf
    ms = oracle.SDF_MAX_STEPS
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=n_rays, max_reflections=K, sdf=True, hit_log=True,
                              rx_radius_scale=sigma)
    n_all = len(s.tx) * n_rays
    gid_all = launch.hit_log[0].cpu().numpy().reshape(n_all, K + 1)
    gt_all = launch.hit_log[1].cpu().numpy().astype(np.float64).reshape(n_all, K + 1)
    grec = launch.records()
    dirs = oracle.fibonacci(n_rays)
    if case == "furnished_room_full":
        sel = _aimed_sample(oracle, s, n_rays, n_random=60)   # direction indices of the single TX
        assert len(s.tx) == 1
    else:
        sel = np.arange(n_all, dtype=np.int64)
    n = len(sel)
    alpha = oracle.ray_spacing(n_rays)
    org = np.asarray(info["origin"], np.float32)
    # the oracle traces the selected rays only (one TX for the sampled case)
    odirs = dirs if case != "furnished_room_full" else dirs[sel]
    args = (s.xyz, s.normal, s.label, org, leaf, s.tx, s.rx, odirs, K, sigma)
    print(f"  [sdf launch] {case}: oracle on {n} rays", flush=True)
    ref = oracle.sdf_launch(*args, alpha=alpha, h=h, eps=eps, max_steps=ms)
    pa = oracle.sdf_launch(*args, alpha=alpha, h=h * (1 + 1e-4), eps=eps * (1 + 1e-2), max_steps=ms + 1,
                           diam_scale=1 + 1e-5, cross_margin=1e-5 * leaf)
    pb = oracle.sdf_launch(*args, alpha=alpha, h=h * (1 - 1e-4), eps=eps * (1 - 1e-2), max_steps=ms - 1,
                           diam_scale=1 - 1e-5, cross_margin=-1e-5 * leaf)
    gid = gid_all[sel]
    gt = gt_all[sel]
    gt = np.where(gid == -1, np.inf, gt)   # miss
    gt = np.where(gid == -2, np.nan, gt)   # not traced
    # labels of the device's hits come from the hit log's point ids
    glab = np.where(gid >= 0, np.asarray(s.label, np.int64)[np.maximum(gid, 0)], -1)
    rt, cos = ref["t"], np.nan_to_num(ref["cos"], nan=1.0)
    full, mism, excused = np.zeros(n, bool), 0, 0
    first_bad = None
    for r in range(n):
        path = 0.0
        ok = True
        for b in range(K + 1):
            r0 = rt[r, b]
            if np.isnan(r0):
                ok = np.isnan(gt[r, b])
                break
            tol = 2 * eps / max(cos[r, b], 0.05) + 4e-6 * (1 + path + (r0 if np.isfinite(r0) else 0.0)) + 1e-5 * path

            def close(x, y):
                return (np.isinf(x) and np.isinf(y)) or (np.isfinite(x) and np.isfinite(y) and abs(x - y) <= tol)
            stable = (close(pa["t"][r, b], r0) and close(pb["t"][r, b], r0) and pa["label"][r, b] ==
                      ref["label"][r, b] == pb["label"][r, b] and ref["label_margin"][r, b] > 1e-6 * h)
            if not stable:
                ok = None
                break
            if not close(gt[r, b], r0) or (np.isfinite(r0) and glab[r, b] != ref["label"][r, b]):
                ok = False
                break
            if not np.isfinite(r0):
                break
            path += r0
        if ok is None:
            excused += 1
        elif ok:
            full[r] = True
        else:
            mism += 1
            if first_bad is None:
                first_bad = (int(sel[r]), b, gt[r], rt[r], glab[r], ref["label"][r])
    # receptions of the rays that matched throughout (oracle ray r is device ray sel[r])
    ok_rays = {int(sel[r]) for r in range(n) if full[r]}
    want = {(int(sel[g]), int(x), int(b)) for g, x, b, got, band in zip(ref["rec_g"], ref["rec_rx"], ref["rec_b"],
            ref["rec_got"], ref["rec_band"]) if got and not band and full[g]}
    banded = {(int(sel[g]), int(x), int(b)) for g, x, b, band in zip(ref["rec_g"], ref["rec_rx"], ref["rec_b"],
              ref["rec_band"]) if band}
    have = {(int(g), int(x), int(b)) for g, x, b in zip(grec["ray"].tolist(), grec["rx"].tolist(),
            grec["n_refl"].tolist()) if int(g) in ok_rays}
    print(f"  [sdf launch] {case}: rays={n} matched={int(full.sum())} excused={excused} mismatch={mism} "
          f"records={len(have)} oracle_records={len(want)} first_bad={first_bad}", flush=True)
    assert mism == 0, first_bad
    # A ray is excused when the oracle's own answer moves under rounding-sized
    # perturbations (h, eps, the step limit, the segment length): that depends on
    # the oracle and the sample only, never on the device, so the bound only keeps
    # the comparison from going vacuous.  The box room and the random scene are
    # excused at most 4.5 %; the full furnished room 28 % (86 of 307 aimed rays:
    # four noisy segments of 1M points, where a march that ends at its step limit
    # or within eps of an edge moves with max_steps +- 1 or eps +- 1 %).
    assert excused <= EXCUSED_MAX[case] * n + 2, (excused, n)
    assert full.sum() >= 0.5 * n
    assert want - have == set()
    assert (have - want) <= banded
    assert len(want) > 0
    # the coarse paths of the launch collect as usual
    p = pcrl.collect_paths(launch)
    assert int(p["n_rows"]) > 0


def test_edge_cases(env):
    torch, pcrl, oracle = env
    s = scenes.box_room()
    scene = _build(env, s)
    o = np.array([[2.0, 2.0, 1.5]] * 5, np.float32)
    d = np.array([[1, 0, 0], [0, 0, 0], [np.nan, 0, 1], [0, 1, 0], [0, 0, -1]], np.float32)
    tr = np.array([[0, np.inf], [0, np.inf], [0, np.inf], [1.0, 0.5], [0, np.inf]], np.float32)
    r = pcrl.sdf_intersect(scene, o, d, t_range=tr)
    t = r["t"].cpu().numpy()
    assert np.isfinite(t[0]) and np.isfinite(t[4])
    assert np.all(np.isinf(t[1:4]))  # zero direction, NaN direction, empty range
    # no rays
    r = pcrl.sdf_intersect(scene, np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32))
    assert r["t"].numel() == 0
    # parameters out of range
    leaf = scene.info()["leaf_size"]
    for kw in (dict(h=0.99 * leaf), dict(max_steps=(1 << 20) + 1)):
        with pytest.raises(pcrl.PcrlError):
            pcrl.sdf_intersect(scene, o, d, **kw)
    # an empty cloud: every ray misses
    e = np.zeros((0, 3), np.float32)
    es = pcrl.build_voxels(e, e, np.zeros(0, np.uint32), (0.5,), 0.1)
    r = pcrl.sdf_intersect(es, o, d)
    assert torch.isinf(r["t"]).all()
    # dynamic points are not part of the surface
    ids = torch.arange(s.n_points, s.n_points + 4, dtype=torch.int32)
    # the SDF launch takes no traversal statistics
    with pytest.raises(pcrl.PcrlError):
        pcrl.launch_rays(scene, s.tx, s.rx, n_rays=100, max_reflections=1, sdf=True, stats=True)
    scene.update_points(ids, s.xyz[:4], s.normal[:4], s.label[:4])
    with pytest.raises(pcrl.PcrlError):
        pcrl.sdf_intersect(scene, o, d)
    with pytest.raises(pcrl.PcrlError):
        pcrl.launch_rays(scene, s.tx, s.rx, n_rays=100, max_reflections=1, sdf=True)
