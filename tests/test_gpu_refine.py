"""GPU path refinement (refine_paths) against the FP64 oracle, through the C ABI.

The coarse rows come from the device launch and collection; the oracle
refines the same rows (the same FP32 coarse points) by brute force.  The
bar, per row:
  * the outcome (status) is the oracle's;
  * for valid rows the label sequence is the oracle's, the length agrees to
    1e-5 relative and the points to 1e-3 m (both converge to the same
    stationary point; FP32 leaves ~1e-7 relative); the surfel of a point is
    the oracle's or a coplanar overlapping one;
  * the gradient steps taken agree to within 2 (the threshold delta is met
    by both at the same step unless the norm lands within rounding of it);
  * `kept` equals the oracle's dedup of the device's refined rows.
Scenes: the empty box room (where the refined paths are the image-method
paths of tests/golden/), random tilted planes and boxes, and the furnished
room at full size (768 rows; the oracle refines a sample, and every valid
device row is checked for validity in FP64).
"""
import math
import os

import numpy as np
import pytest

import scenes
from tests import parity

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2402_13747_amd as pcrl
    oracle.build(force=False)
    return torch, pcrl, oracle


def _golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "box_room_image_paths.txt")):
        if line.startswith("#"):
            continue
        name, l2 = line.split()
        out[() if name == "-" else tuple(int(x) for x in name.split(","))] = float(l2)
    return out


def _device_refine(env, s, K, kappa, n_rays=None, **kw):
    torch, pcrl, _ = env
    n_rays = n_rays or s.n_rays
    print(f"[refine] {s.name}: {s.n_points} pts, {n_rays} rays, K={K}, kappa={kappa}, {kw}", flush=True)
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, float(np.float32(s.surfel_radius)),
                              t_eps=float(np.float32(parity.t_eps_of(s))))
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=n_rays, max_reflections=K)
    P = pcrl.collect_paths(launch, kappa=kappa)
    R = pcrl.refine_paths(scene, s.tx, s.rx, P, **kw)
    return scene, launch, P, parity.to_numpy(P), parity.to_numpy(R)


def _oracle_refine(oracle, s, p, rows, **kw):
    return oracle.refine(s.xyz, s.normal, s.label, float(np.float32(s.surfel_radius)),
                         float(np.float32(parity.t_eps_of(s))), s.tx[p["tx"][rows]].astype(np.float64),
                         s.rx[p["rx"][rows]].astype(np.float64), p["n_refl"][rows],
                         p["points"][rows].astype(np.float64), **kw)


def _compare_rows(s, p, r, o, rows):
    st = r["status"][rows]
    assert np.array_equal(st, o["status"]), np.nonzero(st != o["status"])
    assert np.abs(r["iters"][rows] - o["iters"]).max(initial=0) <= 2
    ok = st == 0
    if not ok.any():
        return 0
    assert np.array_equal(r["key"][rows][ok], o["labels"][ok])
    # overlapping disks of one plane give the same point: either surfel is correct
    gi, oi = r["point_id"][rows][ok], o["ids"][ok]
    for a, b in zip(gi[gi != oi], oi[gi != oi]):
        assert parity._same_plane(int(a), int(b), s.xyz, s.normal, s.label), (a, b)
    rel = np.abs(r["length"][rows][ok] - o["length"][ok]) / o["length"][ok]
    assert rel.max() <= 1e-5, rel.max()
    K = p["points"].shape[1]
    if K:
        dp = np.abs(r["points"][rows][ok] - o["points"][ok])
        assert np.nanmax(dp, initial=0) <= 1e-3
        # NaN exactly past n_refl on both sides
        assert np.array_equal(np.isnan(r["points"][rows][ok]), np.isnan(o["points"][ok]))
    return int(ok.sum())


def _check_kept(oracle, s, p, r):
    grp = p["tx"].astype(np.int64) * 65536 + p["rx"]
    kept = oracle.refine_dedup(grp, p["n_refl"], r["key"], r["points"], r["length"], r["status"],
                               s.tx[p["tx"]].astype(np.float64))
    assert np.array_equal(kept, r["kept"].astype(bool))
    assert int(kept.sum()) == int(r["kept"].sum())


def test_box_room_refines_to_image_paths(env):
    torch, pcrl, oracle = env
    s = scenes.box_room()
    scene, launch, P, p, r = _device_refine(env, s, 2, 5)
    n = p["n_rows"]
    assert (r["status"] == pcrl.REFINE_VALID).all()
    gold = _golden()
    for i in range(n):
        seq = tuple(int(x) for x in r["key"][i, :p["n_refl"][i]])
        L = math.sqrt(gold[seq])
        # the FP64 refinement lands within 1e-7 above L; FP32 adds ~1e-7 either way
        assert L * (1 - 1e-6) <= r["length"][i] <= L * (1 + 1e-6), (seq, r["length"][i], L)
    kept = sorted(tuple(int(x) for x in r["key"][i, :p["n_refl"][i]]) for i in np.nonzero(r["kept"])[0])
    assert kept == sorted(gold) and len(kept) == 25
    o = _oracle_refine(oracle, s, p, np.arange(n))
    assert _compare_rows(s, p, r, o, np.arange(n)) == n
    _check_kept(oracle, s, p, r)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_random_scenes_match_oracle(env, seed):
    torch, pcrl, oracle = env
    s = scenes.random_scene(seed, n_rays=20_000, n_rx=4)
    scene, launch, P, p, r = _device_refine(env, s, 3, 3)
    rows = np.arange(p["n_rows"])
    o = _oracle_refine(oracle, s, p, rows)
    _compare_rows(s, p, r, o, rows)
    _check_kept(oracle, s, p, r)


def test_iteration_limit_matches_oracle(env):
    # the same rows with rho = 25: most stop unconverged at step 25
    torch, pcrl, oracle = env
    s = scenes.random_scene(2, n_rays=20_000, n_rx=4)
    scene, launch, P, p, r = _device_refine(env, s, 3, 3, max_iters=25, step=0.5)
    rows = np.arange(p["n_rows"])
    o = _oracle_refine(oracle, s, p, rows, max_iters=25, step=0.5)
    _compare_rows(s, p, r, o, rows)
    nc = r["status"] == pcrl.REFINE_NOT_CONVERGED
    assert (r["iters"][nc] == 25).all()
    assert np.allclose(r["grad"][nc], o["grad"][nc], rtol=1e-3, atol=1e-6)


def _fp64_valid(s, r_s, t_eps, tx, rx, pts, ids, grad_tol):
    """A refined path checked in FP64 from its points and surfels alone:
    every point on its surfel's disk, tangent-plane gradient below the
    threshold (plus FP32 slack), a reflection at every point and a last
    segment no surfel blocks (brute force over all points)."""
    xyz = s.xyz.astype(np.float64)
    nrm = s.normal.astype(np.float64)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    N = len(ids)
    I = [np.asarray(tx, np.float64)] + [np.asarray(q, np.float64) for q in pts] + [np.asarray(rx, np.float64)]
    gg = 0.0
    for k in range(1, N + 1):
        m = ids[k - 1]
        n = nrm[m]
        w = I[k] - xyz[m]
        if abs(w @ n) > 1e-4 or np.linalg.norm(w - (w @ n) * n) > r_s * (1 + 1e-4):
            return "off its surfel"
        e1 = (I[k] - I[k - 1]) / np.linalg.norm(I[k] - I[k - 1])
        e2 = (I[k] - I[k + 1]) / np.linalg.norm(I[k] - I[k + 1])
        G = e1 + e2
        g = G - (G @ n) * n
        gg += g @ g
        if not ((I[k - 1] - I[k]) @ n) * ((I[k + 1] - I[k]) @ n) > 0:
            return "not a reflection"
    if math.sqrt(gg) >= grad_tol + 2e-5:
        return f"gradient {math.sqrt(gg)}"
    o, e = I[N], I[N + 1] - I[N]
    seg = np.linalg.norm(e)
    d = e / seg
    den = nrm @ d
    with np.errstate(divide="ignore", invalid="ignore"):
        t = ((xyz - o) * nrm).sum(1) / den
        q = o + t[:, None] * d - xyz
    # clear blockers only: inside the disk, past t_eps and short of the RX by margins
    # that FP32 rounding of the device's hit tests cannot cross
    hit = (np.abs(den) > 1e-6) & (t > t_eps * 1.01) & ((q * q).sum(1) <= (r_s * (1 - 1e-4)) ** 2) & \
        (t < seg * (1 - 1e-4))
    if N:
        hit[ids[N - 1]] = False
    if hit.any():
        return "last segment blocked"
    return None


def test_furnished_room_full_size(env):
    torch, pcrl, oracle = env
    s = scenes.furnished_room()
    scene, launch, P, p, r = _device_refine(env, s, 3, 100)
    n = p["n_rows"]
    st = r["status"]
    print(f"[refine] furnished room: {n} rows, status counts {np.bincount(st, minlength=6)}, kept {r['kept'].sum()}",
          flush=True)
    assert n > 500 and (st == pcrl.REFINE_VALID).sum() > 50
    # the oracle on the rows that finish soonest (valid and missed ones; 2000-step rows are covered below)
    rows = np.argsort(r["iters"], kind="stable")[:48]
    o = _oracle_refine(oracle, s, p, rows)
    assert _compare_rows(s, p, r, o, rows) > 10
    # every valid device row is a valid path in FP64
    r_s, t_eps = float(np.float32(s.surfel_radius)), float(np.float32(parity.t_eps_of(s)))
    for i in np.nonzero(st == pcrl.REFINE_VALID)[0]:
        N = p["n_refl"][i]
        why = _fp64_valid(s, r_s, t_eps, s.tx[p["tx"][i]], s.rx[p["rx"][i]], r["points"][i, :N],
                          r["point_id"][i, :N], 1e-4)
        assert why is None, (i, why)
    _check_kept(oracle, s, p, r)
    # rows that did not converge in 2000 steps: the first 20 steps of 16 of them
    slow = np.nonzero(st == pcrl.REFINE_NOT_CONVERGED)[0][:16]
    if len(slow):
        R20 = parity.to_numpy(pcrl.refine_paths(scene, s.tx, s.rx, P, max_iters=20))
        o = _oracle_refine(oracle, s, p, slow, max_iters=20)
        _compare_rows(s, p, R20, o, slow)


def test_canyon_three_levels_brick_masks(env):
    # three voxel levels and the brick-mask traversal (no dense cell table)
    torch, pcrl, oracle = env
    s = scenes.street_canyon(n_points=1_000_000, scale=0.25, n_tx=2, n_rx=16, n_rays=200_000, K=3,
                             levels=(4.0, 0.5, 0.1))
    print(f"[refine] small canyon: {s.n_points} pts, spacing {s.spacing:.3f}", flush=True)
    r_s, t_eps = float(np.float32(s.surfel_radius)), float(np.float32(parity.t_eps_of(s)))
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, r_s, t_eps=t_eps, compact=True)
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=s.n_rays, max_reflections=3)
    P = pcrl.collect_paths(launch, kappa=3)
    p, r = parity.to_numpy(P), parity.to_numpy(pcrl.refine_paths(scene, s.tx, s.rx, P))
    print(f"[refine] small canyon: {p['n_rows']} rows, status {np.bincount(r['status'], minlength=6)}", flush=True)
    assert p["n_rows"] > 20 and (r["status"] == pcrl.REFINE_VALID).sum() > 10
    work = (r["iters"] + 1) * np.maximum(p["n_refl"], 1)
    rows = np.argsort(work, kind="stable")[:40]
    o = _oracle_refine(oracle, s, p, rows)
    assert _compare_rows(s, p, r, o, rows) > 10
    _check_kept(oracle, s, p, r)


@pytest.mark.parametrize("seed", [11, 12])
def test_smoothed_normals_match_oracle(env, seed):
    # random planes and boxes with tilted normals and jittered points
    torch, pcrl, oracle = env
    s = scenes.random_scene(seed, n_rays=20_000, n_rx=4, pos_sigma=0.002, tilt_sigma=0.02, h=0.1)
    h = 0.9 * float(np.float32(s.levels[-1]))
    scene, launch, P, p, r = _device_refine(env, s, 3, 3, smooth_radius=h)
    rows = np.arange(p["n_rows"])
    o = _oracle_refine(oracle, s, p, rows, smooth_radius=h)
    _compare_rows(s, p, r, o, rows)
    _check_kept(oracle, s, p, r)


def test_furnished_room_smoothed_normals(env):
    torch, pcrl, oracle = env
    s = scenes.furnished_room()
    scene, launch, P, p, r = _device_refine(env, s, 3, 100, smooth_radius=0.045)
    st = r["status"]
    print(f"[refine] furnished room, smoothed normals: status counts {np.bincount(st, minlength=6)}, "
          f"kept {r['kept'].sum()}", flush=True)
    rows = np.argsort((r["iters"] + 1) * np.maximum(p["n_refl"], 1), kind="stable")[:32]
    o = _oracle_refine(oracle, s, p, rows, smooth_radius=0.045)
    assert _compare_rows(s, p, r, o, rows) > 10
    _check_kept(oracle, s, p, r)
    # an invalid radius is refused
    with pytest.raises(pcrl.PcrlError) as e:
        pcrl.refine_paths(scene, s.tx, s.rx, P, smooth_radius=0.06)
    assert e.value.status == -1 and "smoothing radius" in e.value.message


def test_edge_cases(env):
    torch, pcrl, oracle = env
    s = scenes.box_room()
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, float(np.float32(s.surfel_radius)),
                              t_eps=float(np.float32(parity.t_eps_of(s))))
    # K = 0: line-of-sight rows only, no iteration, one kept per (TX, RX)
    rx = np.array([[7.0, 5.0, 1.5], [5.0, 1.0, 2.0], [9.0, 7.0, 0.5]], np.float32)
    launch = pcrl.launch_rays(scene, s.tx, rx, n_rays=10_000, max_reflections=0)
    P = pcrl.collect_paths(launch, kappa=4)
    r = parity.to_numpy(pcrl.refine_paths(scene, s.tx, rx, P))
    assert (r["status"] == pcrl.REFINE_VALID).all() and (r["iters"] == 0).all()
    L = np.linalg.norm(rx[P["rx"].cpu().numpy()] - s.tx[0], axis=1)
    assert np.allclose(r["length"], L, rtol=1e-6)
    assert r["n_kept"] == 3
    # no rows
    empty = {k: v[:0] for k, v in P.items() if hasattr(v, "shape")}
    empty["n_rows"] = 0
    assert pcrl.refine_paths(scene, s.tx, rx, empty)["n_kept"] == 0
    # rows out of (tx, rx, n_refl) order, and an RX index out of range, are refused
    launch = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=10_000, max_reflections=2)
    P = pcrl.collect_paths(launch, kappa=2)
    bad = dict(P)
    bad["n_refl"] = P["n_refl"].flip(0).contiguous()
    with pytest.raises(pcrl.PcrlError) as e:
        pcrl.refine_paths(scene, s.tx, s.rx, bad)
    assert e.value.status == -1 and "sorted" in e.value.message
    bad = dict(P)
    bad["rx"] = P["rx"] + 1
    with pytest.raises(pcrl.PcrlError) as e:
        pcrl.refine_paths(scene, s.tx, s.rx, bad)
    assert e.value.status == -1 and "rx" in e.value.message


def test_refine_over_overlay_equals_rebuilt_scene(env):
    # a box of dynamic points inside the room: refinement over base + overlay
    # traces exactly the nearest hits of a scene built from all points
    torch, pcrl, oracle = env
    s = scenes.box_room()
    # its face y = 6 holds the specular point (6, 6, 1.5) of TX (2, 2, 1.5) -> RX (7, 5, 1.5)
    faces = scenes._box_faces((5.5, 6.0, 0.0), (6.5, 7.0, 2.5), label=(9,) * 6, inward=False, bottom=False)
    bx, bn, bl = scenes._sample_faces(faces, 0.1)
    r_s, t_eps = float(np.float32(s.surfel_radius)), float(np.float32(parity.t_eps_of(s)))
    ids = np.arange(s.n_points, s.n_points + len(bx), dtype=np.uint32)
    base = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, r_s, t_eps=t_eps)
    base.update_points(ids, bx.astype(np.float32), bn.astype(np.float32), bl.astype(np.uint32))
    full = pcrl.build_voxels(np.concatenate([s.xyz, bx.astype(np.float32)]),
                             np.concatenate([s.normal, bn.astype(np.float32)]),
                             np.concatenate([s.label, bl.astype(np.uint32)]), s.levels, r_s, t_eps=t_eps)
    res = []
    for sc in (base, full):
        L = pcrl.launch_rays(sc, s.tx, s.rx, n_rays=20_000, max_reflections=2)
        P = pcrl.collect_paths(L, kappa=3)
        res.append((parity.to_numpy(P), parity.to_numpy(pcrl.refine_paths(sc, s.tx, s.rx, P))))
    (p0, r0), (p1, r1) = res
    assert p0["n_rows"] == p1["n_rows"] and np.array_equal(p0["points"], p1["points"], equal_nan=True)
    for k in ("status", "iters", "point_id", "key", "kept"):
        assert np.array_equal(r0[k], r1[k]), k
    for k in ("length", "grad", "points"):
        assert np.array_equal(r0[k], r1[k], equal_nan=True), k
    assert ((r0["key"] == 9).any(axis=1) & (r0["status"] == pcrl.REFINE_VALID)).any()   # off the dynamic box


# --------------------------------------------------------------------------- diffraction (Section 2.3)

CORNER_TX = np.array([(-3.0, 5.0, 3.0), (-3.0, 5.0, 8.0), (-3.0, 5.0, 1.5)], np.float32)
CORNER_RX = np.array([(5.0, -3.0, 1.5), (3.0, 3.0, 1.5), (5.0, -3.0, -1.0)], np.float32)


def _corner_rows(cone):
    """Coarse rows at the corner building, from the oracle only: edge pieces of the vertical edge at
    (0, 0) (oracle/cone.py's edge IEs), ground points placed by hand, and the receptions of the
    oracle's own cone trace (TX 2, one diffraction).  Returns (rows sorted by (tx, rx, n), the
    expected status of the hand-made ones or None)."""
    s = scenes.corner_building()
    E = s.extra["edges"]
    origin, dims = np.array([-10.292, -10.292, -0.292], np.float32), (53, 53, 13)
    eies = cone.edge_ies(E["seg"], E["normals"], E["label"], origin, 0.4, 2, dims)
    on0 = np.nonzero(eies["edge"] == 0)[0]

    def piece(z):
        return eies["pos"][on0[np.argmin(np.abs(eies["pos"][on0, 2] - z))]]
    ground_a = np.array([1.5, -1.2, 0.0])
    V, OFF, WS, OCC = 0, 6, 3, 4
    rows = [  # (tx, rx, points, edges, expected status)
        (0, 0, [piece(1.0)], [0], V), (0, 0, [piece(2.5)], [0], V), (0, 0, [piece(3.7)], [0], V),
        (0, 0, [piece(1.0), ground_a], [0, -1], V),
        (0, 1, [piece(1.0)], [0], WS),                       # RX inside the building
        (0, 2, [piece(1.0)], [0], OCC),                      # RX under the ground
        (1, 0, [piece(3.7)], [0], OFF),                      # the stationary point is at 4.75 m
    ]
    # the oracle's cone trace from TX 2 (the default corner scene): its receptions through the edge
    ies = cone.ie_build(s.xyz, s.normal, s.label, origin, 0.4, 2, dims)
    sc = cone.Scene(s.xyz, s.normal, s.label, s.surfel_radius, s.t_eps_value)
    res = cone.trace(sc, ies, CORNER_TX[2:3], CORNER_RX[0:1], origin, 0.4, 2, dims, K=1, kappa=100,
                     half_angle=math.radians(2.5), edges=eies, max_diff=1)
    C = cone.combine(ies, eies)
    for r in res["records"]:
        if r["exact"]:
            rows.append((2, 0, [C["pos"][e] for e in r["chain"]], [int(C["edge"][e]) for e in r["chain"]], V))
    rows.sort(key=lambda r: (r[0], r[1], len(r[2])))
    return s, rows


def _rows_arrays(rows, K):
    n = len(rows)
    pts = np.full((n, K, 3), np.nan, np.float32)
    eo = np.full((n, K), -1, np.int32)
    for i, (_, _, ps, es, _) in enumerate(rows):
        pts[i, :len(ps)] = np.asarray(ps, np.float32)
        eo[i, :len(es)] = es
    return dict(tx=np.array([r[0] for r in rows], np.int32), rx=np.array([r[1] for r in rows], np.int32),
                n_refl=np.array([len(r[2]) for r in rows], np.int32), points=pts, n_rows=n), eo


def test_refine_diffraction_corner(env):
    """Diffraction points on the corner building's vertical edge against the oracle, row by row:
    outcomes, steps, labels, lengths and points; the closed forms sqrt(136 + 1.5^2) (one
    diffraction, TX at 3 m) and 12.5 (diffraction then ground reflection); Keller's law at
    every valid diffraction point; the dedup against the oracle's."""
    torch, pcrl, oracle = env
    from oracle import cone
    s, rows = _corner_rows(cone)
    K = 2
    p, eo = _rows_arrays(rows, K)
    E = s.extra["edges"]
    r_s, t_eps = float(np.float32(s.surfel_radius)), float(np.float32(parity.t_eps_of(s)))
    print(f"[refine] corner building: {len(rows)} rows with diffraction points", flush=True)
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, r_s, t_eps=t_eps)
    P = {k: torch.from_numpy(v).cuda() if isinstance(v, np.ndarray) else v for k, v in p.items()}
    r = parity.to_numpy(pcrl.refine_paths(scene, CORNER_TX, CORNER_RX, P, edges=E, edge_of=eo))
    o = oracle.refine(s.xyz, s.normal, s.label, r_s, t_eps, CORNER_TX[p["tx"]].astype(np.float64),
                      CORNER_RX[p["rx"]].astype(np.float64), p["n_refl"], p["points"].astype(np.float64),
                      edges=E, edge_of=eo)
    want = np.array([w for *_, w in rows])
    assert np.array_equal(o["status"], want), (o["status"], want)
    rows_all = np.arange(len(rows))
    assert _compare_rows(s, p, r, o, rows_all) == int((want == 0).sum())
    w = np.array([0.0, 0.0, 1.0])
    for i in np.nonzero(r["status"] == 0)[0]:
        N = p["n_refl"][i]
        I = [CORNER_TX[p["tx"][i]].astype(np.float64)] + list(r["points"][i, :N].astype(np.float64)) + \
            [CORNER_RX[p["rx"][i]].astype(np.float64)]
        for k in range(N):
            if eo[i, k] >= 0:
                assert r["point_id"][i, k] == -2 - eo[i, k] and r["key"][i, k] == 100 + eo[i, k]
                u, v = I[k + 1] - I[k], I[k + 2] - I[k + 1]
                assert abs(u @ w / np.linalg.norm(u) - v @ w / np.linalg.norm(v)) <= 1e-3
        if p["tx"][i] == 0 and N == 1:
            L = math.sqrt(136.0 + 1.5 ** 2)
            assert abs(r["length"][i] - L) <= 1e-5 * L
        if p["tx"][i] == 0 and N == 2:
            assert abs(r["length"][i] - 12.5) <= 1e-5 * 12.5
        if p["tx"][i] == 2:
            L = 2.0 * math.sqrt(34.0)
            assert abs(r["length"][i] - L) <= 1e-5 * L
    grp = p["tx"].astype(np.int64) * 65536 + p["rx"]
    kept = oracle.refine_dedup(grp, p["n_refl"], r["key"], r["points"], r["length"], r["status"],
                               CORNER_TX[p["tx"]].astype(np.float64))
    assert np.array_equal(kept, r["kept"].astype(bool))


def test_refine_cone_paths_corner(env):
    """refine_cone_paths on the cone tracer's own coarse paths (two interactions, one diffraction):
    equal to refine_paths given the edges explicitly (each edge's label is 100 + its index); the
    corner diffraction (label 100) is kept with length 2 sqrt(34)."""
    torch, pcrl, oracle = env
    s = scenes.corner_building()
    E = s.extra["edges"]
    r_s, t_eps = float(np.float32(s.surfel_radius)), float(np.float32(parity.t_eps_of(s)))
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, r_s, t_eps=t_eps)
    origin, dims = np.array([-10.292, -10.292, -0.292], np.float32), np.array([53, 53, 13])
    ies = pcrl.ie_build(scene, origin, 0.4, 2, dims)
    ies.add_edges(E["seg"], E["normals"], E["label"])
    L = pcrl.cone_launch(ies, s.tx, s.rx, 2, math.radians(2.5), max_diffractions=1)
    P = pcrl.cone_collect(L, kappa=1 << 20)
    print(f"[refine] corner building cone paths: {P['n_rows']} rows", flush=True)
    r1 = parity.to_numpy(pcrl.refine_cone_paths(L, P))
    key = P["key"].cpu().numpy()
    eo = np.where(key >= 100, key - 100, -1).astype(np.int32)
    r2 = parity.to_numpy(pcrl.refine_paths(scene, s.tx, s.rx, P, edges=E, edge_of=eo))
    for k in ("status", "iters", "point_id", "key", "kept"):
        assert np.array_equal(r1[k], r2[k]), k
    for k in ("grad", "length", "points"):
        assert np.array_equal(r1[k], r2[k], equal_nan=True), k
    kept = [(tuple(int(x) for x in r1["key"][i, :int(P["n_refl"][i])]), float(r1["length"][i]))
            for i in np.nonzero(r1["kept"])[0]]
    Ls = [ln for seq, ln in kept if seq == (100,)]
    assert len(Ls) == 1 and abs(Ls[0] - 2.0 * math.sqrt(34.0)) <= 1e-5 * 2.0 * math.sqrt(34.0)
