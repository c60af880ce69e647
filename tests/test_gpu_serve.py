"""Incremental re-voxelisation and the serving loop.

* base (static points) + overlay (moving points) traces bitwise like a scene
  rebuilt from all points, frame after frame, and matches the FP64 oracle run
  over all points of that frame;
* a served query's records match the oracle's on sampled rays;
* every served query's result equals the same query launched alone on the
  same epoch, also when queries overlap on the device and when the scene
  changes between admission rounds;
* admission respects the memory budget and refuses queries larger than it.
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
def world(env):
    torch, pcrl = env
    sc, mover = scenes.moving_canyon(n_points=120_000, extent=(60.0, 60.0), lots=(2, 2), levels=(4.0, 1.0, 0.25),
                                     seed=5)
    ids = sc.extra["moving_idx"]
    n_static = int(ids[0])
    r_s = float(np.float32(sc.surfel_radius))
    t_eps = float(np.float32(sc.t_eps))
    print(f"[serve] moving canyon: {sc.n_points} points, {len(ids)} moving, h={sc.spacing:.3f}", flush=True)
    base = pcrl.build_voxels(sc.xyz[:n_static], sc.normal[:n_static], sc.label[:n_static], sc.levels, r_s, t_eps=t_eps)
    return sc, mover, base, n_static, r_s, t_eps


def _paths(pcrl, L):
    return parity.to_numpy(pcrl.collect_paths(L, kappa=1 << 30))


def _same_paths(a, b):
    for k in ("tx", "rx", "n_refl", "key", "count", "rank", "ray", "len_poly", "len_unf", "points"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k]), equal_nan=True), k
    assert a["n_rows"] == b["n_rows"] and a["n_keys"] == b["n_keys"]


def test_overlay_equals_full_rebuild(env, world):
    torch, pcrl = env
    sc, mover, base, n_static, r_s, t_eps = world
    tx = sc.tx
    rx = sc.rx[:4]
    for frame in (0, 3, 7):
        idx, xyz, nrm = mover(frame)
        lab = sc.label[idx]
        print(f"[serve] frame {frame}", flush=True)
        base.update_points(idx.astype(np.uint32), xyz, nrm, lab)
        inc = pcrl.launch_rays(base, tx, rx, n_rays=30_000, max_reflections=3, hit_log=True)
        allx = np.concatenate([sc.xyz[:n_static], xyz])
        alln = np.concatenate([sc.normal[:n_static], nrm])
        full_scene = pcrl.build_voxels(allx, alln, sc.label, sc.levels, r_s, t_eps=t_eps)
        full = pcrl.launch_rays(full_scene, tx, rx, n_rays=30_000, max_reflections=3, hit_log=True)
        assert np.array_equal(inc.hit_log[0].cpu().numpy(), full.hit_log[0].cpu().numpy())
        assert np.array_equal(inc.hit_log[1].cpu().numpy(), full.hit_log[1].cpu().numpy(), equal_nan=True)
        _same_paths(_paths(pcrl, inc), _paths(pcrl, full))
        hits = inc.hit_log[0].cpu().numpy()
        assert np.isin(hits, idx.astype(np.int64)).any()          # the moving boxes are actually hit
    assert base.info()["epoch"] >= 3 and base.info()["n_dynamic"] == len(idx)
    # a dynamic disk reaching outside the base grid is refused and the current overlay stays
    info = base.info()
    far = xyz.copy()
    far[0, 0] = info["origin"][0] + 0.5 * r_s
    with pytest.raises(pcrl.PcrlError) as e:
        base.update_points(idx.astype(np.uint32), far, nrm, lab)
    assert e.value.status == -1 and "grid" in e.value.message
    assert base.info()["epoch"] == info["epoch"] and base.info()["n_dynamic"] == len(idx)


def _queries(sc, rng, n):
    out = []
    for k in range(n):
        n_rays = int(rng.integers(2_000, 40_000))
        n_rx = int(rng.integers(1, 5))
        out.append(dict(tx=sc.tx, rx=sc.rx[rng.choice(len(sc.rx), n_rx, replace=False)], n_rays=n_rays,
                        max_reflections=int(rng.integers(1, 4))))
    return out


def _aimed_rays(oracle, tx, rx, n_rays, n_even):
    """Global ray ids (tx * n_rays + j) of the directions within 1.2 ray
    spacings of each RX and of its image in the ground plane z = 0, seen from
    each TX, plus n_even evenly spaced ones: rays that are likely received,
    chosen by geometry alone."""
    d = oracle.fibonacci(n_rays).astype(np.float64)
    alpha = oracle.ray_spacing(n_rays)
    pick = set()
    for i, t in enumerate(np.asarray(tx, np.float64).reshape(-1, 3)):
        for r in np.asarray(rx, np.float64).reshape(-1, 3):
            for z in (r[2], -r[2]):
                u = np.array([r[0], r[1], z]) - t
                u /= np.linalg.norm(u)
                pick.update((i * n_rays + np.nonzero(d @ u > np.cos(1.2 * alpha))[0]).tolist())
        pick.update((i * n_rays + np.linspace(0, n_rays - 1, n_even).astype(np.int64)).tolist())
    return np.array(sorted(pick), np.int64)


def _served_paths(res):
    keys = ("tx", "rx", "n_refl", "key", "count", "rank", "ray", "len_poly", "len_unf", "points", "n_rows", "n_keys")
    return {k: res[k] for k in keys}


@pytest.mark.parametrize("large", [False, True])
def test_served_equals_alone(env, world, large):
    """Small queries share batched rounds; large ones (>= 65536 rays) are launched one by one in a round."""
    torch, pcrl = env
    sc, mover, base, n_static, r_s, t_eps = world
    idx, xyz, nrm = mover(11)
    base.update_points(idx.astype(np.uint32), xyz, nrm, sc.label[idx])
    qs = _queries(sc, np.random.default_rng(0), 14)
    if large:
        qs = [dict(q, n_rays=q["n_rays"] + 70_000) for q in qs[:6]]
    alone = []
    for q in qs:
        L = pcrl.launch_rays(base, **q)
        p = _paths(pcrl, L)
        p["points"] = p["points"].reshape(p["n_rows"], q["max_reflections"], 3)
        alone.append(p)
    srv = pcrl.Server(base, n_streams=3, max_batch=5, kappa=1 << 30)
    tickets = [srv.submit(**q) for q in qs]
    for t in tickets:
        info = srv.poll(t, timeout=60.0)
        assert info["status"] == 2, info
    for t, ref in zip(tickets, alone):
        _same_paths(_served_paths(srv.result(t)), ref)
    st = srv.stats()
    assert st["completed"] == len(qs) and st["p99_ms"] >= st["p50_ms"] > 0
    srv.close()


def test_serve_epochs(env, world):
    torch, pcrl = env
    sc, mover, base, n_static, r_s, t_eps = world
    srv = pcrl.Server(base, n_streams=2, max_batch=3, kappa=1 << 30)
    rng = np.random.default_rng(1)
    for frame in (20, 21):
        idx, xyz, nrm = mover(frame)
        srv.update(idx.astype(np.uint32), xyz, nrm, sc.label[idx])
        epoch = base.info()["epoch"]
        qs = _queries(sc, rng, 6)
        tickets = [srv.submit(**q) for q in qs]
        for t, q in zip(tickets, qs):
            info = srv.poll(t, timeout=60.0)
            assert info["status"] == 2 and info["epoch"] == epoch
            L = pcrl.launch_rays(base, **q)
            ref = _paths(pcrl, L)
            ref["points"] = ref["points"].reshape(ref["n_rows"], q["max_reflections"], 3)
            _same_paths(_served_paths(srv.result(t)), ref)
            srv.release(t)
    srv.close()


def test_serve_budget(env, world):
    torch, pcrl = env
    sc, mover, base, n_static, r_s, t_eps = world
    # what the server charges one query against its budget (its launch's buffers)
    rays, K, n_rx = 20_000, 3, 2
    one = pcrl.serve_query_bytes(len(sc.tx), n_rx, rays, K)
    assert one >= len(sc.tx) * rays * (72 + 16 * K)     # ray state and history at least
    srv = pcrl.Server(base, n_streams=4, max_batch=8, hbm_budget_bytes=int(1.5 * one))
    qs = [dict(tx=sc.tx, rx=sc.rx[:n_rx], n_rays=rays, max_reflections=K) for _ in range(5)]
    tickets = [srv.submit(**q) for q in qs]
    for t in tickets:
        assert srv.poll(t, timeout=60.0)["status"] == 2
    st = srv.stats()
    assert st["rounds"] == 5 and abs(st["mean_batch"] - 1.0) < 1e-9     # one query fits at a time
    with pytest.raises(pcrl.PcrlError) as e:
        srv.submit(sc.tx, sc.rx[:2], n_rays=2_000_000, max_reflections=3)
    assert e.value.status == -5
    srv.close()


def test_serve_cancel(env, world):
    torch, pcrl = env
    sc, mover, base, n_static, r_s, t_eps = world
    rays, K, n_rx = 20_000, 3, 2
    one = pcrl.serve_query_bytes(len(sc.tx), n_rx, rays, K)
    # room for one query at a time: the last two are still queued when cancelled
    srv = pcrl.Server(base, n_streams=4, max_batch=8, hbm_budget_bytes=int(1.5 * one))
    tickets = [srv.submit(sc.tx, sc.rx[:2], n_rays=rays, max_reflections=K) for _ in range(6)]
    srv.cancel(tickets[4])
    srv.cancel(tickets[5])
    for t in tickets[:4]:
        assert srv.poll(t, timeout=60.0)["status"] == 2
    for t in tickets[4:]:
        with pytest.raises(pcrl.PcrlError) as e:
            srv.poll(t, timeout=60.0)
        assert e.value.status == -6
        srv.release(t)
    srv.cancel(tickets[0])                      # finished: left as it is
    assert srv.poll(tickets[0])["status"] == 2 and srv.result(tickets[0])["n_rows"] >= 0
    with pytest.raises(pcrl.PcrlError) as e:
        srv.cancel(1 << 40)
    assert e.value.status == -1
    assert srv.stats()["completed"] == 4
    srv.close()


def _frame_points(sc, n_static, xyz, nrm):
    """All points of a frame, indexed by their global ids (static, then moving)."""
    return (np.ascontiguousarray(np.concatenate([sc.xyz[:n_static], xyz]), np.float32),
            np.ascontiguousarray(np.concatenate([sc.normal[:n_static], nrm]), np.float32))


def test_overlay_matches_oracle(env, world):
    """The overlay kernel variant (base hierarchy, then the dynamic points' overlay)
    against the oracle's brute force over all points of the frame, per ray and
    segment on a sample of rays aimed at the moving boxes and at random."""
    import oracle
    oracle.build(force=False)
    torch, pcrl = env
    sc, mover, base, n_static, r_s, t_eps = world
    idx, xyz, nrm = mover(5)
    base.update_points(idx.astype(np.uint32), xyz, nrm, sc.label[idx])
    n_rays, K = 30_000, 3
    rx = sc.rx[:4]
    L = pcrl.launch_rays(base, sc.tx, rx, n_rays=n_rays, max_reflections=K, hit_log=True)
    ids = L.hit_log[0].cpu().numpy().reshape(n_rays * len(sc.tx), K + 1)
    rec = parity.to_numpy(L.records())
    # rays whose first hit is a moving point, plus an even sample
    moving_first = np.nonzero(ids[:, 0] >= n_static)[0]
    assert len(moving_first) > 20
    sel = np.union1d(moving_first[:: max(1, len(moving_first) // 400)], np.linspace(0, n_rays - 1, 1200).astype(np.int64))
    allx, alln = _frame_points(sc, n_static, xyz, nrm)
    print(f"[serve] overlay vs oracle: {len(sel)} rays over {len(allx)} points", flush=True)
    orc = oracle.launch(allx, alln, sc.label, sc.tx, rx, oracle.fibonacci(n_rays), K=K, r_s=r_s, t_eps=t_eps, sel=sel,
                        parity=True, **parity.fp32_bands(allx, sc.tx, rx))
    rep = parity.compare(orc, ids, rec, allx, alln, sc.label, K)
    print(f"  [overlay vs oracle] {rep.summary()}", flush=True)
    assert rep.ok(), (rep.mismatch[:5], rep.record_missing[:5], rep.record_extra[:5], rep.length_bad[:5],
                      rep.overflow[:5])
    assert rep.exact + rep.equivalent >= 0.95 * rep.segments
    hit_moving = sum(int(np.any((orc["hit_id"][r] >= n_static))) for r in range(len(sel)))
    assert hit_moving > 20


def test_served_matches_oracle(env, world):
    """Queries served together (overlapping rounds on the device) against the
    oracle: on sampled rays whose every segment has a single acceptable answer
    in the oracle, the served rows (every record, kappa unbounded) are exactly
    the oracle's receptions, with the oracle's labels and lengths to 1e-5."""
    import oracle
    oracle.build(force=False)
    torch, pcrl = env
    sc, mover, base, n_static, r_s, t_eps = world
    idx, xyz, nrm = mover(9)
    allx, alln = _frame_points(sc, n_static, xyz, nrm)
    srv = pcrl.Server(base, n_streams=3, max_batch=4, kappa=1 << 30)
    srv.update(idx.astype(np.uint32), xyz, nrm, sc.label[idx])
    rng = np.random.default_rng(4)
    qs = _queries(sc, rng, 5) + [dict(tx=sc.tx, rx=sc.rx[:3], n_rays=70_001, max_reflections=3)]
    tickets = [srv.submit(**q) for q in qs]
    checked = 0
    for t, q in zip(tickets, qs):
        assert srv.poll(t, timeout=120.0)["status"] == 2
        res = srv.result(t)
        K, n_rays = q["max_reflections"], q["n_rays"]
        sel = _aimed_rays(oracle, q["tx"], q["rx"], n_rays, 300)
        orc = oracle.launch(allx, alln, sc.label, q["tx"], q["rx"], oracle.fibonacci(n_rays), K=K, r_s=r_s,
                            t_eps=t_eps, sel=sel, parity=True, **parity.fp32_bands(allx, q["tx"], q["rx"]))
        stable = {}
        for r, g in enumerate(sel):
            traced = orc["hit_id"][r] != -2
            stable[int(g)] = bool(np.all(orc["acc_n"][r][traced] == 1))
        want = {}
        for k in range(orc["n_rec"]):
            g = int(orc["rec_g"][k])
            if not stable[g]:
                continue
            b = int(orc["rec_b"][k])
            key = (g, int(orc["rec_rx"][k]), b)
            r = int(orc["rec_sel"][k])
            want[key] = (int(orc["rec_flags"][k]), tuple(int(x) for x in orc["seq"][r, :b]),
                         float(orc["rec_lpoly"][k]), float(orc["rec_lunf"][k]))
        have = {}
        for i in range(int(res["n_rows"])):
            g = int(res["ray"][i])
            if g in stable and stable[g]:
                b = int(res["n_refl"][i])
                have[(g, int(res["rx"][i]), b)] = (tuple(int(x) for x in np.asarray(res["key"][i])[:b]),
                                                  float(res["len_poly"][i]), float(res["len_unf"][i]))
        for key, (flags, seq, lp, lu) in want.items():
            if flags == 1:
                assert key in have, key
            if key in have:
                dseq, dlp, dlu = have[key]
                assert dseq == seq, (key, dseq, seq)
                assert abs(dlp - lp) <= 1e-5 * lp and abs(dlu - lu) <= 1e-5 * lu, (key, dlp, lp, dlu, lu)
                checked += 1
        assert set(have) <= set(want), sorted(set(have) - set(want))[:5]
        print(f"  [served vs oracle] {n_rays} rays K={K}: stable {sum(stable.values())}/{len(sel)}, "
              f"records {len(have)}", flush=True)
    assert checked >= 10
    srv.close()
