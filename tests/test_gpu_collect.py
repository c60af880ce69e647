"""collect_paths against a plain numpy deduplication of the same launch's records.

The expected rows are built from the launch's own reception records and hit
log (labels of the hit points): sort by (tx, rx, b, label_0 .. label_b-1, then
0 past b), len_poly, ray; keep the first kappa rows of every key.  Small
record sets (one-workgroup path) and large ones (radix-sort path) are both
covered, for several kappa.
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


def _expected(s, L, K, kappa):
    rec = {k: v.cpu().numpy() for k, v in L.records().items()}
    hits = L.hit_log[0].cpu().numpy().reshape(-1, K + 1)
    n_rays = L.n_rays
    rows = []
    for ray, rx, b, lp, lu in zip(rec["ray"], rec["rx"], rec["n_refl"], rec["len_poly"], rec["len_unf"]):
        ray, rx, b = int(ray), int(rx), int(b)
        labels = tuple(int(s.label[hits[ray, k]]) for k in range(b))
        key = (ray // n_rays, rx, b) + tuple(x + 1 for x in labels) + (0,) * (K - b)
        rows.append((key, np.float32(lp).view(np.uint32), ray, labels, np.float32(lp), np.float32(lu)))
    rows.sort(key=lambda r: (r[0], int(r[1]), r[2]))
    out, i = [], 0
    while i < len(rows):
        j = i
        while j < len(rows) and rows[j][0] == rows[i][0]:
            j += 1
        for r in range(min(kappa, j - i)):
            key, _, ray, labels, lp, lu = rows[i + r]
            out.append(dict(tx=key[0], rx=key[1], b=key[2], labels=labels, count=j - i, rank=r, ray=ray, lp=lp, lu=lu))
        i = j
    return out, len(set(r[0] for r in rows))


def _check(pcrl, s, L, K, kappa):
    exp, n_keys = _expected(s, L, K, kappa)
    got = parity.to_numpy(pcrl.collect_paths(L, kappa=kappa))
    assert got["n_rows"] == len(exp) and got["n_keys"] == n_keys
    for i, e in enumerate(exp):
        assert (int(got["tx"][i]), int(got["rx"][i]), int(got["n_refl"][i])) == (e["tx"], e["rx"], e["b"]), i
        assert tuple(int(x) for x in got["key"][i, :e["b"]]) == e["labels"], i
        assert all(int(x) == -1 for x in got["key"][i, e["b"]:])
        assert (int(got["count"][i]), int(got["rank"][i]), int(got["ray"][i])) == (e["count"], e["rank"], e["ray"]), i
        assert np.float32(got["len_poly"][i]) == e["lp"] and np.float32(got["len_unf"][i]) == e["lu"], i
        b = e["b"]
        assert np.isfinite(got["points"][i, :b]).all() and np.isnan(got["points"][i, b:]).all()
    return len(exp), got


@pytest.mark.parametrize("n_rx,n_rays,kappa", [(4, 30_000, 1), (4, 30_000, 3), (64, 200_000, 2), (64, 200_000, 1000)])
def test_collect_matches_numpy_dedup(env, n_rx, n_rays, kappa):
    torch, pcrl = env
    s = scenes.box_room(n_rays=n_rays, K=3)
    rng = np.random.default_rng(n_rx)
    rx = np.concatenate([s.rx, (rng.uniform([1, 1, 0.5], [9, 7, 2.5], (n_rx - len(s.rx), 3))).astype(np.float32)])
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, float(np.float32(s.surfel_radius)),
                              t_eps=float(np.float32(parity.t_eps_of(s))))
    L = pcrl.launch_rays(scene, s.tx, rx, n_rays=n_rays, max_reflections=3, hit_log=True)
    n_rec = int(L.stats()["records"])
    print(f"[collect] {n_rx} RX, {n_rays} rays: {n_rec} records, kappa {kappa}", flush=True)
    # both collection paths are exercised: a single workgroup up to 2048 records, radix sorts above
    assert (n_rec <= 2048) == (n_rx == 4)
    _check(pcrl, s, L, 3, kappa)


def test_collect_capacity_overflow(env):
    torch, pcrl = env
    s = scenes.box_room(n_rays=30_000, K=2)
    scene = pcrl.build_voxels(s.xyz, s.normal, s.label, s.levels, float(np.float32(s.surfel_radius)),
                              t_eps=float(np.float32(parity.t_eps_of(s))))
    L = pcrl.launch_rays(scene, s.tx, s.rx, n_rays=30_000, max_reflections=2)
    full = parity.to_numpy(pcrl.collect_paths(L, kappa=1 << 20))
    # too small a capacity is grown by the binding after the library reports the rows needed
    small = parity.to_numpy(pcrl.collect_paths(L, kappa=1 << 20, capacity=3))
    for k in ("tx", "rx", "n_refl", "key", "count", "rank", "ray", "len_poly", "len_unf"):
        assert np.array_equal(full[k], small[k]), k
