"""Comparison of the HIP path with the CPU oracle (test host logic).

The rule (FP32 device geometry against the FP64 definition):
  * per ray and segment the device hit id must equal the oracle's, unless the
    device id is in the oracle's acceptable set for that segment (near ties
    within 1e-4 relative, or surfels whose disk / t_eps / grazing thresholds
    lie inside the FP32 error band).  After such an excused difference the ray
    is compared further only if both surfels lie on the same plane with the
    same normal and label (the continuation is then identical); otherwise the
    ray is "diverged" from that segment on;
  * every oracle reception that is received, not ambiguous and on a
    non-diverged segment must be a device record, and every device record on a
    non-diverged segment must be an oracle reception or ambiguous reception;
  * matched records agree in len_poly and len_unf within 1e-5 relative.

FP32 error band used for the oracle's acceptable sets: the device keeps
positions to ~2^-24 of the scene extent per operation; 16 ulps of the extent
per segment (times the segment index + 1) plus 16 ulps of direction per unit
length bound what a correct FP32 implementation can deviate by.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def fp32_bands(scene_xyz, tx, rx):
    ext = float(max(np.abs(scene_xyz).max() if scene_xyz.size else 0.0, np.abs(tx).max(),
                    np.abs(rx).max() if rx.size else 0.0, 1.0))
    return dict(err_abs=16 * U32 * ext, err_dir=16 * U32)


class ParityReport:
    def __init__(self):
        self.segments = 0
        self.exact = 0
        self.excused = 0
        self.equivalent = 0
        self.mismatch = []
        self.records_checked = 0
        self.record_missing = []
        self.record_extra = []
        self.length_bad = []
        self.diverged = {}
        self.overflow = []   # segments decided by oracle.accepts (set larger than the stored array)

    def ok(self):
        return not (self.mismatch or self.record_missing or self.record_extra or self.length_bad)

    def summary(self):
        return (f"segments={self.segments} exact={self.exact} excused={self.excused} equivalent={self.equivalent} "
                f"mismatch={len(self.mismatch)} records={self.records_checked} missing={len(self.record_missing)} "
                f"extra={len(self.record_extra)} length_bad={len(self.length_bad)} diverged_rays={len(self.diverged)} "
                f"overflow={len(self.overflow)}")


def _same_plane(m1, m2, xyz, nrm, label):
    if label[m1] != label[m2]:
        return False
    n1, n2 = nrm[m1], nrm[m2]
    if not np.array_equal(n1, n2):
        return False
    n = n1.astype(np.float64)
    n /= np.linalg.norm(n)
    p1 = xyz[m1].astype(np.float64)
    p2 = xyz[m2].astype(np.float64)
    # FP32 inputs put points of one plane up to a few ulps off it
    return abs(float((p1 - p2) @ n)) <= 8 * U32 * (1.0 + float(np.abs(p1).max()))


def compare(orc, gpu_ids, gpu_rec, xyz, nrm, label, K, rel_len=1e-5):
    """orc: oracle.launch(..., parity=True) result; gpu_ids: [n_total, K+1] int array;
    gpu_rec: dict of numpy arrays (ray, rx, n_refl, len_poly, len_unf)."""
    rep = ParityReport()
    sel = orc["sel"]
    diverged_at = {}
    for r, g in enumerate(sel):
        g = int(g)
        for b in range(K + 1):
            o_id = int(orc["hit_id"][r, b])
            d_id = int(gpu_ids[g, b])
            if o_id == -2:
                if d_id != -2:
                    rep.mismatch.append((g, b, o_id, d_id, "device traced a segment the oracle did not"))
                break
            rep.segments += 1
            if o_id == d_id:
                rep.exact += 1
                if o_id < 0:
                    break
                continue
            n_acc = int(orc["acc_n"][r, b])
            cap = orc["acc_id"].shape[2]
            acc = [int(x) for x in orc["acc_id"][r, b, :min(n_acc, cap)]]
            if n_acc > cap and d_id not in acc:
                # the oracle stored only part of the acceptable set: membership
                # of the device's answer is decided by the oracle's band test
                import oracle
                rep.overflow.append((g, b, n_acc))
                if oracle.accepts(orc, r, b, d_id):
                    acc.append(d_id)
            if d_id in acc:
                rep.excused += 1
                if o_id >= 0 and d_id >= 0 and _same_plane(o_id, d_id, xyz, nrm, label):
                    rep.equivalent += 1
                    continue
                diverged_at[g] = b
                break
            rep.mismatch.append((g, b, o_id, d_id, f"acceptable={acc}"))
            diverged_at[g] = b
            break
    rep.diverged = diverged_at
    sel_set = {int(g): r for r, g in enumerate(sel)}

    def live(g, b):
        return g in sel_set and (g not in diverged_at or b < diverged_at[g])

    orc_rec = {}
    for q in range(orc["n_rec"]):
        key = (int(orc["rec_g"][q]), int(orc["rec_rx"][q]), int(orc["rec_b"][q]))
        orc_rec[key] = (int(orc["rec_flags"][q]), float(orc["rec_lpoly"][q]), float(orc["rec_lunf"][q]))
    dev_rec = {}
    for q in range(len(gpu_rec["ray"])):
        key = (int(gpu_rec["ray"][q]), int(gpu_rec["rx"][q]), int(gpu_rec["n_refl"][q]))
        dev_rec[key] = (float(gpu_rec["len_poly"][q]), float(gpu_rec["len_unf"][q]))
    for key, (flags, lp, lu) in orc_rec.items():
        g, _, b = key
        if not live(g, b):
            continue
        if flags == 1:  # received, unambiguous
            rep.records_checked += 1
            if key not in dev_rec:
                rep.record_missing.append(key)
                continue
        if key in dev_rec:
            dlp, dlu = dev_rec[key]
            if abs(dlp - lp) > rel_len * lp or abs(dlu - lu) > rel_len * max(lu, 1e-30):
                rep.length_bad.append((key, lp, dlp, lu, dlu))
    for key in dev_rec:
        g, _, b = key
        if live(g, b) and key not in orc_rec:
            rep.record_extra.append(key)
    return rep


def device_paths(res):
    """collect_paths output (numpy) -> {(tx, rx, b, labels): [rows]}"""
    out = {}
    for i in range(res["n_rows"]):
        b = int(res["n_refl"][i])
        key = (int(res["tx"][i]), int(res["rx"][i]), b, tuple(int(x) for x in res["key"][i, :b]))
        out.setdefault(key, []).append(dict(ray=int(res["ray"][i]), count=int(res["count"][i]),
                                            rank=int(res["rank"][i]), len_poly=float(res["len_poly"][i]),
                                            len_unf=float(res["len_unf"][i])))
    return out


def to_numpy(d):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in d.items()}


def fp32_direction_ulps(a, b):
    """Max difference of two float32 arrays in units of float32 spacing."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    sp = np.spacing(np.maximum(np.abs(a), np.abs(b)).astype(np.float32)).astype(np.float64)
    return float(np.max(np.abs(a.astype(np.float64) - b.astype(np.float64)) / sp)) if a.size else 0.0


def t_eps_of(s):
    return s.t_eps_value
