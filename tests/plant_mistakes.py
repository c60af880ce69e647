"""Plant plausible mistakes in a copy of the oracle and check that its pins fail.

Run by hand (not collected by pytest; several minutes):

    python tests/plant_mistakes.py [group ...]

Groups: launch, refl, diff, sdf, cone, vis.  Each mistake is applied alone to a
fresh copy of oracle/, scenes/ and tests/ in a temporary directory (the C
oracle is rebuilt there), then the group's pin file runs with -x.  A mistake
is caught when that run fails.  Two mistakes only reverse the order of the
merge priorities and of the kappa rows, a convention no pin fixes: they are
expected to pass.  Exit status 1 if any other mistake passes.
"""
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C, PY, CONE = "oracle/oracle.c", "oracle/__init__.py", "oracle/cone.py"

GROUPS = {
    "launch": ("tests/test_oracle_pins.py", [
        ("reflection sign", C,
         "double e[3] = {d[0] - 2.0 * dn * n[0], d[1] - 2.0 * dn * n[1], d[2] - 2.0 * dn * n[2]};",
         "double e[3] = {d[0] + 2.0 * dn * n[0], d[1] + 2.0 * dn * n[1], d[2] + 2.0 * dn * n[2]};"),
        ("reception sphere of the segment only", C, "double rho = a->sigma * (L + s) * w->alpha * inv_sqrt3;",
         "double rho = a->sigma * (s) * w->alpha * inv_sqrt3;"),
        ("tie to the larger index", C, "if (dist2 <= rs2 && (t < tb || (t == tb && m < best))) {",
         "if (dist2 <= rs2 && (t < tb || (t == tb && m > best))) {"),
        ("surfel just left not skipped", C,
         "    for (int64_t m = 0; m < a->n_pts; ++m) {\n        if (m == last) continue;\n"
         "        double den = d[0] * P->nx[m] + d[1] * P->ny[m] + d[2] * P->nz[m];",
         "    for (int64_t m = 0; m < a->n_pts; ++m) {\n"
         "        double den = d[0] * P->nx[m] + d[1] * P->ny[m] + d[2] * P->nz[m];"),
        ("reception past the hit", C, "int received = (s > 0.0) && (s <= tb) && (dist <= rho);",
         "int received = (s > 0.0) && (dist <= rho);"),
        ("disk radius unsquared", C, "const double rs2 = a->r_s * a->r_s;", "const double rs2 = a->r_s;"),
        ("Fibonacci z offset", C, "double z = 1.0 - (double)(2 * j + 1) / (double)n;",
         "double z = 1.0 - (double)(2 * j) / (double)n;"),
        ("kappa keeps the longest", PY, "rows.sort(key=lambda x: (x[0], x[2]))", "rows.sort(key=lambda x: (-x[0], x[2]))"),
        ("t_eps sign", C, "        if (!(t > a->t_eps)) continue;\n        double qx",
         "        if (!(t > -a->t_eps)) continue;\n        double qx"),
    ]),
    "refl": ("tests/test_refine_oracle.py", [
        ("tangent projection sign", C, "g[k - 1][j] = G[j] - gn * n[k - 1][j];", "g[k - 1][j] = G[j] + gn * n[k - 1][j];"),
        ("side test reversed", C, "if (!(sp * sn > 0.0)) status = ORACLE_REF_WRONG_SIDE;",
         "if (!(sp * sn < 0.0)) status = ORACLE_REF_WRONG_SIDE;"),
        ("step times the curvature", C,
         "double step = a->step / (1.0 / dist3(I, IPT(k - 1)) + 1.0 / dist3(I, IPT(k + 1)));",
         "double step = a->step * (1.0 / dist3(I, IPT(k - 1)) + 1.0 / dist3(I, IPT(k + 1)));"),
        ("Fresnel radius without its root", PY, "return float(np.sqrt(wavelength * d1 * d2 / (d1 + d2)))",
         "return float(wavelength * d1 * d2 / (d1 + d2))"),
        ("Fresnel d2 from the start", PY, "r_f = fresnel_radius(d1, float(length[q]) - d1, lam)",
         "r_f = fresnel_radius(d1, float(length[q]), lam)"),
        ("label dedup keeps the longest", PY, "rows.sort(key=lambda p: (float(length[p]), p))",
         "rows.sort(key=lambda p: (-float(length[p]), p))"),
    ]),
    "diff": ("tests/test_refine_oracle.py", [
        ("edge step sign", C, "tp[k - 1] -= step * dot3(g[k - 1], ew[k - 1]);",
         "tp[k - 1] += step * dot3(g[k - 1], ew[k - 1]);"),
        ("no clearance arriving", C, "tb < (k <= N ? len - clear : len)", "tb < len"),
        ("wedge test: and for or", C, "if (!(dot3(v, nn) > 0.0 || dot3(v, nn + 3) > 0.0)) status",
         "if (!(dot3(v, nn) > 0.0 && dot3(v, nn + 3) > 0.0)) status"),
        ("no clearance leaving (iteration)", C, "                skip = clear;", "                skip = 0.0;"),
        ("no clearance leaving (final check)", C, "prev_diff ? clear : 0.0, cc, nn, &mm, &tb);",
         "0.0, cc, nn, &mm, &tb);"),
    ]),
    "cone": ("tests/test_cone_oracle.py", [
        ("Keller count rounded down", CONE, "N = max(1, int(math.ceil(arg)))", "N = max(1, int(math.floor(arg)))"),
        ("sector plane sign", CONE, "math.cos(j * dphi) * e2 - math.sin(j * dphi) * e1",
         "math.cos(j * dphi) * e2 + math.sin(j * dphi) * e1"),
        ("exterior test: and for or", CONE, "ext = max(float(v @ n1), float(v @ n2))", "ext = min(float(v @ n1), float(v @ n2))"),
        ("cone-sphere sine and cosine swapped", CONE, "lateral = rho * cos_t - a * sin_t", "lateral = rho * sin_t - a * cos_t"),
        ("reflected plane sign", CONE, "m_sep = float((pr - o1) @ sep[1]) - tau", "m_sep = float((o1 - pr) @ sep[1]) - tau"),
        ("SplitMix64 constant", CONE, "0xBF58476D1CE4E5B9", "0xBF58476D1CE4E5B8"),
        ("Keller cone reversed", CONE, "axis = cb * w + sb * v", "axis = -cb * w + sb * v"),
        ("sector upper plane left out", CONE, "sep_in = sep[3] and m_lo >= 0 and m_hi < 0", "sep_in = sep[3] and m_lo >= 0"),
        ("IE point is its first point", CONE, 'out["pos"][i] = x64[idx].mean(axis=0)', 'out["pos"][i] = x64[idx[0]]'),
        ("subvoxel by rounding", CONE, "return np.floor(rel * inv).astype(np.int64)", "return np.round(rel * inv).astype(np.int64)"),
        ("no merge", CONE, "        out += head\n", "        out += group\n"),
        ("merge keeps the largest priority (convention)", CONE,
         '    kids.sort(key=lambda c: (c["tx"], c["labels"], c["ie"], c["prio"], c["parent"]))',
         '    kids.sort(key=lambda c: (c["tx"], c["labels"], c["ie"], -c["prio"], c["parent"]))'),
        ("kappa keeps the largest priorities (convention)", CONE,
         'key=lambda r: (r["tx"], r["rx"], len(r["labels"]), r["labels"], r["prio"], r["chain"])',
         'key=lambda r: (r["tx"], r["rx"], len(r["labels"]), r["labels"], -r["prio"], r["chain"])'),
    ]),
    "sdf": ("tests/test_sdf_oracle.py", [
        ("weight squared once", "oracle/sdf.c", "                    w = w * w;\n                    w = w * w;\n",
         "                    w = w * w;\n"),
        ("step over an undefined sample h", "oracle/sdf.c", "            t += 0.5 * a->h;\n", "            t += a->h;\n"),
        ("interpolation from the new sample", "oracle/sdf.c", "*th = tp + (t - tp) * fp / (fp - f);",
         "*th = t + (t - tp) * fp / (fp - f);"),
        ("segment half as long", "oracle/sdf.c", "double ta = tc - 0.5 * D, tb = tc + 0.5 * D;",
         "double ta = tc - 0.25 * D, tb = tc + 0.25 * D;"),
        ("march by twice |f|", "oracle/sdf.c", "        t += fabs(f);\n", "        t += 2.0 * fabs(f);\n"),
    ]),
    "vis": ("tests/test_cone_oracle.py", [
        ("box exit for entry", C, "    return t0 <= t1 ? t0 : INFINITY;\n}", "    return t0 <= t1 ? t1 : INFINITY;\n}"),
        ("blocked up to the target point", C, "w->state[r] = t_clear >= t_in ? 1 : 0; continue; }",
         "w->state[r] = t_clear >= len ? 1 : 0; continue; }"),
        ("slab swap dropped", C, "            if (ta > tb) { double t = ta; ta = tb; tb = t; }\n", ""),
    ]),
}


def run_one(test, f, old, new):
    with tempfile.TemporaryDirectory() as tmp:
        for d in ("oracle", "scenes", "tests"):
            shutil.copytree(os.path.join(ROOT, d), os.path.join(tmp, d),
                            ignore=shutil.ignore_patterns("__pycache__", "*.so"))
        shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp)
        p = os.path.join(tmp, f)
        src = open(p).read()
        if src.count(old) != 1:
            raise SystemExit(f"the line to change occurs {src.count(old)} times in {f}: {old!r}")
        open(p, "w").write(src.replace(old, new))
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", test], cwd=tmp,
                           capture_output=True, text=True)
        failed = [ln.split("::", 1)[1].split(" ")[0] for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
        return r.returncode != 0, failed


def main(groups):
    missed = []
    for g in groups or list(GROUPS):
        test, cases = GROUPS[g]
        for name, f, old, new in cases:
            caught, failed = run_one(test, f, old, new)
            convention = name.endswith("(convention)")
            print(f"{g:7s} {name:48s} {'caught by ' + failed[0] if caught and failed else ('caught' if caught else 'passes')}",
                  flush=True)
            if not caught and not convention:
                missed.append(name)
    if missed:
        print("not caught:", ", ".join(missed))
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
