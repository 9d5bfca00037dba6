"""Mutation check of the oracle's pins (CPU only, test infrastructure).

Each entry plants one plausible mistake (a dropped term, a wrong sign, a
swapped index, an open instead of a closed interval, ...) in a copy of the
oracle made in a temporary directory, and runs the oracle's own pins
(tests/test_oracle_*.py) against the copy: a pin must fail for every
mutation that changes what the oracle computes.  Two entries are
equivalent mutations and survive by construction (see the design notes):
'step voxel zero dir' (step_voxel is only called on an axis whose
direction component is non-zero) and 'electron cut clamp' (the track ends
when its residual range runs out, before the energy can fall below the
cut-off; the clamp only guards the round-off between the step integration
and the range quadrature).

    python oracle/mutation_check.py            # all
    python oracle/mutation_check.py 3 17 40    # some, by index
"""
import json
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

M = [
 # (file, old, new, label)
 ("oracle/oracle.c", "if (v >= edges[j]) k = j;", "if (v > edges[j]) k = j;", "bin ties"),
 ("oracle/oracle.c", "key[i] = (((int64_t)t * n_e + e) * n_y + iy) * n_x + ix;", "key[i] = (((int64_t)t * n_e + e) * n_y + ix) * n_x + iy;", "key x/y swapped"),
 ("oracle/oracle.c", "    for (int64_t i = 0; i < n; ++i) {\n        if (key[i] < 0) continue;", "    for (int64_t i = n - 1; i >= 0; --i) {\n        if (key[i] < 0) continue;", "build unstable"),
 ("oracle/oracle.c", "*s = 2.0 * a * b / r2;", "*s = -2.0 * a * b / r2;", "apr sin sign"),
 ("oracle/oracle.c", "ov[m] = (float)(s * du + c * dv);", "ov[m] = (float)(s * du - c * dv);", "apr dir turn"),
 ("oracle/oracle.c", "owt[m] = (float)((double)wt[i] / (double)k);", "owt[m] = wt[i];", "apr weight"),
 ("oracle/oracle.c", "double f = (sad - z_psl) / (sad - z_jaw);", "double f = (sad - z_jaw) / (sad - z_psl);", "roi magnification"),
 ("oracle/oracle.c", "int keep = ((double)x_edges[ix] < xhi) &&", "int keep = ((double)x_edges[ix] <= xhi) &&", "cull touch"),
 ("oracle/oracle.c", "oracle_roi(Y1[f], Y2[f], z_y, sad, z_psl, &ylo, &yhi);", "oracle_roi(Y1[f], Y2[f], z_x, sad, z_psl, &ylo, &yhi);", "cull y jaw plane"),
 ("oracle/oracle.c", "                         ? (MU[f] / mu_tot) * ((double)nk / (double)N[idx])", "                         ? ((double)nk / (double)N[idx])", "alloc weight MU"),
 ("oracle/oracle.c", "            S += nk;\n            int64_t Fk = (int64_t)(((__int128)Ni * S) / C[f]);", "            int64_t Fk = (int64_t)(((__int128)Ni * S) / C[f]);\n            S += nk;", "alloc prefix off by one"),
 ("oracle/oracle.c", "                            : (int64_t)floor((double)n_sim * m / mu_tot);", "                            : (int64_t)ceil((double)n_sim * m / mu_tot);", "alloc MU floor/ceil"),
 ("oracle/oracle.c", "        double xj = px + tx * (G->z_x - pz);", "        double xj = px + tx * (G->z_y - pz);", "jaw x plane"),
 ("oracle/oracle.c", "        double xlo = F->X1 * G->z_x / G->sad;", "        double xlo = F->X1 * G->sad / G->z_x;", "jaw projection"),
 ("oracle/oracle.c", "        if (!(xj >= xlo && xj <= xhi && yj >= ylo && yj <= yhi)) return 0;", "        if (!(xj > xlo && xj <= xhi && yj >= ylo && yj <= yhi)) return 0;", "jaw open interval"),
 ("oracle/oracle.c", "        double xs = px + (du / dw) * (G->sad - pz);", "        double xs = px + (du / dw) * (G->sad);", "fluence plane"),
 ("oracle/oracle.c", "        double fy = floor((ys - F->f_y0) / F->f_pix);", "        double fy = round((ys - F->f_y0) / F->f_pix);", "fluence pixel round"),
 ("oracle/oracle.c", "    double qz = -F->sin_g * rx + F->cos_g * rz + G->iso[2];", "    double qz = F->sin_g * rx + F->cos_g * rz + G->iso[2];", "gantry pos sign"),
 ("oracle/oracle.c", "    double ew = -F->sin_g * au + F->cos_g * dw;", "    double ew = F->sin_g * au + F->cos_g * dw;", "gantry dir sign"),
 ("oracle/oracle.c", "        double y1 = F->sin_c * rx + F->cos_c * ry;", "        double y1 = -F->sin_c * rx + F->cos_c * ry;", "collimator sign"),
 ("oracle/oracle.c", "        qy = -F->sin_t * sx + F->cos_t * sy + G->iso[1];", "        qy = F->sin_t * sx + F->cos_t * sy + G->iso[1];", "couch pos sign"),
 ("oracle/oracle.c", "        double v2 = -F->sin_t * eu + F->cos_t * ev;", "        double v2 = F->sin_t * eu + F->cos_t * ev;", "couch dir sign"),
 ("oracle/oracle.c", "    double t = tn > 0.0 ? tn : 0.0;", "    double t = tn;", "projection inside box"),
 ("oracle/oracle.c", "    double wgt = (double)wt * fl * gk;", "    double wgt = (double)wt * gk;", "fluence weight dropped"),
 ("oracle/oracle.c", "            uint64_t sk = oracle_splitmix64(seed ^ (uint64_t)k) % (uint64_t)nk;", "            uint64_t sk = oracle_splitmix64(seed + (uint64_t)k) % (uint64_t)nk;", "psl start key"),
 ("oracle/oracle.c", "            uint64_t c = (uint64_t)batch * (uint64_t)Tk + (uint64_t)before;", "            uint64_t c = (uint64_t)batch * (uint64_t)Tk;", "psl cursor fields"),
 ("oracle/oracle.c", "            fl_trigger[n_fl] = r;", "            fl_trigger[n_fl] = r - 1;", "stream trigger"),
 ("oracle/oracle.c", "    for (int b = 0; b < n_bins; ++b) {\n        if (fill[b] == 0) continue;", "    for (int b = n_bins - 1; b >= 0; --b) {\n        if (fill[b] == 0) continue;", "stream end order"),
 ("oracle/oracle.c", "            if (E[p] >= e_edges[k]) e = k;", "            if (E[p] > e_edges[k]) e = k;", "stream energy tie"),
 ("oracle/oracle.c", "        const int64_t p = (int64_t)((s0 + (uint64_t)batch * (uint64_t)n_hist +\n                                     (uint64_t)r) % (uint64_t)n);", "        const int64_t p = (int64_t)((s0 + (uint64_t)batch * (uint64_t)(n_hist + 1) +\n                                     (uint64_t)r) % (uint64_t)n);", "stream batch stride"),
 ("oracle/oracle.c", "    double t3 = (1.0 + 3.0 * k) / (a * a);", "    double t3 = (1.0 + 2.0 * k) / (a * a);", "KN sigma term"),
 ("oracle/oracle.c", "    double L = log(tau * tau * (tau + 2.0) / (2.0 * ir * ir));", "    double L = log(tau * tau * (tau + 2.0) / (2.0 * ir));", "Bethe log"),
 ("oracle/oracle.c", "               (tau * tau / 8.0 - (2.0 * tau + 1.0) * log(2.0)) / (gam * gam);", "               (tau * tau / 8.0 + (2.0 * tau + 1.0) * log(2.0)) / (gam * gam);", "Bethe F sign"),
 ("oracle/oracle.c", "    double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);", "    double left = (m - a) / 6.0 * (fa + 3.0 * flm + fm);", "csda simpson"),
 ("oracle/oracle.c", "        T -= h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);", "        T -= h / 6.0 * (k1 + k2 + k3 + k4) * 1.5;", "csda RK4"),
 ("oracle/oracle.c", "    double th = 13.6 / pbc * sqrt(r) * (1.0 + 0.038 * log(r));", "    double th = 13.6 / pbc * sqrt(r) * (1.0 + 0.088 * log(r));", "Highland log coeff"),
 ("oracle/oracle.c", "        ax = th0 * rr * cos(2.0 * PI * u2);", "        ax = th0 * rr * cos(PI * u2);", "msc box-muller"),
 ("oracle/oracle.c", "        nd[i] = cth * d[i] + sth * (cp * e1[i] + sp * e2[i]);", "        nd[i] = sth * d[i] + cth * (cp * e1[i] + sp * e2[i]);", "deflect cos/sin"),
 ("oracle/oracle.c", "            deposit(C, ijk, T - Tn, wgt);", "            deposit(C, ijk, T - Tn, 1.0);", "electron weight"),
 ("oracle/oracle.c", "            if (Tn < Y->t_cut) Tn = Y->t_cut;\n", "", "electron cut clamp"),
 ("oracle/oracle.c", "            if (dm >= r_left) {     /* residual range runs out here */\n                deposit(C, ijk, T, wgt);", "            if (dm >= r_left) {     /* residual range runs out here */\n                deposit(C, ijk, T - Y->t_cut, wgt);", "electron end deposit"),
 ("oracle/oracle.c", "            double mu = P->rho[vindex(P, ijk)] * mu1;", "            double mu = mu1;", "photon density"),
 ("oracle/oracle.c", "            Pr = 1.0 / (1.0 + k * (1.0 - ct));", "            Pr = 1.0 / (1.0 + k * (1.0 + ct));", "compton kinematics"),
 ("oracle/oracle.c", "            double f = 0.5 * Pr * Pr * (Pr + 1.0 / Pr - (1.0 - ct * ct));", "            double f = 0.5 * Pr * (Pr + 1.0 / Pr - (1.0 - ct * ct));", "KN rejection"),
 ("oracle/oracle.c", "        if (E < Y->p_cut) { deposit(C, ijk, E, wgt); return; }", "        if (E < Y->p_cut) { escape(C, E, d, tr); return; }", "photon cut deposit"),
 ("oracle/oracle.c", "        } else {\n            deposit(C, ijk, T, wgt);\n        }\n        E = Es;", "        } else {\n            C->esc += T;\n        }\n        E = Es;", "sub-cut electron deposit"),
 ("oracle/oracle.c", "        if (f > nn[a] - 1) f = nn[a] - 1;\n", "", "clamp top face"),
 ("oracle/oracle.c", "    ijk[axis] += d[axis] > 0.0 ? 1 : -1;", "    ijk[axis] += d[axis] >= 0.0 ? 1 : -1;", "step voxel zero dir"),
 ("oracle/oracle.c", "        double tau = -log(1.0 - urand(R));", "        double tau = -0.9 * log(1.0 - urand(R));", "photon free path"),
 ("oracle/oracle.c", "    uint64_t res = rotl(s[1] * 5, 7) * 9;", "    uint64_t res = rotl(s[1] * 5, 9) * 7;", "xoshiro output"),
 ("oracle/__init__.py", "    var = np.maximum(s2 - s1 * s1 / B, 0.0) / (B - 1) if B > 1 else \\", "    var = np.maximum(s2 - s1 * s1 / B, 0.0) / B if B > 1 else \\", "Eq5 variance n-1"),
 ("oracle/__init__.py", "    return mean * c, np.sqrt(var / B) * c", "    return mean * c, np.sqrt(var) * c", "Eq5 standard error"),
 ("oracle/__init__.py", "        c = np.where(rho > 0, MEV_PER_G_TO_GY / (rho * V), 0.0) * norm", "        c = np.where(rho > 0, MEV_PER_G_TO_GY / V, 0.0) * norm", "dose mass"),
 ("oracle/__init__.py", "    m = r2 <= radius * radius", "    m = r2 < radius * radius", "dose_point boundary"),
 ("oracle/__init__.py", "    return float(d[m].sum() / n), float(math.sqrt((s[m] ** 2).sum()) / n), n", "    return float(d[m].sum() / n), float(math.sqrt((s[m] ** 2).sum() / n)), n", "dose_point se"),
 ("oracle/analysis.py", "                g2 = d2 / (dta * dta) + ((sh - ref) / dd) ** 2", "                g2 = d2 / (dta * dta) + ((sh - ref) / (2 * dd)) ** 2", "gamma dose crit"),
 ("oracle/analysis.py", "    return t_run * (s / target) ** 2, s", "    return t_run * (s / target), s", "time to uncertainty"),
]
M += [
 ("oracle/unet.py", "        z, yy, xx = o // 9, (o // 3) % 3, o % 3\n        y += xp", "        xx, yy, z = o // 9, (o // 3) % 3, o % 3\n        y += xp", "unet conv tap order"),
 ("oracle/unet.py", "    return x.reshape(N, D // 2, 2, H // 2, 2, W // 2, 2, C).mean((2, 4, 6))", "    return x.reshape(N, D // 2, 2, H // 2, 2, W // 2, 2, C).max((2, 4, 6))", "unet pool max"),
 ("oracle/unet.py", "        cat = np.concatenate([up(h), skips[l]], axis=-1)", "        cat = np.concatenate([skips[l], up(h)], axis=-1)", "unet concat order"),
 ("oracle/unet.py", "    out = dose * scale[:, None, None, None] + h @ wh + bh", "    out = h @ wh + bh", "unet residual"),
 ("oracle/unet.py", "    g = 2.0 * e / e.size", "    g = 2.0 * e", "unet loss scale"),
 ("oracle/unet.py", "            dh = dh * (A[n] > 0)\n            dx, dW, db = conv3_back(A[n + \"_in\"], P[n][0], dh)\n            G[n] = (dW, db)\n            dh = dx\n        cc", "            dx, dW, db = conv3_back(A[n + \"_in\"], P[n][0], dh)\n            G[n] = (dW, db)\n            dh = dx\n        cc", "unet relu mask dec"),
 ("oracle/unet.py", "    scale = np.where(mx > 0, 1.0 / np.where(mx > 0, mx, 1.0), 1.0)", "    scale = np.ones_like(mx)", "unet input scale"),
]


def run(indices=None):
    out = []
    base = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        for i, (f, old, new, label) in enumerate(M):
            if indices is not None and i not in indices:
                continue
            d = os.path.join(base, "%02d" % i)
            os.makedirs(d)
            for sub in ("oracle", "psl_synth"):
                shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub),
                                ignore=shutil.ignore_patterns(
                                    "*.so", "__pycache__"))
            os.makedirs(os.path.join(d, "tests"))
            for fn in os.listdir(os.path.join(ROOT, "tests")):
                if fn.startswith("test_oracle") or fn in ("conftest.py",
                                                          "gpu_util.py"):
                    shutil.copy(os.path.join(ROOT, "tests", fn),
                                os.path.join(d, "tests", fn))
            os.symlink(os.path.join(ROOT, "tests", "golden"),
                       os.path.join(d, "tests", "golden"))
            p = os.path.join(d, f)
            s = open(p).read()
            if old not in s:
                out.append((i, label, "not found"))
                print(i, label, "not found", flush=True)
                continue
            open(p, "w").write(s.replace(old, new, 1))
            try:
                r = subprocess.run(
                    [sys.executable, "-m", "pytest", "tests", "-q", "-x",
                     "-p", "no:cacheprovider", "--timeout", "60"],
                    cwd=d, capture_output=True, text=True, timeout=300)
                killed = r.returncode != 0
                why = [l for l in r.stdout.splitlines()
                       if l.startswith("FAILED")][:1]
            except subprocess.TimeoutExpired:
                killed, why = True, ["timeout"]
            res = "killed" if killed else "SURVIVED"
            out.append((i, label, res))
            print(i, label, res, *why, flush=True)
            shutil.rmtree(d, ignore_errors=True)
    finally:
        shutil.rmtree(base, ignore_errors=True)
    return out


if __name__ == "__main__":
    sel = set(int(a) for a in sys.argv[1:]) or None
    res = run(sel)
    print(json.dumps({"mutations": len(res),
                      "survived": [r for r in res if r[2] != "killed"]}))
