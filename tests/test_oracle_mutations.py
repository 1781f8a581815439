"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutation below is a plausible slip (a dropped term, a wrong sign, index or constant,
a transposed operand) applied to a copy of oracle.c; the copy is built into a temporary
library and the pin suite is run against it in a subprocess.  The suite must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = [
    ("changeover denominator", "2.0 * y * y - 2.0 * y + 1.0", "2.0 * y * y - y + 1.0"),
    ("changeover inner edge", "double y = (r - 0.1 * rc) / (0.9 * rc);", "double y = (r - 0.2 * rc) / (0.8 * rc);"),
    ("pair radius min instead of max",
     "double rcij = rc[i] > rc[j] ? rc[i] : rc[j];\n        double k = pair_weight",
     "double rcij = rc[i] < rc[j] ? rc[i] : rc[j];\n        double k = pair_weight"),
    ("force sign", "double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];\n        double r2 = sep2(dx, dy, dz);\n        double rcij",
     "double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];\n        double r2 = sep2(dx, dy, dz);\n        double rcij"),
    ("r^-3 -> r^-2", "double s = m[j] * k / (r2 * r);", "double s = m[j] * k / (r2);"),
    ("source mass index", "double s = m[j] * k / (r2 * r);", "double s = m[i] * k / (r2 * r);"),
    ("transposed y/z in force", "sy += s * dy;\n        sz += s * dz;", "sy += s * dz;\n        sz += s * dy;"),
    ("energy pair mass index", "s += m[j] / sqrt(sep2(dx, dy, dz));", "s += m[i] / sqrt(sep2(dx, dy, dz));"),
    ("energy kinetic factor", "kin += 0.5 * m[i]", "kin += 1.0 * m[i]"),
    ("energy drops sun term", "out[0] = kin + (px * px + py * py + pz * pz) / (2.0 * mstar) + pot_sun - pot_pair;",
     "out[0] = kin + pot_sun - pot_pair;"),
    ("L cross-product sign", "lx += m[i] * (y[i] * vz[i] - z[i] * vy[i]);", "lx += m[i] * (y[i] * vz[i] + z[i] * vy[i]);"),
    ("Kepler fdot sign", "fd = -a * a * nm * sX / (r * r0);", "fd = a * a * nm * sX / (r * r0);"),
    ("Kepler g term", "g = dt - (X - sX) / nm;", "g = dt - (X + sX) / nm;"),
    ("Kepler equation term", "double F = X - c * sin(X) + s * (1.0 - cos(X)) - target;",
     "double F = X - c * sin(X) - s * (1.0 - cos(X)) - target;"),
    ("hyperbolic fdot", "fd = -A * A * nm * shX / (r * r0);", "fd = A * A * nm * shX / (r * r0);"),
    ("sun drift index", "y[i] += tau * py / mstar;", "y[i] += tau * px / mstar;"),
    ("BS uses K instead of 1-K", "for (int k = 0; k < nlev; ++k) w *= 1.0 - pair_weight(r2, rcij[k]);",
     "for (int k = 0; k < nlev; ++k) w *= pair_weight(r2, rcij[k]);"),
    # (a wrong extrapolation coefficient only costs work: the accepted result is still held
    # to the tolerance by the error estimate, so it is not listed here)
    ("BS acceptance tolerance", "if (err <= tol) done = k;", "if (err <= 1e-5) done = k;"),
    ("BS midpoint end correction", "out[q] = 0.5 * (zm[q] + zc[q] + h * dd[q]);", "out[q] = 0.5 * (zm[q] + zc[q]);"),
    ("drift full sun step", "oracle_sun_drift(n, x, y, z, vx, vy, vz, m, mstar, 0.5 * dt);\n    int64_t *gid",
     "oracle_sun_drift(n, x, y, z, vx, vy, vz, m, mstar, dt);\n    int64_t *gid"),
    ("first half-kick length",
     "kick(n, nm, x, y, z, vx, vy, vz, m, rc, 0.5 * dt, ax, ay, az);\n        int64_t np = oracle_encounters(n, nm, x, y, z, rc, cap, pairs);\n        if (np > cap) {\n            free(pairs);\n            cap = np;",
     "kick(n, nm, x, y, z, vx, vy, vz, m, rc, dt, ax, ay, az);\n        int64_t np = oracle_encounters(n, nm, x, y, z, rc, cap, pairs);\n        if (np > cap) {\n            free(pairs);\n            cap = np;"),
    ("Hill radius factor 3", "double rh = a * cbrt(m[i] / (3.0 * mstar));", "double rh = a * cbrt(m[i] / mstar);"),
    ("Hill radius with the distance for a", "double a = (inv_a > 0.0) ? 1.0 / inv_a : r;", "double a = r;"),
    ("Kepler velocity read as the speed", "double vk = sqrt(mstar / a);", "double vk = sqrt(v2);"),
    ("unbound body keeps |1/inv_a|", "double a = (inv_a > 0.0) ? 1.0 / inv_a : r;",
     "double a = (inv_a > 0.0) ? 1.0 / inv_a : -1.0 / inv_a;"),
    ("osculating 1/a with the speed unsquared", "double inv_a = 2.0 / r - v2 / mstar;",
     "double inv_a = 2.0 / r - sqrt(v2) / mstar;"),
    ("TP2 test bodies interact", "        if (i >= nm && j >= nm) continue; /* two test bodies */\n", ""),
    ("TP2 energy keeps test pairs", "            if (i >= nm && j >= nm) continue;\n            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];\n            s += m[j]",
     "            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];\n            s += m[j]"),
    ("TP2 BS keeps test pairs", "            if (gtest[a] && gtest[b]) continue;\n", ""),
    ("level weight drops the outer levels", "    for (int k = 0; k < l; ++k) w *= 1.0 - pair_weight(r2, rcij[k]);\n", ""),
    ("level kick over a whole sub-step",
     "level_kick(l, nlev, nb, idx, nm, x, y, z, vx, vy, vz, m, rcl, n, 0.5 * h);\n        int64_t np = 0;",
     "level_kick(l, nlev, nb, idx, nm, x, y, z, vx, vy, vz, m, rcl, n, h);\n        int64_t np = 0;"),
    ("level sub-step length", "const double h = tau / nsub;", "const double h = tau / (nsub + 1);"),
    ("deepest integration with level 0 only",
     "if (l == nlev) return bs_group_levels(nb, idx, nm, x, y, z, vx, vy, vz, m, rcl, n, nlev, mstar, tau, tol);",
     "if (l == nlev) return bs_group_levels(nb, idx, nm, x, y, z, vx, vy, vz, m, rcl, n, 1, mstar, tau, tol);"),
    ("level members left undrifted", "if (gid[idx[a]] < 0)\n                bad |= kepler_one",
     "if (gid[idx[a]] < -1)\n                bad |= kepler_one"),
    ("level kick target mass", "double s = m[j] * w / (r2 * r);", "double s = m[i] * w / (r2 * r);"),
    ("collision closest approach unclamped", "            if (t > dt) t = dt;\n", ""),
    ("collision radius sum", "double rs = radius[i] + radius[j];", "double rs = radius[i];"),
    ("collision groups keep dead bodies", "        np = live_pairs(np, pairs, status);\n", ""),
    ("merge velocity weights swapped", "vx[i] = (mi * vx[i] + mj * vx[j]) / mt;", "vx[i] = (mj * vx[i] + mi * vx[j]) / mt;"),
    ("merge radius adds radii", "radius[i] = cbrt(radius[i] * radius[i] * radius[i] + radius[j] * radius[j] * radius[j]);",
     "radius[i] = radius[i] + radius[j];"),
    ("removal inner radius unsquared", "if (r2 < r_min * r_min || r2 > r_max * r_max) {", "if (r2 < r_min || r2 > r_max * r_max) {"),
    ("merge of an already merged body", "        if (status[i] || status[j]) continue;\n        double mi = m[i]", "        double mi = m[i]"),
    ("encounter self pairs counted", "for (int64_t j = i + 1; j < n; ++j) c += is_encounter",
     "for (int64_t j = i; j < n; ++j) c += is_encounter"),
    ("encounter self pairs listed", "for (int64_t j = i + 1; j < n && k < cap; ++j)",
     "for (int64_t j = i; j < n && k < cap; ++j)"),
    ("encounter pair radius min", "    double rcij = rc[i] > rc[j] ? rc[i] : rc[j];\n    return sep2",
     "    double rcij = rc[i] < rc[j] ? rc[i] : rc[j];\n    return sep2"),
]


PIN_FILES = {"pins": "test_oracle_pins.py", "levels": "test_oracle_levels.py"}


PIN_FILES["collisions"] = "test_oracle_collisions.py"


def pin_file(name):
    """Mistakes in the level code are run against the level pins, those in the collision code
    against the collision pins, the others against the main pin suite."""
    if name.startswith(("level", "deepest")):
        return PIN_FILES["levels"]
    if name.startswith(("collision", "merge", "removal")):
        return PIN_FILES["collisions"]
    return PIN_FILES["pins"]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {name}"
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-w",
                           "-o", str(lib), str(mutated), "-lm"])
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", pin_file(name))],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation '{name}' survived the pins:\n{r.stdout[-2000:]}"
