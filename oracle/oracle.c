/*
 * FP64 CPU oracle for the long-range kick path of a GENGA-style hybrid symplectic
 * N-body integrator (Brasser, Grimm, Hatalova & Stadel 2023, "Speeding up the GENGA
 * N-body integrator on consumer-grade graphics cards").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this file.  It shares no code, header, table or
 * constant with the HIP library; it is deliberately plain: double precision,
 * straight loops, j summed in ascending order, no blocking, no fast-math
 * (build with -O2 -ffp-contract=off so that a*b+c is never fused).
 *
 * Units: G = 1, central mass Mstar given per call, lengths in au.  Coordinates are
 * democratic heliocentric: heliocentric positions r_i, barycentric velocities v_i.
 *
 * What the paper fixes and what this file reads into it:
 *  - eq. (1), Sect. 1: r_crit,i = max(n1 R_H,i, n2 dt v_i), R_H,i = a_i (m_i/3Mstar)^(1/3).
 *    a_i is the osculating semi-major axis of the body's Kepler part (heliocentric r,
 *    barycentric v, mu = G Mstar); v_i = sqrt(G Mstar/a_i) is the Kepler velocity.
 *  - Sect. 1: level 0 is a fixed-step symplectic step about the central mass, level 1
 *    Bulirsch-Stoer for close encounters, with a changeover function between them
 *    (the one of Chambers 1999, which the paper cites).  Read here as the force split
 *    F = K F_N (kick) + (1-K) F_N (encounter step), with
 *        K(y) = 0 (y<0),  y^2/(2y^2-2y+1) (0<=y<=1),  1 (y>1),
 *        y = (r_ij - 0.1 r_crit,ij) / (0.9 r_crit,ij),  r_crit,ij = max(r_crit,i, r_crit,j).
 *  - Sect. 1: long-range forces in FP64 (or FP32 on the GPU); the Kepler solver and the
 *    close-encounter forces always in FP64.  This oracle is all FP64.
 *  - Sect. 3.1: Delta E/E = E(t)/E_0 - 1 and Delta L/L = L(t)/L_0 - 1.
 *  - Step order (democratic heliocentric split): Kick(dt/2), Sun drift(dt/2),
 *    [Kepler drift | Bulirsch-Stoer for encounter groups](dt), Sun drift(dt/2), Kick(dt/2).
 *  - TP2 mode (Sect. 3.3): with nm < n, bodies nm..n-1 are test bodies that feel and exert
 *    forces on bodies 0..nm-1 but do not interact with each other; nm = n is the plain
 *    fully self-gravitating system.
 *  - A pair is an encounter pair iff r_ij^2 < r_crit,ij^2, with
 *    r_ij^2 = (dx*dx + dy*dy) + dz*dz evaluated left to right in FP64, at the positions
 *    the kick used.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Number of OpenMP threads the parallel loops use (reported with CPU timings). */
int oracle_num_threads(void)
{
    return omp_get_max_threads();
}

/* Threads of the later parallel loops (timings on one core); the results do not depend on it. */
void oracle_set_num_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}

/* ------------------------------------------------------------------------------------
 * Changeover function (Sect. 1; the Chambers 1999 form cited there).
 * ---------------------------------------------------------------------------------- */
double oracle_changeover(double y)
{
    if (y <= 0.0) return 0.0;
    if (y >= 1.0) return 1.0;
    return (y * y) / (2.0 * y * y - 2.0 * y + 1.0);
}

/* Pair weight K for separation^2 r2 and pair critical radius rc. */
static double pair_weight(double r2, double rc)
{
    if (!(r2 < rc * rc)) return 1.0;
    double r = sqrt(r2);
    double y = (r - 0.1 * rc) / (0.9 * rc);
    return oracle_changeover(y);
}

static double sep2(double dx, double dy, double dz)
{
    return (dx * dx + dy * dy) + dz * dz;
}

/* ------------------------------------------------------------------------------------
 * Critical radius, eq. (1).
 * ---------------------------------------------------------------------------------- */
void oracle_rcrit(int64_t n, const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz, const double *m,
                  double mstar, double n1, double n2, double dt, double *rc)
{
    for (int64_t i = 0; i < n; ++i) {
        double r = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
        double v2 = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
        double inv_a = 2.0 / r - v2 / mstar;       /* osculating 1/a of the Kepler part */
        double a = (inv_a > 0.0) ? 1.0 / inv_a : r; /* unbound: use the distance */
        double rh = a * cbrt(m[i] / (3.0 * mstar));
        double vk = sqrt(mstar / a);
        double t1 = n1 * rh, t2 = n2 * dt * vk;
        rc[i] = (t1 > t2) ? t1 : t2;
    }
}

/* ------------------------------------------------------------------------------------
 * Long-range (changeover-weighted) accelerations: the kick's force, Sect. 1.
 *   a_i = sum_{j != i} m_j K(r_ij) (r_j - r_i) / r_ij^3
 * ---------------------------------------------------------------------------------- */
static void accel_row(int64_t n, int64_t nm, int64_t i, const double *x, const double *y,
                      const double *z, const double *m, const double *rc, double *ax, double *ay,
                      double *az)
{
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        if (i >= nm && j >= nm) continue; /* two test bodies */
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r2 = sep2(dx, dy, dz);
        double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
        double k = pair_weight(r2, rcij);
        if (k == 0.0) continue;
        double r = sqrt(r2);
        double s = m[j] * k / (r2 * r);
        sx += s * dx;
        sy += s * dy;
        sz += s * dz;
    }
    *ax = sx;
    *ay = sy;
    *az = sz;
}

void oracle_accel(int64_t n, int64_t nm, const double *x, const double *y, const double *z,
                  const double *m, const double *rc, double *ax, double *ay, double *az)
{
#pragma omp parallel for schedule(dynamic, 16) if (n >= 256)
    for (int64_t i = 0; i < n; ++i)
        accel_row(n, nm, i, x, y, z, m, rc, &ax[i], &ay[i], &az[i]);
}

/* Same sum for a chosen subset of rows (used for sampled checks at large n). */
void oracle_accel_rows(int64_t n, int64_t nm, const double *x, const double *y, const double *z,
                       const double *m, const double *rc, int64_t nrows, const int64_t *rows,
                       double *ax, double *ay, double *az)
{
#pragma omp parallel for schedule(dynamic, 4) if (nrows >= 64)
    for (int64_t k = 0; k < nrows; ++k)
        accel_row(n, nm, rows[k], x, y, z, m, rc, &ax[k], &ay[k], &az[k]);
}

/* ------------------------------------------------------------------------------------
 * Close-encounter pair list: every (i, j), i < j, with r_ij < r_crit,ij, in
 * lexicographic order.  Returns the number of pairs (which may exceed cap; only the
 * first cap are written).
 * ---------------------------------------------------------------------------------- */
static int is_encounter(int64_t nm, int64_t i, int64_t j, const double *x, const double *y, const double *z,
                        const double *rc)
{
    if (i >= nm && j >= nm) return 0; /* test bodies do not meet each other */
    double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
    double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
    return sep2(dx, dy, dz) < rcij * rcij;
}

/* Rows i in parallel: a first pass counts each row's pairs, their prefix sums place every row
 * in the output, a second pass writes the pairs (i ascending, then j): the order and the
 * decisions are those of the plain double loop. */
int64_t oracle_encounters(int64_t n, int64_t nm, const double *x, const double *y, const double *z,
                          const double *rc, int64_t cap, int32_t *pairs)
{
    int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
#pragma omp parallel for schedule(dynamic, 64) if (n >= 256)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = i + 1; j < n; ++j) c += is_encounter(nm, i, j, x, y, z, rc);
        first[i + 1] = c;
    }
    first[0] = 0;
    for (int64_t i = 0; i < n; ++i) first[i + 1] += first[i];
#pragma omp parallel for schedule(dynamic, 64) if (n >= 256)
    for (int64_t i = 0; i < n; ++i) {
        if (first[i] == first[i + 1] || first[i] >= cap) continue;
        int64_t k = first[i];
        for (int64_t j = i + 1; j < n && k < cap; ++j)
            if (is_encounter(nm, i, j, x, y, z, rc)) {
                pairs[2 * k] = (int32_t)i;
                pairs[2 * k + 1] = (int32_t)j;
                ++k;
            }
    }
    int64_t cnt = first[n];
    free(first);
    return cnt;
}

/* ------------------------------------------------------------------------------------
 * Energy and angular momentum (Sect. 3.1 diagnostics), democratic heliocentric form:
 *   E = sum m v^2/2 + |sum m v|^2/(2 Mstar) - sum Mstar m / r - sum_{i<j} m_i m_j / r_ij
 *   L = sum m r x v
 * out[0] = E, out[1..3] = L.
 * ---------------------------------------------------------------------------------- */
void oracle_energy(int64_t n, int64_t nm, const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz, const double *m,
                   double mstar, double *out)
{
    double kin = 0.0, pot_sun = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    double lx = 0.0, ly = 0.0, lz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        kin += 0.5 * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        pot_sun -= mstar * m[i] / sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
        px += m[i] * vx[i];
        py += m[i] * vy[i];
        pz += m[i] * vz[i];
        lx += m[i] * (y[i] * vz[i] - z[i] * vy[i]);
        ly += m[i] * (z[i] * vx[i] - x[i] * vz[i]);
        lz += m[i] * (x[i] * vy[i] - y[i] * vx[i]);
    }
    double *row = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
#pragma omp parallel for schedule(dynamic, 16) if (n >= 256)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = i + 1; j < n; ++j) {
            if (i >= nm && j >= nm) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            s += m[j] / sqrt(sep2(dx, dy, dz));
        }
        row[i] = m[i] * s;
    }
    double pot_pair = 0.0;
    for (int64_t i = 0; i < n; ++i) pot_pair += row[i];
    free(row);
    out[0] = kin + (px * px + py * py + pz * pz) / (2.0 * mstar) + pot_sun - pot_pair;
    out[1] = lx;
    out[2] = ly;
    out[3] = lz;
}

/* ------------------------------------------------------------------------------------
 * Sun drift: r_i += tau * (sum_j m_j v_j) / Mstar  (the |P|^2/2Mstar part of the split).
 * ---------------------------------------------------------------------------------- */
void oracle_sun_drift(int64_t n, double *x, double *y, double *z, const double *vx,
                      const double *vy, const double *vz, const double *m, double mstar, double tau)
{
    double px = 0.0, py = 0.0, pz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        px += m[i] * vx[i];
        py += m[i] * vy[i];
        pz += m[i] * vz[i];
    }
    for (int64_t i = 0; i < n; ++i) {
        x[i] += tau * px / mstar;
        y[i] += tau * py / mstar;
        z[i] += tau * pz / mstar;
    }
}

/* ------------------------------------------------------------------------------------
 * Kepler drift (always FP64, Sect. 1).  Gauss f and g functions written in the
 * difference of the eccentric anomaly (elliptic) or of the hyperbolic anomaly:
 *   elliptic   : n dt = X - c sin X + s (1 - cos X),  c = 1 - r0/a, s = r0.v0/(n a^2)
 *   hyperbolic : n dt = c sinh X + s (cosh X - 1) - X, c = 1 + r0/A, s = r0.v0/(n A^2), A = -a
 * solved by safeguarded Newton iteration.  Returns 0 on success, 1 if not converged.
 * ---------------------------------------------------------------------------------- */
static int kepler_one(double *rx, double *ry, double *rz, double *wx, double *wy, double *wz,
                      double mu, double dt)
{
    double x0 = *rx, y0 = *ry, z0 = *rz, u0 = *wx, v0 = *wy, w0 = *wz;
    double r0 = sqrt(x0 * x0 + y0 * y0 + z0 * z0);
    double vv = u0 * u0 + v0 * v0 + w0 * w0;
    double rv = x0 * u0 + y0 * v0 + z0 * w0;
    double alpha = 2.0 / r0 - vv / mu; /* 1/a */
    double f, g, fd, gd;
    int ok = 0;
    if (alpha > 0.0) {
        double a = 1.0 / alpha;
        double nm = sqrt(mu * alpha * alpha * alpha);
        double c = 1.0 - r0 / a, s = rv / (nm * a * a);
        double target = nm * dt;
        double X = target, lo = target - 2.0, hi = target + 2.0;
        for (int it = 0; it < 100; ++it) {
            double F = X - c * sin(X) + s * (1.0 - cos(X)) - target;
            double Fp = 1.0 - c * cos(X) + s * sin(X);
            if (F > 0.0) hi = X; else lo = X;
            double step = F / Fp;
            if (fabs(step) <= 1e-15 * (1.0 + fabs(X))) { X -= step; ok = 1; break; }
            double Xn = X - step;
            if (!(Xn > lo && Xn < hi)) Xn = 0.5 * (lo + hi);
            X = Xn;
        }
        double sX = sin(X), cX = cos(X);
        double r = a * (1.0 - c * cX + s * sX);
        f = 1.0 - (a / r0) * (1.0 - cX);
        g = dt - (X - sX) / nm;
        fd = -a * a * nm * sX / (r * r0);
        gd = 1.0 - (a / r) * (1.0 - cX);
    } else if (alpha < 0.0) {
        double A = -1.0 / alpha;
        double nm = sqrt(-mu * alpha * alpha * alpha);
        double c = 1.0 + r0 / A, s = rv / (nm * A * A);
        double target = nm * dt;
        /* G(X) = c sinh X + s (cosh X - 1) - X - target, increasing in X */
        double X = (target > 0.0) ? log(1.0 + 2.0 * target / c) : -log(1.0 - 2.0 * target / c);
        double lo = -1e3, hi = 1e3;
        for (int it = 0; it < 200; ++it) {
            double G = c * sinh(X) + s * (cosh(X) - 1.0) - X - target;
            double Gp = c * cosh(X) + s * sinh(X) - 1.0;
            if (G > 0.0) hi = X; else lo = X;
            double step = G / Gp;
            if (fabs(step) <= 1e-15 * (1.0 + fabs(X))) { X -= step; ok = 1; break; }
            double Xn = X - step;
            if (!(Xn > lo && Xn < hi)) Xn = 0.5 * (lo + hi);
            X = Xn;
        }
        double shX = sinh(X), chX = cosh(X);
        double r = A * (c * chX + s * shX - 1.0);
        f = 1.0 - (A / r0) * (chX - 1.0);
        g = dt - (shX - X) / nm;
        fd = -A * A * nm * shX / (r * r0);
        gd = 1.0 - (A / r) * (chX - 1.0);
    } else {
        return 1; /* exactly parabolic: not met by the workloads */
    }
    *rx = f * x0 + g * u0;
    *ry = f * y0 + g * v0;
    *rz = f * z0 + g * w0;
    *wx = fd * x0 + gd * u0;
    *wy = fd * y0 + gd * v0;
    *wz = fd * z0 + gd * w0;
    return ok ? 0 : 1;
}

int oracle_kepler_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                        double *vz, double mu, double dt, const uint8_t *skip)
{
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (skip && skip[i]) continue;
        bad |= kepler_one(&x[i], &y[i], &z[i], &vx[i], &vy[i], &vz[i], mu, dt);
    }
    return bad;
}

/* ------------------------------------------------------------------------------------
 * Close-encounter step (level 1, Sect. 1): each group of bodies linked by encounter
 * pairs is integrated over dt, in FP64, with Gragg-Bulirsch-Stoer (modified midpoint
 * with n_k = 2k sub-steps, k = 1..8, polynomial extrapolation in h^2) under the
 * Hamiltonian  sum_i (p_i^2/2m_i - Mstar m_i/r_i) - sum_{i<j in group} (1-K_ij) m_i m_j/r_ij.
 * A step H is accepted when the last two extrapolated values agree to tol, measured
 * against the group's position and velocity scales; otherwise H is halved.
 * ---------------------------------------------------------------------------------- */
#define BS_KMAX 8
#define ORACLE_MAX_LEVELS 8

/* Weight of the deepest integration for a pair: prod_{k<nlev} (1 - K_k), rcij[k] being the
 * pair's critical radius of level k (one level: 1 - K). */
static double encounter_weight(double r2, int nlev, const double *rcij)
{
    double w = 1.0;
    for (int k = 0; k < nlev; ++k) w *= 1.0 - pair_weight(r2, rcij[k]);
    return w;
}

/* grc[k * nb + a]: level-k critical radius of member a */
static void group_rhs(int nb, const double *Y, double *D, const double *gm, const double *grc,
                      int nlev, const uint8_t *gtest, double mstar)
{
    /* Y = [x y z vx vy vz] per body, 6 doubles each */
    for (int a = 0; a < nb; ++a) {
        const double *ya = Y + 6 * a;
        double r2 = ya[0] * ya[0] + ya[1] * ya[1] + ya[2] * ya[2];
        double r = sqrt(r2);
        double s = -mstar / (r2 * r);
        D[6 * a + 0] = ya[3];
        D[6 * a + 1] = ya[4];
        D[6 * a + 2] = ya[5];
        D[6 * a + 3] = s * ya[0];
        D[6 * a + 4] = s * ya[1];
        D[6 * a + 5] = s * ya[2];
    }
    /* rows are independent (each a sums over b in index order): threads split the rows only */
#pragma omp parallel for schedule(static) if (nb >= 256)
    for (int a = 0; a < nb; ++a) {
        for (int b = 0; b < nb; ++b) {
            if (b == a) continue;
            if (gtest[a] && gtest[b]) continue;
            const double *ya = Y + 6 * a, *yb = Y + 6 * b;
            double dx = yb[0] - ya[0], dy = yb[1] - ya[1], dz = yb[2] - ya[2];
            double r2 = sep2(dx, dy, dz);
            double rcij[ORACLE_MAX_LEVELS];
            for (int k = 0; k < nlev; ++k)
                rcij[k] = grc[k * nb + a] > grc[k * nb + b] ? grc[k * nb + a] : grc[k * nb + b];
            double w = encounter_weight(r2, nlev, rcij);
            if (w == 0.0) continue;
            double r = sqrt(r2);
            double s = gm[b] * w / (r2 * r);
            D[6 * a + 3] += s * dx;
            D[6 * a + 4] += s * dy;
            D[6 * a + 5] += s * dz;
        }
    }
}

/* modified midpoint over H with nsub sub-steps: Y0 -> out */
static void modified_midpoint(int nb, const double *Y0, double H, int nsub, double *out,
                              double *zm, double *zc, double *dd, const double *gm,
                              const double *grc, int nlev, const uint8_t *gtest, double mstar)
{
    int dim = 6 * nb;
    double h = H / nsub;
    group_rhs(nb, Y0, dd, gm, grc, nlev, gtest, mstar);
    for (int q = 0; q < dim; ++q) {
        zm[q] = Y0[q];
        zc[q] = Y0[q] + h * dd[q];
    }
    for (int k = 1; k < nsub; ++k) {
        group_rhs(nb, zc, dd, gm, grc, nlev, gtest, mstar);
        for (int q = 0; q < dim; ++q) {
            double t = zm[q] + 2.0 * h * dd[q];
            zm[q] = zc[q];
            zc[q] = t;
        }
    }
    group_rhs(nb, zc, dd, gm, grc, nlev, gtest, mstar);
    for (int q = 0; q < dim; ++q) out[q] = 0.5 * (zm[q] + zc[q] + h * dd[q]);
}

/* Integrate one group's state Y (6*nb) over dt.  Step control: after a step accepted at
 * extrapolation column k the next step is doubled (k <= 4), kept (k = 5, 6) or halved
 * (k = 7); a rejected step is multiplied by 0.9 (tol/err)^(1/15), err being the last
 * column's error estimate, kept within [1/50, 1/2].  Returns 1 (failure) if the step falls below
 * dt * 2^-40 or more than 20000 steps are attempted, else 0. */
static int bs_group(int nb, double *Y, const double *gm, const double *grc, int nlev,
                    const uint8_t *gtest, double mstar, double dt, double tol)
{
    int dim = 6 * nb;
    /* tableau T[k][l] (l <= k), each a state vector */
    double *T = (double *)malloc(sizeof(double) * (size_t)dim * (BS_KMAX * BS_KMAX + 3));
    double *zm = T + (size_t)dim * BS_KMAX * BS_KMAX, *zc = zm + dim, *dd = zc + dim;
#define TAB(k, l) (T + (size_t)dim * ((k) * BS_KMAX + (l)))
    double t = 0.0, H = dt;
    int attempts = 0;
    while (t < dt) {
        int last = H >= (dt - t) * (1.0 - 0x1p-30); /* ends the interval (exactly) */
        if (last) H = dt - t;
        if (H < dt * 0x1p-40 || ++attempts > 20000) { free(T); return 1; }
        double sr = 0.0, sv = 0.0;
        for (int a = 0; a < nb; ++a) {
            const double *ya = Y + 6 * a;
            double rr = sqrt(ya[0] * ya[0] + ya[1] * ya[1] + ya[2] * ya[2]);
            double vv = sqrt(ya[3] * ya[3] + ya[4] * ya[4] + ya[5] * ya[5]);
            if (rr > sr) sr = rr;
            if (vv > sv) sv = vv;
        }
        int done = -1;
        double err = 0.0;
        for (int k = 0; k < BS_KMAX && done < 0; ++k) {
            modified_midpoint(nb, Y, H, 2 * (k + 1), TAB(k, 0), zm, zc, dd, gm, grc, nlev, gtest, mstar);
            for (int l = 1; l <= k; ++l) {
                double ratio = (double)(k + 1) / (double)(k + 1 - l); /* n_k / n_{k-l} */
                double den = ratio * ratio - 1.0;
                for (int q = 0; q < dim; ++q)
                    TAB(k, l)[q] = TAB(k, l - 1)[q] + (TAB(k, l - 1)[q] - TAB(k - 1, l - 1)[q]) / den;
            }
            if (k == 0) continue;
            err = 0.0;
            for (int q = 0; q < dim; ++q) {
                double sc = ((q % 6) < 3) ? sr : sv;
                double e = fabs(TAB(k, k)[q] - TAB(k, k - 1)[q]) / sc;
                if (e > err) err = e;
            }
            if (err <= tol) done = k;
        }
        if (done >= 0) {
            memcpy(Y, TAB(done, done), sizeof(double) * (size_t)dim);
            t = last ? dt : t + H;
            if (done <= 4) H = 2.0 * H;
            else if (done == BS_KMAX - 1) H = 0.5 * H;
        } else {
            /* rejected: shrink by the last column's error, between 1/50 and 1/2 */
            double f = 0.9 * pow(tol / err, 1.0 / (2 * BS_KMAX - 1));
            H = H * fmax(0.02, fmin(0.5, f));
        }
    }
#undef TAB
    free(T);
    return 0;
}

/* Integrate bodies idx[0..nb-1] (a group) of the full arrays in place under the pair
 * weight prod_{k<nlev} (1 - K_k); rcl[k * n + i] is body i's level-k critical radius. */
static int bs_group_levels(int nb, const int32_t *idx, int64_t nm, double *x, double *y, double *z,
                           double *vx, double *vy, double *vz, const double *m, const double *rcl,
                           int64_t n, int nlev, double mstar, double dt, double tol)
{
    double *Y = (double *)malloc(sizeof(double) * (size_t)((7 + nlev) * nb));
    double *gm = Y + 6 * nb, *grc = gm + nb;
    uint8_t *gtest = (uint8_t *)malloc((size_t)nb);
    for (int a = 0; a < nb; ++a) {
        int32_t i = idx[a];
        Y[6 * a + 0] = x[i]; Y[6 * a + 1] = y[i]; Y[6 * a + 2] = z[i];
        Y[6 * a + 3] = vx[i]; Y[6 * a + 4] = vy[i]; Y[6 * a + 5] = vz[i];
        gm[a] = m[i];
        for (int k = 0; k < nlev; ++k) grc[k * nb + a] = rcl[k * n + i];
        gtest[a] = i >= nm;
    }
    int st = bs_group(nb, Y, gm, grc, nlev, gtest, mstar, dt, tol);
    for (int a = 0; a < nb; ++a) {
        int32_t i = idx[a];
        x[i] = Y[6 * a + 0]; y[i] = Y[6 * a + 1]; z[i] = Y[6 * a + 2];
        vx[i] = Y[6 * a + 3]; vy[i] = Y[6 * a + 4]; vz[i] = Y[6 * a + 5];
    }
    free(gtest);
    free(Y);
    return st;
}

/* Public wrapper: integrate bodies idx[0..nb-1] (a group) of the full arrays in place. */
int oracle_bs_group(int nb, const int32_t *idx, int64_t nm, double *x, double *y, double *z,
                    double *vx, double *vy, double *vz, const double *m, const double *rc,
                    double mstar, double dt, double tol)
{
    return bs_group_levels(nb, idx, nm, x, y, z, vx, vy, vz, m, rc, 0, 1, mstar, dt, tol);
}

/* ------------------------------------------------------------------------------------
 * Encounter groups: connected components of the pair graph (union-find), each group's
 * members in ascending body order.  Writes group id per body into gid (-1 = none) and
 * returns the number of groups.
 * ---------------------------------------------------------------------------------- */
static int64_t find_root(int64_t *parent, int64_t a)
{
    while (parent[a] != a) a = parent[a];
    return a;
}

int64_t oracle_groups(int64_t n, int64_t npairs, const int32_t *pairs, int64_t *gid)
{
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) parent[i] = i;
    for (int64_t p = 0; p < npairs; ++p) {
        int64_t a = find_root(parent, pairs[2 * p]), b = find_root(parent, pairs[2 * p + 1]);
        if (a == b) continue;
        if (a < b) parent[b] = a; else parent[a] = b; /* the smaller index is the root */
    }
    for (int64_t i = 0; i < n; ++i) gid[i] = -1;
    for (int64_t p = 0; p < npairs; ++p) {
        gid[pairs[2 * p]] = 0;
        gid[pairs[2 * p + 1]] = 0;
    }
    /* number the groups by their smallest member */
    int64_t ng = 0;
    int64_t *label = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) label[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (gid[i] < 0) continue;
        int64_t r = find_root(parent, i);
        if (label[r] < 0) label[r] = ng++;
        gid[i] = label[r];
    }
    free(label);
    free(parent);
    return ng;
}

/* ------------------------------------------------------------------------------------
 * Hierarchical levels (Sect. 1: intermediate symplectic levels with reduced steps between
 * the level-0 step and the Bulirsch-Stoer step).  The paper describes them without formulas;
 * the reading taken here:
 *  - nlev symplectic levels 0..nlev-1; level k has its own critical radius r_crit,k,i
 *    (eq. (1) with the level's step, dt / nsub^k; supplied by the caller, non-increasing in
 *    k) and K_k = K(y; r_crit,k,ij) with r_crit,k,ij = max over the pair.
 *  - The pair force splits as
 *        F = K_0 F + W_1 K_1 F + ... + W_{nlev-1} K_{nlev-1} F + W_nlev F,
 *    W_l = prod_{k<l} (1 - K_k), so that level l's kick carries W_l K_l F and the deepest
 *    integration (Bulirsch-Stoer) carries W_nlev F.  The weights add up to 1 for every r.
 *  - Level 0 is the plain step.  Level l >= 1 integrates each group of level l-1 over its
 *    parent's interval tau in nsub Strang sub-steps of h = tau / nsub: kick(h/2) with
 *    W_l K_l F over every pair of the group; the level-l pairs are the pairs of the group with
 *    r^2 < r_crit,l,ij^2 at that moment; Kepler drift(h) for members in no level-l pair and
 *    level l+1 (Bulirsch-Stoer after the last level) over h for each connected group of
 *    level-l pairs; kick(h/2) with the new positions.
 *  - Test bodies (TP2 mode) never interact with each other at any level.
 * ---------------------------------------------------------------------------------- */

/* Weight of level l's kick (l < nlev): W_l K_l; of the deepest integration (l == nlev):
 * W_nlev.  rcij[k] is the pair's level-k critical radius. */
double oracle_level_weight(double r2, int l, int nlev, const double *rcij)
{
    double w = 1.0;
    for (int k = 0; k < l; ++k) w *= 1.0 - pair_weight(r2, rcij[k]);
    if (l < nlev) w *= pair_weight(r2, rcij[l]);
    return w;
}

static void pair_rc_levels(const double *rcl, int64_t n, int nlev, int64_t i, int64_t j, double *rcij)
{
    for (int k = 0; k < nlev; ++k) rcij[k] = rcl[k * n + i] > rcl[k * n + j] ? rcl[k * n + i] : rcl[k * n + j];
}

/* v += tau * (level-l pair accelerations among the members idx[0..nb-1]) */
static void level_kick(int l, int nlev, int nb, const int32_t *idx, int64_t nm, const double *x,
                       const double *y, const double *z, double *vx, double *vy, double *vz,
                       const double *m, const double *rcl, int64_t n, double tau)
{
    double *acc = (double *)malloc(sizeof(double) * (size_t)(3 * (nb > 0 ? nb : 1)));
    for (int a = 0; a < nb; ++a) {
        int32_t i = idx[a];
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int b = 0; b < nb; ++b) {
            int32_t j = idx[b];
            if (j == i || (i >= nm && j >= nm)) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r2 = sep2(dx, dy, dz);
            double rcij[ORACLE_MAX_LEVELS];
            pair_rc_levels(rcl, n, nlev, i, j, rcij);
            double w = oracle_level_weight(r2, l, nlev, rcij);
            if (w == 0.0) continue;
            double r = sqrt(r2);
            double s = m[j] * w / (r2 * r);
            sx += s * dx;
            sy += s * dy;
            sz += s * dz;
        }
        acc[3 * a] = sx;
        acc[3 * a + 1] = sy;
        acc[3 * a + 2] = sz;
    }
    for (int a = 0; a < nb; ++a) {
        int32_t i = idx[a];
        vx[i] += tau * acc[3 * a];
        vy[i] += tau * acc[3 * a + 1];
        vz[i] += tau * acc[3 * a + 2];
    }
    free(acc);
}

/* Integrate the members idx[0..nb-1] (ascending) of one group of level l-1 over tau. */
static int level_step(int l, int nlev, int nsub, int nb, const int32_t *idx, int64_t nm, double *x,
                      double *y, double *z, double *vx, double *vy, double *vz, const double *m,
                      const double *rcl, int64_t n, double mstar, double tau, double tol)
{
    if (l == nlev) return bs_group_levels(nb, idx, nm, x, y, z, vx, vy, vz, m, rcl, n, nlev, mstar, tau, tol);
    const double h = tau / nsub;
    int bad = 0;
    int64_t cap = 16 * (int64_t)nb + 16;
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * cap));
    int64_t *gid = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *sub = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    for (int s = 0; s < nsub; ++s) {
        level_kick(l, nlev, nb, idx, nm, x, y, z, vx, vy, vz, m, rcl, n, 0.5 * h);
        int64_t np = 0;
        for (int a = 0; a < nb; ++a)
            for (int b = a + 1; b < nb; ++b) {
                int32_t i = idx[a], j = idx[b];
                if (i >= nm && j >= nm) continue;
                double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                double rcij[ORACLE_MAX_LEVELS];
                pair_rc_levels(rcl, n, nlev, i, j, rcij);
                if (sep2(dx, dy, dz) < rcij[l] * rcij[l]) {
                    if (np == cap) {
                        cap *= 2;
                        pairs = (int32_t *)realloc(pairs, sizeof(int32_t) * (size_t)(2 * cap));
                    }
                    pairs[2 * np] = i;
                    pairs[2 * np + 1] = j;
                    ++np;
                }
            }
        int64_t ng = oracle_groups(n, np, pairs, gid);
        for (int a = 0; a < nb; ++a)
            if (gid[idx[a]] < 0)
                bad |= kepler_one(&x[idx[a]], &y[idx[a]], &z[idx[a]], &vx[idx[a]], &vy[idx[a]], &vz[idx[a]], mstar, h);
        for (int64_t g = 0; g < ng; ++g) {
            int k = 0;
            for (int a = 0; a < nb; ++a)
                if (gid[idx[a]] == g) sub[k++] = idx[a];
            bad |= level_step(l + 1, nlev, nsub, k, sub, nm, x, y, z, vx, vy, vz, m, rcl, n, mstar, h, tol);
        }
        level_kick(l, nlev, nb, idx, nm, x, y, z, vx, vy, vz, m, rcl, n, 0.5 * h);
    }
    free(sub);
    free(gid);
    free(pairs);
    return bad;
}

/* The drift with nlev levels: Sun drift(dt/2); Kepler drift(dt) for bodies in no encounter
 * pair and level 1 (Bulirsch-Stoer when nlev = 1) for each group of the level-0 pairs;
 * Sun drift(dt/2).  rcl[k * n + i]: level-k critical radius (rcl[0..n-1] = r_crit of eq. (1)).
 * nlev = 1 is oracle_drift. */
int oracle_drift_levels(int64_t n, int64_t nm, double *x, double *y, double *z, double *vx, double *vy,
                        double *vz, const double *m, const double *rcl, int nlev, int nsub, double mstar,
                        double dt, int64_t npairs, const int32_t *pairs, double tol)
{
    if (nlev < 1 || nlev > ORACLE_MAX_LEVELS || nsub < 1) return 1;
    int bad = 0;
    oracle_sun_drift(n, x, y, z, vx, vy, vz, m, mstar, 0.5 * dt);
    int64_t *gid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *skip = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int32_t *members = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t ng = oracle_groups(n, npairs, pairs, gid);
    for (int64_t i = 0; i < n; ++i) skip[i] = gid[i] >= 0;
    bad |= oracle_kepler_drift(n, x, y, z, vx, vy, vz, mstar, dt, skip);
    for (int64_t g = 0; g < ng; ++g) {
        int nb = 0;
        for (int64_t i = 0; i < n; ++i)
            if (gid[i] == g) members[nb++] = (int32_t)i;
        bad |= level_step(1, nlev, nsub, nb, members, nm, x, y, z, vx, vy, vz, m, rcl, n, mstar, dt, tol);
    }
    free(members);
    free(skip);
    free(gid);
    oracle_sun_drift(n, x, y, z, vx, vy, vz, m, mstar, 0.5 * dt);
    return bad;
}

/* Drift part of the plain step: Sun drift(dt/2), then over dt the Kepler drift for bodies
 * outside encounter groups and Bulirsch-Stoer for each group, then Sun drift(dt/2).
 * Returns 0 on success, 1 if a Kepler solve or a BS step failed. */
int oracle_drift(int64_t n, int64_t nm, double *x, double *y, double *z, double *vx, double *vy,
                 double *vz, const double *m, const double *rc, double mstar, double dt,
                 int64_t npairs, const int32_t *pairs, double tol)
{
    return oracle_drift_levels(n, nm, x, y, z, vx, vy, vz, m, rc, 1, 1, mstar, dt, npairs, pairs, tol);
}

/* ------------------------------------------------------------------------------------
 * Collisions and removal (Sect. 2: collisions are taken as perfect mergers; bodies are
 * removed when they come closer to the star than r_min or farther than r_max).  The paper
 * gives no detection scheme; the reading taken here:
 *  - only encounter pairs can collide within a step; at the start of the drift, a pair (i, j)
 *    of two live bodies collides if the straight-line relative motion brings it within
 *    R_i + R_j during the drift: t* = clamp(-(dr . dv) / |dv|^2, 0, dt), and
 *    |dr + t* dv|^2 < (R_i + R_j)^2;
 *  - after the drift the colliding pairs merge in ascending (i, j) order, skipping a pair with
 *    a body already merged in this step: body i keeps m_i + m_j, the mass-weighted position
 *    and velocity (momentum is kept) and radius (R_i^3 + R_j^3)^(1/3); body j gets m = 0 and
 *    status 1;
 *  - then every live body with |r| < r_min or |r| > r_max gets m = 0 and status 2;
 *  - a body with status != 0 is in no encounter pair from then on: with m = 0 it exerts no
 *    force, and it moves on as a massless particle (kicked by the live bodies' K-weighted
 *    forces, Kepler-drifted) until the arrays are compacted.
 * status: 0 live, 1 merged into another body, 2 removed by distance.
 * ---------------------------------------------------------------------------------- */
int64_t oracle_collisions(int64_t npairs, const int32_t *pairs, const double *x, const double *y,
                          const double *z, const double *vx, const double *vy, const double *vz,
                          const double *radius, const int32_t *status, double dt, int32_t *out)
{
    int64_t nc = 0;
    for (int64_t p = 0; p < npairs; ++p) {
        int32_t i = pairs[2 * p], j = pairs[2 * p + 1];
        if (status[i] || status[j]) continue;
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double ux = vx[j] - vx[i], uy = vy[j] - vy[i], uz = vz[j] - vz[i];
        double uu = sep2(ux, uy, uz);
        double t = 0.0;
        if (uu > 0.0) {
            t = -((dx * ux + dy * uy) + dz * uz) / uu;
            if (t < 0.0) t = 0.0;
            if (t > dt) t = dt;
        }
        double ex = dx + t * ux, ey = dy + t * uy, ez = dz + t * uz;
        double rs = radius[i] + radius[j];
        if (sep2(ex, ey, ez) < rs * rs) {
            out[2 * nc] = i;
            out[2 * nc + 1] = j;
            ++nc;
        }
    }
    return nc;
}

void oracle_merge(int64_t ncol, const int32_t *col, double *x, double *y, double *z, double *vx,
                  double *vy, double *vz, double *m, double *radius, int32_t *status)
{
    for (int64_t c = 0; c < ncol; ++c) {
        int32_t i = col[2 * c], j = col[2 * c + 1];
        if (status[i] || status[j]) continue;
        double mi = m[i], mj = m[j], mt = mi + mj;
        if (mt > 0.0) {
            x[i] = (mi * x[i] + mj * x[j]) / mt;
            y[i] = (mi * y[i] + mj * y[j]) / mt;
            z[i] = (mi * z[i] + mj * z[j]) / mt;
            vx[i] = (mi * vx[i] + mj * vx[j]) / mt;
            vy[i] = (mi * vy[i] + mj * vy[j]) / mt;
            vz[i] = (mi * vz[i] + mj * vz[j]) / mt;
        }
        m[i] = mt;
        radius[i] = cbrt(radius[i] * radius[i] * radius[i] + radius[j] * radius[j] * radius[j]);
        m[j] = 0.0;
        status[j] = 1;
    }
}

/* Keep the pairs of two live bodies (order kept); returns their number. */
static int64_t live_pairs(int64_t npairs, int32_t *pairs, const int32_t *status)
{
    int64_t k = 0;
    for (int64_t p = 0; p < npairs; ++p) {
        int32_t i = pairs[2 * p], j = pairs[2 * p + 1];
        if (status[i] || status[j]) continue;
        pairs[2 * k] = i;
        pairs[2 * k + 1] = j;
        ++k;
    }
    return k;
}

void oracle_remove(int64_t n, const double *x, const double *y, const double *z, double *m,
                   int32_t *status, double r_min, double r_max)
{
    for (int64_t i = 0; i < n; ++i) {
        if (status[i]) continue;
        double r2 = sep2(x[i], y[i], z[i]);
        if (r2 < r_min * r_min || r2 > r_max * r_max) {
            m[i] = 0.0;
            status[i] = 2;
        }
    }
}

/* v += tau * a_K */
static void kick(int64_t n, int64_t nm, const double *x, const double *y, const double *z,
                 double *vx, double *vy, double *vz, const double *m, const double *rc, double tau,
                 double *ax, double *ay, double *az)
{
    oracle_accel(n, nm, x, y, z, m, rc, ax, ay, az);
    for (int64_t i = 0; i < n; ++i) {
        vx[i] += tau * ax[i];
        vy[i] += tau * ay[i];
        vz[i] += tau * az[i];
    }
}

/* ------------------------------------------------------------------------------------
 * Full steps: Kick(dt/2) Sun(dt/2) [Kepler | BS](dt) Sun(dt/2) Kick(dt/2), nsteps times
 * (with nlev > 1 levels, the drift of oracle_drift_levels; the kick and the encounter list
 * use the level-0 critical radii).
 * The encounter list used by a step's drift is the one at the positions of its first
 * half-kick.  If energy != NULL, energy[4*k..] receives (E, Lx, Ly, Lz) after step k
 * when k is a multiple of cadence (k = 0 is the initial state); the caller sizes it.
 * Returns 0 on success.
 * ---------------------------------------------------------------------------------- */
int oracle_step_levels(int64_t n, int64_t nm, double *x, double *y, double *z, double *vx, double *vy,
                       double *vz, const double *m, const double *rcl, int nlev, int nsub, double mstar,
                       double dt, int64_t nsteps, double tol, int64_t cadence, double *energy)
{
    const double *rc = rcl; /* level 0: the kick's changeover and the encounter list */
    double *ax = (double *)malloc(sizeof(double) * (size_t)(3 * (n > 0 ? n : 1)));
    double *ay = ax + n, *az = ay + n;
    int64_t cap = 16 * n + 16;
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * cap));
    int bad = 0;
    int64_t e_idx = 0;
    if (energy && cadence > 0) oracle_energy(n, nm, x, y, z, vx, vy, vz, m, mstar, energy + 4 * e_idx++);
    for (int64_t s = 1; s <= nsteps; ++s) {
        kick(n, nm, x, y, z, vx, vy, vz, m, rc, 0.5 * dt, ax, ay, az);
        int64_t np = oracle_encounters(n, nm, x, y, z, rc, cap, pairs);
        if (np > cap) {
            free(pairs);
            cap = np;
            pairs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * cap));
            np = oracle_encounters(n, nm, x, y, z, rc, cap, pairs);
        }
        bad |= oracle_drift_levels(n, nm, x, y, z, vx, vy, vz, m, rcl, nlev, nsub, mstar, dt, np, pairs, tol);
        kick(n, nm, x, y, z, vx, vy, vz, m, rc, 0.5 * dt, ax, ay, az);
        if (energy && cadence > 0 && s % cadence == 0)
            oracle_energy(n, nm, x, y, z, vx, vy, vz, m, mstar, energy + 4 * e_idx++);
    }
    free(pairs);
    free(ax);
    return bad;
}

int oracle_step(int64_t n, int64_t nm, double *x, double *y, double *z, double *vx, double *vy,
                double *vz, const double *m, const double *rc, double mstar, double dt,
                int64_t nsteps, double tol, int64_t cadence, double *energy)
{
    return oracle_step_levels(n, nm, x, y, z, vx, vy, vz, m, rc, 1, 1, mstar, dt, nsteps, tol, cadence, energy);
}

/* Full steps with collisions and removal: as oracle_step_levels (rcl holds the radii of
 * levels 0..nlev-1, nlev = nsub = 1 for the plain step), with the colliding pairs found at the
 * start of each drift (from the encounter list of the first half-kick, pairs with a body of
 * status != 0 left out) and merged after it, then removal by distance.  m, radius and status
 * are updated. */
int oracle_step_collide(int64_t n, int64_t nm, double *x, double *y, double *z, double *vx, double *vy,
                        double *vz, double *m, const double *rcl, int64_t nlev, int64_t nsub, double *radius,
                        int32_t *status, double mstar, double dt, int64_t nsteps, double tol, double r_min,
                        double r_max)
{
    const double *rc = rcl; /* level 0: the kick's changeover and the encounter list */
    double *ax = (double *)malloc(sizeof(double) * (size_t)(3 * (n > 0 ? n : 1)));
    double *ay = ax + n, *az = ay + n;
    int64_t cap = 16 * n + 16;
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * cap));
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * cap));
    int bad = 0;
    for (int64_t s = 1; s <= nsteps; ++s) {
        kick(n, nm, x, y, z, vx, vy, vz, m, rc, 0.5 * dt, ax, ay, az);
        int64_t np = oracle_encounters(n, nm, x, y, z, rc, cap, pairs);
        if (np > cap) {
            free(pairs);
            free(col);
            cap = np;
            pairs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * cap));
            col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * cap));
            np = oracle_encounters(n, nm, x, y, z, rc, cap, pairs);
        }
        np = live_pairs(np, pairs, status);
        int64_t nc = oracle_collisions(np, pairs, x, y, z, vx, vy, vz, radius, status, dt, col);
        bad |= oracle_drift_levels(n, nm, x, y, z, vx, vy, vz, m, rcl, nlev, nsub, mstar, dt, np, pairs, tol);
        oracle_merge(nc, col, x, y, z, vx, vy, vz, m, radius, status);
        oracle_remove(n, x, y, z, m, status, r_min, r_max);
        kick(n, nm, x, y, z, vx, vy, vz, m, rc, 0.5 * dt, ax, ay, az);
    }
    free(col);
    free(pairs);
    free(ax);
    return bad;
}
