"""Pins of the FP64 oracle against what the mathematics fixes (closed forms, invariants,
independent library integrators, brute force).  CPU only.

Each test names the passage of Brasser et al. (2023) whose computation it pins and what a
plausible mistake it would catch.
"""
import math

import numpy as np
import pytest

import discs
import oracle

MU = 1.0


def state(pos, vel=None, m=None):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = len(pos)
    vel = np.zeros((n, 3)) if vel is None else np.asarray(vel, dtype=np.float64).reshape(-1, 3)
    m = np.ones(n) if m is None else np.asarray(m, dtype=np.float64)
    return dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(),
                vx=vel[:, 0].copy(), vy=vel[:, 1].copy(), vz=vel[:, 2].copy(), m=m.copy())


def vec(st, keys=("x", "y", "z")):
    return np.stack([st[k] for k in keys], axis=1)


# ------------------------------------------------------------------------------------------
# Changeover function K (Sect. 1, the Chambers 1999 function the paper cites)
# ------------------------------------------------------------------------------------------

def test_changeover_special_values():
    K = oracle.changeover
    assert K(-0.3) == 0.0 and K(0.0) == 0.0
    assert K(1.0) == 1.0 and K(1.7) == 1.0
    assert K(0.5) == 0.5                      # y^2/(2y^2-2y+1) at 1/2 is exactly 1/2
    assert abs(K(0.25) - 0.0625 / 0.625) < 1e-16


def test_changeover_symmetry_and_flat_ends():
    K = oracle.changeover
    ys = np.linspace(0.0, 1.0, 1001)
    # K(y) + K(1-y) = 1 holds for the Chambers polynomial ratio; a wrong coefficient breaks it
    sym = max(abs(K(y) + K(1.0 - y) - 1.0) for y in ys)
    assert sym < 4e-16
    # C1 at both ends: K'(0) = K'(1) = 0
    for h in (1e-4, 1e-5):
        assert K(h) / h < 2 * h
        assert (1.0 - K(1.0 - h)) / h < 2 * h
    vals = [K(y) for y in ys]
    assert all(b >= a for a, b in zip(vals, vals[1:]))


# ------------------------------------------------------------------------------------------
# Changeover-weighted long-range force (Sect. 1): closed forms in the Newtonian limit and
# with the weight switched on.
# ------------------------------------------------------------------------------------------

def test_two_body_newtonian():
    st = state([[0.3, -0.2, 0.1], [0.3 + 0.6, -0.2 + 0.8, 0.1]], m=[2e-3, 5e-4])
    rc = np.array([0.01, 0.02])
    ax, ay, az = oracle.accel(st, rc)
    d = 1.0  # |(0.6, 0.8, 0)|
    np.testing.assert_allclose([ax[0], ay[0], az[0]], [5e-4 * 0.6 / d**2, 5e-4 * 0.8 / d**2, 0.0], rtol=1e-15, atol=1e-20)
    np.testing.assert_allclose([ax[1], ay[1], az[1]], [-2e-3 * 0.6, -2e-3 * 0.8, 0.0], rtol=1e-15, atol=1e-20)


def test_two_body_changeover_uses_max_pair_radius():
    # rc_a = 1e-3, rc_b = 2e-3, separation 1.1e-3: inside b's radius only.  With the pair
    # radius max(rc_a, rc_b) = 2e-3: y = (1.1e-3 - 2e-4) / 1.8e-3 = 1/2, so K = 1/2.
    r = 1.1e-3
    st = state([[1.0, 0.0, 0.0], [1.0 + r, 0.0, 0.0]], m=[1e-6, 3e-6])
    ax, _, _ = oracle.accel(st, np.array([1e-3, 2e-3]))
    assert ax[0] == pytest.approx(0.5 * 3e-6 / r**2, rel=1e-12)
    assert ax[1] == pytest.approx(-0.5 * 1e-6 / r**2, rel=1e-12)


def test_changeover_inner_zone_and_boundary():
    rc = np.array([1e-2, 1e-2])
    # inside 0.1 rc the long-range force vanishes
    st = state([[1, 0, 0], [1 + 0.05e-2, 0, 0]], m=[1e-6, 1e-6])
    ax, ay, az = oracle.accel(st, rc)
    assert ax[0] == 0.0 and ax[1] == 0.0
    # at 0.55 rc, K(1/2) = 1/2
    st = state([[1, 0, 0], [1 + 0.55e-2, 0, 0]], m=[1e-6, 1e-6])
    ax, _, _ = oracle.accel(st, rc)
    assert ax[0] == pytest.approx(0.5 * 1e-6 / 0.55e-2**2, rel=1e-12)
    # just outside rc the full Newtonian force applies
    st = state([[1, 0, 0], [1 + 1.0001e-2, 0, 0]], m=[1e-6, 1e-6])
    ax, _, _ = oracle.accel(st, rc)
    assert ax[0] == pytest.approx(1e-6 / 1.0001e-2**2, rel=1e-13)


def test_equilateral_triangle():
    s, m = 0.37, 1e-5
    c = np.array([0.8, -0.4, 0.2])
    pts = c + s / math.sqrt(3) * np.array([[1, 0, 0], [-0.5, math.sqrt(3) / 2, 0], [-0.5, -math.sqrt(3) / 2, 0]])
    st = state(pts, m=[m] * 3)
    a = np.stack(oracle.accel(st, np.zeros(3)), axis=1)
    for k in range(3):
        toward = (c - pts[k]) / np.linalg.norm(c - pts[k])
        mag = math.sqrt(3) * m / s**2
        np.testing.assert_allclose(a[k], mag * toward, rtol=0, atol=1e-14 * mag)


@pytest.mark.parametrize("N", [5, 12, 64])
def test_regular_ngon_ring(N):
    R, m = 0.9, 1e-7
    ang = 2 * np.pi * np.arange(N) / N
    pts = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros(N)], axis=1)
    st = state(pts, m=np.full(N, m))
    a = np.stack(oracle.accel(st, np.zeros(N)), axis=1)
    mag = m / (4 * R * R) * sum(1.0 / math.sin(math.pi * k / N) for k in range(1, N))
    radial = -(a * pts).sum(axis=1) / R
    tang = (a[:, 0] * -np.sin(ang) + a[:, 1] * np.cos(ang))
    np.testing.assert_allclose(radial, mag, rtol=1e-13)
    assert np.max(np.abs(tang)) < 1e-13 * mag
    assert np.max(np.abs(a[:, 2])) == 0.0


def test_brute_force_high_precision():
    """Tiny N, separations placed in every changeover zone; compared with 50-digit mpmath."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(7)
    rc = np.array([2e-3, 1e-3, 3e-3, 2.5e-3, 1.5e-3, 2e-3])
    base = np.array([1.0, 0.2, -0.01])
    fr = [0.0, 0.05, 0.3, 0.55, 0.99, 1.5]  # r / rc relative to body 0's neighbour
    pts = [base]
    for k in range(1, 6):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        pts.append(base + u * max(fr[k], 1e-3) * max(rc[0], rc[k]))
    pts = np.array(pts)
    m = rng.uniform(1e-9, 1e-6, 6)
    st = state(pts, m=m)
    a = np.stack(oracle.accel(st, rc), axis=1)

    def K(y):
        if y <= 0:
            return mpmath.mpf(0)
        if y >= 1:
            return mpmath.mpf(1)
        return y * y / (2 * y * y - 2 * y + 1)

    P = [[mpmath.mpf(float(v)) for v in p] for p in pts]
    for i in range(6):
        acc = [mpmath.mpf(0)] * 3
        for j in range(6):
            if i == j:
                continue
            d = [P[j][q] - P[i][q] for q in range(3)]
            r = mpmath.sqrt(sum(t * t for t in d))
            R = mpmath.mpf(float(max(rc[i], rc[j])))
            w = K((r - R / 10) / (R * 9 / 10)) if r < R else mpmath.mpf(1)
            for q in range(3):
                acc[q] += mpmath.mpf(float(m[j])) * w * d[q] / r**3
        ref = np.array([float(t) for t in acc])
        assert np.max(np.abs(a[i] - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_momentum_and_torque_free_on_disc():
    d = discs.disc_c1()
    st = d.state()
    rc = oracle.rcrit(st, 1.0, 3.0, 0.0, discs.DT_6_DAYS)
    a = np.stack(oracle.accel(st, rc), axis=1)
    m = d.m[:, None]
    scale = np.sum(m * np.abs(a))
    assert np.max(np.abs((m * a).sum(axis=0))) < 1e-14 * scale
    r = vec(st)
    torque = np.cross(r, m * a).sum(axis=0)
    assert np.max(np.abs(torque)) < 1e-13 * np.sum(np.linalg.norm(r, axis=1)[:, None] * m * np.abs(a))


def test_force_is_minus_gradient_of_energy():
    """-dE/dr_i = -Mstar m_i r_i/r_i^3 + m_i a_i (Newtonian limit): pins signs/indices of the
    pair potential in the energy against the kick force."""
    rng = np.random.default_rng(3)
    n = 7
    pts = rng.normal(size=(n, 3)) * 0.3 + np.array([1.0, 0.5, 0.0])
    m = rng.uniform(1e-6, 1e-4, n)
    st = state(pts, m=m)
    a = np.stack(oracle.accel(st, np.zeros(n)), axis=1)
    h = 1e-6
    for i in range(n):
        for q, key in enumerate("xyz"):
            sp, sm = {k: v.copy() for k, v in st.items()}, {k: v.copy() for k, v in st.items()}
            sp[key][i] += h
            sm[key][i] -= h
            g = (oracle.energy(sp, 1.0)[0] - oracle.energy(sm, 1.0)[0]) / (2 * h)
            r = np.linalg.norm(pts[i])
            expect = -m[i] * pts[i, q] / r**3 + m[i] * a[i, q]
            assert -g == pytest.approx(expect, rel=1e-7, abs=1e-12 * m[i])


# ------------------------------------------------------------------------------------------
# Critical radius, eq. (1)
# ------------------------------------------------------------------------------------------

def test_rcrit_eq1_circular_orbits():
    m = np.array([3e-9, 3e-9, 1e-6])
    a = np.array([1.0, 2.5, 0.7])
    pts = np.stack([a, np.zeros(3), np.zeros(3)], axis=1)
    vel = np.stack([np.zeros(3), np.sqrt(1.0 / a), np.zeros(3)], axis=1)
    st = state(pts, vel, m)
    dt = discs.DT_6_DAYS
    rh = a * np.cbrt(m / 3.0)
    np.testing.assert_allclose(oracle.rcrit(st, 1.0, 3.0, 0.0, dt), 3.0 * rh, rtol=1e-14)
    # the paper's typical n1 = 3, n2 = 0.4: the velocity term wins for small bodies
    expect = np.maximum(3.0 * rh, 0.4 * dt * np.sqrt(1.0 / a))
    np.testing.assert_allclose(oracle.rcrit(st, 1.0, 3.0, 0.4, dt), expect, rtol=1e-14)


def _rotation(seed):
    """A proper rotation matrix from a seeded Gaussian matrix (QR, sign-fixed)."""
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("where", ["pericentre", "apocentre"])
def test_rcrit_eq1_eccentric_orbits(where):
    """eq. (1) off the circle: at pericentre r = a(1 - e) with v^2 = M(1 + e)/r, at apocentre
    r = a(1 + e) with v^2 = M(1 - e)/r (Kepler's ellipse, textbook).  R_H uses the semi-major
    axis a, not the distance, and the velocity term the Kepler velocity sqrt(M/a), not |v|;
    on a circle both readings agree; here r/a = 1 -+ e and |v|/sqrt(M/a) = sqrt((1 +- e)/(1 -+ e))
    (upper signs at pericentre)."""
    mstar = 1.3
    a = np.array([0.6, 1.0, 1.7, 3.2])
    e = np.array([0.05, 0.3, 0.6, 0.9])
    m = np.array([2e-9, 4e-10, 3e-7, 1e-12])
    sgn = -1.0 if where == "pericentre" else 1.0
    r = a * (1.0 + sgn * e)
    v = np.sqrt(mstar * (1.0 - sgn * e) / r)
    R = _rotation(7 if where == "pericentre" else 8)
    pos = (R @ np.stack([r, np.zeros(4), np.zeros(4)])).T
    vel = (R @ np.stack([np.zeros(4), v, np.zeros(4)])).T
    st = state(pos, vel, m)
    dt = discs.DT_6_DAYS
    rh = a * np.cbrt(m / (3.0 * mstar))
    np.testing.assert_allclose(oracle.rcrit(st, mstar, 3.0, 0.0, dt), 3.0 * rh, rtol=1e-12)
    # n2 large enough that the velocity term decides every body
    vk = np.sqrt(mstar / a)
    np.testing.assert_allclose(oracle.rcrit(st, mstar, 0.0, 0.4, dt), 0.4 * dt * vk, rtol=1e-12)
    np.testing.assert_allclose(oracle.rcrit(st, mstar, 3.0, 0.4, dt),
                               np.maximum(3.0 * rh, 0.4 * dt * vk), rtol=1e-12)


def test_rcrit_eq1_unbound_orbits():
    """eq. (1) for a body that is not bound to the star (v^2 >= 2M/r: no semi-major axis):
    the distance |r| stands in for a, in R_H and in the Kepler velocity sqrt(M/|r|).  The
    parabolic speed sqrt(2M/r) is the boundary case, a hyperbolic speed the general one."""
    mstar = 1.0
    r = np.array([0.8, 1.5, 2.0])
    v = np.array([1.0, 1.5, 3.0]) * np.sqrt(2.0 * mstar / r)
    m = np.array([3e-9, 1e-6, 5e-10])
    R = _rotation(9)
    pos = (R @ np.stack([r, np.zeros(3), np.zeros(3)])).T
    # the velocity at 60 degrees to the radius: the unbound test must not depend on direction
    vel = (R @ np.stack([0.5 * v, np.sqrt(0.75) * v, np.zeros(3)])).T
    st = state(pos, vel, m)
    dt = discs.DT_6_DAYS
    rh = r * np.cbrt(m / (3.0 * mstar))
    np.testing.assert_allclose(oracle.rcrit(st, mstar, 3.0, 0.0, dt), 3.0 * rh, rtol=1e-12)
    np.testing.assert_allclose(oracle.rcrit(st, mstar, 0.0, 0.4, dt), 0.4 * dt * np.sqrt(mstar / r),
                               rtol=1e-12)


# ------------------------------------------------------------------------------------------
# Encounter list and groups
# ------------------------------------------------------------------------------------------

def test_encounter_list_matches_kdtree():
    from scipy.spatial import cKDTree
    d = discs.make_disc(3000, 2.5, seed=11, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001)
    st = d.state()
    rc = oracle.rcrit(st, 1.0, 3.0, 0.0, discs.DT_6_DAYS)
    got = oracle.encounters(st, rc)
    pts = vec(st)
    cand = cKDTree(pts).query_pairs(r=rc.max(), output_type="ndarray")
    keep = []
    for i, j in cand:
        i, j = min(i, j), max(i, j)
        if np.linalg.norm(pts[j] - pts[i]) < max(rc[i], rc[j]):
            keep.append((i, j))
    ref = np.array(sorted(keep), dtype=np.int32).reshape(-1, 2)
    assert len(ref) > 5
    np.testing.assert_array_equal(got, ref)


def test_groups_match_connected_components():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(5)
    n = 200
    pairs = np.unique(np.sort(rng.integers(0, n, size=(120, 2)), axis=1), axis=0)
    pairs = pairs[pairs[:, 0] != pairs[:, 1]].astype(np.int32)
    gid = oracle.groups(n, pairs)
    A = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    inv = set(pairs.ravel().tolist())
    for i in range(n):
        assert (gid[i] >= 0) == (i in inv)
    for i in inv:
        for j in inv:
            assert (gid[i] == gid[j]) == (lab[i] == lab[j])
    # numbered by smallest member, in increasing order
    firsts = [min(np.where(gid == g)[0]) for g in range(gid.max() + 1)]
    assert firsts == sorted(firsts)


# ------------------------------------------------------------------------------------------
# Kepler drift (FP64, Sect. 1)
# ------------------------------------------------------------------------------------------

def test_kepler_circular_rotation():
    for a, t in ((1.0, 0.7), (2.3, 5.1), (0.5, -1.3)):
        v = math.sqrt(MU / a)
        st = state([[a, 0, 0]], [[0, v, 0]], [0.0])
        s = oracle.kepler_drift(st, MU, t)
        th = t * math.sqrt(MU / a**3)
        np.testing.assert_allclose([s["x"][0], s["y"][0], s["vx"][0], s["vy"][0]],
                                   [a * math.cos(th), a * math.sin(th), -v * math.sin(th), v * math.cos(th)],
                                   atol=1e-14 * max(1, a))


def test_kepler_one_period_returns():
    rng = np.random.default_rng(2)
    for _ in range(20):
        r0 = rng.normal(size=3)
        r0 *= rng.uniform(0.5, 3) / np.linalg.norm(r0)
        vc = math.sqrt(MU / np.linalg.norm(r0))
        v0 = rng.normal(size=3) * 0.3 * vc + np.cross([0, 0, 1], r0) / np.linalg.norm(r0) * vc
        a = 1.0 / (2 / np.linalg.norm(r0) - v0 @ v0 / MU)
        if a <= 0:
            continue
        P = 2 * math.pi * math.sqrt(a**3 / MU)
        s = oracle.kepler_drift(state([r0], [v0], [0.0]), MU, P)
        np.testing.assert_allclose(vec(s)[0], r0, atol=1e-12 * a)
        np.testing.assert_allclose(vec(s, ("vx", "vy", "vz"))[0], v0, atol=1e-12 * vc)


@pytest.mark.parametrize("v0", [0.35, 0.9, 1.2, 1.6, 3.0])
def test_kepler_against_numerical_integration(v0):
    """Elliptic and hyperbolic arcs against scipy's DOP853 at tight tolerance, plus the
    conservation of energy and r x v (equivalent to f gdot - fdot g = 1)."""
    from scipy.integrate import solve_ivp
    y0 = np.array([1.0, 0.2, -0.1, 0.1, v0, 0.3])

    def rhs(t, y):
        r = np.linalg.norm(y[:3])
        return np.concatenate([y[3:], -MU * y[:3] / r**3])

    st = state([y0[:3]], [y0[3:]], [0.0])
    for dt in (0.3, -0.4, 2.5):
        s = oracle.kepler_drift(st, MU, dt)
        got = np.concatenate([vec(s)[0], vec(s, ("vx", "vy", "vz"))[0]])
        ref = solve_ivp(rhs, (0, dt), y0, rtol=1e-13, atol=1e-15, method="DOP853").y[:, -1]
        assert np.max(np.abs(got - ref)) < 3e-12
        h0, h1 = np.cross(y0[:3], y0[3:]), np.cross(got[:3], got[3:])
        assert np.max(np.abs(h1 - h0)) < 1e-14 * np.linalg.norm(h0) * 10
        e0 = 0.5 * y0[3:] @ y0[3:] - MU / np.linalg.norm(y0[:3])
        e1 = 0.5 * got[3:] @ got[3:] - MU / np.linalg.norm(got[:3])
        assert abs(e1 - e0) < 1e-13 * abs(e0) * 10


def test_sun_drift_translation_keeps_L():
    d = discs.make_disc(300, 2.5, seed=9)
    st = d.state()
    tau = 0.05
    s = oracle.sun_drift(st, 1.0, tau)
    P = np.array([np.sum(d.m * st[k]) for k in ("vx", "vy", "vz")])
    # exact up to the rounding of r + shift (|r| <= ~4 au)
    np.testing.assert_allclose(vec(s) - vec(st), np.broadcast_to(tau * P, (d.n, 3)), rtol=0, atol=2e-15)
    L0, L1 = oracle.energy(st, 1.0)[1:], oracle.energy(s, 1.0)[1:]
    assert np.max(np.abs(L1 - L0)) < 1e-14 * np.linalg.norm(L0)


# ------------------------------------------------------------------------------------------
# Close-encounter step: Bulirsch-Stoer (FP64, Sect. 1)
# ------------------------------------------------------------------------------------------

def test_bs_single_body_equals_kepler():
    d = discs.make_disc(5, 2.5, seed=21)
    st = d.state()
    rc = np.full(5, 1e-3)
    for i in range(5):
        bs = oracle.bs_group(st, rc, [i], 1.0, 0.1032)
        kp = oracle.kepler_drift({k: v[i:i + 1] for k, v in st.items()}, 1.0, 0.1032)
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert abs(bs[k][i] - kp[k][0]) < 1e-12


def _group_reference(pts, vel, m, rc, dt):
    """Encounter-group equations of motion (Kepler about the Sun + (1-K) pair forces),
    integrated with scipy's DOP853; K is the pinned oracle changeover."""
    from scipy.integrate import solve_ivp
    n = len(m)

    def rhs(t, y):
        Y = y.reshape(n, 6)
        out = np.zeros_like(Y)
        out[:, :3] = Y[:, 3:]
        for a in range(n):
            r = np.linalg.norm(Y[a, :3])
            out[a, 3:] = -Y[a, :3] / r**3
            for b in range(n):
                if a == b:
                    continue
                dv = Y[b, :3] - Y[a, :3]
                rr = np.linalg.norm(dv)
                R = max(rc[a], rc[b])
                w = 1.0 - (oracle.changeover((rr - 0.1 * R) / (0.9 * R)) if rr < R else 1.0)
                out[a, 3:] += m[b] * w * dv / rr**3
        return out.ravel()

    y0 = np.concatenate([pts, vel], axis=1).ravel()
    return solve_ivp(rhs, (0, dt), y0, rtol=1e-13, atol=1e-16, method="DOP853").y[:, -1].reshape(n, 6)


@pytest.mark.parametrize("sep_frac", [0.05, 0.5])
def test_bs_close_pair_against_numerical_integration(sep_frac):
    """Two bodies deep inside (K = 0, a pure three-body problem) and in the changeover zone."""
    rc = np.array([0.02, 0.02])
    m = np.array([3e-6, 1e-6])
    p0 = np.array([1.0, 0.0, 0.0])
    sep = sep_frac * rc[0]
    pts = np.array([p0, p0 + [0.0, sep, 0.0]])
    vk = 1.0
    vrel = math.sqrt((m[0] + m[1]) / sep)  # bound mutual orbit
    vel = np.array([[0, vk, 0], [-0.5 * vrel, vk, 0.0]])
    st = state(pts, vel, m)
    dt = 0.02
    got = oracle.bs_group(st, rc, [0, 1], 1.0, dt)
    ref = _group_reference(pts, vel, m, rc, dt)
    g = np.stack([vec(got), vec(got, ("vx", "vy", "vz"))], axis=1).reshape(2, 6)
    assert np.max(np.abs(g[:, :3] - ref[:, :3])) < 1e-10
    assert np.max(np.abs(g[:, 3:] - ref[:, 3:])) < 1e-9


# ------------------------------------------------------------------------------------------
# Integrator: second order, angular momentum kept to round-off in FP64
# ------------------------------------------------------------------------------------------

def test_step_is_second_order():
    # Sun + two massive planets, no encounters (rc = 0): the energy error of the split
    # scales as dt^2.
    pts = np.array([[1.0, 0, 0], [0, 1.6, 0.01]])
    vel = np.array([[0, 1.0, 0.0], [-1 / math.sqrt(1.6), 0, 0.0]])
    m = np.array([1e-3, 3e-4])
    st = state(pts, vel, m)
    rc = np.zeros(2)
    T = 20.0
    errs = []
    for nst in (200, 400, 800):
        dt = T / nst
        _, e = oracle.step(st, rc, 1.0, dt, nst, cadence=1)
        errs.append(np.max(np.abs(e[:, 0] / e[0, 0] - 1)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7


def test_step_conserves_L_and_bounds_E_on_disc():
    d = discs.make_disc(800, 2.5, seed=12, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001)
    st = d.state()
    rc = oracle.rcrit(st, 1.0, 3.0, 0.0, discs.DT_6_DAYS)
    s, e = oracle.step(st, rc, 1.0, discs.DT_6_DAYS, 100, cadence=10)
    L = np.linalg.norm(e[:, 1:], axis=1)
    assert np.max(np.abs(L / L[0] - 1)) < 1e-13
    assert np.max(np.abs(e[:, 0] / e[0, 0] - 1)) < 1e-6


def test_kepler_strongly_hyperbolic_converges():
    """A fast unbound orbit whose Newton iterates approach the root from one side only
    (the converged iterate lands on the bracket edge)."""
    from scipy.integrate import solve_ivp
    x0 = np.array([0.9, 0.44, 0.01])
    v0 = np.array([-1.2, 2.9, 0.05])
    st = state([x0], [v0], [0.0])
    for dt in (3.0, 0.2, 12.0):
        s = oracle.kepler_drift(st, MU, dt)
        got = np.concatenate([vec(s)[0], vec(s, ("vx", "vy", "vz"))[0]])

        def rhs(t, y):
            r = np.linalg.norm(y[:3])
            return np.concatenate([y[3:], -MU * y[:3] / r**3])
        ref = solve_ivp(rhs, (0, dt), np.concatenate([x0, v0]), rtol=1e-13, atol=1e-15, method="DOP853").y[:, -1]
        assert np.max(np.abs(got - ref) / np.maximum(1, np.abs(ref))) < 1e-11


def test_step_through_dense_embryo_encounters():
    """Cold annulus with embryos: many strongly focused encounters over 160 steps.  Every
    Bulirsch-Stoer group step must reach the end of its interval (the last sub-step lands
    exactly on dt, and step control does not exhaust a budget of halvings), energy stays
    bounded and L is kept to round-off."""
    d = discs.make_disc(3000, 2.0, seed=5, sigma_e=0.001, sigma_i=0.001, n_embryo=40,
                        embryo_mass_earth=0.05, a_in=0.7, a_out=1.0)
    st = d.state()
    rc = oracle.rcrit(st, 1.0, 3.0, 0.0, discs.DT_6_DAYS)
    assert len(oracle.encounters(st, rc)) > 30
    s, e = oracle.step(st, rc, 1.0, discs.DT_6_DAYS, 160, cadence=20)
    assert np.max(np.abs(e[:, 0] / e[0, 0] - 1)) < 1e-7
    L = np.linalg.norm(e[:, 1:], axis=1)
    assert np.max(np.abs(L / L[0] - 1)) < 1e-13


# ------------------------------------------------------------------------------------------
# TP2 mode (Sect. 3.3): test bodies feel and exert forces on the massive bodies only
# ------------------------------------------------------------------------------------------

def test_tp2_three_body_closed_form():
    pts = np.array([[1.0, 0.0, 0.0], [1.3, 0.4, 0.0], [0.6, -0.3, 0.1]])
    m = np.array([1e-3, 2e-6, 5e-6])
    st = state(pts, m=m)
    a = np.stack(oracle.accel(st, np.zeros(3), n_massive=1), axis=1)

    def term(i, j):
        d = pts[j] - pts[i]
        return m[j] * d / np.linalg.norm(d) ** 3
    np.testing.assert_allclose(a[0], term(0, 1) + term(0, 2), rtol=1e-14)
    np.testing.assert_allclose(a[1], term(1, 0), rtol=1e-14)        # no pull from body 2
    np.testing.assert_allclose(a[2], term(2, 0), rtol=1e-14)
    # all bodies massive: the full sum; none massive: nothing
    full = np.stack(oracle.accel(st, np.zeros(3)), axis=1)
    np.testing.assert_allclose(full[1], term(1, 0) + term(1, 2), rtol=1e-14)
    assert np.all(np.stack(oracle.accel(st, np.zeros(3), n_massive=0)) == 0.0)


def test_tp2_force_is_minus_gradient_of_energy():
    rng = np.random.default_rng(8)
    n, nm = 7, 3
    pts = rng.normal(size=(n, 3)) * 0.3 + np.array([1.0, 0.5, 0.0])
    m = rng.uniform(1e-6, 1e-4, n)
    st = state(pts, m=m)
    a = np.stack(oracle.accel(st, np.zeros(n), n_massive=nm), axis=1)
    h = 1e-6
    for i in range(n):
        for q, key in enumerate("xyz"):
            sp, sm = {k: v.copy() for k, v in st.items()}, {k: v.copy() for k, v in st.items()}
            sp[key][i] += h
            sm[key][i] -= h
            g = (oracle.energy(sp, 1.0, n_massive=nm)[0] - oracle.energy(sm, 1.0, n_massive=nm)[0]) / (2 * h)
            r = np.linalg.norm(pts[i])
            # central differences of an O(1e-4) energy with h = 1e-6: ~1e-14 of round-off
            assert -g == pytest.approx(-m[i] * pts[i, q] / r**3 + m[i] * a[i, q], rel=1e-6, abs=1e-13)
    assert np.max(np.abs((m[:, None] * a).sum(axis=0))) < 1e-14 * np.sum(m[:, None] * np.abs(a))


def test_tp2_encounters_exclude_test_pairs():
    d = discs.make_disc(600, 2.5, seed=13, a_in=0.9, a_out=1.0, sigma_e=0.001, sigma_i=0.001,
                        n_embryo=10, embryo_mass_earth=0.05)
    st = d.state()
    rc = oracle.rcrit(st, 1.0, 3.0, 0.0, discs.DT_6_DAYS)
    full = oracle.encounters(st, rc)
    tp2 = oracle.encounters(st, rc, n_massive=10)
    keep = full[full[:, 0] < 10]
    np.testing.assert_array_equal(tp2, keep)
    assert len(full) > len(tp2) > 0


def test_tp2_bs_group_against_numerical_integration():
    from scipy.integrate import solve_ivp
    rc = np.array([0.02, 0.02, 0.02])
    m = np.array([3e-6, 1e-9, 1e-9])
    p0 = np.array([1.0, 0.0, 0.0])
    pts = np.array([p0, p0 + [0.0, 0.004, 0.0], p0 + [0.004, 0.0, 0.001]])
    vel = np.array([[0, 1.0, 0], [-0.02, 1.0, 0.0], [0.0, 1.02, 0.0]])
    st = state(pts, vel, m)
    dt = 0.02
    got = oracle.bs_group(st, rc, [0, 1, 2], 1.0, dt, n_massive=1)

    def rhs(t, y):
        Y = y.reshape(3, 6)
        out = np.zeros_like(Y)
        out[:, :3] = Y[:, 3:]
        for a_ in range(3):
            out[a_, 3:] = -Y[a_, :3] / np.linalg.norm(Y[a_, :3]) ** 3
            for b in range(3):
                if a_ == b or (a_ >= 1 and b >= 1):
                    continue
                dv = Y[b, :3] - Y[a_, :3]
                rr = np.linalg.norm(dv)
                R = max(rc[a_], rc[b])
                w = 1.0 - (oracle.changeover((rr - 0.1 * R) / (0.9 * R)) if rr < R else 1.0)
                out[a_, 3:] += m[b] * w * dv / rr**3
        return out.ravel()
    y0 = np.concatenate([pts, vel], axis=1).ravel()
    ref = solve_ivp(rhs, (0, dt), y0, rtol=1e-13, atol=1e-16, method="DOP853").y[:, -1].reshape(3, 6)
    g = np.concatenate([vec(got), vec(got, ("vx", "vy", "vz"))], axis=1)
    assert np.max(np.abs(g - ref)) < 1e-10


def test_tp2_step_conserves_its_energy():
    d = discs.make_disc(400, 2.0, seed=14, a_in=0.7, a_out=1.0, n_embryo=5, embryo_mass_earth=0.5)
    st = d.state()
    rc = oracle.rcrit(st, 1.0, 3.0, 0.0, discs.DT_6_DAYS)
    _, e = oracle.step(st, rc, 1.0, discs.DT_6_DAYS, 60, cadence=10, n_massive=5)
    assert np.max(np.abs(e[:, 0] / e[0, 0] - 1)) < 1e-7
    L = np.linalg.norm(e[:, 1:], axis=1)
    assert np.max(np.abs(L / L[0] - 1)) < 1e-13
