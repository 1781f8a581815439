"""Pins of the oracle's collisions and removal (Sect. 2: collisions are perfect mergers; bodies
are removed inside r_min or beyond r_max).  CPU only.

The reading (stated in oracle.c): encounter pairs collide when their straight-line relative
motion over the drift comes within R_i + R_j; colliding pairs merge after the drift in
ascending order, the lower index keeping the summed mass, the mass-weighted position and
velocity and the summed volume; then bodies outside [r_min, r_max] are removed.  Pinned by
closed forms: the closest approach of a straight line, the conservation of mass, momentum and
volume, and the order rules.
"""
import numpy as np
import pytest

import discs
import oracle


def two_bodies(dx, dv, m=(1e-9, 3e-9)):
    """Body 0 at (1, 0, 0) on a circular orbit, body 1 displaced by dx and moving by dv
    relative to it."""
    x0 = np.array([1.0, 0.0, 0.0])
    v0 = np.array([0.0, 1.0, 0.0])
    x1, v1 = x0 + np.asarray(dx, float), v0 + np.asarray(dv, float)
    return dict(x=np.array([x0[0], x1[0]]), y=np.array([x0[1], x1[1]]), z=np.array([x0[2], x1[2]]),
                vx=np.array([v0[0], v1[0]]), vy=np.array([v0[1], v1[1]]), vz=np.array([v0[2], v1[2]]),
                m=np.array(m, dtype=float))


PAIR = np.array([[0, 1]], dtype=np.int32)
DT = discs.DT_5_DAYS


@pytest.mark.parametrize("b,hit", [(0.9e-5, True), (1.1e-5, False)])
def test_detection_is_the_straight_line_closest_approach(b, hit):
    """Impact parameter b, relative speed u along x, closest approach at t = s/u inside the
    drift: the distance there is b, against R_0 + R_1 = 1e-5."""
    s, u = 2e-4, 4e-3          # reaches closest approach at t = 0.05 < dt = 0.086
    st = two_bodies([-s, b, 0.0], [u, 0.0, 0.0])
    col = oracle.collisions(st, PAIR, [0.5e-5, 0.5e-5], [0, 0], DT)
    assert (len(col) == 1) == hit


def test_closest_approach_is_clamped_to_the_drift():
    # approaching, but the closest point lies after the drift: distance at t = dt counts
    s, u = 1e-3, 4e-3          # s / u = 0.25 > dt
    st = two_bodies([-s, 0.0, 0.0], [u, 0.0, 0.0])
    gap = s - u * DT
    assert len(oracle.collisions(st, PAIR, [0.5 * gap * 1.001] * 2, [0, 0], DT)) == 1
    assert len(oracle.collisions(st, PAIR, [0.5 * gap * 0.999] * 2, [0, 0], DT)) == 0
    # receding: the closest point is the start
    st = two_bodies([s, 0.0, 0.0], [u, 0.0, 0.0])
    assert len(oracle.collisions(st, PAIR, [0.5 * s * 1.001] * 2, [0, 0], DT)) == 1
    assert len(oracle.collisions(st, PAIR, [0.5 * s * 0.999] * 2, [0, 0], DT)) == 0
    # no relative motion: the start
    st = two_bodies([s, 0.0, 0.0], [0.0, 0.0, 0.0])
    assert len(oracle.collisions(st, PAIR, [0.5 * s * 1.001] * 2, [0, 0], DT)) == 1


def test_dead_bodies_do_not_collide():
    st = two_bodies([1e-6, 0.0, 0.0], [0.0, 0.0, 0.0])
    assert len(oracle.collisions(st, PAIR, [1e-5, 1e-5], [0, 1], DT)) == 0
    assert len(oracle.collisions(st, PAIR, [1e-5, 1e-5], [2, 0], DT)) == 0


def test_perfect_merger_keeps_mass_momentum_centre_and_volume():
    rng = np.random.default_rng(5)
    st = two_bodies(rng.normal(size=3) * 1e-5, rng.normal(size=3) * 1e-3, m=(2e-9, 5e-9))
    rad = np.array([3e-6, 4e-6])
    out, rad2, stt = oracle.merge(st, PAIR, rad, [0, 0])
    m0, m1 = st["m"]
    assert out["m"][0] == m0 + m1 and out["m"][1] == 0.0
    assert stt.tolist() == [0, 1]
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        before = m0 * st[k][0] + m1 * st[k][1]
        assert abs(out["m"][0] * out[k][0] - before) <= 2e-16 * abs(before) + 1e-30
    assert abs(rad2[0] ** 3 - (3e-6 ** 3 + 4e-6 ** 3)) <= 1e-15 * rad2[0] ** 3
    assert rad2[1] == rad[1]


def test_merge_order_and_chains():
    """A-B then B-C in ascending order: B joins A; B-C is skipped (B is gone), C stays."""
    st = dict(x=np.array([1.0, 1.0 + 1e-6, 1.0 + 2e-6]), y=np.zeros(3), z=np.zeros(3),
              vx=np.zeros(3), vy=np.ones(3), vz=np.zeros(3), m=np.array([1e-9, 2e-9, 3e-9]))
    col = np.array([[0, 1], [1, 2]], dtype=np.int32)
    out, _, stt = oracle.merge(st, col, [1e-5] * 3, [0, 0, 0])
    assert stt.tolist() == [0, 1, 0]
    assert out["m"].tolist() == [1e-9 + 2e-9, 0.0, 3e-9]


def test_removal_by_distance():
    st = dict(x=np.array([0.3, 0.9, 50.0, 0.0, 0.5, 0.0]), y=np.array([0.0, 0.0, 0.0, 39.9, 0.0, 0.39]),
              z=np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.1]), vx=np.zeros(6), vy=np.zeros(6), vz=np.zeros(6),
              m=np.full(6, 1e-9))
    out, stt = oracle.remove(st, [0, 0, 0, 1, 0, 0], 0.4, 40.0)
    assert stt.tolist() == [2, 0, 2, 1, 0, 0]       # |r| = 0.3, 0.9, 50, (dead), 0.5, 0.4026
    assert out["m"].tolist() == [0.0, 1e-9, 0.0, 1e-9, 1e-9, 1e-9]


def test_collide_steps_conserve_mass_and_merge_some_bodies():
    """A cold ring with inflated radii: over 20 steps some bodies merge; the total mass stays
    (removal off), and every dead body has zero mass."""
    d = discs.ring_dense(300)
    st = d.state()
    rc = oracle.rcrit(st, 1.0, 3.0, 0.4, DT)
    rad = np.full(d.n, 2e-3)
    out, rad2, stt = oracle.step_collide(st, rc, rad, np.zeros(d.n, np.int32), 1.0, DT, 20, 0.0, 1e9)
    merged = int((stt == 1).sum())
    print("merged", merged)
    assert merged >= 1
    assert abs(out["m"].sum() - st["m"].sum()) <= 1e-15 * st["m"].sum()
    assert np.all(out["m"][stt != 0] == 0.0) and np.all(out["m"][stt == 0] > 0.0)
    # merged survivors carry the summed volume
    assert abs(np.sum(rad2[stt == 0] ** 3) - np.sum(rad ** 3)) <= 1e-12 * np.sum(rad ** 3)


def test_collide_steps_with_levels():
    """Collisions composed with the hierarchical step (Sect. 1 levels, Sect. 2 mergers): with
    radii of zero nothing collides and the steps equal oracle.step_levels bit for bit; with
    inflated radii mass and volume are conserved and dead bodies have zero mass."""
    d = discs.ring_dense(300)
    st = d.state()
    rcl = oracle.rcrit_levels(st, 1.0, 3.0, 0.4, DT, 2, 2)
    none, r0, s0 = oracle.step_collide(st, rcl, np.zeros(d.n), np.zeros(d.n, np.int32), 1.0, DT, 3, 0.0, 1e9,
                                       nsub=2)
    exp, _ = oracle.step_levels(st, rcl, 2, 1.0, DT, 3)
    assert np.all(s0 == 0)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(none[k], exp[k])
    rad = np.full(d.n, 2e-3)
    out, rad2, stt = oracle.step_collide(st, rcl, rad, np.zeros(d.n, np.int32), 1.0, DT, 10, 0.0, 1e9, nsub=2)
    assert (stt == 1).sum() >= 1
    assert abs(out["m"].sum() - st["m"].sum()) <= 1e-15 * st["m"].sum()
    assert np.all(out["m"][stt != 0] == 0.0)
    assert abs(np.sum(rad2[stt == 0] ** 3) - np.sum(rad ** 3)) <= 1e-12 * np.sum(rad ** 3)


def test_dead_body_leaves_the_encounter_groups():
    """A body that has merged (status 1, m = 0) takes part in no encounter pair.  Placed
    1e-4 au ahead of a live body on the same circular orbit (K = 0 there: well inside
    0.1 r_crit), it must not be integrated with that body, whose (1 - K) force would pull it
    in within a step; it moves on as a massless particle.  With a second live body on the
    opposite side of the orbit (total momentum zero, so the Sun drift is nil) the only force
    on it besides the Sun's is the far body's K = 1 pull (about 2.5e-10), so it follows the
    Sun-only Kepler orbit (scipy DOP853) to 1e-9 au over 10 steps."""
    from scipy.integrate import solve_ivp

    phi = 1e-4
    pos = np.array([[1.0, 0.0, 0.0], [np.cos(phi), np.sin(phi), 0.0], [-1.0, 0.0, 0.0]])
    vel = np.array([[0.0, 1.0, 0.0], [-np.sin(phi), np.cos(phi), 0.0], [0.0, -1.0, 0.0]])
    m = np.array([1e-9, 0.0, 1e-9])
    st = dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), vx=vel[:, 0].copy(),
              vy=vel[:, 1].copy(), vz=vel[:, 2].copy(), m=m)
    dt = discs.DT_6_DAYS
    rc = oracle.rcrit(dict(st, m=np.array([1e-9, 1e-9, 1e-9])), 1.0, 3.0, 0.0, dt)
    assert phi < 0.1 * rc[0]
    out, rad, stt = oracle.step_collide(st, rc, [0.0, 0.0, 0.0], [0, 1, 0], 1.0, dt, 10, 0.0, 1e9)
    assert list(stt) == [0, 1, 0]

    def f(t, y):
        r3 = np.linalg.norm(y[:3]) ** 3
        return np.concatenate([y[3:], -y[:3] / r3])

    sol = solve_ivp(f, (0.0, 10 * dt), np.concatenate([pos[1], vel[1]]), method="DOP853", rtol=1e-13, atol=1e-15)
    got = np.array([out["x"][1], out["y"][1], out["z"][1]])
    assert np.max(np.abs(got - sol.y[:3, -1])) < 1e-9
