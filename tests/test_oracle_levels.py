"""Pins of the oracle's hierarchical levels (Sect. 1: intermediate symplectic levels with
reduced steps between the level-0 step and the Bulirsch-Stoer step).  CPU only.

The paper describes the levels without formulas; the oracle's reading (stated in oracle.c)
is pinned here by what the mathematics fixes, not by re-running the oracle's own formulas:
  - the level weights are a partition of unity of the pair force at every separation;
  - one level is the plain drift;
  - a pair that stays deep inside every level's changeover region is integrated by
    Bulirsch-Stoer alone, whatever the number of levels;
  - the level-1 Strang splitting converges to the exact flow of the level-0 drift
    Hamiltonian (which a one-level Bulirsch-Stoer integration at a tight tolerance is) at
    second order in the sub-step, both for a pair that only the level-1 kick sees and for a
    bound pair that the level-1 kick and the deepest integration share;
  - every sub-step is torque-free, so the total angular momentum is kept to rounding.
"""
import numpy as np
import pytest

import discs
import oracle

DT20 = 4 * discs.DT_5_DAYS


def co_orbital_pair(m, sep):
    """Two bodies of mass m on the same circular orbit at 1 au, sep apart along it."""
    th = sep
    return dict(x=np.array([1.0, np.cos(th)]), y=np.array([0.0, np.sin(th)]), z=np.zeros(2),
                vx=np.array([0.0, -np.sin(th)]), vy=np.array([1.0, np.cos(th)]), vz=np.zeros(2),
                m=np.full(2, m))


def bound_pair(m, sep):
    """A circular binary of two bodies of mass m, separation sep, whose centre of mass is on
    a circular orbit at 1 au (orbital plane = the disc plane)."""
    w = np.sqrt(2.0 * m / sep) / 2.0    # each body's speed about the binary's centre
    return dict(x=np.array([1.0 - sep / 2, 1.0 + sep / 2]), y=np.zeros(2), z=np.zeros(2),
                vx=np.zeros(2), vy=np.array([1.0 - w, 1.0 + w]), vz=np.zeros(2), m=np.full(2, m))


def max_diff(a, b):
    return max(np.max(np.abs(a[k] - b[k])) for k in ("x", "y", "z", "vx", "vy", "vz"))


def ang_mom(s):
    m = s["m"]
    return np.array([np.sum(m * (s["y"] * s["vz"] - s["z"] * s["vy"])),
                     np.sum(m * (s["z"] * s["vx"] - s["x"] * s["vz"])),
                     np.sum(m * (s["x"] * s["vy"] - s["y"] * s["vx"]))])


@pytest.mark.parametrize("nlev", [1, 2, 3, 4])
def test_level_weights_are_a_partition_of_unity(nlev):
    rng = np.random.default_rng(7)
    for _ in range(40):
        rc = np.sort(rng.uniform(0.05, 1.0, nlev))[::-1]      # non-increasing with the level
        for r in np.concatenate([rng.uniform(0.0, 1.3, 25), rc, 0.1 * rc, 0.55 * rc]):
            w = [oracle.level_weight(r * r, l, nlev, rc) for l in range(nlev + 1)]
            assert all(0.0 <= x <= 1.0 for x in w)
            assert abs(sum(w) - 1.0) <= 4e-16 * (nlev + 1)
            # beyond level k's radius nothing reaches the levels below k
            for k in range(nlev):
                if r * r >= rc[k] * rc[k]:
                    assert all(x == 0.0 for x in w[k + 1:])


def test_rcrit_levels_follow_eq1_with_the_level_step():
    d = discs.disc_dense(300, seed=31)
    st = d.state()
    rcl = oracle.rcrit_levels(st, 1.0, 3.0, 0.4, discs.DT_5_DAYS, 3, 2)
    for k in range(3):
        assert np.array_equal(rcl[k], oracle.rcrit(st, 1.0, 3.0, 0.4, discs.DT_5_DAYS / 2 ** k))
    assert np.all(np.diff(rcl, axis=0) <= 0.0)
    flat = oracle.rcrit_levels(st, 1.0, 3.0, 0.0, discs.DT_5_DAYS, 3, 2)
    assert np.array_equal(flat[0], flat[2])     # no velocity term: every level the same


def test_one_level_is_the_plain_drift():
    d = discs.disc_dense(400, seed=32)
    st = d.state()
    rc = oracle.rcrit(st, 1.0, 3.0, 0.4, discs.DT_5_DAYS)
    pairs = oracle.encounters(st, rc)
    assert len(pairs) > 10
    a = oracle.drift(st, rc, 1.0, discs.DT_5_DAYS, pairs)
    b = oracle.drift_levels(st, rc[None, :], 3, 1.0, discs.DT_5_DAYS, pairs)
    assert max_diff(a, b) == 0.0


def test_deep_pair_is_bulirsch_stoer_alone():
    """A bound pair well inside 0.1 r_crit of the deepest level: every level's kick weight is
    zero, so 3 levels of 2 sub-steps give the one-level result (Bulirsch-Stoer over dt), to
    the accuracy Bulirsch-Stoer reaches on this binary of 20 orbits (the trial states of
    rejected steps see different weights, so the step sequences differ)."""
    m = 1e-7
    rc0 = 3.0 * (m / 3.0) ** (1.0 / 3.0)
    rcl = np.array([[rc0] * 2, [0.5 * rc0] * 2, [0.25 * rc0] * 2])
    st = bound_pair(m, 0.012 * rc0)
    pairs = np.array([[0, 1]])
    ref = oracle.drift_levels(st, rcl[:1], 1, 1.0, DT20, pairs)
    for nsub in (1, 2, 3):
        got = oracle.drift_levels(st, rcl, nsub, 1.0, DT20, pairs)
        assert max_diff(got, ref) <= 1e-8


@pytest.mark.parametrize("case", ["kick only", "kick and deepest integration"])
def test_level_splitting_is_second_order(case):
    """Level 1 splits the level-0 drift (Kepler + (1-K_0) F) into kick and drift parts; with
    nsub sub-steps it must approach the exact flow of that drift as nsub^-2."""
    m = 1e-7
    rc0 = 3.0 * (m / 3.0) ** (1.0 / 3.0)
    if case == "kick only":
        rcl = np.array([[rc0] * 2, [0.3 * rc0] * 2])
        st = co_orbital_pair(m, 0.6 * rc0)      # between r_crit,1 and r_crit,0 all the time
    else:
        rcl = np.array([[rc0] * 2, [0.5 * rc0] * 2])
        st = bound_pair(m, 0.25 * rc0)          # in the ramps of levels 0 and 1
    pairs = np.array([[0, 1]])
    exact = oracle.drift_levels(st, rcl[:1], 1, 1.0, DT20, pairs, tol=1e-14)
    errs = [max_diff(oracle.drift_levels(st, rcl, ns, 1.0, DT20, pairs), exact) for ns in (2, 4, 8)]
    assert errs[0] > 1e-9                       # the splitting is really exercised
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.6 <= e0 / e1 <= 4.4, errs


def test_levels_keep_angular_momentum():
    d = discs.disc_dense(500, seed=33, a_in=0.8, a_out=0.9)
    st = d.state()
    st["m"] = st["m"] * np.random.default_rng(34).uniform(0.5, 1.5, d.n)   # unequal masses
    rcl = oracle.rcrit_levels(st, 1.0, 3.0, 0.4, discs.DT_5_DAYS, 3, 2)
    pairs = oracle.encounters(st, rcl[0])
    gid = oracle.groups(d.n, pairs)
    assert np.bincount(gid[gid >= 0]).max() >= 3
    got = oracle.drift_levels(st, rcl, 2, 1.0, discs.DT_5_DAYS, pairs)
    L0, L1 = ang_mom(st), ang_mom(got)
    assert np.linalg.norm(L1 - L0) <= 1e-14 * np.linalg.norm(L0)
