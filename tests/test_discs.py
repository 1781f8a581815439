"""The seeded synthetic discs have the shapes the workloads state (CPU only)."""
import math

import numpy as np
from scipy import stats

import discs


def test_seeded_and_reproducible():
    a, b = discs.disc_c1(), discs.disc_c1()
    for k in ("x", "y", "z", "vx", "vy", "vz", "m"):
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k))
    assert a.n == 2048


def test_masses_and_sizes():
    assert abs(discs.disc_c1().m.sum() - 2.5 * discs.EARTH_MASS) < 1e-18
    c3 = discs.disc_c3()
    assert c3.n == 40000 and abs(c3.m.sum() - 5 * discs.EARTH_MASS) < 1e-18
    c5 = discs.disc_c5()
    assert c5.n == 20040
    np.testing.assert_allclose(c5.m[:40], 0.05 * discs.EARTH_MASS)
    assert abs(c5.m[40:].sum() - 2 * discs.EARTH_MASS) < 1e-18
    b = discs.batch_c4()
    ns = [d.n for d in b]
    assert len(b) == 64 and min(ns) >= 2000 and max(ns) <= 8000


def test_semi_major_axis_distribution():
    # dN/da ~ a^-1/2 on [0.5, 4]: CDF (sqrt(a) - sqrt(0.5)) / (2 - sqrt(0.5))
    d = discs.make_disc(20000, 2.5, seed=31, sigma_e=1e-9, sigma_i=1e-9)
    r = np.sqrt(d.x**2 + d.y**2 + d.z**2)   # e ~ 0: r = a
    cdf = lambda a: (np.sqrt(a) - math.sqrt(0.5)) / (2 - math.sqrt(0.5))
    assert stats.kstest(r, cdf).pvalue > 1e-3
    assert r.min() >= 0.5 - 1e-6 and r.max() <= 4.0 + 1e-6


def test_barycentric_velocities_and_kepler_speeds():
    d = discs.disc_c2()
    P = [np.sum(d.m * v) for v in (d.vx, d.vy, d.vz)]
    # barycentric frame: the bodies' momentum balances the Sun's, which is -P
    r = np.sqrt(d.x**2 + d.y**2 + d.z**2)
    v = np.sqrt(d.vx**2 + d.vy**2 + d.vz**2)
    assert np.median(np.abs(v * np.sqrt(r) - 1.0)) < 0.02     # near-circular: v ~ r^-1/2
    assert max(abs(p) for p in P) < d.m.sum()
