"""Seeded synthetic planetesimal discs: the inputs shared by the oracle and the GPU path.

This module only draws random orbital elements and turns them into Cartesian
initial conditions.  It holds none of the method's arithmetic (no forces, no
changeover, no drift, no energy): both the CPU oracle and the HIP library take
its arrays as plain inputs.

Units (G = 1): masses in solar masses, lengths in au, time in units of 1/k days
with k the Gaussian gravitational constant, so one orbit at 1 au lasts 2*pi.

Disc recipe (the paper's workloads are planetesimal annuli; the synthetic
stand-ins use these shapes):
  * semi-major axes from a surface density Sigma ~ a^-1.5 on [a_in, a_out],
    i.e. dN/da ~ a^-0.5, sampled by the inverse CDF
    a = (sqrt(a_in) + u (sqrt(a_out) - sqrt(a_in)))^2;
  * eccentricity and inclination Rayleigh-distributed (scales sigma_e, sigma_i);
  * node, argument of pericentre and mean anomaly uniform on [0, 2 pi);
  * equal masses inside one population;
  * heliocentric positions/velocities from the elements (mu = G (M_* + m_i)),
    then velocities shifted to the barycentric frame, which is the democratic
    heliocentric choice: heliocentric positions, barycentric velocities.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List

import numpy as np

GAUSS_K = 0.01720209895            # Gaussian gravitational constant (au^1.5 / day / Msun^0.5)
EARTH_MASS = 1.0 / 332946.0487     # Earth mass in solar masses
MSTAR = 1.0


def days_to_code(days: float) -> float:
    """Convert a time in days to code units (G = 1, M_sun = 1, au)."""
    return days * GAUSS_K


DT_6_DAYS = days_to_code(6.0)


@dataclasses.dataclass
class Disc:
    """One planetary system: the Sun plus n bodies, structure-of-arrays float64."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray
    mstar: float = MSTAR
    seed: int = 0
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def state(self) -> Dict[str, np.ndarray]:
        return {k: getattr(self, k) for k in ("x", "y", "z", "vx", "vy", "vz", "m")}

    def copy(self) -> "Disc":
        return Disc(*(np.array(getattr(self, k), copy=True) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                    mstar=self.mstar, seed=self.seed, name=self.name)


def _solve_kepler_equation(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly E with E - e sin E = M (vectorised Newton, e < 1)."""
    E = M + e * np.sin(M)
    for _ in range(60):
        f = E - e * np.sin(E) - M
        d = f / (1.0 - e * np.cos(E))
        E = E - d
        if np.max(np.abs(d)) < 1e-15:
            break
    return E


def elements_to_cartesian(a, e, inc, node, peri, mean_anom, mu):
    """Heliocentric position/velocity arrays from elliptic orbital elements."""
    E = _solve_kepler_equation(np.mod(mean_anom, 2 * np.pi), e)
    cE, sE = np.cos(E), np.sin(E)
    rt = np.sqrt(1.0 - e * e)
    # perifocal frame
    xp = a * (cE - e)
    yp = a * rt * sE
    r = a * (1.0 - e * cE)
    nmean = np.sqrt(mu / a**3)
    vxp = -a * nmean * sE / (1.0 - e * cE)
    vyp = a * nmean * rt * cE / (1.0 - e * cE)
    cO, sO = np.cos(node), np.sin(node)
    cw, sw = np.cos(peri), np.sin(peri)
    ci, si = np.cos(inc), np.sin(inc)
    P = np.stack([cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si])
    Q = np.stack([-cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si])
    pos = P * xp + Q * yp
    vel = P * vxp + Q * vyp
    del r
    return pos, vel


def _draw_population(rng: np.random.Generator, n: int, a_in: float, a_out: float,
                     sigma_e: float, sigma_i: float):
    u = rng.random(n)
    a = (math.sqrt(a_in) + u * (math.sqrt(a_out) - math.sqrt(a_in))) ** 2
    e = np.minimum(rng.rayleigh(sigma_e, n), 0.9)
    inc = rng.rayleigh(sigma_i, n)
    node = rng.uniform(0.0, 2 * np.pi, n)
    peri = rng.uniform(0.0, 2 * np.pi, n)
    mean_anom = rng.uniform(0.0, 2 * np.pi, n)
    return a, e, inc, node, peri, mean_anom


def make_disc(n: int, total_mass_earth: float, seed: int, *, a_in: float = 0.5, a_out: float = 4.0,
              sigma_e: float = 0.01, sigma_i: float = 0.005,
              n_embryo: int = 0, embryo_mass_earth: float = 0.0, name: str = "") -> Disc:
    """Draw one disc: n_embryo embryos (listed first) then n equal-mass planetesimals.

    Every random number comes from numpy's PCG64 stream seeded with ``seed``; the draw
    order is fixed (embryo elements, then planetesimal elements), so a seed always gives
    the same bytes.
    """
    rng = np.random.default_rng(seed)
    pops = []
    if n_embryo > 0:
        pops.append((n_embryo, embryo_mass_earth * EARTH_MASS) + _draw_population(rng, n_embryo, a_in, a_out, sigma_e, sigma_i))
    m_p = total_mass_earth * EARTH_MASS / n if n > 0 else 0.0
    pops.append((n, m_p) + _draw_population(rng, n, a_in, a_out, sigma_e, sigma_i))
    xs, vs, ms = [], [], []
    for cnt, mass, a, e, inc, node, peri, ma in pops:
        if cnt == 0:
            continue
        mu = MSTAR + mass
        pos, vel = elements_to_cartesian(a, e, inc, node, peri, ma, mu)
        xs.append(pos)
        vs.append(vel)
        ms.append(np.full(cnt, mass))
    if xs:
        pos = np.concatenate(xs, axis=1)
        vel = np.concatenate(vs, axis=1)
        m = np.concatenate(ms)
    else:
        pos = np.zeros((3, 0))
        vel = np.zeros((3, 0))
        m = np.zeros(0)
    # heliocentric -> barycentric velocities (positions stay heliocentric)
    mtot = MSTAR + m.sum()
    vcm = (vel * m).sum(axis=1) / mtot
    vel = vel - vcm[:, None]
    return Disc(np.ascontiguousarray(pos[0]), np.ascontiguousarray(pos[1]), np.ascontiguousarray(pos[2]),
                np.ascontiguousarray(vel[0]), np.ascontiguousarray(vel[1]), np.ascontiguousarray(vel[2]),
                np.ascontiguousarray(m), MSTAR, seed, name)


# ---------------------------------------------------------------------------------------------
# The five workloads: sizes, masses and distributions of the paper's experiments, synthetic.
# ---------------------------------------------------------------------------------------------

def disc_c1() -> Disc:
    """2048 equal-mass planetesimals, 2.5 Earth masses, 0.5-4 au, e~R(0.01), i~R(0.005)."""
    return make_disc(2048, 2.5, seed=1, name="c1_n2048")


def disc_c2() -> Disc:
    """6600 planetesimals, same disc (2.5 Earth masses)."""
    return make_disc(6600, 2.5, seed=2, name="c2_n6600")


def disc_c3() -> Disc:
    """40000 planetesimals, 5 Earth masses, 0.5-4 au."""
    return make_disc(40000, 5.0, seed=3, name="c3_n40000")


def batch_c4(n_sys: int = 64, n_lo: int = 2000, n_hi: int = 8000) -> List[Disc]:
    """64 independent discs with n uniform in [2000, 8000], 2.5 Earth masses each, seeds 1000+s."""
    rng = np.random.default_rng(4)
    sizes = rng.integers(n_lo, n_hi + 1, size=n_sys)
    return [make_disc(int(sizes[s]), 2.5, seed=1000 + s, name=f"c4_s{s}") for s in range(n_sys)]


def disc_c5() -> Disc:
    """40 embryos of 0.05 Earth masses + 20000 planetesimals (2 Earth masses), cold disc."""
    return make_disc(20000, 2.0, seed=5, sigma_e=0.001, sigma_i=0.001,
                     n_embryo=40, embryo_mass_earth=0.05, name="c5_mixed")


# ---------------------------------------------------------------------------------------------
# The encounter-dominated regime: the paper's dense annulus (6600 planetesimals between 0.7
# and 1 au, 2 Earth masses, 5-day step) with r_crit from the full eq. (1), n1 = 3, n2 = 0.4.
# There r_crit (about 0.037 au) exceeds the mean spacing and the encounter groups percolate.
# ---------------------------------------------------------------------------------------------
DT_5_DAYS = days_to_code(5.0)
DENSE_N1, DENSE_N2 = 3.0, 0.4


def disc_dense(n: int = 6600, seed: int = 11, a_in: float = 0.7, a_out: float = 1.0,
               mass_earth: float = 0.0) -> Disc:
    """n planetesimals in [a_in, a_out] au, cold: e~R(0.002), i~R(0.001), carrying mass_earth
    Earth masses (default: 2 per 6600 bodies, the paper's surface density).  The default is
    the paper's first experiment: one encounter group of all 6600 bodies at n2 = 0.4."""
    m = mass_earth if mass_earth > 0.0 else 2.0 * n / 6600.0
    return make_disc(n, m, seed, a_in=a_in, a_out=a_out, sigma_e=0.002, sigma_i=0.001, name=f"dense_n{n}")


def disc_dense_40k(seed: int = 13) -> Disc:
    """The paper's high-resolution run: 40322 planetesimals (2 Earth masses) in 0.7-1 au."""
    return disc_dense(40322, seed, mass_earth=2.0)


def ring_dense(n: int = 1000, seed: int = 12) -> Disc:
    """A narrower dense ring (0.8-0.9 au) of n bodies at the same surface density scale: a few
    groups of some hundred bodies each at n2 = 0.4 (1000 bodies: 4 groups, the largest 511)."""
    return disc_dense(n, seed, a_in=0.8, a_out=0.9)


def concat(discs: List[Disc]):
    """Flatten several systems into CSR form: (state dict, sys_off int32[n_sys+1], mstar[n_sys])."""
    off = np.zeros(len(discs) + 1, dtype=np.int32)
    off[1:] = np.cumsum([d.n for d in discs])
    st = {k: np.concatenate([getattr(d, k) for d in discs]) if discs else np.zeros(0)
          for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    mstar = np.array([d.mstar for d in discs], dtype=np.float64)
    return st, off, mstar
