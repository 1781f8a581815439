"""FP64 CPU oracle for the changeover-weighted kick path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  It wraps ``oracle.c`` (plain C, FP64, j summed in ascending
order, built with ``-O2 -ffp-contract=off -fopenmp``) through ctypes and shares no
code with the HIP library.

Every function follows a passage of Brasser et al. (2023): the changeover-weighted
long-range force and the FP64 Kepler drift / close-encounter step of Sect. 1, the
critical radius of eq. (1), and the energy / angular-momentum diagnostics of Sect. 3.1.
The readings taken where the paper is silent are stated in ``oracle.c``'s header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a planted-mistake test points this at a mutated build of oracle.c
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB_OVERRIDE")

BS_TOL = 1e-12


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build(force=False)
            L = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_set_num_threads.restype = None
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_changeover.restype = ctypes.c_double
        L.oracle_changeover.argtypes = [ctypes.c_double]
        L.oracle_rcrit.argtypes = [i64] + [d] * 7 + [ctypes.c_double] * 4 + [d]
        L.oracle_accel.argtypes = [i64, i64] + [d] * 5 + [d] * 3
        L.oracle_accel_rows.argtypes = [i64, i64] + [d] * 5 + [i64, ctypes.POINTER(ctypes.c_int64)] + [d] * 3
        L.oracle_encounters.restype = i64
        L.oracle_encounters.argtypes = [i64, i64, d, d, d, d, i64, ctypes.POINTER(ctypes.c_int32)]
        L.oracle_energy.argtypes = [i64, i64] + [d] * 7 + [ctypes.c_double, d]
        L.oracle_sun_drift.argtypes = [i64] + [d] * 7 + [ctypes.c_double, ctypes.c_double]
        L.oracle_kepler_drift.restype = ctypes.c_int
        L.oracle_kepler_drift.argtypes = [i64] + [d] * 6 + [ctypes.c_double, ctypes.c_double,
                                                            ctypes.POINTER(ctypes.c_uint8)]
        L.oracle_bs_group.restype = ctypes.c_int
        L.oracle_bs_group.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int32), i64] + [d] * 8 + \
            [ctypes.c_double] * 3
        L.oracle_groups.restype = i64
        L.oracle_groups.argtypes = [i64, i64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
        L.oracle_drift.restype = ctypes.c_int
        L.oracle_drift.argtypes = [i64, i64] + [d] * 8 + [ctypes.c_double, ctypes.c_double, i64,
                                                          ctypes.POINTER(ctypes.c_int32), ctypes.c_double]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_step.argtypes = [i64, i64] + [d] * 8 + [ctypes.c_double, ctypes.c_double, i64,
                                                         ctypes.c_double, i64, d]
        L.oracle_level_weight.restype = ctypes.c_double
        L.oracle_level_weight.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, d]
        L.oracle_drift_levels.restype = ctypes.c_int
        L.oracle_drift_levels.argtypes = [i64, i64] + [d] * 8 + [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                                 ctypes.c_double, i64, ctypes.POINTER(ctypes.c_int32),
                                                                 ctypes.c_double]
        L.oracle_step_levels.restype = ctypes.c_int
        L.oracle_step_levels.argtypes = [i64, i64] + [d] * 8 + [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                                ctypes.c_double, i64, ctypes.c_double, i64, d]
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.oracle_collisions.restype = i64
        L.oracle_collisions.argtypes = [i64, i32p] + [d] * 7 + [i32p, ctypes.c_double, i32p]
        L.oracle_merge.argtypes = [i64, i32p] + [d] * 8 + [i32p]
        L.oracle_remove.argtypes = [i64] + [d] * 4 + [i32p, ctypes.c_double, ctypes.c_double]
        L.oracle_step_collide.restype = ctypes.c_int
        L.oracle_step_collide.argtypes = [i64, i64] + [d] * 8 + [i64, i64, d, i32p] + [ctypes.c_double] * 2 + \
            [i64] + [ctypes.c_double] * 3
        _lib = L
    return _lib


def _p(a: np.ndarray, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# -------------------------------------------------------------------------------------------
# Functions on one system (the Sun plus n bodies).  State dicts hold float64 arrays
# x, y, z, vx, vy, vz, m (heliocentric positions, barycentric velocities).
# -------------------------------------------------------------------------------------------

def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (results do not depend on it)."""
    lib().oracle_set_num_threads(int(n))


def num_threads() -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return int(lib().oracle_num_threads())


def changeover(y: float) -> float:
    """K(y) of the changeover (Sect. 1, the Chambers 1999 function the paper cites)."""
    return lib().oracle_changeover(float(y))


def rcrit(st: Dict[str, np.ndarray], mstar: float, n1: float, n2: float, dt: float) -> np.ndarray:
    """Critical radius of every body, eq. (1)."""
    n = len(st["x"])
    rc = np.zeros(n)
    a = [_f64(st[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")]
    lib().oracle_rcrit(n, *[_p(v) for v in a], float(mstar), float(n1), float(n2), float(dt), _p(rc))
    return rc


def _nm(n: int, n_massive: Optional[int]) -> int:
    return n if n_massive is None else int(n_massive)


def accel(st: Dict[str, np.ndarray], rc: np.ndarray, n_massive: Optional[int] = None
          ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Changeover-weighted long-range accelerations a_i (the kick force, Sect. 1).  With
    n_massive < n, bodies n_massive.. are TP2 test bodies (Sect. 3.3)."""
    n = len(st["x"])
    ax, ay, az = np.zeros(n), np.zeros(n), np.zeros(n)
    a = [_f64(st[k]) for k in ("x", "y", "z", "m")] + [_f64(rc)]
    lib().oracle_accel(n, _nm(n, n_massive), *[_p(v) for v in a], _p(ax), _p(ay), _p(az))
    return ax, ay, az


def accel_rows(st: Dict[str, np.ndarray], rc: np.ndarray, rows: np.ndarray, n_massive: Optional[int] = None):
    """a_i for the listed rows only (for sampled checks at large n)."""
    n = len(st["x"])
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    k = len(rows)
    ax, ay, az = np.zeros(k), np.zeros(k), np.zeros(k)
    a = [_f64(st[k_]) for k_ in ("x", "y", "z", "m")] + [_f64(rc)]
    lib().oracle_accel_rows(n, _nm(n, n_massive), *[_p(v) for v in a], k, _p(rows, ctypes.c_int64),
                            _p(ax), _p(ay), _p(az))
    return ax, ay, az


def encounters(st: Dict[str, np.ndarray], rc: np.ndarray, cap: Optional[int] = None,
               n_massive: Optional[int] = None) -> np.ndarray:
    """Encounter pairs (i < j, r_ij < r_crit,ij), lexicographic, as an int32 array [P, 2]."""
    n = len(st["x"])
    if cap is None:
        cap = 16 * n + 16
    pairs = np.zeros((cap, 2), dtype=np.int32)
    a = [_f64(st[k]) for k in ("x", "y", "z")] + [_f64(rc)]
    cnt = lib().oracle_encounters(n, _nm(n, n_massive), *[_p(v) for v in a], cap, _p(pairs, ctypes.c_int32))
    if cnt > cap:
        return encounters(st, rc, cap=int(cnt), n_massive=n_massive)
    return pairs[:cnt].copy()


def energy(st: Dict[str, np.ndarray], mstar: float, n_massive: Optional[int] = None) -> np.ndarray:
    """(E, Lx, Ly, Lz) of the system (Sect. 3.1 diagnostics)."""
    n = len(st["x"])
    out = np.zeros(4)
    a = [_f64(st[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")]
    lib().oracle_energy(n, _nm(n, n_massive), *[_p(v) for v in a], float(mstar), _p(out))
    return out


def _mut(st):
    return {k: _f64(st[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz", "m")}


def sun_drift(st: Dict[str, np.ndarray], mstar: float, tau: float) -> Dict[str, np.ndarray]:
    """Positions shifted by tau * (sum m v) / M_star; returns a new state."""
    s = _mut(st)
    n = len(s["x"])
    lib().oracle_sun_drift(n, *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")], float(mstar), float(tau))
    return s


def kepler_drift(st: Dict[str, np.ndarray], mu: float, dt: float, skip: Optional[np.ndarray] = None):
    """Every body advanced on its two-body orbit about mu over dt (FP64, Sect. 1)."""
    s = _mut(st)
    n = len(s["x"])
    sk = None
    if skip is not None:
        sk_arr = np.ascontiguousarray(skip, dtype=np.uint8)
        sk = _p(sk_arr, ctypes.c_uint8)
    bad = lib().oracle_kepler_drift(n, *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz")],
                                    float(mu), float(dt), sk)
    if bad:
        raise RuntimeError("oracle Kepler solve did not converge")
    return s


def bs_group(st: Dict[str, np.ndarray], rc: np.ndarray, members, mstar: float, dt: float, tol: float = BS_TOL,
             n_massive: Optional[int] = None):
    """One encounter group integrated over dt with Bulirsch-Stoer (FP64, Sect. 1)."""
    s = _mut(st)
    idx = np.ascontiguousarray(members, dtype=np.int32)
    bad = lib().oracle_bs_group(len(idx), _p(idx, ctypes.c_int32), _nm(len(s["x"]), n_massive),
                                *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")],
                                _p(_f64(rc)), float(mstar), float(dt), float(tol))
    if bad:
        raise RuntimeError("oracle Bulirsch-Stoer step did not converge")
    return s


def groups(n: int, pairs: np.ndarray) -> np.ndarray:
    """Group id per body (-1 = not in an encounter); groups numbered by smallest member."""
    p = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    gid = np.zeros(n, dtype=np.int64)
    lib().oracle_groups(n, len(p), _p(p, ctypes.c_int32), _p(gid, ctypes.c_int64))
    return gid


def drift(st, rc, mstar: float, dt: float, pairs: np.ndarray, tol: float = BS_TOL,
          n_massive: Optional[int] = None):
    """Sun drift(dt/2), Kepler drift or BS per group (dt), Sun drift(dt/2)."""
    s = _mut(st)
    n = len(s["x"])
    p = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    bad = lib().oracle_drift(n, _nm(n, n_massive), *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")], _p(_f64(rc)),
                             float(mstar), float(dt), len(p), _p(p, ctypes.c_int32), float(tol))
    if bad:
        raise RuntimeError("oracle drift failed")
    return s


def step(st, rc, mstar: float, dt: float, nsteps: int, cadence: int = 0, tol: float = BS_TOL,
         n_massive: Optional[int] = None):
    """nsteps full steps; returns (new state, energy rows [k, 4] at the cadence or None)."""
    s = _mut(st)
    n = len(s["x"])
    e = None
    ep = None
    if cadence > 0:
        e = np.zeros((nsteps // cadence + 1, 4))
        ep = _p(e)
    bad = lib().oracle_step(n, _nm(n, n_massive), *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")], _p(_f64(rc)),
                            float(mstar), float(dt), int(nsteps), float(tol), int(cadence), ep)
    if bad:
        raise RuntimeError("oracle step failed")
    return s, e


# -------------------------------------------------------------------------------------------
# Hierarchical levels (Sect. 1: intermediate symplectic levels with reduced steps between the
# level-0 step and the Bulirsch-Stoer step).  The reading is stated in oracle.c.
# -------------------------------------------------------------------------------------------

def rcrit_levels(st: Dict[str, np.ndarray], mstar: float, n1: float, n2: float, dt: float,
                 nlev: int, nsub: int) -> np.ndarray:
    """Critical radius of every body at levels 0..nlev-1: eq. (1) with the level's step
    dt / nsub^k.  Shape (nlev, n)."""
    return np.stack([rcrit(st, mstar, n1, n2, dt / float(nsub) ** k) for k in range(nlev)])


def level_weight(r2: float, level: int, nlev: int, rcij) -> float:
    """Share of the pair force carried by level `level`'s kick (level < nlev) or by the
    deepest Bulirsch-Stoer integration (level == nlev)."""
    rc = _f64(rcij)
    return lib().oracle_level_weight(float(r2), int(level), int(nlev), _p(rc))


def drift_levels(st, rcl: np.ndarray, nsub: int, mstar: float, dt: float, pairs: np.ndarray,
                 tol: float = BS_TOL, n_massive: Optional[int] = None):
    """The drift with len(rcl) levels and nsub sub-steps per level; rcl[k] is the level-k
    critical radius of every body (rcl[0] the r_crit of the kick)."""
    s = _mut(st)
    n = len(s["x"])
    rc = _f64(np.asarray(rcl).reshape(-1, n))
    p = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    bad = lib().oracle_drift_levels(n, _nm(n, n_massive), *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")],
                                    _p(rc), rc.shape[0], int(nsub), float(mstar), float(dt), len(p),
                                    _p(p, ctypes.c_int32), float(tol))
    if bad:
        raise RuntimeError("oracle drift failed")
    return s


def step_levels(st, rcl: np.ndarray, nsub: int, mstar: float, dt: float, nsteps: int, cadence: int = 0,
                tol: float = BS_TOL, n_massive: Optional[int] = None):
    """nsteps full steps with the drift of drift_levels; returns (state, energy rows or None)."""
    s = _mut(st)
    n = len(s["x"])
    rc = _f64(np.asarray(rcl).reshape(-1, n))
    e = None
    ep = None
    if cadence > 0:
        e = np.zeros((nsteps // cadence + 1, 4))
        ep = _p(e)
    bad = lib().oracle_step_levels(n, _nm(n, n_massive), *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")],
                                   _p(rc), rc.shape[0], int(nsub), float(mstar), float(dt), int(nsteps), float(tol),
                                   int(cadence), ep)
    if bad:
        raise RuntimeError("oracle step failed")
    return s, e


# -------------------------------------------------------------------------------------------
# Collisions and removal (Sect. 2: perfect mergers; removal inside r_min / beyond r_max).  The
# reading is stated in oracle.c.  status: 0 live, 1 merged into another body, 2 removed.
# -------------------------------------------------------------------------------------------

def collisions(st, pairs: np.ndarray, radius, status, dt: float) -> np.ndarray:
    """Encounter pairs whose straight-line relative motion over dt comes within R_i + R_j."""
    p = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.zeros((max(len(p), 1), 2), dtype=np.int32)
    stt = np.ascontiguousarray(status, dtype=np.int32)
    a = [_f64(st[k]) for k in ("x", "y", "z", "vx", "vy", "vz")]
    nc = lib().oracle_collisions(len(p), _p(p, ctypes.c_int32), *[_p(v) for v in a], _p(_f64(radius)),
                                 _p(stt, ctypes.c_int32), float(dt), _p(out, ctypes.c_int32))
    return out[:nc].copy()


def merge(st, col: np.ndarray, radius, status):
    """Perfect mergers of the colliding pairs in order; returns (state, radius, status)."""
    s = _mut(st)
    rad = np.array(radius, dtype=np.float64)
    stt = np.array(status, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32).reshape(-1, 2)
    lib().oracle_merge(len(c), _p(c, ctypes.c_int32), *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")],
                       _p(rad), _p(stt, ctypes.c_int32))
    return s, rad, stt


def remove(st, status, r_min: float, r_max: float):
    """Removal by distance to the star; returns (state, status)."""
    s = _mut(st)
    stt = np.array(status, dtype=np.int32)
    lib().oracle_remove(len(s["x"]), *[_p(s[k]) for k in ("x", "y", "z", "m")], _p(stt, ctypes.c_int32),
                        float(r_min), float(r_max))
    return s, stt


def step_collide(st, rc, radius, status, mstar: float, dt: float, nsteps: int, r_min: float, r_max: float,
                 tol: float = BS_TOL, n_massive: Optional[int] = None, nsub: int = 1):
    """nsteps full steps with collisions and removal; returns (state, radius, status).  rc is
    the r_crit array, or [nlev][n] radii of levels 0..nlev-1 for the hierarchical step with
    nsub sub-steps per level."""
    s = _mut(st)
    n = len(s["x"])
    rcl = np.ascontiguousarray(np.atleast_2d(np.asarray(rc, dtype=np.float64)))
    nlev = rcl.shape[0]
    rad = np.array(radius, dtype=np.float64)
    stt = np.array(status, dtype=np.int32)
    bad = lib().oracle_step_collide(n, _nm(n, n_massive), *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")],
                                    _p(rcl), int(nlev), int(nsub if nlev > 1 else 1), _p(rad),
                                    _p(stt, ctypes.c_int32), float(mstar), float(dt), int(nsteps), float(tol),
                                    float(r_min), float(r_max))
    if bad:
        raise RuntimeError("oracle step failed")
    return s, rad, stt
