"""Python binding of the gfx950 kick library (libgenga.so).

Argument marshalling only: every step of the kick path (pair forces, encounter list, drift,
close-encounter step, energy) runs in the HIP kernels behind the C ABI declared in
include/genga.h.  PyTorch provides device memory and streams.  There is no CPU fallback:
if libgenga.so is missing or no GPU is present, the calls raise.

The functions carry the C names (genga_create, genga_kick, ...) and take the same
arguments, with torch tensors in place of device pointers.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgenga.so")

GENGA_OK = 0
GENGA_ERR_ARG = -1
GENGA_ERR_HIP = -2
GENGA_ERR_CAPACITY = -3
GENGA_ERR_NONFINITE = -4
GENGA_ERR_NOCONVERGE = -5
GENGA_ERR_STATE = -6

GENGA_KICK_FP64 = 0
GENGA_KICK_FP32 = 1

GENGA_ACC_FP64 = 0
GENGA_ACC_KAHAN32 = 1

# every entry point of include/genga.h
ENTRY_POINTS = (
    "genga_create", "genga_destroy", "genga_set_systems", "genga_set_test_bodies", "genga_set_large_groups",
    "genga_set_levels", "genga_tune_levels", "genga_set_collisions", "genga_compact", "genga_sort_bodies",
    "genga_rcrit", "genga_accel", "genga_accel_noalloc",
    "genga_kick", "genga_encounter_list", "genga_drift", "genga_energy", "genga_step",
    "genga_graph_capture", "genga_graph_launch", "genga_autotune", "genga_set_kick_shape",
    "genga_get_kick_shape", "genga_poll_status", "genga_last_error",
)


class GengaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"genga status {status}: {message}")
        self.status = status


class genga_bodies(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rcrit")]


_lib: Optional[ctypes.CDLL] = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgenga.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2309_08217_amd.build` "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    bp = ctypes.POINTER(genga_bodies)
    sig = {
        "genga_create": [ctypes.POINTER(vp), ctypes.c_int],
        "genga_destroy": [vp],
        "genga_set_systems": [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), i32],
        "genga_set_test_bodies": [vp, ctypes.POINTER(i32)],
        "genga_set_large_groups": [vp, i32],
        "genga_set_levels": [vp, i32, i32, vp],
        "genga_set_collisions": [vp, vp, vp, vp, dbl, dbl],
        "genga_compact": [vp, bp, vp, vp, ctypes.POINTER(i32)],
        "genga_sort_bodies": [vp, bp, vp, vp],
        "genga_tune_levels": [vp, bp, dbl, dbl, dbl, i32, i32, i32, ctypes.c_int, ctypes.POINTER(i32),
                              ctypes.POINTER(i32), vp],
        "genga_rcrit": [vp, bp, dbl, dbl, dbl, vp, vp],
        "genga_accel": [vp, bp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp],
        "genga_accel_noalloc": [bp, i32, vp, vp, vp, vp, i32, vp, vp, ctypes.c_int, ctypes.c_int, vp],
        "genga_kick": [vp, bp, dbl, ctypes.c_int, ctypes.c_int, vp],
        "genga_encounter_list": [vp, bp, vp, i32, vp, vp],
        "genga_drift": [vp, bp, dbl, vp, vp, vp],
        "genga_energy": [vp, bp, vp, vp],
        "genga_step": [vp, bp, dbl, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp],
        "genga_graph_capture": [vp, bp, dbl, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp],
        "genga_graph_launch": [vp, ctypes.c_int, vp],
        "genga_autotune": [vp, bp, ctypes.c_int, ctypes.c_char_p, vp],
        "genga_set_kick_shape": [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int],
        "genga_get_kick_shape": [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
        "genga_poll_status": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.genga_last_error.argtypes = []
    L.genga_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int) -> int:
    if status < 0:
        msg = load_library().genga_last_error().decode(errors="replace")
        raise GengaError(status, msg)
    return status


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Bodies:
    """Device SoA state (float64 CUDA tensors, length n_total) and its C view."""

    KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "rcrit")

    def __init__(self, **tensors):
        import torch
        for k in self.KEYS:
            t = tensors.get(k)
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda):
                raise TypeError(f"{k} must be a float64 CUDA tensor")
            setattr(self, k, t)

    @classmethod
    def from_numpy(cls, state: dict, rcrit=None, device: str = "cuda"):
        import torch
        t = {k: torch.as_tensor(np.ascontiguousarray(state[k], dtype=np.float64), device=device)
             for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
        if rcrit is not None:
            t["rcrit"] = torch.as_tensor(np.ascontiguousarray(rcrit, dtype=np.float64), device=device)
        return cls(**t)

    def to_numpy(self) -> dict:
        return {k: getattr(self, k).cpu().numpy() for k in ("x", "y", "z", "vx", "vy", "vz", "m")}

    def c(self) -> genga_bodies:
        return genga_bodies(*[_ptr(getattr(self, k)) for k in self.KEYS])


# ----------------------------------------------------------------------------------------------
# Entry points, same names and argument order as include/genga.h
# ----------------------------------------------------------------------------------------------

def genga_create(device: int = 0) -> int:
    L = load_library()
    h = ctypes.c_void_p()
    _check(L.genga_create(ctypes.byref(h), int(device)))
    return h.value


def genga_destroy(ctx: int) -> None:
    _check(load_library().genga_destroy(ctx))


def genga_set_systems(ctx: int, sys_off: Sequence[int], mstar: Sequence[float], pair_capacity: int = 0) -> None:
    off = np.ascontiguousarray(sys_off, dtype=np.int32)
    ms = np.ascontiguousarray(mstar, dtype=np.float64)
    if len(off) != len(ms) + 1:
        raise ValueError("sys_off must have n_sys + 1 entries")
    _check(load_library().genga_set_systems(ctx, len(ms), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(pair_capacity)))


def genga_set_test_bodies(ctx: int, n_massive: Optional[Sequence[int]]) -> None:
    """TP2 mode: per system, the number of massive bodies listed first (None: all massive)."""
    if n_massive is None:
        _check(load_library().genga_set_test_bodies(ctx, None))
        return
    nm = np.ascontiguousarray(n_massive, dtype=np.int32)
    _check(load_library().genga_set_test_bodies(ctx, nm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))


def genga_set_large_groups(ctx: int, enable: bool) -> None:
    """Encounter groups above 64 bodies: integrate them (True) or flag them (False, default)."""
    _check(load_library().genga_set_large_groups(ctx, int(enable)))


def genga_set_levels(ctx: int, n_levels: int, n_sub: int, rcrit_levels=None) -> None:
    """Hierarchical levels: n_levels symplectic levels (1 = the plain step) with n_sub
    sub-steps per level; rcrit_levels a device float64 tensor [n_levels - 1, n_total] with the
    critical radii of levels 1..n_levels-1 (copied)."""
    ptr = None
    if rcrit_levels is not None:
        import torch
        if rcrit_levels.dtype != torch.float64:
            raise TypeError("rcrit_levels must be float64")
        ptr = _ptr(rcrit_levels)
    _check(load_library().genga_set_levels(ctx, int(n_levels), int(n_sub), ptr))


def genga_tune_levels(ctx: int, b: Bodies, dt: float, n1: float, n2: float, max_levels: int, max_sub: int,
                      trial_steps: int, prec: int, stream=None):
    """Try the level configurations, keep the fastest; returns (n_levels, n_sub)."""
    cb = b.c()
    lv, sub = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load_library().genga_tune_levels(ctx, ctypes.byref(cb), float(dt), float(n1), float(n2), int(max_levels),
                                            int(max_sub), int(trial_steps), int(prec), ctypes.byref(lv),
                                            ctypes.byref(sub), _stream(stream)))
    return lv.value, sub.value


def genga_set_collisions(ctx: int, b: Bodies, radius, status, r_min: float, r_max: float) -> None:
    """Perfect mergers and removal by distance on b's masses; radius (float64) and status
    (int32) device tensors of n_total entries.  b = None turns collisions off."""
    if b is None:
        _check(load_library().genga_set_collisions(ctx, None, None, None, 0.0, 0.0))
        return
    import torch
    if radius.dtype != torch.float64 or status.dtype != torch.int32:
        raise TypeError("radius must be float64 and status int32")
    _check(load_library().genga_set_collisions(ctx, _ptr(b.m), _ptr(radius), _ptr(status), float(r_min),
                                               float(r_max)))


def genga_compact(ctx: int, b: Bodies, radius, status) -> int:
    """Remove the bodies with status != 0 in place; returns the new n_total (the tensors keep
    their length, the first n_total entries hold the survivors)."""
    cb = b.c()
    n = ctypes.c_int32(0)
    _check(load_library().genga_compact(ctx, ctypes.byref(cb), _ptr(radius), _ptr(status), ctypes.byref(n)))
    return n.value


def genga_sort_bodies(ctx: int, b: Bodies, perm_out=None, stream=None) -> None:
    """Reorder the bodies in space in place (ring, then azimuth, per system and kind); perm_out
    (int32 device tensor of n_total, optional) receives the old index of each new place."""
    cb = b.c()
    _check(load_library().genga_sort_bodies(ctx, ctypes.byref(cb), _ptr(perm_out), _stream(stream)))


def genga_rcrit(ctx: int, b: Bodies, n1: float, n2: float, dt: float, rc_out, stream=None) -> None:
    cb = b.c()
    _check(load_library().genga_rcrit(ctx, ctypes.byref(cb), float(n1), float(n2), float(dt), _ptr(rc_out),
                                      _stream(stream)))


def genga_accel(ctx: int, b: Bodies, ax, ay, az, prec: int, acc: int = GENGA_ACC_FP64, stream=None) -> None:
    cb = b.c()
    _check(load_library().genga_accel(ctx, ctypes.byref(cb), _ptr(ax), _ptr(ay), _ptr(az), int(prec), int(acc),
                                      _stream(stream)))


GENGA_NOALLOC_MAX_BODIES = 65536


def genga_accel_noalloc(b: Optional[Bodies], n: int, ax, ay, az, pairs, pair_cap: int, d_count, d_status,
                        prec: int, acc: int = GENGA_ACC_FP64, stream=None) -> None:
    """Accelerations and encounter pairs of one system of n bodies with no context and no
    allocation (scratch in a static device array); d_count / d_status: device int32 words."""
    cb = b.c() if b is not None else None
    _check(load_library().genga_accel_noalloc(ctypes.byref(cb) if cb is not None else None, int(n), _ptr(ax),
                                              _ptr(ay), _ptr(az), _ptr(pairs), int(pair_cap), _ptr(d_count),
                                              _ptr(d_status), int(prec), int(acc), _stream(stream)))


def genga_kick(ctx: int, b: Bodies, tau: float, prec: int, acc: int = GENGA_ACC_FP64, stream=None) -> None:
    cb = b.c()
    _check(load_library().genga_kick(ctx, ctypes.byref(cb), float(tau), int(prec), int(acc), _stream(stream)))


def genga_encounter_list(ctx: int, b: Optional[Bodies], pairs, cap: int, d_count, stream=None) -> None:
    """b = None: the list of the last kick; else the list of b's positions, computed alone."""
    cb = b.c() if b is not None else None
    _check(load_library().genga_encounter_list(ctx, ctypes.byref(cb) if cb is not None else None, _ptr(pairs),
                                               int(cap), _ptr(d_count), _stream(stream)))


def genga_drift(ctx: int, b: Bodies, dt: float, pairs=None, d_count=None, stream=None) -> None:
    """pairs = None: the context's encounter list; else a device int32 tensor of pairs and a
    device int32 count."""
    cb = b.c()
    _check(load_library().genga_drift(ctx, ctypes.byref(cb), float(dt), _ptr(pairs), _ptr(d_count),
                                      _stream(stream)))


def genga_energy(ctx: int, b: Bodies, d_out, stream=None) -> None:
    cb = b.c()
    _check(load_library().genga_energy(ctx, ctypes.byref(cb), _ptr(d_out), _stream(stream)))


def genga_step(ctx: int, b: Bodies, dt: float, nsteps: int, prec: int, acc: int = GENGA_ACC_FP64,
               energy_cadence: int = 0, d_energy=None, stream=None) -> None:
    cb = b.c()
    _check(load_library().genga_step(ctx, ctypes.byref(cb), float(dt), int(nsteps), int(prec), int(acc),
                                     int(energy_cadence), _ptr(d_energy), _stream(stream)))


def genga_graph_capture(ctx: int, b: Bodies, dt: float, nsteps: int, prec: int, acc: int = GENGA_ACC_FP64,
                        energy_cadence: int = 0, d_energy=None, stream=None) -> None:
    cb = b.c()
    _check(load_library().genga_graph_capture(ctx, ctypes.byref(cb), float(dt), int(nsteps), int(prec), int(acc),
                                              int(energy_cadence), _ptr(d_energy), _stream(stream)))


def genga_graph_launch(ctx: int, repeats: int, stream=None) -> None:
    _check(load_library().genga_graph_launch(ctx, int(repeats), _stream(stream)))


def genga_autotune(ctx: int, b: Bodies, prec: int, cache_path: Optional[str] = None, stream=None) -> None:
    """Time the kick's launch shapes and keep the fastest; cache_path: a text file of earlier
    results (read, and appended to on a miss)."""
    cb = b.c()
    path = os.fsencode(cache_path) if cache_path is not None else None
    _check(load_library().genga_autotune(ctx, ctypes.byref(cb), int(prec), path, _stream(stream)))


def genga_set_kick_shape(ctx: int, prec: int, waves: int, split: int = 0) -> None:
    _check(load_library().genga_set_kick_shape(ctx, int(prec), int(waves), int(split)))


def genga_get_kick_shape(ctx: int, prec: int):
    """(waves per workgroup, source split) of the kick for `prec`."""
    w, s = ctypes.c_int(), ctypes.c_int()
    _check(load_library().genga_get_kick_shape(ctx, int(prec), ctypes.byref(w), ctypes.byref(s)))
    return w.value, s.value


def genga_poll_status(ctx: int) -> int:
    """Returns the deferred device status (0 or a negative genga_status) without raising."""
    return load_library().genga_poll_status(ctx)


def genga_last_error() -> str:
    return load_library().genga_last_error().decode(errors="replace")


class Context:
    """Owns one genga_ctx; thin convenience wrapper over the entry points."""

    def __init__(self, device: int = 0):
        self.handle = genga_create(device)

    def close(self):
        if self.handle:
            genga_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
