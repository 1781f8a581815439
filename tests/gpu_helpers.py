"""Helpers shared by the GPU parity tests: build device state from seeded discs, run the
library through its C ABI, and compare with the FP64 oracle."""
from __future__ import annotations

import numpy as np

import discs
import oracle
import paper_2309_08217_amd as genga

N1_HILL = 3.0
N2_VEL = 0.0
DT = discs.DT_6_DAYS


def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch


class System:
    """A set of discs laid out in CSR form on the device, with a context."""

    def __init__(self, disc_list, pair_capacity: int = 0, rcrit=None):
        torch = torch_mod()
        self.discs = disc_list
        self.state, self.off, self.mstar = discs.concat(disc_list)
        if rcrit is None:
            rcrit = np.concatenate([oracle.rcrit(d.state(), d.mstar, N1_HILL, N2_VEL, DT) for d in disc_list]) \
                if disc_list else np.zeros(0)
        self.rc = np.ascontiguousarray(rcrit, dtype=np.float64)
        self.ctx = genga.Context()
        genga.genga_set_systems(self.ctx.handle, self.off, self.mstar, pair_capacity)
        self.b = genga.Bodies.from_numpy(self.state, self.rc)
        self.n = len(self.state["x"])
        self.torch = torch

    def zeros(self, n=None, dtype=None):
        torch = self.torch
        return torch.zeros(self.n if n is None else n, dtype=dtype or torch.float64, device="cuda")

    def accel(self, prec):
        ax, ay, az = self.zeros(), self.zeros(), self.zeros()
        genga.genga_accel(self.ctx.handle, self.b, ax, ay, az, prec)
        self.torch.cuda.synchronize()
        return np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], axis=1)

    def encounter_list(self, cap=None, standalone=False):
        """Canonical pair list: the last kick's (standalone=False) or computed from the
        current positions (standalone=True)."""
        torch = self.torch
        cap = 16 * self.n + 16 if cap is None else cap
        pairs = torch.zeros(max(cap, 1) * 2, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        genga.genga_encounter_list(self.ctx.handle, self.b if standalone else None, pairs, cap, cnt)
        torch.cuda.synchronize()
        c = int(cnt.item())
        return pairs[: 2 * min(c, cap)].cpu().numpy().reshape(-1, 2), c

    def energy(self):
        out = self.zeros(4 * len(self.discs))
        genga.genga_energy(self.ctx.handle, self.b, out)
        self.torch.cuda.synchronize()
        return out.cpu().numpy().reshape(-1, 4)

    def numpy_state(self):
        self.torch.cuda.synchronize()
        return self.b.to_numpy()

    def system_slice(self, s):
        return slice(int(self.off[s]), int(self.off[s + 1]))

    def close(self):
        self.ctx.close()


def oracle_accel_systems(sysm: System):
    out = np.zeros((sysm.n, 3))
    for s, d in enumerate(sysm.discs):
        sl = sysm.system_slice(s)
        st = {k: v[sl] for k, v in sysm.state.items()}
        out[sl] = np.stack(oracle.accel(st, sysm.rc[sl]), axis=1)
    return out


def force_errors(a, ref):
    """rms and max per-body relative error |a - a_ref| / |a_ref| (the per-body force metric)."""
    num = np.linalg.norm(a - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    den = np.where(den > 0, den, 1.0)
    e = num / den
    return float(np.sqrt(np.mean(e * e))), float(np.max(e))
