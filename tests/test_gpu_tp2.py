"""TP2 mode (Sect. 3.3) on the GPU against the oracle: test bodies feel and exert forces on
the massive bodies only."""
import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import DT, System, force_errors

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32


def tp2_disc(n_test, n_massive, seed):
    return discs.make_disc(n_test, 2.0, seed=seed, a_in=0.7, a_out=1.0, sigma_e=0.002, sigma_i=0.002,
                           n_embryo=n_massive, embryo_mass_earth=0.3)


def oracle_accel_tp2(s, nms):
    out = np.zeros((s.n, 3))
    for k, d in enumerate(s.discs):
        sl = s.system_slice(k)
        st = {key: v[sl] for key, v in s.state.items()}
        out[sl] = np.stack(oracle.accel(st, s.rc[sl], n_massive=nms[k]), axis=1)
    return out


def test_tp2_accel_encounters_energy_batch():
    ds = [tp2_disc(1500, 12, 81), tp2_disc(700, 0, 82), tp2_disc(300, 5, 83), tp2_disc(200, 70, 84)]
    nms = [12, 0, 5, 270]       # the last system is fully massive
    s = System(ds)
    genga.genga_set_test_bodies(s.ctx.handle, nms)
    ref = oracle_accel_tp2(s, nms)
    for prec, bar in ((FP64, 1e-12), (FP32, 1e-5)):
        a = s.accel(prec)
        for k in range(len(ds)):
            sl = s.system_slice(k)
            rms, mx = force_errors(a[sl], ref[sl])
            print(f"[tp2 accel] sys={k} n_massive={nms[k]} prec={prec} rms={rms:.3e}", flush=True)
            assert rms <= bar
        got, cnt = s.encounter_list()
        exp = np.concatenate([oracle.encounters({q: v[s.system_slice(k)] for q, v in s.state.items()},
                                                s.rc[s.system_slice(k)], n_massive=nms[k]) + s.off[k]
                              for k in range(len(ds))]).astype(np.int32)
        assert cnt == len(exp) and cnt > 0
        np.testing.assert_array_equal(got, exp)
    E = s.energy()
    for k, d in enumerate(ds):
        e = oracle.energy(d.state(), 1.0, n_massive=nms[k])
        assert abs(E[k, 0] - e[0]) <= 1e-13 * abs(e[0])
    # switching back to all-massive gives the plain sums
    genga.genga_set_test_bodies(s.ctx.handle, None)
    full = s.accel(FP64)
    sl = s.system_slice(0)
    rms, _ = force_errors(full[sl], np.stack(oracle.accel(ds[0].state(), s.rc[sl]), axis=1))
    assert rms <= 1e-12
    s.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_tp2_steps_against_oracle(prec):
    d = tp2_disc(1200, 8, 85)
    s = System([d])
    genga.genga_set_test_bodies(s.ctx.handle, [8])
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    print(f"[tp2 steps] pairs at t=0: {cnt}", flush=True)
    genga.genga_step(s.ctx.handle, s.b, DT, 3, prec)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    exp, _ = oracle.step(d.state(), s.rc, 1.0, DT, 3, n_massive=8)
    tol = 1e-9 if prec == FP64 else 1e-7
    for k in ("x", "y", "z"):
        err = np.max(np.abs(got[k] - exp[k]))
        print(f"[tp2 steps prec={prec}] {k} max err {err:.2e}", flush=True)
        assert err <= tol
    s.close()


def test_tp2_group_with_test_members():
    """Encounter groups that contain test bodies: the (1-K) forces between two test members
    are left out on both sides."""
    d = tp2_disc(600, 3, 86)
    st = d.state()
    rng = np.random.default_rng(86)
    rc = oracle.rcrit(st, 1.0, 3.0, 0.0, DT)
    # plant test bodies around embryo 0 inside its critical radius
    for k in range(6):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        for q, key in enumerate(("x", "y", "z")):
            st[key][10 + k] = st[key][0] + u[q] * (0.2 + 0.1 * k) * rc[0]
        for key in ("vx", "vy", "vz"):
            st[key][10 + k] = st[key][0] + rng.normal(scale=2e-3)
    dd = discs.Disc(**st)
    s = System([dd], rcrit=rc)
    genga.genga_set_test_bodies(s.ctx.handle, [3])
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    gid = oracle.groups(dd.n, pairs)
    assert np.bincount(gid[gid >= 0]).max() >= 7
    exp = oracle.drift(st, rc, 1.0, DT, pairs, n_massive=3)
    genga.genga_drift(s.ctx.handle, s.b, DT)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        err = np.max(np.abs(got[k] - exp[k]))
        print(f"[tp2 group] {k} max err {err:.2e}", flush=True)
        assert err <= 1e-10
    s.close()
