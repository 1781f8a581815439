"""Hierarchical levels (Sect. 1: intermediate symplectic levels with reduced steps between
the level-0 step and the Bulirsch-Stoer step) on the GPU against the oracle's
drift_levels / step_levels, on the GPU's own encounter list.  Level k's radius is eq. (1)
with the level's step dt / n_sub^k (n1 = 3, n2 = 0.4), as in the encounter-dominated runs."""
import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import System

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32
DT5 = discs.DT_5_DAYS


def level_system(d, nlev, nsub):
    rcl = oracle.rcrit_levels(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5, nlev, nsub)
    s = System([d], rcrit=rcl[0])
    genga.genga_set_large_groups(s.ctx.handle, True)
    if nlev > 1:
        t = s.torch.tensor(np.ascontiguousarray(rcl[1:]), dtype=s.torch.float64, device="cuda")
        genga.genga_set_levels(s.ctx.handle, nlev, nsub, t)
        s.torch.cuda.synchronize()
    return s, rcl


def compare(label, got, exp, gid, bar_in=1e-10, bar_out=1e-13):
    inside = gid >= 0
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        e_in = np.max(np.abs(got[k][inside] - exp[k][inside])) if inside.any() else 0.0
        e_out = np.max(np.abs(got[k][~inside] - exp[k][~inside])) if (~inside).any() else 0.0
        print(f"[{label}] {k} groups err {e_in:.2e} others err {e_out:.2e}", flush=True)
        assert e_in <= bar_in
        assert e_out <= bar_out


def test_chains_two_levels_more_tiles_than_cus():
    """150 chains of 70 bodies of 1e-10 solar masses on a circle (level 0: r_crit 2.5
    spacings, level 1: 1.5; the chains 10 spacings apart), 2 levels x 2 sub-steps: 300 target
    tiles in multi-tile groups, more than one workgroup per CU, so the level kick runs 8 waves
    per tile, and the level-1 groups of 70 go to the grid-wide Bulirsch-Stoer."""
    per, gap, ng = 70, 10, 150
    npos = ng * (per + gap)
    keep = (np.arange(npos) % (per + gap)) < per
    th = 2.0 * np.pi * np.arange(npos)[keep] / npos
    c, sn, z = np.cos(th), np.sin(th), np.zeros(len(th))
    d = discs.Disc(c, sn, z.copy(), -sn, c.copy(), z.copy(), np.full(len(th), 1e-10), name="chains")
    spacing = 2.0 * np.pi / npos
    rcl = np.stack([np.full(d.n, 2.5 * spacing), np.full(d.n, 1.5 * spacing)])
    s = System([d], rcrit=rcl[0])
    genga.genga_set_large_groups(s.ctx.handle, True)
    t = s.torch.tensor(np.ascontiguousarray(rcl[1:]), dtype=s.torch.float64, device="cuda")
    genga.genga_set_levels(s.ctx.handle, 2, 2, t)
    s.torch.cuda.synchronize()
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    gid = oracle.groups(d.n, pairs)
    sizes = np.bincount(gid[gid >= 0])
    print(f"[chains 2x2] pairs={cnt} groups={len(sizes)} sizes {sizes.min()}..{sizes.max()}", flush=True)
    assert len(sizes) == ng and sizes.min() == per and int(np.sum((sizes + 63) // 64)) > 256
    b0 = s.numpy_state()
    exp = oracle.drift_levels(b0, rcl, 2, 1.0, DT5, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    compare("chains 2x2", got, exp, gid)
    s.close()


def test_levels_in_a_batch_of_two_systems():
    """Two rings in one batch (300 and 500 bodies), 2 levels x 2 sub-steps: each system's
    drift against the oracle's drift_levels of that system alone."""
    ds = [discs.ring_dense(300, seed=31), discs.ring_dense(500, seed=32)]
    rcls = [oracle.rcrit_levels(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5, 2, 2) for d in ds]
    rcl = np.concatenate(rcls, axis=1)
    s = System(ds, rcrit=rcl[0])
    genga.genga_set_large_groups(s.ctx.handle, True)
    t = s.torch.tensor(np.ascontiguousarray(rcl[1:]), dtype=s.torch.float64, device="cuda")
    genga.genga_set_levels(s.ctx.handle, 2, 2, t)
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    b0 = s.numpy_state()
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    for k, d in enumerate(ds):
        sl = s.system_slice(k)
        lo, hi = sl.start, sl.stop
        mine = pairs[(pairs[:, 0] >= lo) & (pairs[:, 0] < hi)] - lo
        assert np.all((mine >= 0) & (mine < d.n))
        st0 = {key: b0[key][sl] for key in b0}
        exp = oracle.drift_levels(st0, rcls[k], 2, d.mstar, DT5, mine)
        gid = oracle.groups(d.n, mine)
        print(f"[batch {k}] pairs={len(mine)} groups={gid.max() + 1}", flush=True)
        compare(f"batch {k}", {key: got[key][sl] for key in got}, exp, gid)
    s.close()


def test_levels_resume_is_bit_identical():
    """Two calls of two steps with 3 levels x 2 sub-steps in one context equal two steps, a
    save of the state to the host, a fresh context from it and two more steps (FP32 kick).
    The checkpoint sits at a call boundary in both runs: within one call the closing and
    opening half-kicks of consecutive steps are merged into one kick."""
    d = discs.ring_dense(1000)
    s, rcl = level_system(d, 3, 2)
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP32)
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP32)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    whole = s.numpy_state()
    s.close()
    s, _ = level_system(d, 3, 2)
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP32)
    saved = s.numpy_state()
    s.close()
    d2 = discs.Disc(*(saved[k] for k in ("x", "y", "z", "vx", "vy", "vz", "m")), mstar=d.mstar)
    s = System([d2], rcrit=rcl[0])
    genga.genga_set_large_groups(s.ctx.handle, True)
    t = s.torch.tensor(np.ascontiguousarray(rcl[1:]), dtype=s.torch.float64, device="cuda")
    genga.genga_set_levels(s.ctx.handle, 3, 2, t)
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP32)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    resumed = s.numpy_state()
    s.close()
    for k in whole:
        np.testing.assert_array_equal(whole[k], resumed[k])


def test_levels_with_no_encounters_equal_the_plain_path():
    """Degenerate case: radii so small that no pair is listed at any level; three steps with
    3 levels x 2 sub-steps equal those of the plain path bit for bit."""
    d = discs.ring_dense(1000)
    out = []
    for nlev in (1, 3):
        s = System([d], rcrit=np.full(d.n, 1e-9))
        genga.genga_set_large_groups(s.ctx.handle, True)
        if nlev > 1:
            t = s.torch.full((nlev - 1, d.n), 1e-10, dtype=s.torch.float64, device="cuda")
            genga.genga_set_levels(s.ctx.handle, nlev, 2, t)
        genga.genga_set_kick_shape(s.ctx.handle, FP64, 8, 1)
        genga.genga_step(s.ctx.handle, s.b, DT5, 3, FP64)
        assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
        out.append(s.numpy_state())
        s.close()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_array_equal(out[0][k], out[1][k])


@pytest.mark.parametrize("nlev,nsub", [(2, 2), (3, 2), (2, 3), (4, 2)])
def test_ring_drift_with_levels(nlev, nsub):
    d = discs.ring_dense(1000)
    s, rcl = level_system(d, nlev, nsub)
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    gid = oracle.groups(d.n, pairs)
    print(f"[ring {nlev}x{nsub}] pairs={cnt} level-0 groups={gid.max() + 1}", flush=True)
    b0 = s.numpy_state()
    exp = oracle.drift_levels(b0, rcl, nsub, 1.0, DT5, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    compare(f"ring {nlev}x{nsub}", got, exp, gid)
    s.close()


def test_whole_disc_group_with_three_levels():
    """The 6600-body annulus, one level-0 group of every body, integrated by 3 levels of 2
    sub-steps (level-2 groups go to Bulirsch-Stoer)."""
    d = discs.disc_dense()
    s, rcl = level_system(d, 3, 2)
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    gid = oracle.groups(d.n, pairs)
    assert np.bincount(gid[gid >= 0]).max() == d.n
    b0 = s.numpy_state()
    exp = oracle.drift_levels(b0, rcl, 2, 1.0, DT5, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    compare("dense 6600 3x2", got, exp, gid)
    s.close()


def test_steps_with_levels_against_oracle():
    """Five full steps (kick, list, drift with 3 levels, kick) in FP64 and FP32."""
    d = discs.ring_dense(1000)
    rcl = oracle.rcrit_levels(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5, 3, 2)
    exp, _ = oracle.step_levels(d.state(), rcl, 2, 1.0, DT5, 5)
    for prec, bar in ((FP64, 1e-10), (FP32, 1e-8)):
        s, _ = level_system(d, 3, 2)
        genga.genga_step(s.ctx.handle, s.b, DT5, 5, prec)
        got = s.numpy_state()
        assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            err = np.max(np.abs(got[k] - exp[k]))
            print(f"[ring steps 3x2 prec={prec}] {k} max err {err:.2e}", flush=True)
            assert err <= bar
        s.close()


def test_one_level_is_the_plain_large_group_drift():
    """genga_set_levels(1) gives the large-group drift bit for bit."""
    d = discs.ring_dense(1000)
    out = []
    for use_levels in (False, True):
        s, rcl = level_system(d, 1, 1)
        if use_levels:
            genga.genga_set_levels(s.ctx.handle, 1, 1, None)
        s.accel(FP64)
        genga.genga_drift(s.ctx.handle, s.b, DT5)
        out.append(s.numpy_state())
        s.close()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(out[0][k], out[1][k])


def test_set_levels_argument_and_state_checks():
    d = discs.ring_dense(1000)
    rcl = oracle.rcrit_levels(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5, 3, 2)
    s = System([d], rcrit=rcl[0])
    t = s.torch.tensor(np.ascontiguousarray(rcl[1:]), dtype=s.torch.float64, device="cuda")
    with pytest.raises(genga.GengaError) as e:          # large groups off
        genga.genga_set_levels(s.ctx.handle, 3, 2, t)
    assert e.value.status == genga.GENGA_ERR_STATE
    genga.genga_set_large_groups(s.ctx.handle, True)
    for bad in ((0, 2), (5, 2), (3, 0), (3, 65)):
        with pytest.raises(genga.GengaError) as e:
            genga.genga_set_levels(s.ctx.handle, bad[0], bad[1], t)
        assert e.value.status == genga.GENGA_ERR_ARG
    grow = s.torch.tensor(np.ascontiguousarray(rcl[[2, 1]]), dtype=s.torch.float64, device="cuda")
    with pytest.raises(genga.GengaError) as e:          # radii growing with the level
        genga.genga_set_levels(s.ctx.handle, 3, 2, grow)
    assert e.value.status == genga.GENGA_ERR_ARG
    genga.genga_set_levels(s.ctx.handle, 3, 2, t)
    stream = s.torch.cuda.Stream()
    with pytest.raises(genga.GengaError) as e:          # host round trips: no graph capture
        genga.genga_graph_capture(s.ctx.handle, s.b, DT5, 2, FP32, stream=stream)
    assert e.value.status == genga.GENGA_ERR_STATE
    s.close()


def test_tune_levels_keeps_the_state_and_sets_the_fastest():
    """Self-tuning (Sect. 1): every configuration up to 3 levels x 3 sub-steps is tried from
    the current state; the state comes back bit for bit and the chosen configuration is then
    the one genga_drift uses (checked against the oracle's drift_levels)."""
    d = discs.ring_dense(1000)
    s, rc0 = level_system(d, 1, 1)
    b0 = s.numpy_state()
    nl, ns = genga.genga_tune_levels(s.ctx.handle, s.b, DT5, discs.DENSE_N1, discs.DENSE_N2, 3, 3, 2, FP64)
    print(f"[tune] chose {nl} levels x {ns} sub-steps", flush=True)
    assert 1 <= nl <= 3 and (ns == 1 if nl == 1 else 2 <= ns <= 3)
    after = s.numpy_state()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(after[k], b0[k])
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK
    rcl = oracle.rcrit_levels(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5, nl, max(ns, 1))
    s.accel(FP64)
    pairs, _ = s.encounter_list()
    gid = oracle.groups(d.n, pairs)
    exp = oracle.drift_levels(b0, rcl, max(ns, 1), 1.0, DT5, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    compare(f"tuned {nl}x{ns}", got, exp, gid)
    for bad in ((0, 3, 2), (5, 3, 2), (3, 1, 2), (3, 3, 0)):
        with pytest.raises(genga.GengaError) as e:
            genga.genga_tune_levels(s.ctx.handle, s.b, DT5, 3.0, 0.4, *bad, FP64)
        assert e.value.status == genga.GENGA_ERR_ARG
    genga.genga_set_large_groups(s.ctx.handle, False)
    with pytest.raises(genga.GengaError) as e:
        genga.genga_tune_levels(s.ctx.handle, s.b, DT5, 3.0, 0.4, 3, 3, 2, FP64)
    assert e.value.status == genga.GENGA_ERR_STATE
    s.close()


def test_levels_with_test_bodies():
    """TP2 mode (Sect. 3.3) under 3 levels of 2 sub-steps: the last 400 of 1000 ring bodies
    are test bodies, which never interact with each other at any level."""
    d = discs.ring_dense(1000)
    nm = 600
    s, rcl = level_system(d, 3, 2)
    genga.genga_set_test_bodies(s.ctx.handle, np.array([nm], dtype=np.int32))
    t = s.torch.tensor(np.ascontiguousarray(rcl[1:]), dtype=s.torch.float64, device="cuda")
    genga.genga_set_levels(s.ctx.handle, 3, 2, t)
    s.accel(FP64)
    pairs, _ = s.encounter_list()
    assert not np.any((pairs[:, 0] >= nm) & (pairs[:, 1] >= nm))
    gid = oracle.groups(d.n, pairs)
    b0 = s.numpy_state()
    exp = oracle.drift_levels(b0, rcl, 2, 1.0, DT5, pairs, n_massive=nm)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    compare("ring 3x2 TP2", got, exp, gid)
    s.close()
