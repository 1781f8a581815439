"""Encounter-dominated regime (Sect. 3.5): with the full eq. (1) (n1 = 3, n2 = 0.4) on the
paper's dense annulus the encounter groups grow past one wavefront, up to the whole disc.
The grid-wide Bulirsch-Stoer path (genga_set_large_groups) against the oracle's drift and
steps, on the GPU's own input state."""
import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import System

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32
DT5 = discs.DT_5_DAYS


def dense_system(d, large=True, pair_capacity=0):
    rc = oracle.rcrit(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5)
    s = System([d], pair_capacity=pair_capacity, rcrit=rc)
    if large:
        genga.genga_set_large_groups(s.ctx.handle, True)
    return s


def compare_drift(d, label, pair_capacity=0):
    s = dense_system(d, pair_capacity=pair_capacity)
    s.accel(FP64)                       # the encounter list of this state
    pairs, cnt = s.encounter_list(cap=pair_capacity or None)
    b0 = s.numpy_state()
    gid = oracle.groups(d.n, pairs)
    sizes = np.bincount(gid[gid >= 0])
    print(f"[{label}] pairs={cnt} groups={len(sizes)} largest={sizes.max()} above 64={(sizes > 64).sum()}", flush=True)
    assert sizes.max() > 64
    exp = oracle.drift(b0, s.rc, 1.0, DT5, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    inside = gid >= 0
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        e_bs = np.max(np.abs(got[k][inside] - exp[k][inside]))
        e_kep = np.max(np.abs(got[k][~inside] - exp[k][~inside])) if (~inside).any() else 0.0
        print(f"[{label}] {k} BS err {e_bs:.2e} Kepler err {e_kep:.2e}", flush=True)
        assert e_bs <= 1e-10
        assert e_kep <= 1e-13
    s.close()


def test_ring_groups_of_hundreds():
    """1000 bodies, 0.8-0.9 au: 4 groups, three above 64 bodies (the largest 511)."""
    compare_drift(discs.ring_dense(1000), "ring 1000")


def test_annulus_mixed_group_sizes():
    """2000 bodies, 0.7-1 au: large groups and groups of 2-64 in the same drift."""
    compare_drift(discs.disc_dense(2000, seed=14), "annulus 2000")


def test_whole_disc_is_one_group():
    """The paper's first experiment at n2 = 0.4: all 6600 bodies form one encounter group."""
    compare_drift(discs.disc_dense(), "dense 6600")


def test_more_members_than_one_workgroup_builds():
    """20000 bodies in 1-3 au: 15280 bodies in 2794 groups (more than the one-workgroup group
    builder holds), six of them above 64 bodies, the largest 2891."""
    compare_drift(discs.disc_dense(20000, seed=23, a_in=1.0, a_out=3.0), "wide 20000")


def test_ring_steps_against_oracle():
    """Five full steps (kick, list, drift with large groups, kick) in FP64 and FP32."""
    d = discs.ring_dense(1000)
    for prec, bar in ((FP64, 1e-10), (FP32, 1e-8)):
        s = dense_system(d)
        genga.genga_step(s.ctx.handle, s.b, DT5, 5, prec)
        got = s.numpy_state()
        assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
        exp, _ = oracle.step(d.state(), s.rc, 1.0, DT5, 5)
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            err = np.max(np.abs(got[k] - exp[k]))
            print(f"[ring steps prec={prec}] {k} max err {err:.2e}", flush=True)
            assert err <= bar
        s.close()


def ring_chain(n):
    """n bodies of 1e-12 solar masses equally spaced on a circular orbit at 1 au."""
    th = 2.0 * np.pi * np.arange(n) / n
    c, s = np.cos(th), np.sin(th)
    z = np.zeros(n)
    return discs.Disc(c, s, z.copy(), -s, c.copy(), z.copy(), np.full(n, 1e-12), name=f"chain_n{n}")


def test_many_large_groups_more_tiles_than_cus():
    """150 chains of 70 bodies of 1e-10 solar masses (each body within r_crit of two neighbours
    on either side, the chains 10 spacings apart): 300 target tiles, more than one workgroup
    per CU, so the sub-steps run the 8-wave tile kernel.  The drift against the oracle's (the
    pair forces move the bodies by about 1e-6 au over the step)."""
    per, gap, ng = 70, 10, 150
    npos = ng * (per + gap)
    keep = (np.arange(npos) % (per + gap)) < per
    full = ring_chain(npos)
    d = discs.Disc(*(getattr(full, k)[keep] for k in ("x", "y", "z", "vx", "vy", "vz")),
                   np.full(int(keep.sum()), 1e-10), name="chains")
    spacing = 2.0 * np.pi / npos
    rc = np.full(d.n, 2.5 * spacing)
    s = System([d], rcrit=rc)
    genga.genga_set_large_groups(s.ctx.handle, True)
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    gid = oracle.groups(d.n, pairs)
    sizes = np.bincount(gid[gid >= 0])
    tiles = int(np.sum((sizes + 63) // 64))
    print(f"[chains] groups={len(sizes)} sizes {sizes.min()}..{sizes.max()} tiles={tiles}", flush=True)
    assert len(sizes) == ng and sizes.min() == per and tiles > 256
    b0 = s.numpy_state()
    exp = oracle.drift(b0, rc, 1.0, DT5, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        err = np.max(np.abs(got[k] - exp[k]))
        print(f"[chains] {k} max err {err:.2e}", flush=True)
        assert err <= 1e-10
    s.close()


def test_large_groups_with_no_encounters_equal_the_plain_path():
    """Degenerate case: r_crit so small that no pair is listed; with the large-group mode on,
    three steps equal those of the plain path bit for bit (Kepler and Sun drifts only), in
    both kick precisions."""
    d = discs.ring_dense(1000)
    rc = np.full(d.n, 1e-9)
    for prec in (FP64, FP32):
        out = []
        for large in (False, True):
            s = System([d], rcrit=rc)
            genga.genga_set_large_groups(s.ctx.handle, large)
            genga.genga_set_kick_shape(s.ctx.handle, prec, 8, 1)
            genga.genga_step(s.ctx.handle, s.b, DT5, 3, prec)
            assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
            assert s.encounter_list()[1] == 0
            out.append(s.numpy_state())
            s.close()
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            np.testing.assert_array_equal(out[0][k], out[1][k])


def test_group_above_limit_refused_before_drift():
    """66000 bodies in a chain (each within r_crit of its two neighbours on either side) form
    one group above the 65536-body limit: the drift is refused with GENGA_ERR_CAPACITY and the
    bodies are untouched.  On the same context a drift whose list holds one group of 104
    bodies then matches the oracle."""
    n = 66000
    d = ring_chain(n)
    spacing = 2.0 * np.pi / n
    s = System([d], rcrit=np.full(n, 2.5 * spacing))
    genga.genga_set_large_groups(s.ctx.handle, True)
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    assert cnt == 2 * n
    b0 = s.numpy_state()
    with pytest.raises(genga.GengaError) as e:
        genga.genga_drift(s.ctx.handle, s.b, DT5)
    assert e.value.status == genga.GENGA_ERR_CAPACITY
    got = s.numpy_state()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(got[k], b0[k])
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK

    rc2 = np.full(n, 0.4 * spacing)
    rc2[:100] = 2.5 * spacing
    s.b = genga.Bodies.from_numpy(d.state(), rc2)
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    gid = oracle.groups(n, pairs)
    assert np.bincount(gid[gid >= 0]).tolist() == [104]
    b0 = s.numpy_state()
    exp = oracle.drift(b0, rc2, 1.0, DT5, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    inside = gid >= 0
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.max(np.abs(got[k][inside] - exp[k][inside])) <= 1e-10
        assert np.max(np.abs(got[k][~inside] - exp[k][~inside])) <= 1e-13
    s.close()


def test_large_groups_off_flags_capacity_and_graph_refused():
    """Without the switch a group above 64 bodies is flagged; with it, graph capture is refused."""
    d = discs.ring_dense(1000)
    s = dense_system(d, large=False)
    s.accel(FP64)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    s.torch.cuda.synchronize()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_ERR_CAPACITY
    genga.genga_set_large_groups(s.ctx.handle, True)
    stream = s.torch.cuda.Stream()
    with pytest.raises(genga.GengaError) as e:
        genga.genga_graph_capture(s.ctx.handle, s.b, DT5, 2, FP32, stream=stream)
    assert e.value.status == genga.GENGA_ERR_STATE
    with pytest.raises(genga.GengaError):
        genga.genga_set_large_groups(s.ctx.handle, 2)
    s.close()


def test_tight_binary_inside_a_large_group():
    """A binary of two 1e-4 solar-mass bodies 3e-3 au apart inside the 0.8-0.9 au ring: their
    mutual pull (about 10 in these units, against the star's 1.3) bends their paths far from the
    straight lines the grid-wide step's neighbour lists are built on, so attempts are voided and
    listed again with wider margins until the bound holds.  The drift against the oracle's."""
    d0 = discs.ring_dense(1000)
    st = d0.state()
    m, sep = 1e-4, 3e-3
    r0 = np.array([st["x"][0], st["y"][0], st["z"][0]])
    v0 = np.array([st["vx"][0], st["vy"][0], st["vz"][0]])
    u = r0 / np.linalg.norm(r0)
    w = np.cross([0.0, 0.0, 1.0], u)
    vrel = np.sqrt(2.0 * m / sep)
    for q, key in enumerate(("x", "y", "z")):
        st[key][1] = r0[q] + sep * u[q]
        st["v" + key][1] = v0[q] + vrel * w[q]
    st["m"][0] = st["m"][1] = m
    compare_drift(discs.Disc(**st, name="ring with binary"), "tight binary")


def test_lists_over_capacity_fall_back_to_the_tile_path():
    """1400 bodies on a jittered lattice 0.02 au across (spacing 5e-4 au), all inside each
    other's r_crit (about 0.037 au here): every member would list the other 1399, more than a
    list holds (8 segments of 128) and from more source tiles than a target tile stages (16),
    so the steps' attempts run on the tile path.  The drift against the oracle's."""
    d0 = discs.disc_dense(2000, seed=14)
    st = d0.state()
    rng = np.random.default_rng(5)
    side = 38
    n_c = 1400
    ij = np.stack(np.meshgrid(np.arange(side), np.arange(side), indexing="ij"), -1).reshape(-1, 2)[:n_c]
    spacing = 0.02 / side
    off = np.zeros((n_c, 3))
    off[:, :2] = (ij - side / 2) * spacing + rng.uniform(-0.1, 0.1, (n_c, 2)) * spacing
    off[:, 2] = rng.uniform(-0.1, 0.1, n_c) * spacing
    r0 = np.array([st["x"][0], st["y"][0], st["z"][0]])
    v0 = np.array([st["vx"][0], st["vy"][0], st["vz"][0]])
    for q, key in enumerate(("x", "y", "z")):
        st[key][:n_c] = r0[q] + off[:, q]
        st["v" + key][:n_c] = v0[q] * (1.0 + rng.normal(0.0, 1e-5, n_c))
    # about 1.0e6 pairs: the list's default capacity (16 per body) is raised
    compare_drift(discs.Disc(**st, name="clump"), "clump 1400", pair_capacity=1 << 21)


def test_large_groups_with_test_bodies():
    """TP2 mode (Sect. 3.3) on the grid-wide path: the last 400 of the 1000 ring bodies are
    test bodies; groups above 64 bodies mix both kinds, and no two test members exert a force
    on each other.  The drift against the oracle's."""
    d = discs.ring_dense(1000)
    nm = 600
    s = dense_system(d)
    genga.genga_set_test_bodies(s.ctx.handle, np.array([nm], dtype=np.int32))
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    assert not np.any((pairs[:, 0] >= nm) & (pairs[:, 1] >= nm))
    gid = oracle.groups(d.n, pairs)
    sizes = np.bincount(gid[gid >= 0])
    big = np.flatnonzero(sizes > 64)
    assert len(big) >= 1 and np.any(np.isin(gid[nm:], big))
    b0 = s.numpy_state()
    exp = oracle.drift(b0, s.rc, 1.0, DT5, pairs, n_massive=nm)
    genga.genga_drift(s.ctx.handle, s.b, DT5)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        err = np.max(np.abs(got[k] - exp[k]))
        print(f"[tp2 large groups] {k} max err {err:.2e}", flush=True)
        assert err <= 1e-10
    s.close()


def test_large_groups_resume_is_bit_identical():
    """The grid-wide path's neighbour lists depend only on the step's starting state: two calls
    of two steps in one context equal two steps, a save to the host, a fresh context from it
    and two more steps (FP32 kick; the ring's groups of hundreds of bodies)."""
    d = discs.ring_dense(1000)
    s = dense_system(d)
    rc = s.rc
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP32)
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP32)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    whole = s.numpy_state()
    s.close()
    s = dense_system(d)
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP32)
    saved = s.numpy_state()
    s.close()
    d2 = discs.Disc(*(saved[k] for k in ("x", "y", "z", "vx", "vy", "vz", "m")), mstar=d.mstar)
    s = System([d2], rcrit=rc)
    genga.genga_set_large_groups(s.ctx.handle, True)
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP32)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    resumed = s.numpy_state()
    s.close()
    for k in whole:
        np.testing.assert_array_equal(whole[k], resumed[k])
