"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

Bars: FP64 kick rms per-body relative force error <= 1e-12, FP32 kick <= 1e-5 (the
stated targets); encounter lists bit-exact; drift and energy to the FP64 rounding level;
Bulirsch-Stoer results to its tolerance.
"""
import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import DT, System, force_errors, oracle_accel_systems

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32


def _sizes_disc(n, seed, **kw):
    return discs.make_disc(n, 2.5, seed=seed, **kw)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 127, 257, 1000, 2049])
def test_accel_ragged_sizes_fp64_and_fp32(n):
    print(f"[accel ragged] n={n}", flush=True)
    d = _sizes_disc(n, seed=100 + n, a_in=0.7, a_out=1.0)
    s = System([d])
    ref = oracle_accel_systems(s)
    for prec, bar in ((FP64, 1e-12), (FP32, 1e-5)):
        a = s.accel(prec)
        if n == 1:
            assert np.all(a == 0.0)
            continue
        rms, mx = force_errors(a, ref)
        print(f"  prec={prec} rms={rms:.3e} max={mx:.3e}", flush=True)
        assert rms <= bar
    s.close()


@pytest.mark.parametrize("split", [1, 2, 3, 4])
def test_accel_c1_disc_and_launch_shapes(split):
    d = discs.disc_c1()
    s = System([d])
    ref = oracle_accel_systems(s)
    for w in (4, 8, 16):
        for prec, bar in ((FP64, 1e-12), (FP32, 1e-5)):
            genga.genga_set_kick_shape(s.ctx.handle, prec, w, split)
            a = s.accel(prec)
            rms, mx = force_errors(a, ref)
            print(f"[accel c1] waves={w} split={split} prec={prec} rms={rms:.3e} max={mx:.3e}", flush=True)
            assert rms <= bar
            assert mx <= (1e-10 if prec == FP64 else 1e-3)
            got, cnt = s.encounter_list()
            np.testing.assert_array_equal(got, oracle.encounters(d.state(), s.rc))
    s.close()


def test_changeover_zone_and_inner_zone_pairs():
    """Bodies placed inside 0.1 r_crit, in the changeover zone and just outside."""
    rng = np.random.default_rng(5)
    base = discs.make_disc(200, 2.5, seed=77, a_in=0.9, a_out=1.0)
    st = base.state()
    rc = np.full(base.n, 2e-3)
    # plant partners at chosen fractions of r_crit next to the first 60 bodies
    fr = np.array([0.03, 0.08, 0.2, 0.5, 0.9, 0.999, 1.001, 1.5] * 8)[:60]
    for k in range(60):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        for key, q in zip(("x", "y", "z"), range(3)):
            st[key][100 + k] = st[key][k] + u[q] * fr[k] * 2e-3
    d = discs.Disc(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["m"])
    s = System([d], rcrit=rc)
    ref = oracle_accel_systems(s)
    for prec, bar in ((FP64, 1e-12), (FP32, 1e-5)):
        rms, mx = force_errors(s.accel(prec), ref)
        print(f"[changeover zones] prec={prec} rms={rms:.3e} max={mx:.3e}", flush=True)
        assert rms <= bar
        got, cnt = s.encounter_list()
        exp = oracle.encounters(st, rc)
        assert cnt == len(exp) and len(exp) >= 40
        np.testing.assert_array_equal(got, exp)
    s.close()


def test_encounter_list_dense_cold_disc():
    d = discs.make_disc(3000, 2.0, seed=55, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001,
                        n_embryo=40, embryo_mass_earth=0.05)
    s = System([d])
    exp = oracle.encounters(d.state(), s.rc)
    for prec in (FP32, FP64):
        s.accel(prec)
        got, cnt = s.encounter_list()
        print(f"[encounters dense] prec={prec} count={cnt} oracle={len(exp)}", flush=True)
        assert cnt == len(exp)
        np.testing.assert_array_equal(got, exp)
    assert len(exp) > 20
    s.close()


def test_rcrit_eq1():
    d = discs.disc_c1()
    s = System([d])
    rc = s.zeros()
    for n1, n2 in ((3.0, 0.0), (3.0, 0.4)):
        genga.genga_rcrit(s.ctx.handle, s.b, n1, n2, DT, rc)
        s.torch.cuda.synchronize()
        ref = oracle.rcrit(d.state(), 1.0, n1, n2, DT)
        np.testing.assert_allclose(rc.cpu().numpy(), ref, rtol=2e-15)
    s.close()


def test_kick_updates_velocity():
    d = discs.disc_c1()
    s = System([d])
    tau = 0.37 * DT
    genga.genga_kick(s.ctx.handle, s.b, tau, FP64)
    got = s.numpy_state()
    a = np.stack(oracle.accel(d.state(), s.rc), axis=1)
    for q, k in enumerate(("vx", "vy", "vz")):
        exp = d.state()[k] + tau * a[:, q]
        np.testing.assert_allclose(got[k], exp, rtol=0, atol=1e-15 * np.max(np.abs(exp)))
    for k in ("x", "y", "z"):
        np.testing.assert_array_equal(got[k], d.state()[k])
    s.close()


def test_drift_without_encounters():
    d = discs.disc_c1()
    rc = np.zeros(d.n)      # no pairs: every body is Kepler-drifted
    s = System([d], rcrit=rc)
    s.accel(FP64)           # refresh the (empty) encounter list
    genga.genga_drift(s.ctx.handle, s.b, DT)
    got = s.numpy_state()
    exp = oracle.drift(d.state(), rc, 1.0, DT, np.zeros((0, 2), np.int32))
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        err = np.max(np.abs(got[k] - exp[k]))
        print(f"[drift no-enc] {k} max abs err {err:.2e}", flush=True)
        assert err <= 1e-13 * max(1.0, np.max(np.abs(exp[k])))
    s.close()


def test_drift_long_and_hyperbolic_kepler():
    """Kepler drift over many orbits and on unbound orbits (universal variables vs the
    oracle's eccentric/hyperbolic-anomaly f and g)."""
    rng = np.random.default_rng(3)
    n = 300
    r = rng.uniform(0.5, 3, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    vfac = np.concatenate([rng.uniform(0.6, 1.3, n - 60), rng.uniform(1.5, 3.0, 60)])  # last 60 unbound
    st = dict(x=r * np.cos(ang), y=r * np.sin(ang), z=rng.normal(0, 0.05, n),
              vx=-vfac * np.sin(ang) / np.sqrt(r), vy=vfac * np.cos(ang) / np.sqrt(r), vz=rng.normal(0, 0.02, n),
              m=np.zeros(n))
    d = discs.Disc(**st)
    s = System([d], rcrit=np.zeros(n))
    s.accel(FP64)
    for dt in (0.05, 3.0, 40.0):
        b0 = s.numpy_state()
        genga.genga_drift(s.ctx.handle, s.b, dt)
        got = s.numpy_state()
        exp = oracle.drift(b0, np.zeros(n), 1.0, dt, np.zeros((0, 2), np.int32))
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            err = np.max(np.abs(got[k] - exp[k]) / np.maximum(1.0, np.abs(exp[k])))
            print(f"[kepler dt={dt}] {k} max err {err:.2e}", flush=True)
            assert err <= 5e-12
    s.close()


def test_drift_with_encounter_groups():
    d = discs.make_disc(2000, 2.0, seed=56, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001,
                        n_embryo=40, embryo_mass_earth=0.05)
    s = System([d])
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    assert cnt > 5
    exp = oracle.drift(d.state(), s.rc, 1.0, DT, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK
    gid = oracle.groups(d.n, pairs)
    inside = gid >= 0
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        e_kep = np.max(np.abs(got[k][~inside] - exp[k][~inside]))
        e_bs = np.max(np.abs(got[k][inside] - exp[k][inside]))
        print(f"[drift enc] {k} kepler err {e_kep:.2e} BS err {e_bs:.2e} ({inside.sum()} in groups)", flush=True)
        assert e_kep <= 1e-13
        assert e_bs <= 1e-10
    s.close()


def test_energy_parity():
    for d in (discs.disc_c1(), _sizes_disc(77, 9)):
        s = System([d])
        got = s.energy()[0]
        exp = oracle.energy(d.state(), 1.0)
        print(f"[energy] n={d.n} E={got[0]:.15e} oracle={exp[0]:.15e}", flush=True)
        assert abs(got[0] - exp[0]) <= 1e-13 * abs(exp[0])
        np.testing.assert_allclose(got[1:], exp[1:], rtol=1e-13, atol=1e-13 * np.linalg.norm(exp[1:]))
        s.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_full_steps_against_oracle(prec):
    d = discs.make_disc(1500, 2.0, seed=57, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001,
                        n_embryo=20, embryo_mass_earth=0.05)
    s = System([d])
    nst = 3
    genga.genga_step(s.ctx.handle, s.b, DT, nst, prec)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK
    exp, _ = oracle.step(d.state(), s.rc, 1.0, DT, nst)
    # FP64: the groups' Bulirsch-Stoer accepts at 1e-12 of their position scale (about 1 au,
    # reading R10), so three steps differ by a few 1e-12 at most (measured 5.6e-13); FP32: the
    # kick's 1e-7 relative force error moves positions by ~1e-11 over three steps
    tol_r = 1e-11 if prec == FP64 else 1e-9
    for k in ("x", "y", "z"):
        err = np.max(np.abs(got[k] - exp[k]))
        print(f"[step prec={prec}] {k} max err {err:.2e}", flush=True)
        assert err <= tol_r
    for k in ("vx", "vy", "vz"):
        err = np.max(np.abs(got[k] - exp[k]))
        assert err <= 10 * tol_r
    s.close()


def test_batched_systems_match_single_systems():
    ds = [_sizes_disc(n, seed=300 + n) for n in (130, 64, 1, 700, 65, 2000)]
    s = System(ds)
    ref = oracle_accel_systems(s)
    for prec, bar in ((FP64, 1e-12), (FP32, 1e-5)):
        a = s.accel(prec)
        for k in range(len(ds)):
            sl = s.system_slice(k)
            if ds[k].n < 2:
                assert np.all(a[sl] == 0)
                continue
            rms, _ = force_errors(a[sl], ref[sl])
            assert rms <= bar
    E = s.energy()
    for k, d in enumerate(ds):
        exp = oracle.energy(d.state(), 1.0)
        assert abs(E[k, 0] - exp[0]) <= 1e-13 * abs(exp[0])
    # two steps of the batch equal two steps of each system alone (to FP64 rounding)
    genga.genga_step(s.ctx.handle, s.b, DT, 2, FP64)
    got = s.numpy_state()
    for k, d in enumerate(ds):
        single = System([d], rcrit=s.rc[s.system_slice(k)])
        genga.genga_step(single.ctx.handle, single.b, DT, 2, FP64)
        one = single.numpy_state()
        for key in ("x", "vx"):
            np.testing.assert_array_equal(got[key][s.system_slice(k)], one[key])
        single.close()
    s.close()


def _empty_disc():
    return discs.Disc(*(np.zeros(0) for _ in range(7)))


def test_empty_systems_in_a_batch():
    """Systems with no bodies between and around non-empty ones: the others' forces, lists,
    energies and steps are exactly those of the batch without the empty systems, the empty
    systems' energy rows are zero."""
    full = [_sizes_disc(n, seed=400 + n, a_in=0.7, a_out=1.0) for n in (90, 65)]
    ds = [_empty_disc(), full[0], _empty_disc(), _empty_disc(), full[1], _empty_disc()]
    s, t = System(ds), System(full)
    ref = oracle_accel_systems(t)
    for prec, bar in ((FP64, 1e-12), (FP32, 1e-5)):
        a, b = s.accel(prec), t.accel(prec)
        np.testing.assert_array_equal(a, b)
        assert force_errors(a, ref)[0] <= bar
    np.testing.assert_array_equal(s.encounter_list()[0], t.encounter_list()[0])
    E, F = s.energy(), t.energy()
    assert np.all(E[[0, 2, 3, 5]] == 0.0)
    np.testing.assert_array_equal(E[[1, 4]], F)
    for prec in (FP64, FP32):
        genga.genga_step(s.ctx.handle, s.b, DT, 3, prec)
        genga.genga_step(t.ctx.handle, t.b, DT, 3, prec)
        assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
        got, exp = s.numpy_state(), t.numpy_state()
        for k in got:
            np.testing.assert_array_equal(got[k], exp[k])
    s.close()
    t.close()


def test_all_systems_empty():
    """n_total = 0: every call is a successful no-op; the energy rows are zero."""
    s = System([_empty_disc(), _empty_disc()])
    assert s.n == 0
    for prec in (FP64, FP32):
        genga.genga_kick(s.ctx.handle, s.b, DT, prec)
        genga.genga_step(s.ctx.handle, s.b, DT, 2, prec)
    genga.genga_drift(s.ctx.handle, s.b, DT)
    # the drift moved the (zero) bodies: the last kick's list is stale and is refused
    with pytest.raises(genga.GengaError) as ei:
        s.encounter_list()
    assert ei.value.status == genga.GENGA_ERR_STATE
    assert s.encounter_list(standalone=True)[1] == 0
    assert np.all(s.energy() == 0.0)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    s.close()


def test_deterministic_reruns():
    d = discs.disc_c1()
    s = System([d])
    a1, a2 = s.accel(FP32), s.accel(FP32)
    np.testing.assert_array_equal(a1, a2)
    genga.genga_step(s.ctx.handle, s.b, DT, 3, FP32)
    st1 = s.numpy_state()
    s2 = System([d])
    genga.genga_step(s2.ctx.handle, s2.b, DT, 3, FP32)
    st2 = s2.numpy_state()
    for k in st1:
        np.testing.assert_array_equal(st1[k], st2[k])
    s.close()
    s2.close()


def test_capacity_overflow_is_flagged():
    d = discs.make_disc(2000, 2.0, seed=58, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001,
                        n_embryo=40, embryo_mass_earth=0.05)
    s = System([d], pair_capacity=2)
    s.accel(FP64)
    pairs, cnt = s.encounter_list(cap=2)
    exp = oracle.encounters(d.state(), s.rc)
    assert cnt == len(exp) and cnt > 2 and len(pairs) == 2
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_ERR_CAPACITY
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK   # cleared
    s.close()


def test_nonfinite_is_flagged():
    d = _sizes_disc(300, 12)
    st = d.state()
    st["m"][7] = np.nan
    s = System([discs.Disc(**st)], rcrit=np.zeros(300))
    s.accel(FP32)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_ERR_NONFINITE
    s.close()


def test_graph_replays_match_eager():
    d = discs.make_disc(1200, 2.0, seed=59, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001,
                        n_embryo=10, embryo_mass_earth=0.05)
    torch = pytest.importorskip("torch")
    g = System([d])
    e = System([d])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        genga.genga_graph_capture(g.ctx.handle, g.b, DT, 2, FP32, stream=stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            genga.genga_graph_launch(g.ctx.handle, 1, stream=stream)
        stream.synchronize()
        genga.genga_step(e.ctx.handle, e.b, DT, 2, FP32)
        torch.cuda.synchronize()
        _ = torch.ones(10, device="cuda").sum().item()   # unrelated eager work between replays
        a, b = g.numpy_state(), e.numpy_state()
        for k in a:
            np.testing.assert_array_equal(a[k], b[k])
        print(f"[graph] replay {rep} identical to eager", flush=True)
    g.close()
    e.close()


def test_c3_full_size_all_rows():
    """N = 40000 disc in the benchmark's launch configuration (autotuned shape): every row of
    the FP64 kick, the FP32 kick with FP64 folding and with Kahan-compensated FP32 folding,
    against the oracle's full sum; the encounter list bit-exact; momentum balance."""
    d = discs.disc_c3()
    s = System([d])
    ref = np.stack(oracle.accel(d.state(), s.rc), axis=1)
    for prec, acc, bar in ((FP64, genga.GENGA_ACC_FP64, 1e-12), (FP32, genga.GENGA_ACC_FP64, 1e-5),
                           (FP32, genga.GENGA_ACC_KAHAN32, 1e-5)):
        genga.genga_autotune(s.ctx.handle, s.b, prec)
        ax, ay, az = s.zeros(), s.zeros(), s.zeros()
        genga.genga_accel(s.ctx.handle, s.b, ax, ay, az, prec, acc)
        s.torch.cuda.synchronize()
        a = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], axis=1)
        rms, mx = force_errors(a, ref)
        print(f"[c3 all rows] prec={prec} acc={acc} shape={genga.genga_get_kick_shape(s.ctx.handle, prec)} "
              f"rms={rms:.3e} max={mx:.3e}", flush=True)
        assert rms <= bar
        assert mx <= (1e-11 if prec == FP64 else 1e-3)
        if prec == FP32:
            p = (d.m[:, None] * a).sum(axis=0)
            assert np.max(np.abs(p)) <= 1e-6 * np.sum(d.m[:, None] * np.abs(a))
        got, cnt = s.encounter_list()
        exp = oracle.encounters(d.state(), s.rc)
        assert cnt == len(exp)
        np.testing.assert_array_equal(got, exp)
    s.close()


def _chain_disc(n_chain, n_field=300, spacing=0.45, rc0=2e-3, seed=61):
    """A field disc plus a chain of n_chain bodies spaced `spacing` r_crit apart, so that the
    chain forms one encounter group."""
    base = discs.make_disc(n_field, 2.5, seed=seed, a_in=0.7, a_out=1.0)
    st = base.state()
    rng = np.random.default_rng(seed)
    p0 = np.array([0.95, 0.1, 0.0])
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    vk = np.array([-p0[1], p0[0], 0.0]) / np.linalg.norm(p0) ** 1.5
    pts = p0 + np.outer(np.arange(n_chain) * spacing * rc0, u)
    vel = vk + rng.normal(scale=1e-3, size=(n_chain, 3))
    for q, k in enumerate(("x", "y", "z")):
        st[k] = np.concatenate([st[k], pts[:, q]])
        st["v" + k] = np.concatenate([st["v" + k], vel[:, q]])
    st["m"] = np.concatenate([st["m"], np.full(n_chain, 1e-9)])
    rc = np.concatenate([oracle.rcrit(base.state(), 1.0, 3.0, 0.0, DT), np.full(n_chain, rc0)])
    return discs.Disc(**st), rc


@pytest.mark.parametrize("n_chain", [5, 8, 9, 12, 40])
def test_drift_large_groups(n_chain):
    """Groups of up to 8 bodies take the column-parallel path, 9..64 the lane-per-member path;
    both must agree with the oracle's Bulirsch-Stoer to its tolerance."""
    d, rc = _chain_disc(n_chain)
    s = System([d], rcrit=rc)
    s.accel(FP64)
    pairs, cnt = s.encounter_list()
    gid = oracle.groups(d.n, pairs)
    big = np.bincount(gid[gid >= 0]).max()
    assert big >= n_chain
    exp = oracle.drift(d.state(), rc, 1.0, DT, pairs)
    genga.genga_drift(s.ctx.handle, s.b, DT)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    inside = gid >= 0
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        e_bs = np.max(np.abs(got[k][inside] - exp[k][inside]))
        print(f"[large group n={n_chain} (largest {big})] {k} BS err {e_bs:.2e}", flush=True)
        assert e_bs <= 1e-10
    s.close()


def test_group_over_capacity_is_flagged():
    d, rc = _chain_disc(70)
    s = System([d], rcrit=rc)
    s.accel(FP64)
    genga.genga_drift(s.ctx.handle, s.b, DT)
    s.torch.cuda.synchronize()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_ERR_CAPACITY
    st = s.numpy_state()
    assert all(np.all(np.isfinite(st[k])) for k in st)
    s.close()


@pytest.mark.parametrize("layout", ["random", "mixed_blocks"])
def test_accel_unequal_masses(layout):
    """Masses that differ from body to body, or only in some 64-source blocks, against the
    oracle (the discs elsewhere have equal planetesimal masses)."""
    d = _sizes_disc(1500, seed=71, a_in=0.7, a_out=1.0)
    st = d.state()
    rng = np.random.default_rng(71)
    if layout == "random":
        st["m"] = 10 ** rng.uniform(-10, -7, d.n)
    else:
        st["m"][:200] = 10 ** rng.uniform(-10, -7, 200)     # blocks 0..3 mixed, rest one mass
        st["m"][1000:1064] = 3e-8                          # a one-mass block of another mass
    dd = discs.Disc(**st)
    s = System([dd])
    ref = oracle_accel_systems(s)
    for prec, bar in ((FP64, 1e-12), (FP32, 1e-5)):
        for split in (1, 3):
            genga.genga_set_kick_shape(s.ctx.handle, prec, 8, split)
            rms, mx = force_errors(s.accel(prec), ref)
            print(f"[unequal masses {layout}] prec={prec} split={split} rms={rms:.3e} max={mx:.3e}", flush=True)
            assert rms <= bar
    s.close()
