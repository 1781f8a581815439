"""Collisions as perfect mergers and removal by distance (Sect. 2) on the GPU against the
oracle's step_collide, and the compaction of the arrays afterwards.  The ring's radii are
inflated (2e-3 au) so that a few tens of steps see several mergers."""
import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import System

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32
DT5 = discs.DT_5_DAYS
R = 2e-3


def collide_system(d, r_min, r_max):
    rc = oracle.rcrit(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5)
    s = System([d], rcrit=rc)
    genga.genga_set_large_groups(s.ctx.handle, True)
    torch = s.torch
    rad = torch.full((d.n,), R, dtype=torch.float64, device="cuda")
    status = torch.zeros(d.n, dtype=torch.int32, device="cuda")
    genga.genga_set_collisions(s.ctx.handle, s.b, rad, status, r_min, r_max)
    return s, rc, rad, status


def check_against_oracle(label, s, rad, status, exp, erad, est, bar, n=None):
    got = s.numpy_state()
    n = len(est) if n is None else n
    gst = status.cpu().numpy()[:n]
    print(f"[{label}] merged {int((est == 1).sum())} removed {int((est == 2).sum())}", flush=True)
    assert np.array_equal(gst, est)
    assert np.array_equal(got["m"][:n], exp["m"])
    assert np.allclose(rad.cpu().numpy()[:n], erad, rtol=4e-16, atol=0)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        err = np.max(np.abs(got[k][:n] - exp[k]))
        print(f"[{label}] {k} max err {err:.2e}", flush=True)
        assert err <= bar


@pytest.mark.parametrize("prec,bar", [(FP64, 1e-10), (FP32, 1e-8)])
def test_mergers_against_oracle(prec, bar):
    d = discs.ring_dense(300)
    s, rc, rad, status = collide_system(d, 0.0, 1e9)
    exp, erad, est = oracle.step_collide(d.state(), rc, np.full(d.n, R), np.zeros(d.n, np.int32), 1.0, DT5, 20,
                                         0.0, 1e9)
    assert (est == 1).sum() >= 3
    genga.genga_step(s.ctx.handle, s.b, DT5, 20, prec)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    check_against_oracle(f"mergers prec={prec}", s, rad, status, exp, erad, est, bar)
    s.close()


def test_removal_compaction_and_more_steps():
    """Removal inside 0.82 au and beyond 0.88 au together with mergers over 10 steps; then the
    arrays are compacted and 5 more steps run on the survivors, against the oracle."""
    d = discs.ring_dense(300)
    s, rc, rad, status = collide_system(d, 0.82, 0.88)
    exp, erad, est = oracle.step_collide(d.state(), rc, np.full(d.n, R), np.zeros(d.n, np.int32), 1.0, DT5, 10,
                                         0.82, 0.88)
    assert (est == 2).sum() >= 1
    genga.genga_step(s.ctx.handle, s.b, DT5, 10, FP64)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    check_against_oracle("removal", s, rad, status, exp, erad, est, 1e-10)
    before = s.numpy_state()
    keep = est == 0
    n_new = genga.genga_compact(s.ctx.handle, s.b, rad, status)
    assert n_new == int(keep.sum())
    after = s.numpy_state()
    for k in ("x", "y", "z", "vx", "vy", "vz", "m"):
        assert np.array_equal(after[k][:n_new], before[k][keep])
    assert np.array_equal(s.b.rcrit.cpu().numpy()[:n_new], rc[keep])
    assert np.all(status.cpu().numpy()[:n_new] == 0)
    # five more steps on the survivors
    st2 = {k: exp[k][keep] for k in exp}
    exp2, erad2, est2 = oracle.step_collide(st2, rc[keep], erad[keep], np.zeros(n_new, np.int32), 1.0, DT5, 5,
                                            0.82, 0.88)
    genga.genga_step(s.ctx.handle, s.b, DT5, 5, FP64)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    check_against_oracle("after compaction", s, rad, status, exp2, erad2, est2, 1e-10, n=n_new)
    s.close()


def test_collision_argument_checks():
    d = discs.ring_dense(300)
    s, rc, rad, status = collide_system(d, 0.0, 1e9)
    torch = s.torch
    with pytest.raises(genga.GengaError) as e:
        genga.genga_set_collisions(s.ctx.handle, s.b, rad, status, 1.0, 0.5)
    assert e.value.status == genga.GENGA_ERR_ARG
    other = genga.Bodies.from_numpy(d.state(), rc)
    genga.genga_set_collisions(s.ctx.handle, other, rad, status, 0.0, 1e9)
    s.accel(FP64)
    with pytest.raises(genga.GengaError) as e:       # the bodies' m is not the collision mass array
        genga.genga_drift(s.ctx.handle, s.b, DT5)
    assert e.value.status == genga.GENGA_ERR_ARG
    genga.genga_set_collisions(s.ctx.handle, None, None, None, 0.0, 0.0)
    genga.genga_drift(s.ctx.handle, s.b, DT5)          # off again: a plain drift
    torch.cuda.synchronize()
    s.close()


def test_mergers_with_test_bodies():
    """TP2 mode: the last 100 of 300 ring bodies are massless test bodies (no mutual forces or
    encounters); a test body that hits a massive one merges into it with weight zero."""
    d = discs.ring_dense(300)
    nm = 200
    s, rc, rad, status = collide_system(d, 0.0, 1e9)
    genga.genga_set_test_bodies(s.ctx.handle, np.array([nm], dtype=np.int32))
    st = d.state()
    st["m"] = st["m"].copy()
    st["m"][nm:] = 0.0
    s.b.m.copy_(s.torch.tensor(st["m"], dtype=s.torch.float64, device="cuda"))
    exp, erad, est = oracle.step_collide(st, rc, np.full(d.n, R), np.zeros(d.n, np.int32), 1.0, DT5, 20, 0.0, 1e9,
                                         n_massive=nm)
    genga.genga_step(s.ctx.handle, s.b, DT5, 20, FP64)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    check_against_oracle("mergers TP2", s, rad, status, exp, erad, est, 1e-10)
    s.close()


def test_mergers_with_levels():
    """Collisions with the hierarchical step (2 levels x 2 sub-steps): 10 FP64 steps of the
    ring with inflated radii against the oracle's step_collide over the same levels."""
    d = discs.ring_dense(300)
    rcl = oracle.rcrit_levels(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5, 2, 2)
    s = System([d], rcrit=rcl[0])
    genga.genga_set_large_groups(s.ctx.handle, True)
    torch = s.torch
    t = torch.tensor(np.ascontiguousarray(rcl[1:]), dtype=torch.float64, device="cuda")
    genga.genga_set_levels(s.ctx.handle, 2, 2, t)
    rad = torch.full((d.n,), R, dtype=torch.float64, device="cuda")
    status = torch.zeros(d.n, dtype=torch.int32, device="cuda")
    genga.genga_set_collisions(s.ctx.handle, s.b, rad, status, 0.0, 1e9)
    exp, erad, est = oracle.step_collide(d.state(), rcl, np.full(d.n, R), np.zeros(d.n, np.int32), 1.0, DT5, 10,
                                         0.0, 1e9, nsub=2)
    assert (est == 1).sum() >= 1
    genga.genga_step(s.ctx.handle, s.b, DT5, 10, FP64)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    check_against_oracle("mergers with levels", s, rad, status, exp, erad, est, 1e-10)
    s.close()


def test_collisions_in_a_batch_then_compaction():
    """Two rings in one batch with mergers and removal inside 0.82 au / beyond 0.88 au over
    10 steps, each system against the oracle's step_collide of that system alone; then the
    compaction keeps every system's survivors in order."""
    ds = [discs.ring_dense(300, seed=41), discs.ring_dense(400, seed=42)]
    rcs = [oracle.rcrit(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5) for d in ds]
    s = System(ds, rcrit=np.concatenate(rcs))
    genga.genga_set_large_groups(s.ctx.handle, True)
    torch = s.torch
    rad = torch.full((s.n,), R, dtype=torch.float64, device="cuda")
    status = torch.zeros(s.n, dtype=torch.int32, device="cuda")
    genga.genga_set_collisions(s.ctx.handle, s.b, rad, status, 0.82, 0.88)
    genga.genga_step(s.ctx.handle, s.b, DT5, 10, FP64)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    got = s.numpy_state()
    gst, grad = status.cpu().numpy(), rad.cpu().numpy()
    keep = []
    for k, d in enumerate(ds):
        sl = s.system_slice(k)
        exp, erad, est = oracle.step_collide(d.state(), rcs[k], np.full(d.n, R), np.zeros(d.n, np.int32), 1.0, DT5,
                                             10, 0.82, 0.88)
        print(f"[batch {k}] merged {int((est == 1).sum())} removed {int((est == 2).sum())}", flush=True)
        assert np.array_equal(gst[sl], est)
        assert np.array_equal(got["m"][sl], exp["m"])
        assert np.allclose(grad[sl], erad, rtol=4e-16, atol=0)
        for key in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.max(np.abs(got[key][sl] - exp[key])) <= 1e-10
        keep.append(est == 0)
    keep = np.concatenate(keep)
    assert (~keep).sum() >= 2
    n_new = genga.genga_compact(s.ctx.handle, s.b, rad, status)
    assert n_new == int(keep.sum())
    after = s.numpy_state()
    for key in ("x", "y", "z", "vx", "vy", "vz", "m"):
        assert np.array_equal(after[key][:n_new], got[key][keep])
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP64)   # the compacted batch steps on
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    s.close()


def test_collisions_in_graph_replays_match_eager():
    """Collisions on the plain path (r_crit of 3 Hill radii, groups of a few bodies) inside a
    captured two-step HIP graph: three replays, with eager work between them, equal eager
    steps bit for bit, radii and status included."""
    d = discs.ring_dense(300)
    rc = oracle.rcrit(d.state(), d.mstar, 3.0, 0.0, DT5)
    torch = pytest.importorskip("torch")
    sides = []
    for _ in range(2):
        s = System([d], rcrit=rc)
        rad = torch.full((d.n,), R, dtype=torch.float64, device="cuda")
        status = torch.zeros(d.n, dtype=torch.int32, device="cuda")
        genga.genga_set_collisions(s.ctx.handle, s.b, rad, status, 0.0, 1e9)
        sides.append((s, rad, status))
    (g, grad, gst), (e, erad, est) = sides
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        genga.genga_graph_capture(g.ctx.handle, g.b, DT5, 2, FP64, stream=stream)
    merged = 0
    for rep in range(3):
        with torch.cuda.stream(stream):
            genga.genga_graph_launch(g.ctx.handle, 1, stream=stream)
        stream.synchronize()
        genga.genga_step(e.ctx.handle, e.b, DT5, 2, FP64)
        torch.cuda.synchronize()
        _ = torch.ones(10, device="cuda").sum().item()   # unrelated eager work between replays
        a, b = g.numpy_state(), e.numpy_state()
        for k in a:
            np.testing.assert_array_equal(a[k], b[k])
        np.testing.assert_array_equal(gst.cpu().numpy(), est.cpu().numpy())
        np.testing.assert_array_equal(grad.cpu().numpy(), erad.cpu().numpy())
        merged = int((est.cpu().numpy() == 1).sum())
        print(f"[graph collisions] replay {rep} identical to eager, merged so far {merged}", flush=True)
    assert genga.genga_poll_status(g.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    assert merged >= 1
    # collisions cannot be switched off under a graph that holds their launches
    with pytest.raises(genga.GengaError) as err:
        genga.genga_set_collisions(g.ctx.handle, None, None, None, 0.0, 0.0)
    assert err.value.status == genga.GENGA_ERR_STATE
    with torch.cuda.stream(stream):
        genga.genga_graph_launch(g.ctx.handle, 1, stream=stream)     # the graph still runs
    stream.synchronize()
    assert genga.genga_poll_status(g.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    g.close()
    e.close()


def test_physical_radius_mergers_and_dead_bodies():
    """Radii of 500 km (3.3e-6 au, the paper's planetesimal sizes) on the ring, with three
    pairs planted on colliding paths (impact parameter 4e-6 au < R_i + R_j, relative speed
    0.05 above the mutual escape speed): 10 FP64 steps against the oracle's step_collide, the
    three mergers happen, and afterwards no absorbed body is in an encounter pair (it moves on
    as a massless particle, outside every Bulirsch-Stoer group)."""
    d0 = discs.ring_dense(300)
    st = d0.state()
    rng = np.random.default_rng(77)
    rad0 = 500.0 / 1.495978707e8
    for k, j in ((0, 250), (1, 251), (2, 252)):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        w = np.cross(u, rng.normal(size=3))
        w /= np.linalg.norm(w)
        pos = np.array([st["x"][k], st["y"][k], st["z"][k]]) + 2e-5 * u + 4e-6 * w
        vel = np.array([st["vx"][k], st["vy"][k], st["vz"][k]]) - 0.05 * u
        for q, key in enumerate(("x", "y", "z")):
            st[key][j] = pos[q]
            st["v" + key][j] = vel[q]
    d = discs.Disc(**st)
    rc = oracle.rcrit(st, d.mstar, 3.0, 0.0, DT5)
    s = System([d], rcrit=rc)
    torch = s.torch
    rad = torch.full((d.n,), rad0, dtype=torch.float64, device="cuda")
    status = torch.zeros(d.n, dtype=torch.int32, device="cuda")
    genga.genga_set_collisions(s.ctx.handle, s.b, rad, status, 0.0, 1e9)
    exp, erad, est = oracle.step_collide(st, rc, np.full(d.n, rad0), np.zeros(d.n, np.int32), 1.0, DT5, 10, 0.0, 1e9)
    assert (est[250:253] == 1).all() or (est[:3] == 1).all()
    genga.genga_step(s.ctx.handle, s.b, DT5, 10, FP64)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    check_against_oracle("physical radius", s, rad, status, exp, erad, est, 1e-10)
    dead = np.flatnonzero(status.cpu().numpy() != 0)
    pairs, cnt = s.encounter_list()
    assert len(dead) >= 3 and not np.isin(pairs, dead).any()
    s.close()


def _cluster_ring(n_clusters=600, m=1e-9):
    """Clusters of 4 bodies on a circular ring at 1 au, each cluster moving with one velocity
    (radii 1e-3 au, inside r_crit = 2.1e-3 au): even clusters are stars (every pair closer than
    R_i + R_j), odd clusters chains with only neighbours touching.  In a star the first body absorbs the three others; in a chain
    (0,1) merges, (1,2) is skipped (1 was absorbed), (2,3) merges."""
    x, y, z, vx, vy, vz = ([] for _ in range(6))
    for k in range(n_clusters):
        th = 2 * np.pi * k / n_clusters
        c = np.array([np.cos(th), np.sin(th), 0.0])
        t = np.array([-np.sin(th), np.cos(th), 0.0])
        v = t * np.sqrt(1.0 / 1.0)
        if k % 2 == 0:
            offs = [np.zeros(3), 1e-3 * c, 1e-3 * t, 1e-3 * np.array([0.0, 0.0, 1.0])]
        else:
            offs = [q * 1.5e-3 * t for q in range(4)]
        for o in offs:
            p = c + o
            x.append(p[0]); y.append(p[1]); z.append(p[2])
            vx.append(v[0]); vy.append(v[1]); vz.append(v[2])
    n = len(x)
    return discs.Disc(np.array(x), np.array(y), np.array(z), np.array(vx), np.array(vy), np.array(vz),
                      np.full(n, m))


def test_many_mergers_in_one_drift():
    """About 2700 colliding pairs in the first drift (stars and chains of 4): the merges follow
    the ascending (i, j) order with already-absorbed bodies skipped, as the oracle's, over two
    FP64 steps."""
    d = _cluster_ring()
    st = d.state()
    rc = oracle.rcrit(st, d.mstar, 3.0, 0.0, DT5)
    rad0 = 1e-3
    s = System([d], rcrit=rc)
    torch = s.torch
    rad = torch.full((d.n,), rad0, dtype=torch.float64, device="cuda")
    status = torch.zeros(d.n, dtype=torch.int32, device="cuda")
    genga.genga_set_collisions(s.ctx.handle, s.b, rad, status, 0.0, 1e9)
    exp, erad, est = oracle.step_collide(st, rc, np.full(d.n, rad0), np.zeros(d.n, np.int32), 1.0, DT5, 2, 0.0, 1e9)
    stars = np.arange(0, d.n, 8)
    assert (est[stars] == 0).all() and (est[stars + 1] == 1).all() and (est[stars + 3] == 1).all()
    chains = np.arange(4, d.n, 8)
    assert (est[chains] == 0).all() and (est[chains + 1] == 1).all() and (est[chains + 2] == 0).all()
    assert (est[chains + 3] == 1).all()
    genga.genga_step(s.ctx.handle, s.b, DT5, 2, FP64)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    check_against_oracle("many mergers", s, rad, status, exp, erad, est, 1e-10)
    s.close()
