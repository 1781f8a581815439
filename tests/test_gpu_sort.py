"""genga_sort_bodies: the bodies reordered in space on the device.  The order is free (the
paper fixes none), so the tests check what must hold for any order: a permutation that keeps
each system's massive and test bodies in their own runs, every per-body array moved with it bit
for bit, a second sort that changes nothing, neighbours in space close in the new order, and
steps after the sort that match the oracle run on the original order (mapped by the
permutation) to the same bars as without the sort."""
import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import System

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32
DT5 = discs.DT_5_DAYS
KEYS = ("x", "y", "z", "vx", "vy", "vz", "m")


def sort(s, stream=None):
    perm = s.torch.full((max(s.n, 1),), -1, dtype=s.torch.int32, device="cuda")
    genga.genga_sort_bodies(s.ctx.handle, s.b, perm, stream)
    s.torch.cuda.synchronize()
    return perm.cpu().numpy()[: s.n].astype(np.int64)


def runs(off, nm):
    """(start, end) of the massive and the test bodies of each system."""
    out = []
    for k in range(len(off) - 1):
        out += [(int(off[k]), int(off[k]) + int(nm[k])), (int(off[k]) + int(nm[k]), int(off[k + 1]))]
    return out


def test_permutation_keeps_runs_and_moves_every_array():
    """Two systems (2048 and 3000 bodies, the second with 600 test bodies at its end): the
    permutation maps each run onto itself, the arrays move bit for bit, and sorting again
    gives the identity."""
    ds = [discs.disc_c1(), discs.make_disc(3000, 2.5, seed=41, name="c1b")]
    s = System(ds)
    nm = np.array([ds[0].n, ds[1].n - 600], dtype=np.int32)
    genga.genga_set_test_bodies(s.ctx.handle, nm)
    before = s.numpy_state()
    rc0 = s.rc.copy()
    perm = sort(s)
    assert np.array_equal(np.sort(perm), np.arange(s.n))
    for a, b in runs(s.off, nm):
        assert np.all((perm[a:b] >= a) & (perm[a:b] < b)), (a, b)
    after = s.numpy_state()
    for k in KEYS:
        assert np.array_equal(after[k], before[k][perm]), k
    assert np.array_equal(s.b.rcrit.cpu().numpy(), rc0[perm])
    assert not np.array_equal(perm, np.arange(s.n))
    again = sort(s)
    assert np.array_equal(again, np.arange(s.n))
    s.close()


def test_neighbours_in_space_are_close_in_the_order():
    """On the 40000-body disc the mean distance between bodies adjacent in the order drops far
    below the random order's, and most bodies in one 64-body block lie within a few r_crit of
    each other."""
    d = discs.disc_c3()
    s = System([d])
    x0, y0 = d.x.copy(), d.y.copy()
    perm = sort(s)
    st = s.numpy_state()
    step_before = np.mean(np.hypot(np.diff(x0), np.diff(y0)))
    step_after = np.mean(np.hypot(np.diff(st["x"]), np.diff(st["y"])))
    print(f"[sort c3] mean consecutive distance {step_before:.3f} -> {step_after:.4f} au", flush=True)
    assert step_after < 0.05 * step_before
    # the extent of each 64-body block: far smaller than the disc
    nb = d.n // 64
    ext = [np.ptp(st["x"][64 * k:64 * (k + 1)]) + np.ptp(st["y"][64 * k:64 * (k + 1)]) for k in range(nb)]
    print(f"[sort c3] 64-body block extent median {np.median(ext):.3f} au", flush=True)
    assert np.median(ext) < 1.0
    assert np.array_equal(np.sort(perm), np.arange(d.n))
    s.close()


@pytest.mark.parametrize("prec,bar", [(FP64, 1e-11), (FP32, 1e-9)])
def test_steps_after_the_sort_match_the_oracle(prec, bar):
    """c1 (2048 bodies), sorted, then 4 steps: against the oracle's 4 steps from the original
    order, mapped by the permutation."""
    d = discs.disc_c1()
    s = System([d])
    perm = sort(s)
    genga.genga_step(s.ctx.handle, s.b, discs.DT_6_DAYS, 4, prec)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    exp, _ = oracle.step(d.state(), s.rc, d.mstar, discs.DT_6_DAYS, 4)  # s.rc: the original order
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        err = np.max(np.abs(got[k] - exp[k][perm]))
        print(f"[sorted step prec={prec}] {k} max err {err:.2e}", flush=True)
        assert err <= bar
    s.close()


def test_levels_and_collisions_follow_the_permutation():
    """The dense ring (300 bodies) with 2 levels x 2 sub-steps and collisions (radii about
    2e-3 au, all different): after the sort the level radii and the radius array follow the
    bodies, so 10 steps match the oracle's step_collide on the sorted inputs (the state, level
    radii and radii permuted on the host).  The merge rule keeps the lower index of a pair, so
    the survivor of a merger is a matter of the order: the comparison is in the new order."""
    d = discs.ring_dense(300)
    nlev, nsub = 2, 2
    rcl = oracle.rcrit_levels(d.state(), d.mstar, discs.DENSE_N1, discs.DENSE_N2, DT5, nlev, nsub)
    s = System([d], rcrit=rcl[0])
    torch = s.torch
    genga.genga_set_large_groups(s.ctx.handle, True)
    t = torch.tensor(np.ascontiguousarray(rcl[1:]), dtype=torch.float64, device="cuda")
    genga.genga_set_levels(s.ctx.handle, nlev, nsub, t)
    rad0 = 2e-3 * (1.0 + 0.25 * np.cos(np.arange(d.n)))  # distinct radii, so a wrong move shows
    rad = torch.tensor(rad0, dtype=torch.float64, device="cuda")
    status = torch.zeros(d.n, dtype=torch.int32, device="cuda")
    genga.genga_set_collisions(s.ctx.handle, s.b, rad, status, 0.0, 1e9)
    torch.cuda.synchronize()
    perm = sort(s)
    assert not np.array_equal(perm, np.arange(d.n))
    assert np.array_equal(rad.cpu().numpy(), rad0[perm])
    st = {k: np.ascontiguousarray(v[perm]) for k, v in d.state().items()}
    exp, erad, est = oracle.step_collide(st, np.ascontiguousarray(rcl[:, perm]), rad0[perm],
                                         np.zeros(d.n, np.int32), 1.0, DT5, 10, 0.0, 1e9, nsub=nsub)
    assert (est == 1).sum() >= 1
    genga.genga_step(s.ctx.handle, s.b, DT5, 10, FP64)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    got = s.numpy_state()
    print(f"[sorted levels+collisions] merged {int((est == 1).sum())}", flush=True)
    assert np.array_equal(status.cpu().numpy(), est)
    assert np.array_equal(got["m"], exp["m"])
    assert np.allclose(rad.cpu().numpy(), erad, rtol=4e-16, atol=0)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        err = np.max(np.abs(got[k] - exp[k]))
        print(f"[sorted levels+collisions] {k} max err {err:.2e}", flush=True)
        assert err <= 1e-10
    s.close()


def test_the_context_list_is_refused_after_a_sort():
    """The last kick's list names bodies by their old places: asking for it after a sort is a
    state error, and a standalone list on the new order equals the oracle's."""
    d = discs.disc_c1()
    s = System([d])
    s.accel(FP64)
    perm = sort(s)
    torch = s.torch
    pairs = torch.zeros(2 * 1024, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(genga.GengaError) as e:
        genga.genga_encounter_list(s.ctx.handle, None, pairs, 1024, cnt)
    assert e.value.status == genga.GENGA_ERR_STATE
    got, c = s.encounter_list(standalone=True)
    st = s.numpy_state()
    exp = oracle.encounters(st, s.b.rcrit.cpu().numpy())
    assert c == len(exp)
    assert np.array_equal(np.unique(got, axis=0), np.unique(np.asarray(exp).reshape(-1, 2), axis=0))
    assert np.array_equal(np.sort(perm), np.arange(d.n))
    s.close()


def test_empty_system_and_stream():
    """A layout with no bodies sorts to nothing; on a caller stream the sort is ordered before
    the following step."""
    s0 = System([discs.Disc(*(np.zeros(0) for _ in range(7)), name="empty")])
    genga.genga_sort_bodies(s0.ctx.handle, s0.b, None)
    s0.close()
    d = discs.disc_c1()
    s = System([d])
    torch = s.torch
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        perm = torch.zeros(d.n, dtype=torch.int32, device="cuda")
        genga.genga_sort_bodies(s.ctx.handle, s.b, perm, st)
        genga.genga_step(s.ctx.handle, s.b, discs.DT_6_DAYS, 2, FP64, stream=st)
    torch.cuda.synchronize()
    p = perm.cpu().numpy().astype(np.int64)
    exp, _ = oracle.step(d.state(), s.rc, d.mstar, discs.DT_6_DAYS, 2)
    got = s.numpy_state()
    for k in ("x", "vx"):
        assert np.max(np.abs(got[k] - exp[k][p])) <= 1e-11
    s.close()


def test_capture_is_refused():
    """Under graph capture the sort refuses (its radix sort would record memset nodes) and
    enqueues nothing: the bodies are unchanged."""
    d = discs.disc_c1()
    s = System([d])
    torch = s.torch
    before = s.numpy_state()
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    dummy = torch.zeros(4, device="cuda")
    err = None
    with torch.cuda.graph(g, stream=st):
        dummy += 1.0
        try:
            genga.genga_sort_bodies(s.ctx.handle, s.b, None, st)
        except genga.GengaError as e:
            err = e
    torch.cuda.synchronize()
    assert err is not None and err.status == genga.GENGA_ERR_STATE
    after = s.numpy_state()
    for k in KEYS:
        assert np.array_equal(after[k], before[k])
    s.close()


def test_empty_runs_between_systems():
    """Three systems, the middle one empty and the last with 100 test bodies at its end: every
    run (massive or test, empty ones included) maps onto itself and the arrays move with it,
    so the search for a position's run passes over the empty runs."""
    empty = discs.Disc(*(np.zeros(0) for _ in range(7)), name="empty")
    ds = [discs.make_disc(700, 2.5, seed=51, name="a"), empty, discs.make_disc(500, 2.5, seed=52, name="b")]
    s = System(ds)
    nm = np.array([700, 0, 400], dtype=np.int32)
    genga.genga_set_test_bodies(s.ctx.handle, nm)
    before = s.numpy_state()
    perm = sort(s)
    assert np.array_equal(np.sort(perm), np.arange(s.n))
    for a_, b_ in runs(s.off, nm):
        assert np.all((perm[a_:b_] >= a_) & (perm[a_:b_] < b_)), (a_, b_)
    after = s.numpy_state()
    for k in KEYS:
        assert np.array_equal(after[k], before[k][perm]), k
    assert not np.array_equal(perm, np.arange(s.n))
    s.close()
