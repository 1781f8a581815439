"""The boundary's selectors and pair-list hand-offs through the C ABI (the level-0 kick and
drift of Sect. 1; FP32 forces as the "Do Kick in single precision" switch of Sect. 4):

- the accumulator selector of the FP32 kick (FP64 folding or Kahan-compensated FP32) against
  the oracle, and what the compensation changes;
- the encounter list of a state computed on its own, and the refusal to hand out a list that
  no longer belongs to the positions;
- the drift with a pair list the caller supplies (the oracle's), an invalid list, and a list
  in another order;
- the autotune cache file; graph replays that record the energy cadence; the stream-scoped
  status poll.
"""
import os

import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import DT, System, force_errors, oracle_accel_systems

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32
ACC64, KAHAN = genga.GENGA_ACC_FP64, genga.GENGA_ACC_KAHAN32


def _cold(n, seed, n_emb=20):
    return discs.make_disc(n, 2.0, seed=seed, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001,
                           n_embryo=n_emb, embryo_mass_earth=0.05)


def _accel(s, prec, acc):
    ax, ay, az = s.zeros(), s.zeros(), s.zeros()
    genga.genga_accel(s.ctx.handle, s.b, ax, ay, az, prec, acc)
    s.torch.cuda.synchronize()
    return np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], axis=1)


@pytest.mark.parametrize("n", [5, 64, 65, 1000, 2049])
def test_kahan_accumulator_against_oracle(n):
    d = discs.make_disc(n, 2.5, seed=500 + n, a_in=0.7, a_out=1.0)
    s = System([d])
    ref = oracle_accel_systems(s)
    for split in (1, 3):
        genga.genga_set_kick_shape(s.ctx.handle, FP32, 8, split)
        a64 = _accel(s, FP32, ACC64)
        ak = _accel(s, FP32, KAHAN)
        r64, m64 = force_errors(a64, ref)
        rk, mk = force_errors(ak, ref)
        # the two folds differ only by the rounding of the cross-block sum, far below the
        # FP32 pair terms' own error
        dk, _ = force_errors(ak, a64)
        print(f"[kahan n={n} split={split}] rms fp64-fold={r64:.3e} kahan={rk:.3e} max {m64:.3e}/{mk:.3e} "
              f"kahan-vs-fp64fold={dk:.3e}", flush=True)
        assert rk <= 1e-5 and r64 <= 1e-5
        assert dk <= 1e-6
        np.testing.assert_array_equal(ak, _accel(s, FP32, KAHAN))   # deterministic
    s.close()


def test_kahan_steps_against_oracle():
    d = _cold(1500, 57)
    s = System([d])
    genga.genga_step(s.ctx.handle, s.b, DT, 3, FP32, KAHAN)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    got = s.numpy_state()
    exp, _ = oracle.step(d.state(), s.rc, 1.0, DT, 3)
    err = max(np.max(np.abs(got[k] - exp[k])) for k in ("x", "y", "z"))
    print(f"[kahan steps] max position err {err:.2e}", flush=True)
    assert err <= 1e-7
    s.close()


def test_standalone_encounter_list():
    """After a drift the last kick's list is stale: b = NULL is refused; with the bodies the
    list of the new positions is computed on its own and equals the oracle's, and it is the
    list that the next drift uses."""
    d = _cold(3000, 55, 40)
    s = System([d])
    torch = s.torch
    cap = 16 * d.n
    pairs = torch.zeros(2 * cap, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(genga.GengaError) as e:      # no kick has run yet
        genga.genga_encounter_list(s.ctx.handle, None, pairs, cap, cnt)
    assert e.value.status == genga.GENGA_ERR_STATE
    s.accel(FP32)
    got, c0 = s.encounter_list()
    np.testing.assert_array_equal(got, oracle.encounters(d.state(), s.rc))
    genga.genga_drift(s.ctx.handle, s.b, DT)
    with pytest.raises(genga.GengaError) as e:
        genga.genga_encounter_list(s.ctx.handle, None, pairs, cap, cnt)
    assert e.value.status == genga.GENGA_ERR_STATE
    genga.genga_encounter_list(s.ctx.handle, s.b, pairs, cap, cnt)
    torch.cuda.synchronize()
    c1 = int(cnt.item())
    st = s.numpy_state()
    exp = oracle.encounters(st, s.rc)
    print(f"[standalone list] pairs before {c0}, after the drift {c1} (oracle {len(exp)})", flush=True)
    assert c1 == len(exp) and c1 > 10
    np.testing.assert_array_equal(pairs[: 2 * c1].cpu().numpy().reshape(-1, 2), exp)
    # now valid for these positions: b = NULL hands out the same list
    got2, c2 = s.encounter_list()
    np.testing.assert_array_equal(got2, exp)
    # the next drift integrates the groups of this list, as the oracle's drift with it does
    genga.genga_drift(s.ctx.handle, s.b, DT)
    got = s.numpy_state()
    ref = oracle.drift(st, s.rc, 1.0, DT, exp)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    err = max(np.max(np.abs(got[k] - ref[k])) for k in ("x", "y", "z", "vx", "vy", "vz"))
    print(f"[standalone list] drift err {err:.2e}", flush=True)
    assert err <= 1e-10
    s.close()


def test_standalone_list_tp2():
    """TP2: test bodies (after the first 500) meet massive bodies only, in the standalone
    list as in the kick's."""
    d = _cold(2000, 58, 20)
    s = System([d])
    genga.genga_set_test_bodies(s.ctx.handle, [500])
    cap = 16 * d.n
    pairs = s.torch.zeros(2 * cap, dtype=s.torch.int32, device="cuda")
    cnt = s.torch.zeros(1, dtype=s.torch.int32, device="cuda")
    genga.genga_encounter_list(s.ctx.handle, s.b, pairs, cap, cnt)
    s.torch.cuda.synchronize()
    c = int(cnt.item())
    exp = oracle.encounters(d.state(), s.rc, n_massive=500)
    assert c == len(exp)
    np.testing.assert_array_equal(pairs[: 2 * c].cpu().numpy().reshape(-1, 2), exp)
    s.accel(FP32)
    np.testing.assert_array_equal(s.encounter_list()[0], exp)
    s.close()


def _device_pairs(torch, p):
    t = torch.as_tensor(np.ascontiguousarray(p, dtype=np.int32).reshape(-1), device="cuda")
    c = torch.tensor([len(p)], dtype=torch.int32, device="cuda")
    return t, c


def test_drift_with_caller_pair_list():
    """The oracle's list handed to genga_drift gives the same state, bit for bit, as the
    context's own list (from the kick on the same positions), in any order of the pairs."""
    d = _cold(2000, 56, 40)
    a, b = System([d]), System([d])
    torch = a.torch
    a.accel(FP64)
    exp_pairs = oracle.encounters(d.state(), a.rc)
    assert len(exp_pairs) > 5
    genga.genga_drift(a.ctx.handle, a.b, DT)
    rev = exp_pairs[::-1].copy()
    p, c = _device_pairs(torch, rev)
    genga.genga_drift(b.ctx.handle, b.b, DT, p, c)
    assert genga.genga_poll_status(b.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    ga, gb = a.numpy_state(), b.numpy_state()
    for k in ga:
        np.testing.assert_array_equal(ga[k], gb[k])
    a.close()
    b.close()


@pytest.mark.parametrize("bad", ["index_out_of_range", "i_not_below_j", "negative_count", "two_systems"])
def test_drift_refuses_an_invalid_pair_list(bad):
    d1, d2 = _cold(300, 61, 0), _cold(200, 62, 0)
    s = System([d1, d2])
    torch = s.torch
    s.accel(FP64)
    good = oracle.encounters(d1.state(), s.rc[:300])
    p = np.concatenate([good, [[1, 2]]]).astype(np.int32)
    cnt = len(p)
    if bad == "index_out_of_range":
        p[-1] = [3, 10 ** 6]
    elif bad == "i_not_below_j":
        p[-1] = [7, 7]
    elif bad == "two_systems":
        p[-1] = [5, 300 + 4]
    t, c = _device_pairs(torch, p)
    if bad == "negative_count":
        c.fill_(-3)
    before = s.numpy_state()
    genga.genga_drift(s.ctx.handle, s.b, DT, t, c)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_ERR_ARG
    got = s.numpy_state()
    # the list was dropped: every body was Kepler-drifted, as with an empty list
    ref = {k: np.concatenate([oracle.drift({q: before[q][:300] for q in before}, s.rc[:300], 1.0, DT,
                                           np.zeros((0, 2), np.int32))[k],
                              oracle.drift({q: before[q][300:] for q in before}, s.rc[300:], 1.0, DT,
                                           np.zeros((0, 2), np.int32))[k]]) for k in ("x", "vx")}
    for k in ("x", "vx"):
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-13
    assert cnt > 0
    s.close()


def test_autotune_cache(tmp_path):
    d = discs.disc_c1()
    s = System([d])
    path = str(tmp_path / "tune.txt")
    genga.genga_autotune(s.ctx.handle, s.b, FP32, path)
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("genga-autotune v1 ")
    shape = genga.genga_get_kick_shape(s.ctx.handle, FP32)
    assert lines[0].split()[-2:] == [str(shape[0]), str(shape[1])]
    # a second context with the same layout takes the cached shape without timing
    t = System([d])
    genga.genga_set_kick_shape(t.ctx.handle, FP32, 4 if shape[0] != 4 else 8, 1)
    genga.genga_autotune(t.ctx.handle, t.b, FP32, path)
    assert genga.genga_get_kick_shape(t.ctx.handle, FP32) == shape
    assert open(path).read().splitlines() == lines
    # another precision or layout is a miss: timed and appended
    genga.genga_autotune(t.ctx.handle, t.b, FP64, path)
    assert len(open(path).read().splitlines()) == 2
    with pytest.raises(genga.GengaError) as e:
        genga.genga_autotune(t.ctx.handle, t.b, FP32, str(tmp_path))     # a directory
    assert e.value.status == genga.GENGA_ERR_ARG
    s.close()
    t.close()


def test_graph_records_the_energy_cadence():
    """A captured graph of 20 steps with the energy every 10 steps: each replay writes the same
    records as 20 eager steps, bit for bit, with eager work between the replays."""
    torch = pytest.importorskip("torch")
    d = _cold(1200, 59, 10)
    g, e = System([d]), System([d])
    stream = torch.cuda.Stream()
    rec_g = torch.zeros(2 * 4, dtype=torch.float64, device="cuda")
    rec_e = torch.zeros(2 * 4, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        genga.genga_graph_capture(g.ctx.handle, g.b, DT, 20, FP32, KAHAN, energy_cadence=10, d_energy=rec_g,
                                  stream=stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            genga.genga_graph_launch(g.ctx.handle, 1, stream=stream)
        stream.synchronize()
        genga.genga_step(e.ctx.handle, e.b, DT, 20, FP32, KAHAN, energy_cadence=10, d_energy=rec_e)
        torch.cuda.synchronize()
        _ = torch.ones(10, device="cuda").sum().item()
        np.testing.assert_array_equal(rec_g.cpu().numpy(), rec_e.cpu().numpy())
        a, b = g.numpy_state(), e.numpy_state()
        for k in a:
            np.testing.assert_array_equal(a[k], b[k])
        assert np.all(rec_g.cpu().numpy()[[0, 4]] < 0)
    assert genga.genga_poll_status(g.ctx.handle) == genga.GENGA_OK
    g.close()
    e.close()


def test_poll_status_on_the_call_stream():
    torch = pytest.importorskip("torch")
    d = discs.make_disc(300, 2.5, seed=12)
    st = d.state()
    st["m"][7] = np.nan
    s = System([discs.Disc(**st)], rcrit=np.zeros(300))
    stream = torch.cuda.Stream()
    ax, ay, az = s.zeros(), s.zeros(), s.zeros()
    with torch.cuda.stream(stream):
        genga.genga_accel(s.ctx.handle, s.b, ax, ay, az, FP32, stream=stream)
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_ERR_NONFINITE
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK
    s.close()
