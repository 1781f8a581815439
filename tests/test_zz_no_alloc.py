"""The allocation-free accelerations (genga_accel_noalloc) against genga_accel on the same
system: two calls in a row, the second with fewer bodies, for both kick precisions and both
accumulators; the encounter pairs as a set against the context's canonical list."""
import numpy as np
import pytest

import discs
import paper_2309_08217_amd as genga
from gpu_helpers import System, torch_mod

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32


def _disc(n, seed):
    # a cold annulus with embryos, so the encounter list is not empty
    return discs.make_disc(n, 2.0, seed=seed, a_in=0.7, a_out=1.0, sigma_e=0.001, sigma_i=0.001,
                           n_embryo=min(20, n // 50), embryo_mass_earth=0.05)


def _noalloc(sysm, prec, acc, pair_cap):
    torch = torch_mod()
    n = sysm.n
    ax, ay, az = sysm.zeros(), sysm.zeros(), sysm.zeros()
    pairs = torch.full((2 * max(pair_cap, 1),), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    genga.genga_accel_noalloc(sysm.b, n, ax, ay, az, pairs, pair_cap, cnt, status, prec, acc)
    torch.cuda.synchronize()
    a = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], axis=1)
    c = int(cnt.item())
    p = pairs[: 2 * min(c, pair_cap)].cpu().numpy().reshape(-1, 2)
    p = p[np.lexsort((p[:, 1], p[:, 0]))] if len(p) else p
    return a, p, c, int(status.item())


@pytest.mark.parametrize("prec,acc", [(FP64, genga.GENGA_ACC_FP64), (FP32, genga.GENGA_ACC_FP64),
                                      (FP32, genga.GENGA_ACC_KAHAN32)])
def test_noalloc_equals_accel_two_calls(prec, acc):
    for n, seed in ((5000, 71), (1300, 72)):  # the second call is smaller
        print(f"[noalloc] n={n} seed={seed} prec={prec} acc={acc}", flush=True)
        s = System([_disc(n, seed)])
        exp = np.zeros((n, 3))
        ax, ay, az = s.zeros(), s.zeros(), s.zeros()
        genga.genga_accel(s.ctx.handle, s.b, ax, ay, az, prec, acc)
        s.torch.cuda.synchronize()
        exp = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], axis=1)
        exp_pairs, exp_cnt = s.encounter_list()
        assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
        a, p, c, st = _noalloc(s, prec, acc, 16 * n)
        # same kernels, same launch shape: bit for bit
        np.testing.assert_array_equal(a, exp)
        assert st == 0
        assert c == exp_cnt and c > 0
        np.testing.assert_array_equal(p, exp_pairs)
        s.close()


def test_noalloc_small_pair_buffer_and_empty():
    s = System([_disc(2000, 73)])
    exp_pairs, exp_cnt = (None, None)
    genga.genga_accel(s.ctx.handle, s.b, s.zeros(), s.zeros(), s.zeros(), FP32)
    exp_pairs, exp_cnt = s.encounter_list()
    assert exp_cnt >= 2
    # a list that does not fit: the full count, bit 1 of the status
    a, p, c, st = _noalloc(s, FP32, genga.GENGA_ACC_FP64, 1)
    assert c == exp_cnt and st == 1
    assert len(p) == 1 and any((p[0] == q).all() for q in exp_pairs)
    # n = 0 clears both words and writes nothing
    torch = torch_mod()
    cnt = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    status = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    genga.genga_accel_noalloc(None, 0, None, None, None, None, 0, cnt, status, FP32)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0 and int(status.item()) == 0
    s.close()


def test_noalloc_refuses_more_bodies_than_its_scratch():
    torch = torch_mod()
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(genga.GengaError) as ei:
        genga.genga_accel_noalloc(None, genga.GENGA_NOALLOC_MAX_BODIES + 1, None, None, None, None, 0, cnt, cnt,
                                  FP32)
    assert ei.value.status == genga.GENGA_ERR_ARG
    assert "allocation-free" in genga.genga_last_error()
