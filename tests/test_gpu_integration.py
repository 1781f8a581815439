"""Workload-sized runs on the GPU: energy and angular-momentum drift of the FP32 and FP64
kicks over many steps, encounter lists on the dense mixed disc step by step, and the batched
64-disc layout on sampled rows.  The oracle checks the GPU state it is fed at checkpoints.
"""
import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import DT, System, force_errors

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32


def run_series(sysm, prec, nsteps, cadence):
    torch = sysm.torch
    nsys = len(sysm.discs)
    e0 = sysm.energy()
    rec = torch.zeros((nsteps // cadence) * 4 * nsys, dtype=torch.float64, device="cuda")
    genga.genga_step(sysm.ctx.handle, sysm.b, DT, nsteps, prec, cadence, rec)
    torch.cuda.synchronize()
    assert genga.genga_poll_status(sysm.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    r = rec.cpu().numpy().reshape(-1, nsys, 4)
    dE = r[:, :, 0] / e0[None, :, 0] - 1.0
    dL = np.linalg.norm(r[:, :, 1:], axis=2) / np.linalg.norm(e0[:, 1:], axis=1)[None, :] - 1.0
    return dE, dL


def test_c2_energy_drift_fp32_within_twice_fp64():
    """N = 6600 disc, 1000 steps: max |dE/E| of the FP32 kick within 2x that of the FP64 kick;
    FP64 keeps |L| to round-off."""
    d = discs.disc_c2()
    out = {}
    for prec in (FP64, FP32):
        s = System([d])
        out[prec] = run_series(s, prec, 1000, 10)
        # the energy the GPU reports for its final state equals the oracle's for that state
        st = s.numpy_state()
        e_gpu = s.energy()[0]
        e_or = oracle.energy(st, 1.0)
        assert abs(e_gpu[0] - e_or[0]) <= 1e-12 * abs(e_or[0])
        s.close()
    m64 = np.max(np.abs(out[FP64][0]))
    m32 = np.max(np.abs(out[FP32][0]))
    l64 = np.max(np.abs(out[FP64][1]))
    l32 = np.max(np.abs(out[FP32][1]))
    print(f"[c2 1000 steps] max|dE/E| fp64={m64:.3e} fp32={m32:.3e}  max|dL/L| fp64={l64:.3e} fp32={l32:.3e}",
          flush=True)
    assert m32 <= 2.0 * m64
    assert l64 <= 1e-12


def test_c5_encounter_lists_step_by_step():
    """Mixed disc (40 embryos + 20000 planetesimals, cold): after every step the GPU's encounter
    list equals the oracle's on the GPU's positions, and the step stays within BS capacity."""
    d = discs.disc_c5()
    s = System([d])
    torch = s.torch
    for k in range(4):
        ax = s.zeros()
        genga.genga_accel(s.ctx.handle, s.b, FP32, ax, s.zeros(), s.zeros())
        got, cnt = s.encounter_list()
        st = s.numpy_state()
        exp = oracle.encounters(st, s.rc)
        print(f"[c5 step {k}] pairs gpu={cnt} oracle={len(exp)}", flush=True)
        assert cnt == len(exp)
        np.testing.assert_array_equal(got, exp)
        genga.genga_step(s.ctx.handle, s.b, DT, 1, FP32)
        torch.cuda.synchronize()
        assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    s.close()


def test_c5_energy_drift_500_steps():
    d = discs.disc_c5()
    res = {}
    for prec in (FP64, FP32):
        s = System([d])
        res[prec] = run_series(s, prec, 500, 10)
        s.close()
    m64, m32 = (np.max(np.abs(res[p][0])) for p in (FP64, FP32))
    l64, l32 = (np.max(np.abs(res[p][1])) for p in (FP64, FP32))
    print(f"[c5 500 steps] max|dE/E| fp64={m64:.3e} fp32={m32:.3e}  max|dL/L| fp64={l64:.3e} fp32={l32:.3e}",
          flush=True)
    # encounter-dominated: both paths share the encounter machinery; report and bound
    assert max(m32, m64) < 1e-5
    assert l64 <= 1e-12


def test_c4_batched_sampled_rows():
    """64 discs of uneven N in one layout: FP32 and FP64 accelerations of 16 sampled rows per
    disc against the oracle, and every disc's encounter list."""
    ds = discs.batch_c4()
    s = System(ds)
    a32, a64 = s.accel(FP32), s.accel(FP64)
    got, cnt = s.encounter_list()
    rng = np.random.default_rng(1)
    exp_pairs = []
    worst = {FP32: 0.0, FP64: 0.0}
    for k, d in enumerate(ds):
        sl = s.system_slice(k)
        rows = rng.choice(d.n, 16, replace=False)
        ax, ay, az = oracle.accel_rows(d.state(), s.rc[sl], rows)
        ref = np.stack([ax, ay, az], axis=1)
        for prec, a in ((FP32, a32), (FP64, a64)):
            rms, _ = force_errors(a[sl][rows], ref)
            worst[prec] = max(worst[prec], rms)
        p = oracle.encounters(d.state(), s.rc[sl])
        exp_pairs.append(p + sl.start)
    print(f"[c4 sampled] worst rms fp32={worst[FP32]:.3e} fp64={worst[FP64]:.3e} pairs={cnt}", flush=True)
    assert worst[FP32] <= 1e-5 and worst[FP64] <= 1e-12
    exp = np.concatenate(exp_pairs).astype(np.int32)
    exp = exp[np.lexsort((exp[:, 1], exp[:, 0]))]
    assert cnt == len(exp)
    np.testing.assert_array_equal(got, exp)
    s.close()


def test_checkpoint_resume_is_bit_identical():
    """Halting and resuming (Sect. 1: regular halting and resuming on shared systems): a run
    that writes its state to host memory after 5 steps and continues in a fresh context from
    those bytes ends bit-identical to the uninterrupted run (the kernels are deterministic)."""
    d = discs.make_disc(2500, 2.0, seed=91, a_in=0.7, a_out=1.0, sigma_e=0.002, sigma_i=0.002,
                        n_embryo=10, embryo_mass_earth=0.1)
    a = System([d])
    genga.genga_step(a.ctx.handle, a.b, DT, 5, FP32)
    ckpt = a.numpy_state()                      # host copy of the state, as a checkpoint holds it
    genga.genga_step(a.ctx.handle, a.b, DT, 5, FP32)
    end_a = a.numpy_state()
    b = System([discs.Disc(**ckpt)], rcrit=a.rc)
    genga.genga_step(b.ctx.handle, b.b, DT, 5, FP32)
    end_b = b.numpy_state()
    for k in end_a:
        np.testing.assert_array_equal(end_a[k], end_b[k])
    a.close()
    b.close()


def test_c2_force_error_at_checkpoints():
    """Force error of both kicks against the oracle at steps 0, 100 and 200 of the N = 6600
    disc, feeding the GPU's own state to the oracle at each checkpoint."""
    d = discs.disc_c2()
    s = System([d])
    for k in range(3):
        st = s.numpy_state()
        ref = np.stack(oracle.accel(st, s.rc), axis=1)
        for prec, bar in ((FP64, 1e-12), (FP32, 1e-5)):
            rms, mx = force_errors(s.accel(prec), ref)
            print(f"[c2 checkpoint step {100 * k}] prec={prec} rms={rms:.3e} max={mx:.3e}", flush=True)
            assert rms <= bar
        genga.genga_step(s.ctx.handle, s.b, DT, 100, FP32)
    s.close()
