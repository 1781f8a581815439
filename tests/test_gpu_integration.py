"""Workload-sized runs on the GPU: energy and angular-momentum drift of the FP32 and FP64
kicks over many steps, encounter lists on the dense mixed disc step by step, and the batched
64-disc layout on sampled rows.  The oracle checks the GPU state it is fed at checkpoints.
"""
import numpy as np
import pytest

import discs
import oracle
import paper_2309_08217_amd as genga
from gpu_helpers import DT, System, force_errors, oracle_accel_systems

pytestmark = pytest.mark.gpu

FP64, FP32 = genga.GENGA_KICK_FP64, genga.GENGA_KICK_FP32
# c1: FP64 kick, Kepler drift and Bulirsch-Stoer (tolerance 1e-12 on the group's scales)
C1_BAR = 1e-11


def run_series(sysm, prec, nsteps, cadence):
    torch = sysm.torch
    nsys = len(sysm.discs)
    e0 = sysm.energy()
    rec = torch.zeros((nsteps // cadence) * 4 * nsys, dtype=torch.float64, device="cuda")
    genga.genga_step(sysm.ctx.handle, sysm.b, DT, nsteps, prec, energy_cadence=cadence, d_energy=rec)
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


def test_c5_lists_and_energy_500_steps():
    """Mixed disc (40 embryos + 20000 planetesimals, cold; the paper's embryo runs, Sect. 3.2),
    500 steps of each kick precision: every 10 steps the GPU's encounter list equals the
    oracle's on the GPU's positions (the list of the step's last kick), the step stays within
    the close-encounter capacity, and max |dE/E| (Sect. 3.1) of the FP32 kick is within 2x that
    of the FP64 kick; FP64 keeps |L| to round-off."""
    d = discs.disc_c5()
    res = {}
    for prec in (FP64, FP32):
        s = System([d])
        torch = s.torch
        e0 = s.energy()[0]
        rec = torch.zeros(4, dtype=torch.float64, device="cuda")
        dE, dL, npairs = [], [], []
        for k in range(50):
            genga.genga_step(s.ctx.handle, s.b, DT, 10, prec, energy_cadence=10, d_energy=rec)
            torch.cuda.synchronize()
            assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
            r = rec.cpu().numpy()
            dE.append(r[0] / e0[0] - 1.0)
            dL.append(np.linalg.norm(r[1:]) / np.linalg.norm(e0[1:]) - 1.0)
            got, cnt = s.encounter_list()
            exp = oracle.encounters(s.numpy_state(), s.rc)
            assert cnt == len(exp), (prec, 10 * (k + 1), cnt, len(exp))
            np.testing.assert_array_equal(got, exp)
            npairs.append(cnt)
        res[prec] = (np.max(np.abs(dE)), np.max(np.abs(dL)))
        print(f"[c5 prec={prec}] 50 list checks, pairs min {min(npairs)} max {max(npairs)}", flush=True)
        s.close()
    (m64, l64), (m32, l32) = res[FP64], res[FP32]
    print(f"[c5 500 steps] max|dE/E| fp64={m64:.3e} fp32={m32:.3e}  max|dL/L| fp64={l64:.3e} fp32={l32:.3e}",
          flush=True)
    assert m32 <= 2.0 * m64
    assert max(m32, m64) < 1e-5
    assert l64 <= 1e-12


def test_c1_ten_fp64_steps_against_oracle():
    """The oracle-sized run (N = 2048, 10 FP64 steps of the level-0 step, Sect. 1) element by
    element against the oracle's 10 steps."""
    d = discs.disc_c1()
    s = System([d])
    genga.genga_step(s.ctx.handle, s.b, DT, 10, FP64)
    got = s.numpy_state()
    assert genga.genga_poll_status(s.ctx.handle) == genga.GENGA_OK, genga.genga_last_error()
    exp, _ = oracle.step(d.state(), s.rc, 1.0, DT, 10)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        err = np.max(np.abs(got[k] - exp[k]))
        rel = np.max(np.abs(got[k] - exp[k]) / np.maximum(np.abs(exp[k]), 1e-3))
        print(f"[c1 10 steps] {k} max abs err {err:.2e} rel {rel:.2e}", flush=True)
        assert err <= C1_BAR
    s.close()


def test_c4_batched_all_rows():
    """64 discs of uneven N in one layout: every row of the FP32 kick with Kahan-compensated
    FP32 folding (the batched configuration), the FP32 kick with FP64 folding and the FP64
    kick against the oracle, and every disc's encounter list."""
    ds = discs.batch_c4()
    s = System(ds)
    ref = oracle_accel_systems(s)
    worst = {}
    for prec, acc, bar in ((FP32, genga.GENGA_ACC_KAHAN32, 1e-5), (FP32, genga.GENGA_ACC_FP64, 1e-5),
                           (FP64, genga.GENGA_ACC_FP64, 1e-12)):
        ax, ay, az = s.zeros(), s.zeros(), s.zeros()
        genga.genga_accel(s.ctx.handle, s.b, ax, ay, az, prec, acc)
        s.torch.cuda.synchronize()
        a = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], axis=1)
        w = 0.0
        for k in range(len(ds)):
            sl = s.system_slice(k)
            rms, _ = force_errors(a[sl], ref[sl])
            w = max(w, rms)
        worst[(prec, acc)] = w
        assert w <= bar, (prec, acc, w)
    got, cnt = s.encounter_list()
    exp = np.concatenate([oracle.encounters(d.state(), s.rc[s.system_slice(k)]) + s.system_slice(k).start
                          for k, d in enumerate(ds)]).astype(np.int32)
    exp = exp[np.lexsort((exp[:, 1], exp[:, 0]))]
    print(f"[c4 all rows] worst per-disc rms {worst} pairs={cnt}", flush=True)
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
