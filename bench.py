"""Benchmark of the changeover-weighted kick path on one MI355X.

Workload: a single synthetic planetesimal disc, N = 40000 equal-mass bodies (5 Earth
masses, 0.5-4 au, Sigma ~ a^-1.5, Rayleigh e and i), r_crit = 3 Hill radii, dt = 6 days.
A step is the whole hot path: the FP32-pair-arithmetic kick with its encounter list, the
Sun drift, the FP64 Kepler drift and close-encounter step, and the FP64 energy /
angular-momentum diagnostic every 10 steps.  `value` is pair interactions N(N-1) per step
times steps per second, for state already resident in HBM.  The K timed steps are one
captured HIP graph of K steps with the energy diagnostic inside it (replayed once untimed
after the W eager warm-up steps, then once timed); eager steps are reported beside it.

Also reported: the FP64 kick path, kick-only rates and their ratio, the roofline of the
kick kernel (HIP events on the launch stream), a batched run of 64 uneven discs in one
launch per kernel vs a loop of single-disc launches, the encounter-dominated regime (dense
0.7-1 au annuli of 6600 and 40322 bodies with the full eq. (1), whose encounter groups span
most of the disc, on the grid-wide Bulirsch-Stoer path), Delta E/E and Delta L/L over the
timed steps, collisions with merging radii, and the FP64 CPU oracle timed on a bounded
sample of the same workload (on the host's cores and on one thread, with the CPU model).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import discs  # noqa: E402
import paper_2309_08217_amd as genga  # noqa: E402

FLOP_PER_PAIR = 18            # 3 sub + 5 (r^2) + 1 rsqrt + 2 (r^-3) + 1 (m) + 6 (3 FMA)
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector (packed FMA)
PEAK_FP32_NONPACKED = 78.6    # 256 CU x 64 lanes x 2.4 GHz x 2 flop (unpacked FMA)
PEAK_FP64_TFLOPS = 78.6
CADENCE = 10
N1, N2 = 3.0, 0.0
DT = discs.DT_6_DAYS


def rcrit_device(ctx, b, torch):
    rc = torch.zeros_like(b.x)
    genga.genga_rcrit(ctx, b, N1, N2, DT, rc)
    b.rcrit = rc
    return rc


def setup(disc_list, torch):
    st, off, mstar = discs.concat(disc_list)
    ctx = genga.Context(0)
    genga.genga_set_systems(ctx.handle, off, mstar)
    b = genga.Bodies.from_numpy(st, device="cuda:0")
    rcrit_device(ctx.handle, b, torch)
    torch.cuda.synchronize()
    return ctx, b, st, off


def time_kicks(ctx, b, prec, reps, torch, stream):
    """Average duration of one genga_kick (prep + kick kernel) over `reps` launches,
    measured with HIP events on the launch stream."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        for _ in range(3):
            genga.genga_kick(ctx.handle, b, 0.0, prec, stream=stream)
        e0.record(stream)
        for _ in range(reps):
            genga.genga_kick(ctx.handle, b, 0.0, prec, stream=stream)
        e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def time_steps(ctx, b, prec, steps, warmup, n_sys, torch, stream):
    """Run warmup then `steps` timed steps (energy every CADENCE steps); returns
    (seconds, energy records, initial energy)."""
    with torch.cuda.stream(stream):
        if warmup > 0:
            genga.genga_step(ctx.handle, b, DT, warmup, prec, stream=stream)
        e_init = torch.zeros(4 * n_sys, dtype=torch.float64, device="cuda:0")
        genga.genga_energy(ctx.handle, b, e_init, stream=stream)
        nrec = max(steps // CADENCE, 0)
        e_rec = torch.zeros(max(nrec, 1) * 4 * n_sys, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        genga.genga_step(ctx.handle, b, DT, steps, prec, energy_cadence=CADENCE, d_energy=e_rec, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    status = genga.genga_poll_status(ctx.handle)
    return t1 - t0, e_rec.cpu().numpy().reshape(-1, n_sys, 4)[:nrec], e_init.cpu().numpy().reshape(n_sys, 4), status


def time_graph(ctx, b, prec, steps, torch, stream, per_graph=50):
    """Steps replayed from a captured HIP graph of `per_graph` steps (no diagnostics; every
    graph starts and ends with a half kick, so it holds per_graph + 1 force evaluations)."""
    with torch.cuda.stream(stream):
        genga.genga_graph_capture(ctx.handle, b, DT, per_graph, prec, stream=stream)
        genga.genga_graph_launch(ctx.handle, 1, stream=stream)
    torch.cuda.synchronize()
    reps = max(1, steps // per_graph)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        genga.genga_graph_launch(ctx.handle, reps, stream=stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / (reps * per_graph)


def time_graph_steps(ctx, b, prec, steps, n_sys, torch, stream):
    """The timed steps as one captured HIP graph of `steps` steps with the energy diagnostic at
    the cadence inside it: captured after the eager warm-up, replayed once untimed (the graph's
    first launch uploads it), then replayed once timed.  Returns (seconds, energy records,
    energy before the timed replay, status)."""
    nrec = max(steps // CADENCE, 0)
    e_rec = torch.zeros(max(nrec, 1) * 4 * n_sys, dtype=torch.float64, device="cuda:0")
    e_init = torch.zeros(4 * n_sys, dtype=torch.float64, device="cuda:0")
    with torch.cuda.stream(stream):
        genga.genga_graph_capture(ctx.handle, b, DT, steps, prec, energy_cadence=CADENCE, d_energy=e_rec,
                                  stream=stream)
        genga.genga_graph_launch(ctx.handle, 1, stream=stream)
        genga.genga_energy(ctx.handle, b, e_init, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        genga.genga_graph_launch(ctx.handle, 1, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    status = genga.genga_poll_status(ctx.handle)
    return t, e_rec.cpu().numpy().reshape(-1, n_sys, 4)[:nrec], e_init.cpu().numpy().reshape(n_sys, 4), status


def drift_stats(e_init, e_rec):
    E0 = e_init[:, 0]
    L0 = np.linalg.norm(e_init[:, 1:], axis=1)
    if len(e_rec) == 0:
        return {"max_abs_dE_over_E": None, "max_abs_dL_over_L": None}
    dE = e_rec[:, :, 0] / E0[None, :] - 1.0
    dL = np.linalg.norm(e_rec[:, :, 1:], axis=2) / L0[None, :] - 1.0
    return {"max_abs_dE_over_E": float(np.max(np.abs(dE))), "final_dE_over_E": float(dE[-1].mean()),
            "max_abs_dL_over_L": float(np.max(np.abs(dL))), "final_dL_over_L": float(dL[-1].mean()),
            "records": int(len(e_rec)), "cadence": CADENCE}


def kick_traffic(pairs):
    """HBM bytes per kick launch from committed rocprofv3 counter runs, if they were taken
    on the current kick source (else null)."""
    path = os.path.join(ROOT, "profiles", "kick32_c3_traffic.json")
    src = os.path.join(ROOT, "paper_2309_08217_amd", "csrc", "kick.hip")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if rec.get("kick_hip_sha256") != sha:
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(st, n):
    """The FP64 oracle's kick on the same disc, timed on the host cores over whole kicks
    (about 10-30 s of CPU work), in the metric's unit."""
    import oracle
    rc = oracle.rcrit(st, 1.0, N1, N2, DT)
    oracle.accel({k: v[:512] for k, v in st.items()}, rc[:512])  # load / warm the library
    reps, t_total = 0, 0.0
    while reps < 8 and (t_total < 10.0 or reps < 1):
        t0 = time.perf_counter()
        oracle.accel(st, rc)
        t_total += time.perf_counter() - t0
        reps += 1
    pairs = float(n) * (n - 1) * reps
    cores = oracle.num_threads()
    # the same oracle on one thread, over rows of the same disc (each row is n - 1 pairs)
    rows = np.arange(0, n, max(1, n // 5000), dtype=np.int64)
    oracle.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.accel_rows(st, rc, rows)
        t1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(cores)
    one = len(rows) * float(n - 1) / t1 / 1e9
    return {"value": pairs / t_total / 1e9, "unit": "G pair-interactions/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{reps} full FP64 oracle kick(s) of the N={n} disc ({pairs:.3e} pair interactions, "
                      f"{t_total:.1f} s); the oracle's drift is O(N) and not included",
            "one_thread": {"value": one, "unit": "G pair-interactions/s", "cores": 1,
                           "sample": f"{len(rows)} rows of the same disc ({len(rows) * (n - 1):.3e} pair "
                                     f"interactions, {t1:.1f} s)"},
            "host_cpu": host_cpu_model(), "host_cpus_visible": os.cpu_count()}


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def batched(torch, stream, steps=10, warmup=2):
    """64 discs, N uniform in [2000, 8000]: one launch per kernel for all discs vs a loop of
    64 single-disc contexts."""
    ds = discs.batch_c4()
    ctx, b, st, off = setup(ds, torch)
    genga.genga_autotune(ctx.handle, b, genga.GENGA_KICK_FP32)
    t, e_rec, e_init, status = time_steps(ctx, b, genga.GENGA_KICK_FP32, steps, warmup, len(ds), torch, stream)
    t_graph = time_graph(ctx, b, genga.GENGA_KICK_FP32, steps, torch, stream)
    pairs = float(sum(d.n * (d.n - 1) for d in ds))
    # the same discs stepped one context after another (64 launches per kernel per step)
    singles = []
    for d in ds:
        c1, b1, _, _ = setup([d], torch)
        w, _ = genga.genga_get_kick_shape(ctx.handle, genga.GENGA_KICK_FP32)
        genga.genga_set_kick_shape(c1.handle, genga.GENGA_KICK_FP32, w, 0)
        singles.append((c1, b1))
    with torch.cuda.stream(stream):
        for c1, b1 in singles:
            genga.genga_step(c1.handle, b1, DT, warmup, genga.GENGA_KICK_FP32, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for c1, b1 in singles:
            genga.genga_step(c1.handle, b1, DT, steps, genga.GENGA_KICK_FP32, stream=stream)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    for c1, _ in singles:
        c1.close()
    ctx.close()
    return {"workload": "64 discs, N uniform in [2000, 8000] (seeds 1000+s), 2.5 Earth masses each",
            "n_total": int(off[-1]), "steps": steps, "steps_per_s": steps / t,
            "graph_steps_per_s": 1.0 / t_graph,
            "pair_interactions_per_s_G": pairs * steps / t / 1e9,
            "loop_of_single_disc_launches_steps_per_s": steps / t_loop,
            "speedup_vs_loop": t_loop / t, "status": status, **drift_stats(e_init, e_rec)}


_D40K = ("dense annulus N=40322, 0.7-1 au, 2 Earth masses, e~R(0.002), i~R(0.001), "
         "r_crit = max(3 R_H, 0.4 dt v), dt = 5 d, seed 13")
# name: (workload, disc, (symplectic levels, sub-steps per level))
DENSE_WORKLOADS = {
    "dense": ("dense annulus N=6600, 0.7-1 au, 2 Earth masses, e~R(0.002), i~R(0.001), "
              "r_crit = max(3 R_H, 0.4 dt v), dt = 5 d, seed 11", discs.disc_dense, (1, 1)),
    "dense_40k": (_D40K, discs.disc_dense_40k, (1, 1)),
    "dense_40k_levels": (_D40K + "; hierarchical levels and sub-steps chosen by genga_tune_levels (up to 4 "
                         "levels x 3 sub-steps, 2 trial steps each), level k's r_crit from eq. (1) with "
                         "dt / n_sub^k", discs.disc_dense_40k, ("tune", 4, 3)),
}
# the 6600-body annulus again with collisions (perfect mergers) and removal inside 0.4 au /
# beyond 40 au: every body of radius 500 km (the paper's planetesimal sizes; mergers are rare),
# and with radii of 2e-3 au, where tens of pairs merge in every step
COLLIDE_RADII_AU = {"dense_collisions": 500.0 / 1.495978707e8, "dense_collisions_merging": 2e-3}
DENSE_WORKLOADS["dense_collisions"] = (DENSE_WORKLOADS["dense"][0] + "; perfect mergers (radius 500 km) and "
                                       "removal inside 0.4 au / beyond 40 au", discs.disc_dense, (1, 1))
DENSE_WORKLOADS["dense_collisions_merging"] = (DENSE_WORKLOADS["dense"][0] + "; perfect mergers (radius 2e-3 au) "
                                               "and removal inside 0.4 au / beyond 40 au", discs.disc_dense, (1, 1))


# steps between two spatial sorts of the bodies in the dense runs (Keplerian shear mixes a
# ring's azimuths by about a tile's width in some tens of 5-day steps)
SORT_EVERY = 10


def dense(torch, stream, which="dense", steps=10, warmup=2):
    """Encounter-dominated regime: a dense annulus (0.7-1 au, 2 Earth masses, 5-day step) with
    r_crit from the full eq. (1), n2 = 0.4, where the encounter groups span most of the disc;
    the grid-wide Bulirsch-Stoer path integrates them (host round trips per attempt, so eager
    steps only).  "dense": the 6600-body disc (one group of all bodies); "dense_40k": the
    40322-body disc of the paper's high-resolution run.  The bodies are sorted in space
    (genga_sort_bodies) after set-up and then every SORT_EVERY steps inside the timed
    region."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    label, make, lv = DENSE_WORKLOADS[which]
    tune = lv[0] == "tune"
    nlev, nsub = (1, 1) if tune else lv
    d = make()
    st, off, mstar = discs.concat([d])
    cap = 64 * d.n
    ctx = genga.Context(0)
    genga.genga_set_systems(ctx.handle, off, mstar, cap)
    genga.genga_set_large_groups(ctx.handle, True)
    b = genga.Bodies.from_numpy(st, device="cuda:0")
    rc = torch.zeros_like(b.x)
    genga.genga_rcrit(ctx.handle, b, discs.DENSE_N1, discs.DENSE_N2, discs.DT_5_DAYS, rc)
    b.rcrit = rc
    genga.genga_sort_bodies(ctx.handle, b)
    collide = which in COLLIDE_RADII_AU
    if collide:
        radius = torch.full((d.n,), COLLIDE_RADII_AU[which], dtype=torch.float64, device="cuda:0")
        col_status = torch.zeros(d.n, dtype=torch.int32, device="cuda:0")
        genga.genga_set_collisions(ctx.handle, b, radius, col_status, 0.4, 40.0)
    if nlev > 1:
        # level k's critical radius: eq. (1) with the level's step dt / nsub^k
        rcl = torch.zeros((nlev - 1, d.n), dtype=torch.float64, device="cuda:0")
        for k in range(1, nlev):
            genga.genga_rcrit(ctx.handle, b, discs.DENSE_N1, discs.DENSE_N2, discs.DT_5_DAYS / nsub ** k, rcl[k - 1])
        genga.genga_set_levels(ctx.handle, nlev, nsub, rcl)
    tune_s = None
    if tune:
        # GENGA-style self-tuning before the run (trial steps of every configuration)
        t_tune = time.perf_counter()
        nlev, nsub = genga.genga_tune_levels(ctx.handle, b, discs.DT_5_DAYS, discs.DENSE_N1, discs.DENSE_N2,
                                             lv[1], lv[2], 2, genga.GENGA_KICK_FP32)
        tune_s = time.perf_counter() - t_tune
    genga.genga_autotune(ctx.handle, b, genga.GENGA_KICK_FP32)
    # group sizes of the initial state, from the GPU's encounter list
    genga.genga_kick(ctx.handle, b, 0.0, genga.GENGA_KICK_FP32)
    pairs = torch.zeros(2 * cap, dtype=torch.int32, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    genga.genga_encounter_list(ctx.handle, None, pairs, cap, cnt)
    torch.cuda.synchronize()
    npair = int(cnt.item())
    assert npair <= cap, "encounter list above its capacity"
    p = pairs[: 2 * npair].cpu().numpy().reshape(-1, 2)
    adj = coo_matrix((np.ones(npair), (p[:, 0], p[:, 1])), shape=(d.n, d.n))
    _, lab = connected_components(adj, directed=False)
    sizes = np.bincount(lab)
    e0 = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    genga.genga_energy(ctx.handle, b, e0)

    def run(n):
        # sort, then up to SORT_EVERY steps, until n steps are done
        with torch.cuda.stream(stream):
            k = 0
            while k < n:
                c = min(SORT_EVERY, n - k)
                genga.genga_sort_bodies(ctx.handle, b, None, stream)
                genga.genga_step(ctx.handle, b, discs.DT_5_DAYS, c, genga.GENGA_KICK_FP32, stream=stream)
                k += c

    run(warmup)
    torch.cuda.synchronize()
    dead_before = int((col_status != 0).sum().item()) if collide else 0
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    e1 = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    genga.genga_energy(ctx.handle, b, e1)
    torch.cuda.synchronize()
    status = genga.genga_poll_status(ctx.handle)
    # the sort alone (the state is already in order: the same work as any sort)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        ev0.record(stream)
        for _ in range(10):
            genga.genga_sort_bodies(ctx.handle, b, None, stream)
        ev1.record(stream)
    torch.cuda.synchronize()
    sort_ms = ev0.elapsed_time(ev1) / 10
    kick_ms = time_kicks(ctx, b, genga.GENGA_KICK_FP32, 10, torch, stream)
    E0, E1 = e0.cpu().numpy(), e1.cpu().numpy()
    ctx.close()
    extra = {"tuning_s": tune_s} if tune else {}
    if collide:
        stt = col_status.cpu().numpy()
        extra = {"radius_au": COLLIDE_RADII_AU[which], "merged": int((stt == 1).sum()),
                 "removed": int((stt == 2).sum()),
                 "merged_or_removed_in_timed_steps": int((stt != 0).sum()) - dead_before}
    return {"workload": label, "n": d.n, "levels": [nlev, nsub], **extra,
            "encounter_pairs_at_start": npair, "largest_group_at_start": int(sizes.max()),
            "groups_above_64_at_start": int((sizes > 64).sum()),
            "steps": steps, "warmup": warmup, "steps_per_s": steps / t, "ms_per_step": 1e3 * t / steps,
            "kick_ms": kick_ms, "non_kick_ms_per_step": 1e3 * t / steps - kick_ms,
            "sort_ms": sort_ms, "sort_every": SORT_EVERY,
            "dE_over_E": float(E1[0] / E0[0] - 1.0),
            "dL_over_L": float(np.linalg.norm(E1[1:]) / np.linalg.norm(E0[1:]) - 1.0),
            "status": status}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kick-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--only-kick", type=int, default=0,
                    help="profiling aid: run this many kicks of the N=40000 disc and exit")
    ap.add_argument("--kick-prec", choices=("fp32", "fp64"), default="fp32",
                    help="precision of the --only-kick kicks")
    ap.add_argument("--batched-only", action="store_true",
                    help="profiling aid: run only the 64-disc batched measurement")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the encounter-dominated dense-annulus measurement")
    ap.add_argument("--dense-only", action="store_true",
                    help="profiling aid: run only the dense-annulus measurement")
    ap.add_argument("--dense-which", default="",
                    help="profiling aid: with --dense-only, run only these dense workloads (comma-separated)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="profiling aid: copy a 256 MiB buffer 4 times (a plain copy of known size, "
                         "to scale HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the kick of one disc "
              "fits one MI355X, and sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP GPU", file=sys.stderr)
        sys.exit(2)
    genga.load_library()
    stream = torch.cuda.Stream()
    if args.copy_calibration:
        src = torch.ones(256 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8, "copies": 4}))
        return
    if args.batched_only:
        print(json.dumps(batched(torch, stream)))
        return
    if args.dense_only:
        which = [w for w in args.dense_which.split(",") if w] or list(DENSE_WORKLOADS)
        print(json.dumps({w: dense(torch, stream, w) for w in which}))
        return
    d = discs.disc_c3()
    if args.only_kick > 0:
        prec = genga.GENGA_KICK_FP32 if args.kick_prec == "fp32" else genga.GENGA_KICK_FP64
        ctx, b, st, _ = setup([d], torch)
        genga.genga_autotune(ctx.handle, b, prec)
        with torch.cuda.stream(stream):
            for _ in range(args.only_kick):
                genga.genga_kick(ctx.handle, b, 0.0, prec, stream=stream)
        torch.cuda.synchronize()
        print(json.dumps({"kicks": args.only_kick, "prec": args.kick_prec,
                          "shape": genga.genga_get_kick_shape(ctx.handle, prec)}))
        ctx.close()
        return
    n = d.n
    pairs = float(n) * (n - 1)
    result = {}
    for name, prec in (("fp32", genga.GENGA_KICK_FP32), ("fp64", genga.GENGA_KICK_FP64)):
        ctx, b, st, _ = setup([d], torch)
        genga.genga_autotune(ctx.handle, b, prec)
        kick_ms = time_kicks(ctx, b, prec, args.kick_reps, torch, stream)
        t_eager, e_rec, e_init, status = time_steps(ctx, b, prec, args.steps, args.warmup, 1, torch, stream)
        eager_stats = drift_stats(e_init, e_rec)
        t, e_rec, e_init, status_g = time_graph_steps(ctx, b, prec, args.steps, 1, torch, stream)
        status = status or status_g
        t_graph = time_graph(ctx, b, prec, args.steps, torch, stream)
        result[name] = {"step_seconds": t, "ms_per_step": 1e3 * t / args.steps,
                        "eager_ms_per_step": 1e3 * t_eager / args.steps, "eager_energy": eager_stats,
                        "graph_ms_per_step_no_diagnostics": 1e3 * t_graph,
                        "value": pairs * args.steps / t / 1e9,
                        "kick_ms": kick_ms, "kick_G_pairs_per_s": pairs / (kick_ms * 1e-3) / 1e9,
                        "kick_tflops": FLOP_PER_PAIR * pairs / (kick_ms * 1e-3) / 1e12,
                        "shape": genga.genga_get_kick_shape(ctx.handle, prec), "status": status,
                        **drift_stats(e_init, e_rec)}
        ctx.close()
    f32, f64 = result["fp32"], result["fp64"]
    out = {
        "metric": "G pair-interactions/s of the FP32-pair-arithmetic kick step at N=40000 (full step: kick, "
                  "encounter list, drift, close-encounter step, energy every 10 steps)",
        "value": f32["value"],
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single disc N=40000, 5 Earth masses, 0.5-4 au, Sigma~a^-1.5, e~R(0.01), "
                               "i~R(0.005), r_crit = 3 R_H, dt = 6 d, seed 3",
                   "n": n, "dt_days": 6.0, "energy_cadence": CADENCE,
                   "kick_waves_split": f32["shape"]},
        "roofline": {"bound": "alu", "kernel": "kick32_kernel",
                     "achieved": f32["kick_tflops"], "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": f32["kick_tflops"] / PEAK_FP32_TFLOPS,
                     "frac_of_unpacked_fp32_peak": f32["kick_tflops"] / PEAK_FP32_NONPACKED,
                     "flop_per_pair": FLOP_PER_PAIR, "pairs_per_launch": pairs,
                     "launch_ms": f32["kick_ms"], "traffic": kick_traffic(pairs)},
        "fp32_kick": {"G_pair_interactions_per_s": f32["kick_G_pairs_per_s"], "kick_ms": f32["kick_ms"]},
        "timing": {"method": "the K timed steps are one captured HIP graph holding the energy diagnostic every "
                             "10 steps (K + 1 force evaluations), replayed once untimed after the W eager warm-up "
                             "steps, then once timed",
                   "eager_fp32_ms_per_step": f32["eager_ms_per_step"],
                   "eager_fp64_ms_per_step": f64["eager_ms_per_step"],
                   "graph_50_steps_no_diagnostics_fp32_ms_per_step": f32["graph_ms_per_step_no_diagnostics"],
                   "graph_50_steps_no_diagnostics_fp64_ms_per_step": f64["graph_ms_per_step_no_diagnostics"]},
        "fp64": {"value": f64["value"], "ms_per_step": f64["ms_per_step"],
                 "G_pair_interactions_per_s_kick": f64["kick_G_pairs_per_s"], "kick_ms": f64["kick_ms"],
                 "roofline": {"bound": "alu", "achieved": f64["kick_tflops"], "peak": PEAK_FP64_TFLOPS,
                              "unit": "TFLOP/s", "frac": f64["kick_tflops"] / PEAK_FP64_TFLOPS},
                 "kick_waves_split": f64["shape"]},
        "fp32_over_fp64": {"kick": f64["kick_ms"] / f32["kick_ms"], "step": f64["ms_per_step"] / f32["ms_per_step"]},
        "energy": {"fp32": {k: v for k, v in f32.items() if "dE" in k or "dL" in k or k in ("records", "cadence")},
                   "fp64": {k: v for k, v in f64.items() if "dE" in k or "dL" in k or k in ("records", "cadence")}},
        "status": {"fp32": f32["status"], "fp64": f64["status"]},
    }
    if not args.no_batched:
        out["batched"] = batched(torch, stream)
    if not args.no_dense:
        for w in DENSE_WORKLOADS:
            out[w] = dense(torch, stream, w)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d.state(), n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
