"""Benchmark of the DG hot path on one MI355X.

Workload (one "step" = one SSP-RK3 step of dg_step: the CFL reduction and three
fused stage launches): modal DG, k = 3 (20 modes, 4^3 Gauss points), 256^3
cells, periodic unit box, gamma = 5/3, the seeded turbulence surrogate at rms
Mach 0.3 (synthetic: solenoidal k^-5/3 velocity field, rho = p = 1), with the
solenoidal Ornstein-Uhlenbeck driving on 1 <= |n| <= 3 when the library
supports it.

Metric: DOF-updates/s per RK stage = 5 N(k) cells * 3 * steps / elapsed, for
the FP32-grade tier (value) with the FP64 path and the BF16 tier reported
beside it.  Roofline of the stage kernel from HIP events around each launch on
the library's stream; algorithmic bytes per launch: stage 1 reads and writes one state, stages 2 and 3 read two and write one.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--k 3]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_MATRIX_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores
FP64_VECTOR_TFLOPS = 78.6   # MI355X vector FP64
FP32_VECTOR_TFLOPS = 157.3  # MI355X vector FP32
FP32_MATRIX_TFLOPS = 157.3  # MI355X dense FP32 matrix cores
FP64_MATRIX_TFLOPS = 78.6   # MI355X dense FP64 matrix cores


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=256)
    p.add_argument("--k", type=int, default=3)
    p.add_argument("--tiers", default="bf16x3,fp32,bf16,fp64")
    p.add_argument("--primary", default="auto", help="tier reported as value (auto: fastest FP32-grade)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-n", type=int, default=32, help="mesh of the oracle's timed sample")
    p.add_argument("--quiet", action="store_true")
    p.add_argument("--no-forcing", action="store_true", help="operator only (no driving source)")
    p.add_argument("--diagnostics", action="store_true", help="also time the spectrum, PDF and Mach diagnostics")
    p.add_argument("--no-limiter", action="store_true", help="skip the limiter and isothermal-reset timings")
    p.add_argument("--k4-n", type=int, default=64, help="mesh of the k = 4 timing (0: skip it)")
    p.add_argument("--no-configs", action="store_true",
                   help="skip the other workloads (k=2 on 64^3 FP64/FP32, k=3 on 128^3 in every tier) and the "
                        "operator-only figure")
    p.add_argument("--copy-calibration", type=float, default=0.0,
                   help="GiB: also run a plain device copy of this size (reference for counter-based traffic)")
    return p.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def stage_bytes(N, cells, elem):
    """Algorithmic HBM bytes of the three stages of one step: stage 1 reads y and
    writes y1 (2 states); stages 2 and 3 read y^(s), y^(0) and write (3 states)."""
    st = 5 * N * cells * elem
    return [2 * st, 3 * st, 3 * st]


# Algorithmic floating-point operations per cell of one stage at k = 3 (dense contractions as
# written, an FMA counts 2): modal -> volume points 2*5*N*Q, volume integral 2*3*5*N*Q, driving
# source projection 2*4*N*Q, face traces 2*6*5*N*16, lift 2*6*5*N*16 (N = 20, Q = 64): 89 600;
# the vector remainder (point fluxes, HLLC on 48 face points, update) about 7 980.
K3_CONTRACTION_FLOPS = 89600
K3_VECTOR_FLOPS = 7980


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("dg_kernels.hip", "stage_k3.hip", "stage_k4.hip", "dg_device.h", "dg_host.cpp", "dg_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1602_09079_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


# Driving: the solenoidal OU field on 1 <= |n| <= 3 (43 modes and their
# conjugates), one OU update from the stationary start.  a0 is fixed by the scale
# estimate a ~ v_rms^2 / L for Mach 0.3 (v_rms = 0.387, rms |a| ~ 5 a0).
A0 = 0.03
OU_SEED = 1602


def driving_table(dg):
    from paper_1602_09079_amd import synth
    nvec = synth.forcing_modes(1.0, 3.0)
    th = synth.ou_stationary_start(OU_SEED, len(nvec))
    z = synth.ou_normals(OU_SEED, len(nvec), 1)[0]
    ts = 0.5 / (0.3 * math.sqrt(5.0 / 3.0))  # t_s = L / (2 M c)
    _, ahat = dg.ou_update(nvec, th, z, math.exp(-0.1), 1.0, A0, 1.0, 3.0)  # dt_drive = 0.1 t_s
    return nvec, ahat, ts


def measure_tier(args, dg, torch, prec, qp_dev, n, k):
    s = dg.Solver(k, n, precision=prec, cfl=0.3, forcing=not args.no_forcing)
    drive_ms = None
    if not args.no_forcing:
        nvec, ahat, _ = driving_table(dg)
        s.set_forcing(nvec, ahat)
        # one driving update (OU step done on the host): table upload and the cache of the
        # acceleration at every volume point; dg_set_forcing synchronises its stream
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_forcing(nvec, ahat)
        drive_ms = (time.perf_counter() - t0) * 1e3
    y = s.project(qp_dev.to(s.dtype))
    N = s.N
    cells = n ** 3
    torch.cuda.synchronize()
    # warmup
    for _ in range(args.warmup):
        s.step_async(y, 1, 0.0)
    torch.cuda.synchronize()
    # timed region: exactly `steps` steps of dg_step
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s.stream)
    s.step_async(y, args.steps, 0.0)
    e1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    dof_stage = 5 * N * cells
    rate = dof_stage * 3 * args.steps / (ms / 1e3)
    # per-launch durations of the stage kernel (events around each dg_stage call)
    w1 = torch.empty_like(y)
    w2 = torch.empty_like(y)
    h = s.dt(y)
    evs = []
    for rep in range(max(2, args.steps)):
        trip = []
        for (y0, yin, out, a, b) in ((y, y, w1, 0.0, 1.0), (y, w1, w2, 0.75, 0.25), (y, w2, w1, 1 / 3, 2 / 3)):
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record(s.stream)
            s.stage(y0, yin, out, a, b, h)
            eb.record(s.stream)
            trip.append((ea, eb))
        evs.append(trip)
    torch.cuda.synchronize()
    durs = [[ea.elapsed_time(eb) for ea, eb in trip] for trip in evs]
    avg_stage_ms = sum(sum(t) for t in durs) / (3 * len(durs))
    elem = 8 if prec == "fp64" else 4
    sb = stage_bytes(N, cells, elem)
    achieved = (sum(sb) / 3) / (avg_stage_ms / 1e3) / 1e9
    finite = bool(torch.isfinite(y).all().item())
    del w1, w2
    out = dict(prec=prec, ms_per_step=ms_step, wall_s=wall, dof_updates_per_s=rate, stage_ms=avg_stage_ms,
               stage_ms_each=[sum(t[i] for t in durs) / len(durs) for i in range(3)],
               achieved_GBs=achieved, bytes_per_stage_avg=sum(sb) / 3, finite=finite, driving_update_ms=drive_ms)
    log(args, f"[bench] {prec}: {ms_step:.3f} ms/step, {rate:.3e} DOF-updates/s/stage, stage {avg_stage_ms:.3f} ms "
              f"({', '.join(f'{v:.2f}' for v in out['stage_ms_each'])}), "
              f"{achieved:.0f} GB/s algorithmic, finite={finite}")
    del s, y
    torch.cuda.empty_cache()
    return out


def config_cost(args, dg, torch, k, n, tiers, forcing=True):
    """Another workload of the same recipe (seeded turbulence surrogate at Mach 0.3, driving on
    1 <= |n| <= 3): k, n^3 cells, each tier's dg_step rate and stage-launch roofline."""
    from paper_1602_09079_amd import synth
    qp = synth.turbulence(n, dg.gauss_nodes(k + 1), seed=9079, mach=0.3, device="cuda", dtype=torch.float32)
    sub = argparse.Namespace(**vars(args))
    sub.no_forcing = not forcing
    out = dict(k=k, n=n, cells=n ** 3, dof=5 * dg.nmodes(k) * n ** 3, forcing=forcing, tiers={})
    for prec in tiers:
        r = measure_tier(sub, dg, torch, prec, qp, n, k)
        out["tiers"][prec] = dict(dof_updates_per_s=r["dof_updates_per_s"], ms_per_step=r["ms_per_step"],
                                  stage_ms=r["stage_ms"], stage_ms_each=r["stage_ms_each"],
                                  hbm_frac=round(r["achieved_GBs"] / HBM_PEAK_GBS, 4))
    if "fp64" in out["tiers"]:
        base = out["tiers"]["fp64"]["dof_updates_per_s"]
        out["speedup_vs_fp64"] = {p: round(v["dof_updates_per_s"] / base, 3) for p, v in out["tiers"].items()
                                  if p != "fp64"}
    del qp
    torch.cuda.empty_cache()
    return out


def share_cost(args, dg, torch, prec, qp_dev, n, k, parts=8):
    """One GPU's share of the mesh split into `parts` z slabs (n x n x n/parts cells, halo planes
    instead of the periodic wrap): stage launch time, and the two halo planes a stage needs (their
    bytes, and a device-to-device copy of them standing in for the transfer)."""
    dz = n // parts
    s = dg.Solver(k, (n, n, dz), box=(1.0, 1.0, dz / n), precision=prec, cfl=0.3, forcing=not args.no_forcing,
                  zhalo=True)
    s.set_slab(0, n)
    if not args.no_forcing:
        nvec, ahat, _ = driving_table(dg)
        s.set_forcing(nvec, ahat)
    y = s.project(qp_dev[:, :, :, :, :dz].contiguous().to(s.dtype))
    lo, hi = torch.empty_like(y[0]), torch.empty_like(y[0])
    src_lo, src_hi = y[-1].clone(), y[0].clone()
    s.set_halo(lo, hi)
    w1 = torch.empty_like(y)
    lo.copy_(src_lo)
    hi.copy_(src_hi)
    h = s.dt(y)
    s.stage(y, y, w1, 0.0, 1.0, h)
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(s.stream)
    for _ in range(reps):
        lo.copy_(src_lo)
        hi.copy_(src_hi)
    ev[1].record(s.stream)
    for _ in range(reps):
        s.stage(y, y, w1, 0.0, 1.0, h)
    ev[2].record(s.stream)
    torch.cuda.synchronize()
    copy_ms = ev[0].elapsed_time(ev[1]) / reps
    ms = ev[1].elapsed_time(ev[2]) / reps
    plane = lo.numel() * lo.element_size()
    log(args, f"[bench] {prec} one GPU's share of a {parts}-way z split ({n}x{n}x{dz}): stage 1 {ms:.3f} ms, "
              f"halo planes 2 x {plane / 1e6:.1f} MB, device copy {copy_ms:.3f} ms")
    del s, y, w1, lo, hi, src_lo, src_hi
    torch.cuda.empty_cache()
    return dict(tier=prec, parts=parts, cells=[n, n, dz], stage1_ms=ms, halo_plane_bytes=plane,
                halo_copy_ms=copy_ms)


def exact_riemann_cost(args, dg, torch, prec, qp_dev, n, k):
    """Stage launches of the primary tier with the exact Riemann solver as the face flux."""
    s = dg.Solver(k, n, precision=prec, cfl=0.3, forcing=not args.no_forcing, riemann="exact")
    if not args.no_forcing:
        nvec, ahat, _ = driving_table(dg)
        s.set_forcing(nvec, ahat)
    y = s.project(qp_dev.to(s.dtype))
    w1 = torch.empty_like(y)
    h = s.dt(y)
    s.stage(y, y, w1, 0.0, 1.0, h)
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    ea = torch.cuda.Event(enable_timing=True)
    eb = torch.cuda.Event(enable_timing=True)
    ea.record(s.stream)
    for _ in range(reps):
        s.stage(y, y, w1, 0.0, 1.0, h)
    eb.record(s.stream)
    torch.cuda.synchronize()
    ms = ea.elapsed_time(eb) / reps
    log(args, f"[bench] {prec} stage 1 with the exact Riemann solver: {ms:.3f} ms")
    del s, y, w1
    torch.cuda.empty_cache()
    return dict(tier=prec, stage1_ms=ms)


# Algorithmic floating-point operations per cell of one k = 4 stage in the quadrature form
# (N = 35, Q = 125 volume points, 150 face points; an FMA counts 2; the contractions, nearly all
# of it, run on the matrix cores): point states 2*5*N*Q,
# point fluxes 40*Q, volume contraction 2*3*5*N*Q, driving source 2*4*N*Q + 8*Q, face traces
# 2*2*5*N*150, face fluxes about 60*150 (HLLC), lift 2*5*N*150, stage update 4*5*N.
def k4_flops_per_cell(forcing):
    N, Q, F = 35, 125, 150
    f = 2 * 5 * N * Q + 40 * Q + 2 * 3 * 5 * N * Q + 2 * 2 * 5 * N * F + 60 * F + 2 * 5 * N * F + 4 * 5 * N
    if forcing:
        f += 2 * 4 * N * Q + 8 * Q
    return f


def k4_cost(args, dg, torch):
    """Stage launches at k = 4 (the matrix-core kernel) in FP64 and FP32 on a k4_n^3 mesh with the
    same workload recipe; the algorithmic flops per cell above against the matrix-core peak."""
    from paper_1602_09079_amd import synth
    n, k = args.k4_n, 4
    out = dict(n=n, k=k, flops_per_cell=k4_flops_per_cell(not args.no_forcing))
    qp = synth.turbulence(n, dg.gauss_nodes(k + 1), seed=9079, mach=0.3, device="cuda", dtype=torch.float32)
    for prec, peak, unit in (("fp64", FP64_MATRIX_TFLOPS, "mfma"), ("fp32", FP32_MATRIX_TFLOPS, "mfma")):
        s = dg.Solver(k, n, precision=prec, cfl=0.3, forcing=not args.no_forcing)
        if not args.no_forcing:
            nvec, ahat, _ = driving_table(dg)
            s.set_forcing(nvec, ahat)
        y = s.project(qp.to(s.dtype))
        w1 = torch.empty_like(y)
        h = s.dt(y)
        s.stage(y, y, w1, 0.0, 1.0, h)
        torch.cuda.synchronize()
        reps = max(3, args.steps)
        ea = torch.cuda.Event(enable_timing=True)
        eb = torch.cuda.Event(enable_timing=True)
        ea.record(s.stream)
        for _ in range(reps):
            s.stage(y, y, w1, 0.0, 1.0, h)
        eb.record(s.stream)
        torch.cuda.synchronize()
        ms = ea.elapsed_time(eb) / reps
        tf = out["flops_per_cell"] * n ** 3 / (ms / 1e3) / 1e12
        out[prec] = dict(stage_ms=ms, dof_updates_per_s=5 * dg.nmodes(k) * n ** 3 / (ms / 1e3), bound=unit,
                         TFLOPs=round(tf, 2), peak_TFLOPs=peak, frac=round(tf / peak, 4))
        log(args, f"[bench] k=4 {prec} stage 1 on {n}^3: {ms:.3f} ms, {tf:.2f} TFLOP/s")
        del s, y, w1
        torch.cuda.empty_cache()
    del qp
    torch.cuda.empty_cache()
    return out


def k0_cost(args, dg, torch):
    """Stage launches at k = 0 (first-order finite volume, one thread per cell) in FP64 and FP32
    on the benchmark's 256^3 mesh with the same recipe; HBM roof: stage 1 reads and writes one
    state, 2 x 5 values per cell."""
    from paper_1602_09079_amd import synth
    k, n = 0, args.n
    qp = synth.turbulence(n, dg.gauss_nodes(1), seed=9079, mach=0.3, device="cuda", dtype=torch.float32)
    nvec, ahat, _ = driving_table(dg)
    out = dict(n=n, k=k)
    for prec in ("fp64", "fp32"):
        s = dg.Solver(k, n, precision=prec, cfl=0.3, forcing=not args.no_forcing)
        if not args.no_forcing:
            s.set_forcing(nvec, ahat)
        y = s.project(qp.to(s.dtype))
        w1 = torch.empty_like(y)
        h = s.dt(y)
        s.stage(y, y, w1, 0.0, 1.0, h)
        torch.cuda.synchronize()
        reps = max(10, 4 * args.steps)
        ea = torch.cuda.Event(enable_timing=True)
        eb = torch.cuda.Event(enable_timing=True)
        ea.record(s.stream)
        for _ in range(reps):
            s.stage(y, y, w1, 0.0, 1.0, h)
        eb.record(s.stream)
        torch.cuda.synchronize()
        ms = ea.elapsed_time(eb) / reps
        elem = 8 if prec == "fp64" else 4
        gbs = 2 * 5 * n ** 3 * elem / (ms / 1e3) / 1e9
        out[prec] = dict(stage_ms=ms, dof_updates_per_s=5 * n ** 3 / (ms / 1e3), algorithmic_GBs=round(gbs, 1),
                         hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
        log(args, f"[bench] k=0 {prec} stage 1 on {n}^3: {ms:.3f} ms, {gbs:.0f} GB/s algorithmic")
        del s, y, w1
        torch.cuda.empty_cache()
    del qp
    torch.cuda.empty_cache()
    return out


CLOSURE_SHAPE = (140, 128, 128, 20)
CLOSURE_FLOPS_PER_CELL = 2 * (140 * 128 + 128 * 128 + 128 * 20)  # the three dense layers


def closure_cost(args, dg, torch):
    """The learned closure's inference in the stage (k = 1 on 64^3, FP32, driving on; random
    Xavier weights of the 140-128-128-20 network, no cell falling back): stage 1 with and
    without it; the difference is the closure's cost, against the FP32 matrix-core peak."""
    import numpy as np

    from paper_1602_09079_amd import synth
    k, n = 1, 64
    qp = synth.turbulence(n, dg.gauss_nodes(k + 1), seed=9079, mach=0.3, device="cuda", dtype=torch.float32)
    nvec, ahat, _ = driving_table(dg)
    out = dict(k=k, n=n, tier="fp32", flops_per_cell=CLOSURE_FLOPS_PER_CELL)
    for name, closure in (("plain", False), ("closure", True)):
        s = dg.Solver(k, n, precision="fp32", cfl=0.3, forcing=True, closure=closure)
        s.set_forcing(nvec, ahat)
        if closure:
            p = synth.xavier_params(CLOSURE_SHAPE, seed=4)
            s.set_closure(p, np.zeros(140), np.ones(140), np.full(20, 1e-3), np.full(20, 1e30))
        y = s.project(qp)
        w1 = torch.empty_like(y)
        h = s.dt(y)
        s.stage(y, y, w1, 0.0, 1.0, h)
        torch.cuda.synchronize()
        reps = max(10, 4 * args.steps)
        ea = torch.cuda.Event(enable_timing=True)
        eb = torch.cuda.Event(enable_timing=True)
        ea.record(s.stream)
        for _ in range(reps):
            s.stage(y, y, w1, 0.0, 1.0, h)
        eb.record(s.stream)
        torch.cuda.synchronize()
        out[f"stage1_ms_{name}"] = ea.elapsed_time(eb) / reps
        if closure:
            out["fallbacks"] = s.closure_fallbacks()
        del s, y, w1
        torch.cuda.empty_cache()
    d = out["stage1_ms_closure"] - out["stage1_ms_plain"]
    out["closure_ms"] = d
    tf = CLOSURE_FLOPS_PER_CELL * n ** 3 / (d / 1e3) / 1e12 if d > 0 else None
    out["closure_TFLOPs"] = tf
    out["closure_frac_of_fp32_matrix_peak"] = tf / FP32_MATRIX_TFLOPS if tf else None
    log(args, f"[bench] closure inference k=1 {n}^3: stage 1 {out['stage1_ms_plain']:.3f} ms plain, "
              f"{out['stage1_ms_closure']:.3f} ms with the closure")
    del qp
    torch.cuda.empty_cache()
    return out


def limiter_cost(args, dg, torch, prec, qp_dev, n, k):
    """Stage launches of the primary tier with the positivity limiter of Sec. 2.5 on the
    stage input (the paper applies it every stage; the smooth workload never needs it, so this
    is the cost of checking)."""
    s = dg.Solver(k, n, precision=prec, cfl=0.3, forcing=not args.no_forcing, limit=True)
    if not args.no_forcing:
        nvec, ahat, _ = driving_table(dg)
        s.set_forcing(nvec, ahat)
    y = s.project(qp_dev.to(s.dtype))
    w1 = torch.empty_like(y)
    w2 = torch.empty_like(y)
    h = s.dt(y)
    s.stage(y, y, w1, 0.0, 1.0, h)
    torch.cuda.synchronize()
    evs = []
    for rep in range(max(2, args.steps)):
        for (y0, yin, out, a, b) in ((y, y, w1, 0.0, 1.0), (y, w1, w2, 0.75, 0.25), (y, w2, w1, 1 / 3, 2 / 3)):
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record(s.stream)
            s.stage(y0, yin, out, a, b, h)
            eb.record(s.stream)
            evs.append((ea, eb))
    torch.cuda.synchronize()
    ms = sum(ea.elapsed_time(eb) for ea, eb in evs) / len(evs)
    changed = s.limiter_stats()
    log(args, f"[bench] {prec} with the positivity limiter: stage {ms:.3f} ms, cells changed {changed}")
    del s, y, w1, w2
    torch.cuda.empty_cache()
    return dict(tier=prec, stage_ms=ms, cells_changed=changed)


def reset_cost(args, dg, torch, prec, qp_dev, n, k):
    """The isothermal reset of Sec. 3.2 (once per step in the paper's runs) on the benchmark state:
    average launch time and its rate over the algorithmic bytes (reads rho, m and the energy mean,
    writes the energy weights)."""
    s = dg.Solver(k, n, precision=prec)
    s.set_isothermal(1.0, 1.0)
    y = s.project(qp_dev.to(s.dtype))
    s.isothermal_reset(y)
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    ea = torch.cuda.Event(enable_timing=True)
    eb = torch.cuda.Event(enable_timing=True)
    ea.record(s.stream)
    for _ in range(reps):
        s.isothermal_reset(y)
    eb.record(s.stream)
    torch.cuda.synchronize()
    ms = ea.elapsed_time(eb) / reps
    el = 8 if prec == "fp64" else 4
    alg = (5 * s.N + 1) * el * n ** 3
    s.dissipated()
    log(args, f"[bench] {prec} isothermal reset: {ms:.3f} ms, {alg / ms / 1e6:.0f} GB/s algorithmic")
    del s, y
    torch.cuda.empty_cache()
    return dict(tier=prec, reset_ms=ms, algorithmic_GBs=alg / ms / 1e6, hbm_frac=alg / ms / 1e6 / HBM_PEAK_GBS)


def diagnostics_cost(args, dg, torch, prec, qp_dev, n, k):
    """The diagnostics of Sec. 3.3, 4.1, 4.4 on the benchmark state, 4^3 sub-cell points per cell
    (a 4n grid per axis): velocity shell spectrum (three real-to-complex FFTs), log-density PDF,
    rms Mach.  Wall time per call after a first call (which makes the FFT plan)."""
    s = dg.Solver(k, n, precision=prec)
    y = s.project(qp_dev.to(s.dtype))
    work = torch.empty(dg.lib().dg_spectrum_workspace_bytes(s._ctx, 4), dtype=torch.uint8, device=s.device)
    out = {}
    for name, fn in (("spectrum", lambda: s.velocity_spectrum(y, 4, 4 * n, work=work)),
                     ("pdf", lambda: s.density_pdf(y, 4, -0.5, 0.5, 200)),
                     ("rms_mach", lambda: s.rms_mach(y, 4))):
        t0 = time.perf_counter()
        fn()
        first = time.perf_counter() - t0
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        out[name + "_ms"] = (time.perf_counter() - t0) / reps * 1e3
        out[name + "_first_ms"] = first * 1e3
    log(args, f"[bench] {prec} diagnostics on the {4 * n}^3 sub-cell grid: " +
        ", ".join(f"{kk} {v:.1f}" for kk, v in out.items()))
    del s, y, work
    torch.cuda.empty_cache()
    return dict(tier=prec, grid=4 * n, **out)


def cpu_baseline(args, k):
    """Oracle (FP64 C, OpenMP) on a bounded sample: one SSP stage on a cpu_n^3 mesh."""
    import numpy as np

    import oracle as O
    from paper_1602_09079_amd import synth
    n = args.cpu_n
    cfg = O.make_cfg(k, n)
    x = O.gauss_legendre(k + 1)[0]
    y = O.project(cfg, synth.turbulence(n, x, seed=9079, mach=0.3).numpy())
    h = O.dt(cfg, y)
    O.stage(cfg, y, y, 0.0, 1.0, h)  # warm-up
    reps = 0
    t0 = time.perf_counter()
    while True:
        O.stage(cfg, y, y, 0.0, 1.0, h)
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 or reps >= 20:
            break
    per_stage = el / reps
    dof = 5 * O.nmodes(k) * n ** 3
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = dict(value=dof / per_stage, unit="DOF-updates/s per RK stage", cores=threads, kind="oracle",
               sample=f"{reps} SSP stage(s) of the FP64 oracle, k={k}, {n}^3 cells (same per-cell work as the "
                      f"workload), {per_stage:.3f} s per stage, OMP threads={threads}")
    # the same on one thread (a child process: the thread count is fixed when OpenMP starts), 16^3 cells
    code = ("import sys, time; sys.path.insert(0, %r); import oracle as O; from paper_1602_09079_amd import synth; "
            "n, k = 16, %d; cfg = O.make_cfg(k, n); x = O.gauss_legendre(k + 1)[0]; "
            "y = O.project(cfg, synth.turbulence(n, x, seed=9079, mach=0.3).numpy()); h = O.dt(cfg, y); "
            "O.stage(cfg, y, y, 0.0, 1.0, h); t = time.perf_counter(); O.stage(cfg, y, y, 0.0, 1.0, h); "
            "O.stage(cfg, y, y, 0.0, 1.0, h); print((time.perf_counter() - t) / 2)") % (os.path.dirname(
                os.path.abspath(__file__)), k)
    try:
        import subprocess
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
        t1 = float(r.stdout.strip().splitlines()[-1])
        out["single_thread_value"] = 5 * O.nmodes(k) * 16 ** 3 / t1
        out["single_thread_sample"] = f"2 SSP stages of the FP64 oracle, k={k}, 16^3 cells, one thread"
    except Exception as e:  # the one-thread figure is context only
        out["single_thread_value"] = None
        out["single_thread_sample"] = f"not measured: {e}"
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: --gpus must be 1; one GPU's share of a z-slab split "
                                   "is timed as z_slab_share, the transfers between GPUs are not built"}))
        sys.exit(2)
    import torch

    from paper_1602_09079_amd import dg, synth
    dg.lib()
    torch.cuda.set_device(0)
    k, n = args.k, args.n
    x = dg.gauss_nodes(k + 1)
    log(args, f"[bench] generating turbulence surrogate k={k} n={n}")
    qp = synth.turbulence(n, x, seed=9079, mach=0.3, device="cuda", dtype=torch.float32)
    torch.cuda.synchronize()
    results = {}
    for prec in args.tiers.split(","):
        results[prec] = measure_tier(args, dg, torch, prec, qp, n, k)
    fp32_grade0 = [p for p in ("bf16x3", "fp32") if p in results]
    prim0 = args.primary if args.primary != "auto" else max(fp32_grade0 or list(results),
                                                            key=lambda p: results[p]["dof_updates_per_s"])
    lim = None if args.no_limiter else limiter_cost(args, dg, torch, prim0, qp, n, k)
    iso = None if args.no_limiter else reset_cost(args, dg, torch, prim0, qp, n, k)
    diag = diagnostics_cost(args, dg, torch, prim0, qp, n, k) if args.diagnostics else None
    ers = None if args.no_limiter else exact_riemann_cost(args, dg, torch, prim0, qp, n, k)
    shr = None if args.no_limiter else share_cost(args, dg, torch, prim0, qp, n, k)
    k4 = None if (args.no_limiter or args.k4_n <= 0 or k == 4) else k4_cost(args, dg, torch)
    clo = None if args.no_limiter else closure_cost(args, dg, torch)
    k0 = None if (args.no_limiter or k == 0) else k0_cost(args, dg, torch)
    opo = None
    if not args.no_configs and not args.no_forcing:
        # the operator alone (no driving source) on the same state, the primary tier
        sub = argparse.Namespace(**vars(args))
        sub.no_forcing = True
        r = measure_tier(sub, dg, torch, prim0, qp, n, k)
        opo = dict(tier=prim0, forcing=False, dof_updates_per_s=r["dof_updates_per_s"], ms_per_step=r["ms_per_step"],
                   stage_ms=r["stage_ms"], stage_ms_each=r["stage_ms_each"], achieved_GBs=round(r["achieved_GBs"], 1),
                   hbm_frac=round(r["achieved_GBs"] / HBM_PEAK_GBS, 4))
    del qp
    torch.cuda.empty_cache()
    # the box's own copy bandwidth (2 GiB device-to-device, read + write bytes), the second roof
    nel = (2 << 30) // 4
    src = torch.ones(nel, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ea.record()
    for _ in range(5):
        dst.copy_(src)
    eb.record()
    torch.cuda.synchronize()
    copy_GBs = 2 * nel * 4 * 5 / (ea.elapsed_time(eb) / 1e3) / 1e9
    log(args, f"[bench] device copy bandwidth {copy_GBs:.0f} GB/s")
    del src, dst
    torch.cuda.empty_cache()
    if args.copy_calibration > 0:
        nel = int(args.copy_calibration * (1 << 30)) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        # the same bytes in 64-byte segments (the first 16 floats of every 32): the stage kernels
        # read and write 64-byte row segments, the plain copy whole 128-byte lines
        sv, dv = src.view(-1, 32)[:, :16], dst.view(-1, 32)[:, :16]
        for _ in range(3):
            dv.copy_(sv)
        torch.cuda.synchronize()
        log(args, f"[bench] copy calibration: 3 copies of {nel * 4} bytes, then 3 of {nel * 2} bytes in 64-byte segments")
        del src, dst
        torch.cuda.empty_cache()
    fp32_grade = [p for p in ("bf16x3", "fp32") if p in results]
    primary = args.primary if args.primary != "auto" else max(fp32_grade or list(results),
                                                               key=lambda p: results[p]["dof_updates_per_s"])
    r = results[primary]
    N = dg.nmodes(k)
    # achieved: algorithmic bytes over the stage kernel's average launch time (events around each
    # launch); step_achieved_GBs: the same bytes over dg_step's time per step (CFL reduction included)
    roof = dict(bound="hbm", achieved=round(r["achieved_GBs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(r["achieved_GBs"] / HBM_PEAK_GBS, 4), traffic=None,
                step_achieved_GBs=round(3 * r["bytes_per_stage_avg"] / (r["ms_per_step"] / 1e3) / 1e9, 1),
                copy_GBs=round(copy_GBs, 1), frac_of_copy=round(r["achieved_GBs"] / copy_GBs, 4))
    tf = os.path.join(ROOT, "profiles", f"traffic_stage_k{k}_n{n}_{primary}.json")
    if os.path.exists(tf):
        t = json.load(open(tf))
        if t.get("source_hash") == kernel_source_hash():
            roof["traffic"] = t.get("bytes_per_launch")
    cfgs = None
    if not args.no_configs:
        cfgs = {"k2_n64": config_cost(args, dg, torch, 2, 64, ("fp64", "fp32")),
                "k3_n128": config_cost(args, dg, torch, 3, 128, ("fp64", "fp32", "bf16x3", "bf16"))}
    # compute roof of the primary tier at k = 3: algorithmic contraction flops against the dense BF16
    # matrix peak (BF16X3 issues three products per algorithmic one), vector flops against FP32
    comp = None
    if k == 3:
        sec = r["stage_ms"] / 1e3
        mf = K3_CONTRACTION_FLOPS * n ** 3 / sec / 1e12
        vf = K3_VECTOR_FLOPS * n ** 3 / sec / 1e12
        comp = dict(contraction_TFLOPs=round(mf, 2), matrix_peak_TFLOPs=BF16_MATRIX_TFLOPS if primary.startswith("bf16")
                    else FP32_MATRIX_TFLOPS, vector_TFLOPs=round(vf, 2), vector_peak_TFLOPs=FP32_VECTOR_TFLOPS,
                    products_per_contraction=3 if primary == "bf16x3" else 1)
        comp["matrix_frac"] = round(mf * comp["products_per_contraction"] / comp["matrix_peak_TFLOPs"], 4)
        cf = os.path.join(ROOT, "profiles", f"counters_stage_k{k}_n{n}_{primary}.json")
        if os.path.exists(cf):
            c = json.load(open(cf))
            if c.get("source_hash") == kernel_source_hash():
                comp["counters"] = {kk: c[kk] for kk in ("valu_busy", "mfma_busy", "wait_frac") if kk in c}
    cpu = None
    if not args.no_cpu_baseline:
        log(args, "[bench] timing the oracle on the host")
        cpu = cpu_baseline(args, k)
    line = {
        "metric": "DOF-updates/s per RK stage",
        "value": r["dof_updates_per_s"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"modal DG Euler k={k} ({N} modes, {(k + 1) ** 3} Gauss pts), {n}^3 cells, periodic "
                               f"unit box, gamma=5/3, turbulence surrogate Mach 0.3"
                               f"{'' if args.no_forcing else ' with solenoidal OU driving on 1<=|n|<=3'}"
                               f", SSP-RK3 with device CFL dt 0.3",
                   "k": k, "cells": n ** 3, "dof": 5 * N * n ** 3, "tier": primary,
                   "forcing": not args.no_forcing},
        "roofline": roof,
        "cpu_baseline": cpu,
        "tiers": {p: {"dof_updates_per_s": v["dof_updates_per_s"], "ms_per_step": v["ms_per_step"],
                      "stage_ms": v["stage_ms"], "hbm_frac": round(v["achieved_GBs"] / HBM_PEAK_GBS, 4),
                      "driving_update_ms": v["driving_update_ms"]}
                  for p, v in results.items()},
    }
    if "fp64" in results:
        line["speedup_vs_fp64"] = r["dof_updates_per_s"] / results["fp64"]["dof_updates_per_s"]
    if lim is not None:
        line["limiter"] = dict(lim, stage_ms_without=r["stage_ms"])
    if iso is not None:
        line["isothermal_reset"] = iso
    if diag is not None:
        line["diagnostics"] = diag
    if ers is not None:
        line["exact_riemann"] = dict(ers, stage1_ms_hllc=results[ers["tier"]]["stage_ms_each"][0])
    if shr is not None:
        line["z_slab_share"] = dict(shr, whole_stage1_ms=results[shr["tier"]]["stage_ms_each"][0])
    if k4 is not None:
        line["k4_stage"] = k4
    if clo is not None:
        line["closure_inference"] = clo
    if k0 is not None:
        line["k0_stage"] = k0
    if comp is not None:
        line["compute_roof"] = comp
    if opo is not None:
        line["operator_only"] = opo
    if cfgs is not None:
        line["configs"] = cfgs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
