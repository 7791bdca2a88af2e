#!/usr/bin/env python3
"""PCEXP benchmark on one MI355X: DOF-updates/s of the PCEXP step on the 2D
isentropic-vortex workload (periodic [0,20]^2, 128x128 squares split into
32768 jittered triangles, DG P2, Roe flux, Krylov dimension m = 30, CFL 20).

A step is one full PCEXP step (both stages, two Arnoldi runs of m JVPs with
re-orthogonalised Gram-Schmidt, the device-side Hessenberg phi, the corrector)
through the C ABI; the timed steps run in one pcexp_advance call, which keeps
the state in the internal basis between steps.  Inputs are resident in HBM
before the timed region.

Each step takes dt from eq. (x3d) at its own u_n (CFL 20) on the device;
the time reached is read back from the call and the exact solution (the
translated vortex) is evaluated there.

Prints one JSON line.  `value` is the FP64 tangent-JVP variant; the FP64
finite-difference JVP and the mixed FP32/FP64 tangent variants, and ETD2
(eq. (s7), FP64 tangent, dt fixed from u_0), are timed on the same workload
and reported in `variants` with their solution error.  The default run adds
sections (progress on stderr): `measurement` (cold-cache standalone JVP and
the timed 1 GiB copy), `adjoint` (the 40-step checkpointed gradient),
`channel` (the steady bump channel converged to ||R(rho)|| <= 1e-10 in FP64
and mixed precision), `vortex3d` (the 48^3 x 6 tetrahedral P2 vortex, mixed
precision), and `cpu_baseline` (one full step of the FP64 oracle on the
host).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# profiling class -> HIP kernel(s) it times on the 128x128 P2 Roe vortex (FP64)
HIP_KERNELS = {
    "residual": "pcexp::dg_apply<2, 2, 1, double, 0, 28, 256>",
    "jvp": "pcexp::dg_apply<2, 2, 1, double, 1, 28, 256>",
    "gs_reduce": "pcexp::gs_colsum_kernel (each Arnoldi iteration; its dot products run inside the JVP launch) "
                 "and pcexp::dcgs_reduce<double, NV, PW, true> (closing pass)",
    "gs_update": "pcexp::dcgs_fin_update<double, NV, PW, CV> (all vector-count buckets)",
    "gs_close": "pcexp::dcgs_close_finalize",
    "combine": "pcexp::combine_kernel<double, double>",
}
KERNEL_SOURCES = ("dg_kernels.hpp", "dg_physics.hpp", "dg2.hip", "krylov_kernels.hip", "krylov_kernels.hpp",
                  "wave_reduce.hpp", "pcexp.hip")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1801_06300_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch(cls):
    """HBM bytes per launch of the class's kernel from the committed PMC summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when no summary exists or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{cls}_vortex2d_p2_128.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    return float(vals["traffic_bytes_per_launch"])


def log(msg):
    """Progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--workload", default="vortex2d",
                    choices=["vortex2d", "channel", "vortex3d", "stiffvortex", "reverse"],
                    help="vortex2d: the headline PCEXP step benchmark; channel: steady bump channel to "
                         "||R(rho)|| <= 1e-10 with the CFL ramp; vortex3d: 3D P2 vortex, mixed precision; "
                         "reverse: the discrete adjoint of one step of the headline workload alone")
    ap.add_argument("--channel-iters", type=int, default=12000,
                    help="iteration cap of the steady channel runs (a short cap serves profiling)")
    ap.add_argument("--sections", default="all",
                    help="extra sections of the default run, comma separated: measurement, adjoint, channel, "
                         "vortex3d; 'all' (default) or 'none'")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counter calibration)")
    return ap.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mesh, cfg, u0_np, K):
    """Time one full PCEXP step of the FP64 oracle (2 residuals, 2m + 1
    complex-step JVPs, two modified Gram-Schmidt Arnoldi runs, expm of the
    Hessenberg matrices, the corrector) on the host, on the same workload
    and state, dt from eq. (x3d) at u_0.  `cores` is the parallelism the
    step actually used: process CPU time over wall time (NumPy's
    elementwise work, most of the residual and JVP, runs on one thread;
    BLAS calls may use the threads OMP/OPENBLAS_NUM_THREADS allow)."""
    from oracle.dg import DG
    from oracle.integrators import ExactJacobian, pcexp_step, stable_dt

    g = DG(mesh, cfg["p"], cfg["flux"])
    dt = stable_dt(g, u0_np, cfg["cfl"])
    log("cpu baseline: one oracle PCEXP step at full size")
    c0, t0 = time.process_time(), time.perf_counter()
    pcexp_step(ExactJacobian(g), u0_np, dt, cfg["m"])
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    return dict(value=K / wall, unit="DOF-updates/s", cores=round(cpu / wall, 2), kind="oracle",
                sample=(f"one full FP64 oracle PCEXP step on the 128x128 P2 Roe vortex (K = {K}, m = {cfg['m']}, "
                        f"{2 * cfg['m'] + 1} complex-step JVPs), measured: {wall:.1f} s wall, {cpu:.1f} s CPU"),
                seconds_per_step=wall, cpu_model=_cpu_model(), affinity_cpus=len(os.sched_getaffinity(0)),
                thread_env=env,
                note="NumPy elementwise work is single-threaded; cores = CPU time / wall time of the step")


def section_channel(dev, max_iter=12000):
    """Steady subsonic flow over a Gaussian bump (384x128x2 jittered
    triangles, P2 Roe, Mach 0.5; slip wall along the bump, characteristic
    far field at inflow, outflow and top): pseudo-time PCEXP from the
    uniform free stream with the paper's steady settings (m = 30, the CFL
    ramp of eq. (cfl) to CFL_max 1000, Krylov tolerance 1e-5 controlling
    the predictor's dt), in FP64 and in mixed precision, until
    ||R(rho)|| <= 1e-10 or max_iter iterations.  Reports iterations, wall
    time and DOF-updates/s per precision and the relative difference of the
    two converged states."""
    import torch
    import workloads as W
    from paper_1801_06300_amd import PCEXP, PcexpError

    cfg = W.get_config("channel_bump_p2_384x128")
    mesh = W.build_mesh(cfg)
    prim = W.freestream_prim(2, mach=cfg["mach"], angle_deg=cfg["angle_deg"])
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"], farfield_prim=prim, device=dev)
    xq = ctx.quad_points().cpu().numpy()
    Uq = W.uniform_state(xq.reshape(-1, 2), prim).reshape(ctx.nE, ctx.nq, ctx.nv)
    u0 = ctx.project(torch.as_tensor(Uq, device=dev)).contiguous()
    ctx.set_krylov_tol(cfg["krylov_tol"])
    res, states = {}, {}
    for prec in ("f64", "mixed"):
        log(f"channel: steady run, {prec}")
        ctx.steady(u0.clone(), cfl_max=cfg["cfl_max"], tol=1.0, max_iter=1, m=cfg["m"], prec=prec)   # warm-up
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            info = ctx.steady(u, cfl_max=cfg["cfl_max"], tol=cfg["target_residual"], max_iter=max_iter,
                              check_every=100, m=cfg["m"], prec=prec)
        except PcexpError as e:
            res[prec] = dict(error=str(e))
            continue
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[prec] = dict(info, seconds=wall, ms_per_iteration=1e3 * wall / info["iterations"],
                         dofs_per_s=ctx.K * info["iterations"] / wall)
        states[prec] = u
    ctx.set_krylov_tol(0.0)
    out = dict(workload="steady bump channel 384x128x2 jittered (98304 triangles), DG P2, Roe, Mach 0.5, "
                        "PCEXP m=30, CFL ramp eq. (cfl) to 1000, Krylov tolerance 1e-5, target ||R(rho)|| 1e-10",
               K=ctx.K, runs=res)
    if len(states) == 2:
        out["converged_state_rel_diff_mixed_vs_f64"] = float(
            torch.linalg.norm(states["mixed"] - states["f64"]) / torch.linalg.norm(states["f64"]))
    return out


def calibration_copy(dev):
    """A plain 1 GiB device copy (1 GiB read, 1 GiB written), three times: the
    reference the HBM counters of a profiled run are scaled by."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"read": src.numel() * 8, "write": dst.numel() * 8, "launches": 3}


def bench_channel(args, dev):
    out = section_channel(dev, max_iter=args.channel_iters)
    if args.calibrate_copy:
        out["copy_calibration_bytes"] = calibration_copy(dev)
    main = out["runs"].get("mixed", {})
    line = {
        "metric": "PCEXP DOF-updates/s (steady channel to ||R(rho)|| <= 1e-10)",
        "value": round(main.get("dofs_per_s", 0.0), 1), "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": main.get("iterations", 0), "warmup": 1,
        "ms_per_step": round(main.get("ms_per_iteration", 0.0), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": out["workload"] + ", mixed precision", "K": out["K"]},
        "channel": out,
    }
    print(json.dumps(line))


def bench_stiffvortex(args, dev):
    """The paper's stiff vortex (Sec. 5.1): the beta = 0.2, R = 0.05 vortex of
    radial equilibrium on the clustered 24x24x2 mesh of [0, 0.1]^2 (spacing
    3e-5 .. 0.0115), Roe, advected for one period T = L / U.  For p = 0..3:
    PCEXP at CFL 1000 with m = 30 (dt from eq. (x3d) at u_0, rounded down to a
    divisor of T); the same with the Krylov tolerance 1e-5 (adaptive dimension
    checked every 5 iterations, dt halved by the predictor's estimate; the
    run marches to T with the dt each step took); and CFL 50 for reference.
    The error is |u_h(T) - u_h(0)| / |u_h(0)| (the exact solution at one
    period is the initial one; the paper's vortex fills half the box and is
    not smooth across the periodic boundary, which sets the spatial floor).
    `unphysical` marks runs that passed through rho <= 0 or p <= 0 at a
    quadrature point (the device flags, read at the end of the run)."""
    import math
    import torch
    import workloads as W
    from paper_1801_06300_amd import PCEXP, PcexpError

    mesh = W.stretched_square(24, 0.1)
    T = 0.1 / (0.5 * math.sqrt(W.GAMMA))
    runs = {}
    total_dofs, total_s = 0.0, 0.0
    for p in (0, 1, 2, 3):
        ctx = PCEXP(mesh, p, "roe", device=dev)
        xq = ctx.quad_points().cpu().numpy()
        Uq = W.paper_vortex(xq.reshape(-1, 2)).reshape(ctx.nE, ctx.nq, ctx.nv)
        u0 = ctx.project(torch.as_tensor(Uq, device=dev)).contiguous()
        for name, cfl, tol in (("cfl1000", 1000.0, 0.0), ("cfl1000_tol1e-5", 1000.0, 1e-5), ("cfl50", 50.0, 0.0)):
            ctx.set_krylov_tol(tol)
            ctx.set_krylov_adapt(5 if tol > 0 else 0)
            dt_max = ctx.stable_dt(u0, cfl)
            u = u0.clone()
            unphysical = False
            steps, t = 0, 0.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                if tol > 0:
                    while t < T * (1 - 1e-12) and steps < 20000:
                        info = ctx.step(u, dt=min(dt_max, T - t), m=30, info=True)
                        t += info["dt"]
                        steps += 1
                else:
                    n = max(1, math.ceil(T / dt_max))
                    steps, t = n, T   # the flags are read with the last step, after it completed
                    for i in range(n):
                        ctx.step(u, dt=T / n, m=30, info=(i == n - 1))
                torch.cuda.synchronize()
            except PcexpError as e:
                if "UNPHYSICAL" not in str(e):
                    runs[f"p{p}_{name}"] = dict(steps=steps, error=str(e))
                    continue
                unphysical = True
                if tol > 0:
                    runs[f"p{p}_{name}"] = dict(steps=steps, t=t, unphysical=True)
                    continue
            wall = time.perf_counter() - t0
            err = float(torch.linalg.norm(u - u0) / torch.linalg.norm(u0))
            runs[f"p{p}_{name}"] = dict(steps=steps, t=t, rel_error=err, unphysical=unphysical, seconds=wall,
                                        ms_per_step=1e3 * wall / steps)
            if name == "cfl1000":
                total_dofs += ctx.K * steps
                total_s += wall
        ctx.set_krylov_tol(0.0)
        ctx.set_krylov_adapt(0)
    nst = sum(r.get("steps", 0) for k, r in runs.items() if k.endswith("_cfl1000"))
    out = {
        "metric": "PCEXP DOF-updates/s (stiff stretched-mesh vortex, CFL 1000)",
        "value": round(total_dofs / total_s, 1) if total_s > 0 else 0.0, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": nst, "warmup": 0, "ms_per_step": round(1e3 * total_s / max(1, nst), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "paper vortex (beta 0.2, R 0.05, Mach 0.5) on the 24x24x2 clustered mesh of "
                               "[0,0.1]^2, Roe, p = 0..3, one period at CFL 1000 (fixed m = 30, and with the "
                               "Krylov tolerance 1e-5) and at CFL 50 for reference, FP64"},
        "runs": runs,
    }
    print(json.dumps(out))


def section_vortex3d(dev, steps, warmup):
    """3D vortex column (48^3 cubes x 6 tetrahedra, P2, LF), mixed precision,
    m = 30, CFL 10 (dt from eq. (x3d) at each step's u_n), `steps` PCEXP steps
    in one pcexp_advance call; then two profiled steps for the per-kernel
    event times (the FP32 JVP's algorithmic GB/s among them)."""
    import torch
    import workloads as W
    from paper_1801_06300_amd import PCEXP

    cfg = W.get_config("vortex3d_p2_48cube_lf")
    log("vortex3d: mesh and context")
    mesh = W.build_mesh(cfg)
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"], device=dev)
    xq = ctx.quad_points().cpu().numpy()
    c = cfg["vortex_center"]
    Uq = W.isentropic_vortex(xq.reshape(-1, 3), center=c, period=mesh.period).reshape(ctx.nE, ctx.nq, ctx.nv)
    u0 = ctx.project(torch.as_tensor(Uq, device=dev))
    u0 = (u0 + torch.as_tensor(W.perturbation(tuple(u0.shape), cfg["pert_seed"]), device=dev)).contiguous()
    del xq, Uq
    u = u0.clone()
    if warmup > 0:
        ctx.advance(u, warmup, cfl=cfg["cfl"], m=cfg["m"], prec="mixed")
    u = u0.clone()
    log(f"vortex3d: {steps} timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ctx.advance(u, steps, cfl=cfg["cfl"], m=cfg["m"], prec="mixed", info=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile("start")
    u = u0.clone()
    ctx.advance(u, 2, cfl=cfg["cfl"], m=cfg["m"], prec="mixed")
    prof = ctx.profile("read")
    ctx.profile("stop")
    kern = {k: dict(ms_total=v[0], launches=v[1], avg_us=(1e3 * v[0] / v[1]) if v[1] else 0.0,
                    gbs=(v[2] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else 0.0) for k, v in prof.items() if v[1]}
    out = dict(workload="3D isentropic vortex column, periodic [0,10]^3, 48^3 cubes x 6 tetrahedra (663552), "
                        "DG P2, LF, m=30, CFL 10 (dt from eq. x3d each step), mixed precision",
               K=ctx.K, steps=steps, warmup=warmup, ms_per_step=1e3 * wall / steps, dofs_per_s=ctx.K * steps / wall,
               t_advanced=info["t_advanced"], kernels=kern)
    del ctx, u, u0
    torch.cuda.empty_cache()
    return out


def bench_vortex3d(args, dev):
    steps = min(args.steps, 20)
    out = section_vortex3d(dev, steps, args.warmup)
    line = {
        "metric": "PCEXP DOF-updates/s (3D vortex, mixed)", "value": round(out["dofs_per_s"], 1),
        "unit": "DOF-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(out["ms_per_step"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": out["workload"], "K": out["K"]}, "vortex3d": out,
    }
    print(json.dumps(line))


def bench_reverse(args, ctx, u0, dt0, m, K):
    """The discrete adjoint of one PCEXP step of the headline workload
    (dt frozen from u_0, m = 30, FP64): step_vjp recomputes the forward step
    with both Krylov bases, then runs the reverse sweep.  Reports its time
    per call against a forward step with the same dt."""
    import torch
    import workloads as W

    ub = torch.as_tensor(W.random_unit_vector(tuple(u0.shape), 501), device=u0.device)
    log(f"reverse: {args.warmup} warm-up and {args.steps} timed reverse steps")
    for _ in range(max(args.warmup, 1)):
        ctx.step_vjp(u0, ub, dt0, m=m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = ctx.step_vjp(u0, ub, dt0, m=m)
    torch.cuda.synchronize()
    rev = (time.perf_counter() - t0) / args.steps
    u = u0.clone()
    ctx.step(u, dt=dt0, m=m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        u = u0.clone()
        ctx.step(u, dt=dt0, m=m)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / args.steps
    out = dict(metric="reverse (discrete adjoint) PCEXP step time", value=round(1e3 * rev, 4), unit="ms",
               n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=round(1e3 * rev, 4),
               higher_is_better=False, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload="discrete adjoint of one PCEXP step, 2D isentropic vortex 128x128x2 jittered, "
                                    "DG P2, Roe, m=30, dt frozen from u_0 (CFL 20), FP64", K=K, m=m),
               forward_ms_per_step=round(1e3 * fwd, 4), ratio_to_forward=round(rev / fwd, 4),
               gradient_norm=float(torch.linalg.norm(g)))
    print(json.dumps(out), flush=True)


def section_adjoint(dev, ctx, u0, dt_fixed):
    """Gradient of J(u_0) = sum_{n=1}^{40} dt int (p_h(t_n) - 1)^2 dx through 40
    PCEXP steps (dt frozen from u_0, m = 30, checkpoints every 8) on the
    headline mesh and state, behind torch.autograd: forward time, gradient
    (forward + reverse) time, their ratio, and the peak device memory the
    gradient call holds beyond what was allocated before it."""
    import torch
    import workloads as W
    from paper_1801_06300_amd.adjoint import Trajectory, objective

    cfg = W.get_config("adjoint_vortex2d_p2_128x128_roe")
    traj = Trajectory(ctx, dt_fixed, nsteps=cfg["steps"], m=cfg["m"], every=cfg["checkpoint_every"])
    log("adjoint: 40-step trajectory gradient")
    traj.value(u0)                                 # warm-up (allocations, kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    val = traj.value(u0)
    t_fwd = time.perf_counter() - t0
    x = u0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(dev)
    torch.cuda.reset_peak_memory_stats(dev)
    t0 = time.perf_counter()
    J = objective(traj)(x)
    J.backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    peak = torch.cuda.max_memory_allocated(dev) - base
    return dict(workload="gradient of sum_n dt int (p_h - 1)^2 through 40 PCEXP steps on the 128x128 P2 Roe vortex, "
                         "dt frozen from u_0 (CFL 20), m=30, checkpoints every 8, FP64, torch.autograd.Function",
                value=val, forward_s=t_fwd, gradient_s=t_grad, gradient_over_forward=t_grad / t_fwd,
                peak_bytes_beyond_inputs=int(peak),
                states_held=traj.peak_states())


def section_measurement(dev, ctx, u0):
    """Cold-cache standalone JVP and the measured copy bandwidth.  Each timed
    JVP launch follows a write of a 1 GiB buffer (larger than the 256 MB
    Infinity Cache and the L2s), so its inputs come from HBM; the kernel's
    own execution time comes from the library's event pair on its dispatch.
    The copy is a 1 GiB device-to-device copy timed with HIP events
    (2 GiB moved per copy)."""
    import torch
    import workloads as W

    out = {}
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    v = torch.as_tensor(W.random_unit_vector(tuple(u0.shape), 7), device=dev)
    for prec in ("f64", "mixed"):
        ctx.jvp(u0, v, "tangent", prec)
        ctx.profile("start")
        for i in range(10):
            flush.fill_(float(i))
            ctx.jvp(u0, v, "tangent", prec)
        prof = ctx.profile("read")
        ctx.profile("stop")
        ms, n, nbytes = prof["jvp"]
        out[f"jvp_cold_{prec}"] = dict(avg_us=1e3 * ms / n, launches=n, bytes_per_launch=nbytes / n,
                                       gbs=nbytes / (ms * 1e-3) / 1e9)
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    s = ev0.elapsed_time(ev1) / 1e3 / 10
    out["copy_1gib"] = dict(seconds=s, gbs=2 * src.numel() * 8 / s / 1e9,
                            note="read 1 GiB + write 1 GiB per copy; the measured-copy denominator")
    for k in ("jvp_cold_f64", "jvp_cold_mixed"):
        out[k]["frac_of_copy"] = out[k]["gbs"] / out["copy_1gib"]["gbs"]
        out[k]["frac_of_8tbs"] = out[k]["gbs"] / HBM_PEAK_GBS
    del flush, src, dst
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1801_06300_amd import PCEXP

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "channel":
        return bench_channel(args, dev)
    if args.workload == "stiffvortex":
        return bench_stiffvortex(args, dev)
    if args.workload == "vortex3d":
        return bench_vortex3d(args, dev)
    cfg = W.get_config("vortex2d_p2_128x128_jitter_roe")
    log("vortex2d: mesh and context")
    mesh = W.build_mesh(cfg)
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"], device=dev)
    K = ctx.K
    c = cfg["vortex_center"]
    xq = ctx.quad_points().cpu().numpy()
    Uq = W.isentropic_vortex(xq.reshape(-1, 2), center=c, period=mesh.period).reshape(ctx.nE, ctx.nq, ctx.nv)
    u0 = ctx.project(torch.as_tensor(Uq, device=dev))
    u0 = u0 + torch.as_tensor(W.perturbation(tuple(u0.shape), cfg["pert_seed"]), device=dev)
    u0 = u0.contiguous()
    cfl = cfg["cfl"]
    dt0 = ctx.stable_dt(u0, cfl)
    m = cfg["m"]
    steps, warm = args.steps, args.warmup
    if args.workload == "reverse":
        return bench_reverse(args, ctx, u0, dt0, m, K)

    def run(prec, jvp, nsteps, profile=False):
        # the steps of a timed region run through one pcexp_advance call: the
        # state stays in the internal basis between them, and each step takes
        # dt from eq. (x3d) at its own u_n (CFL 20) on the device
        u = u0.clone()
        if warm > 0:
            ctx.advance(u, warm, cfl=cfl, m=m, prec=prec, jvp=jvp)
        u = u0.clone()
        torch.cuda.synchronize()
        if profile:
            ctx.profile("start")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        info = ctx.advance(u, nsteps, cfl=cfl, m=m, prec=prec, jvp=jvp, info=True)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = None
        if profile:
            prof = ctx.profile("read")
            ctx.profile("stop")
        return u, wall, ev0.elapsed_time(ev1) / 1e3, prof, info["t_advanced"]

    log(f"vortex2d: {steps} timed FP64 tangent steps")
    u_t64, wall, gpu_s, _, tN = run("f64", "tangent", steps)
    value = K * steps / wall

    def err(u, t):
        # L2 (coefficient 2-norm) error against the projected exact solution: the vortex translated to time t
        Ue = W.isentropic_vortex(xq.reshape(-1, 2), t=t, center=c, period=mesh.period).reshape(ctx.nE, ctx.nq,
                                                                                               ctx.nv)
        ue = ctx.project(torch.as_tensor(Ue, device=dev))
        return float(torch.linalg.norm(u - ue).item())

    variants = {"t64": dict(dofs_per_s=value, ms_per_step=1e3 * wall / steps, t_final=tN, l2_error=err(u_t64, tN))}
    if not args.no_variants:
        for name, prec, jvp in (("fd64", "f64", "fd"), ("tmix", "mixed", "tangent")):
            log(f"vortex2d: variant {name}")
            u, w_s, _, _, t_v = run(prec, jvp, steps)
            variants[name] = dict(dofs_per_s=K * steps / w_s, ms_per_step=1e3 * w_s / steps, t_final=t_v,
                                  l2_error=err(u, t_v),
                                  rel_diff_vs_t64=float((torch.linalg.norm(u - u_t64) /
                                                         torch.linalg.norm(u_t64)).item()))

        # ETD2 (eq. (s7)) with dt fixed from u_0 (its difference quotient assumes a constant step);
        # the first step is ETD1, later ones use one step of history
        def run_etd2(nsteps):
            u = u0.clone()
            u_prev, r_prev = torch.empty_like(u0), torch.empty_like(u0)
            for i in range(warm):
                ctx.step_etd2(u, u_prev, r_prev, i > 0, dt0, m=m)
            u = u0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(nsteps):
                ctx.step_etd2(u, u_prev, r_prev, i > 0, dt0, m=m)
            torch.cuda.synchronize()
            return u, time.perf_counter() - t0

        log("vortex2d: variant etd2")
        u, w_s = run_etd2(steps)
        variants["etd2"] = dict(dofs_per_s=K * steps / w_s, ms_per_step=1e3 * w_s / steps, t_final=steps * dt0,
                                l2_error=err(u, steps * dt0),
                                rel_diff_vs_t64=float((torch.linalg.norm(u - u_t64) /
                                                       torch.linalg.norm(u_t64)).item()),
                                note="dt fixed from u_0")

    # reverse mode (discrete adjoint of one step, fixed dt): time per step_vjp vs forward step
    reverse = None
    if not args.no_variants:
        log("vortex2d: reverse step")
        ub = torch.as_tensor(W.random_unit_vector(tuple(u0.shape), 501), device=dev)
        ctx.step_vjp(u0, ub, dt0, m=m)
        torch.cuda.synchronize()
        nrev = 3
        t0 = time.perf_counter()
        for _ in range(nrev):
            ctx.step_vjp(u0, ub, dt0, m=m)
        torch.cuda.synchronize()
        rev_s = (time.perf_counter() - t0) / nrev
        reverse = dict(ms_per_step_vjp=1e3 * rev_s, ratio_to_forward=rev_s / (wall / steps),
                       workspace_bytes=int(ctx.lib.pcexp_step_vjp_workspace_bytes(ctx.ctx, m)),
                       note="recomputes the forward step with both Krylov bases, then the reverse sweep")

    # live per-kernel timing (HIP events on the step's stream) over a second timed region
    log("vortex2d: profiled steps")
    _, _, _, prof, _ = run("f64", "tangent", steps, profile=True)
    kern = {k: dict(ms_total=v[0], launches=v[1], avg_us=(1e3 * v[0] / v[1]) if v[1] else 0.0,
                    gbs=(v[2] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else 0.0) for k, v in prof.items() if v[1]}
    # dominant kernel: most GPU time among the kernels that move HBM bytes
    dom = max((k for k in prof if prof[k][2] > 0), key=lambda k: prof[k][0])
    d_ms, d_n, d_bytes = prof[dom]
    achieved = d_bytes / (d_ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic_per_launch(dom),
                    kernel=dom, hip_kernel=HIP_KERNELS[dom], launches=d_n, bytes_per_launch=d_bytes / d_n,
                    avg_launch_us=1e3 * d_ms / d_n)
    jv = prof["jvp"]
    jvp_gbs = jv[2] / (jv[0] * 1e-3) / 1e9 if jv[0] > 0 else 0.0

    out = {
        "metric": "PCEXP DOF-updates/s + JVP HBM GB/s; mixed tangent vs FP64 FD-JVP at equal error",
        "value": round(value, 1),
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(1e3 * wall / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D isentropic vortex, periodic [0,20]^2, 128x128x2 jittered triangles (32768), "
                               "DG P2, Roe, m=30, CFL 20 (dt from eq. x3d at each step's u_n), FP64 tangent JVP",
                   "K": K, "n_elem": ctx.nE, "p": cfg["p"], "flux": cfg["flux"], "m": m, "cfl": cfl,
                   "dt_first": dt0, "t_final": tN},
        "jvp_gbs": round(jvp_gbs, 1),
        "roofline": roofline,
        "variants": variants,
        "reverse": reverse,
        "kernels": kern,
        "gpu_event_seconds": gpu_s,
    }
    if args.calibrate_copy:
        out["copy_calibration_bytes"] = calibration_copy(dev)
    sections = set(args.sections.split(",")) if args.sections != "all" else {"measurement", "adjoint", "channel",
                                                                             "vortex3d"}
    if "measurement" in sections:
        log("measurement: cold-cache JVP and timed copy")
        out["measurement"] = section_measurement(dev, ctx, u0)
    if "adjoint" in sections:
        out["adjoint"] = section_adjoint(dev, ctx, u0, dt0)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, cfg, u0.cpu().numpy(), K)
    del ctx
    torch.cuda.empty_cache()
    if "channel" in sections:
        out["channel"] = section_channel(dev, max_iter=args.channel_iters)
    if "vortex3d" in sections:
        out["vortex3d"] = section_vortex3d(dev, 20, 2)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
