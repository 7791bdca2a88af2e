#!/usr/bin/env python3
"""PCEXP benchmark on one MI355X: DOF-updates/s of the PCEXP step on the 2D
isentropic-vortex workload (periodic [0,20]^2, 128x128 squares split into
32768 jittered triangles, DG P2, Roe flux, Krylov dimension m = 30, CFL 20).

A step is one full PCEXP step (both stages, two Arnoldi runs of m JVPs with
re-orthogonalised Gram-Schmidt, the device-side Hessenberg phi, the corrector)
through the C ABI; the timed steps run in one pcexp_advance call, which keeps
the state in the internal basis between steps.  Inputs are resident in HBM
before the timed region.

Prints one JSON line.  `value` is the FP64 tangent-JVP variant; the FP64
finite-difference JVP and the mixed FP32/FP64 tangent variants, and ETD2
(eq. (s7), FP64 tangent), are timed on the same workload and time levels and
reported in `variants` with their solution error.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--workload", default="vortex2d", choices=["vortex2d", "channel", "vortex3d", "stiffvortex"],
                    help="vortex2d: the headline PCEXP step benchmark; channel: steady bump channel to "
                         "||R(rho)|| <= 1e-10 with the CFL ramp; vortex3d: 3D P2 vortex, mixed precision")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(mesh, cfg, u0_np, K):
    """Time the FP64 oracle on a bounded sample of the same workload (about
    10 s on 16 cores): two residuals, 24 complex-step JVPs and the 30
    modified Gram-Schmidt projections of one late Arnoldi iteration, all at
    full size.  A PCEXP step costs 2 residuals + (2m+1) JVPs + two MGS
    Arnoldi runs (sum_{j<m} (j+1) projections each), from which seconds per
    step are extrapolated."""
    import numpy as np
    from oracle.dg import DG
    from oracle.derivatives import jvp_cs
    import workloads as W

    threads = len(os.sched_getaffinity(0))
    g = DG(mesh, cfg["p"], cfg["flux"])
    u = u0_np
    t0 = time.perf_counter()
    for _ in range(2):
        R = g.residual(u)
    t_res = (time.perf_counter() - t0) / 2
    v = W.random_unit_vector(u.shape, 1)
    njvp = 24
    t0 = time.perf_counter()
    for _ in range(njvp):
        jvp_cs(g, u, v)
    t_jvp = (time.perf_counter() - t0) / njvp
    m = cfg["m"]
    nproj = m
    Vb = np.random.default_rng(0).standard_normal((K, nproj))
    w = R.ravel().copy()
    t0 = time.perf_counter()
    for i in range(nproj):
        h = Vb[:, i] @ w
        w = w - h * Vb[:, i]
    t_proj = (time.perf_counter() - t0) / nproj
    t_gs = t_proj * (m * (m + 1) / 2)     # MGS of one Arnoldi run
    s_step = 2 * t_res + (2 * m + 1) * t_jvp + 2 * t_gs
    sample_s = 2 * t_res + njvp * t_jvp + nproj * t_proj
    return dict(value=K / s_step, unit="DOF-updates/s", cores=threads, kind="oracle",
                sample=(f"128x128 P2 vortex size, FP64 NumPy oracle, {sample_s:.1f} s measured: 2 residuals "
                        f"({t_res:.2f} s each), {njvp} complex-step JVPs ({t_jvp:.2f} s each), {nproj} MGS "
                        f"projections ({1e3 * t_proj:.1f} ms each); per step = 2 R + {2 * m + 1} JVP + "
                        f"2 Arnoldi MGS = {s_step:.1f} s extrapolated"),
                seconds_per_step=s_step)


def bench_channel(args, dev):
    """Steady subsonic channel over a Gaussian bump (384x128x2 jittered
    triangles, P2 Roe, Mach 0.5): pseudo-time PCEXP with the CFL ramp of
    eq. (cfl) (CFL_max 1000, m = 30) from the uniform free stream, in FP64
    and in mixed precision, for at most `--steps` pseudo-time steps or until
    ||R(rho)|| <= 1e-10.  With a fixed Krylov dimension this P2 case does not
    converge at the ramp's CFL (it does on small P1 channels); the line then
    reports the throughput and the residual reached."""
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
    res = {}
    for prec in ("f64", "mixed"):
        u = u0.clone()
        ctx.steady(u.clone(), cfl_max=cfg["cfl_max"], tol=1.0, max_iter=1, m=cfg["m"], prec=prec)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            info = ctx.steady(u, cfl_max=cfg["cfl_max"], tol=cfg["target_residual"], max_iter=args.steps,
                              check_every=10, m=cfg["m"], prec=prec)
        except PcexpError as e:
            res[prec] = dict(error=str(e))
            continue
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[prec] = dict(info, seconds=wall, ms_per_iteration=1e3 * wall / info["iterations"],
                         dofs_per_s=ctx.K * info["iterations"] / wall)
    main = res.get("mixed", {})
    out = {
        "metric": "PCEXP DOF-updates/s (steady channel, CFL ramp)",
        "value": round(main.get("dofs_per_s", 0.0), 1), "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": main.get("iterations", 0), "warmup": 1,
        "ms_per_step": round(main.get("ms_per_iteration", 0.0), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": "steady bump channel, 384x128x2 jittered triangles (98304), DG P2, Roe, "
                               "Mach 0.5, m=30, CFL ramp to 1000, mixed precision", "K": ctx.K},
        "runs": res,
    }
    print(json.dumps(out))


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


def bench_vortex3d(args, dev):
    """3D vortex column (48^3 cubes x 6 tetrahedra, P2, LF), mixed precision,
    m = 30, CFL 10 (dt from eq. (x3d) at u_0), `steps` PCEXP steps."""
    import torch
    import workloads as W
    from paper_1801_06300_amd import PCEXP

    cfg = W.get_config("vortex3d_p2_48cube_lf")
    mesh = W.build_mesh(cfg)
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"], device=dev)
    xq = ctx.quad_points().cpu().numpy()
    c = cfg["vortex_center"]
    Uq = W.isentropic_vortex(xq.reshape(-1, 3), center=c, period=mesh.period).reshape(ctx.nE, ctx.nq, ctx.nv)
    u0 = ctx.project(torch.as_tensor(Uq, device=dev))
    u0 = (u0 + torch.as_tensor(W.perturbation(tuple(u0.shape), cfg["pert_seed"]), device=dev)).contiguous()
    dt = ctx.stable_dt(u0, cfg["cfl"])
    steps = min(args.steps, cfg["steps"])
    u = u0.clone()
    if args.warmup > 0:
        ctx.advance(u, args.warmup, dt=dt, m=cfg["m"], prec="mixed")
    u = u0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(u, steps, dt=dt, m=cfg["m"], prec="mixed")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile("start")
    u = u0.clone()
    ctx.advance(u, 2, dt=dt, m=cfg["m"], prec="mixed")
    prof = ctx.profile("read")
    ctx.profile("stop")
    kern = {k: dict(ms_total=v[0], launches=v[1], avg_us=(1e3 * v[0] / v[1]) if v[1] else 0.0,
                    gbs=(v[2] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else 0.0) for k, v in prof.items() if v[1]}
    out = {
        "metric": "PCEXP DOF-updates/s (3D vortex, mixed)", "value": round(ctx.K * steps / wall, 1),
        "unit": "DOF-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": "3D isentropic vortex column, periodic [0,10]^3, 48^3 cubes x 6 tetrahedra "
                               "(663552), DG P2, LF, m=30, CFL 10, mixed precision", "K": ctx.K, "dt": dt},
        "kernels": kern,
    }
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
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
    mesh = W.build_mesh(cfg)
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"], device=dev)
    K = ctx.K
    L = mesh.period[0]
    c = cfg["vortex_center"]
    xq = ctx.quad_points().cpu().numpy()
    Uq = W.isentropic_vortex(xq.reshape(-1, 2), center=c, period=mesh.period).reshape(ctx.nE, ctx.nq, ctx.nv)
    u0 = ctx.project(torch.as_tensor(Uq, device=dev))
    u0 = u0 + torch.as_tensor(W.perturbation(tuple(u0.shape), cfg["pert_seed"]), device=dev)
    u0 = u0.contiguous()
    dt = ctx.stable_dt(u0, cfg["cfl"])
    m = cfg["m"]
    steps, warm = args.steps, args.warmup

    def run(prec, jvp, nsteps, profile=False):
        # the steps of a timed region run through pcexp_advance: the state stays
        # in the internal basis between them (one change of basis in and out)
        u = u0.clone()
        if warm > 0:
            ctx.advance(u, warm, dt=dt, m=m, prec=prec, jvp=jvp)
        u = u0.clone()
        torch.cuda.synchronize()
        if profile:
            ctx.profile("start")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        ctx.advance(u, nsteps, dt=dt, m=m, prec=prec, jvp=jvp)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = None
        if profile:
            prof = ctx.profile("read")
            ctx.profile("stop")
        return u, wall, ev0.elapsed_time(ev1) / 1e3, prof

    u_t64, wall, gpu_s, _ = run("f64", "tangent", steps)
    value = K * steps / wall

    # exact solution at t_N (translation of the vortex), projected; L2 error of the coefficients
    tN = steps * dt
    Ue = W.isentropic_vortex(xq.reshape(-1, 2), t=tN, center=c, period=mesh.period).reshape(ctx.nE, ctx.nq, ctx.nv)
    ue = ctx.project(torch.as_tensor(Ue, device=dev))

    def err(u):
        return float(torch.linalg.norm(u - ue).item())

    variants = {"t64": dict(dofs_per_s=value, ms_per_step=1e3 * wall / steps, l2_error=err(u_t64))}
    if not args.no_variants:
        for name, prec, jvp in (("fd64", "f64", "fd"), ("tmix", "mixed", "tangent")):
            u, w_s, _, _ = run(prec, jvp, steps)
            variants[name] = dict(dofs_per_s=K * steps / w_s, ms_per_step=1e3 * w_s / steps, l2_error=err(u),
                                  rel_diff_vs_t64=float((torch.linalg.norm(u - u_t64) /
                                                         torch.linalg.norm(u_t64)).item()))
        # ETD2 (eq. (s7)) on the same time levels: the first step is ETD1, later ones use one step of history
        def run_etd2(nsteps):
            u = u0.clone()
            u_prev, r_prev = torch.empty_like(u0), torch.empty_like(u0)
            for i in range(warm):
                ctx.step_etd2(u, u_prev, r_prev, i > 0, dt, m=m)
            u = u0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(nsteps):
                ctx.step_etd2(u, u_prev, r_prev, i > 0, dt, m=m)
            torch.cuda.synchronize()
            return u, time.perf_counter() - t0

        u, w_s = run_etd2(steps)
        variants["etd2"] = dict(dofs_per_s=K * steps / w_s, ms_per_step=1e3 * w_s / steps, l2_error=err(u),
                                rel_diff_vs_t64=float((torch.linalg.norm(u - u_t64) /
                                                       torch.linalg.norm(u_t64)).item()))

    # reverse mode (discrete adjoint of one step, fixed dt): time per step_vjp vs forward step
    reverse = None
    if not args.no_variants:
        ub = torch.as_tensor(W.random_unit_vector(tuple(u0.shape), 501), device=dev)
        ctx.step_vjp(u0, ub, dt, m=m)
        torch.cuda.synchronize()
        nrev = 3
        t0 = time.perf_counter()
        for _ in range(nrev):
            ctx.step_vjp(u0, ub, dt, m=m)
        torch.cuda.synchronize()
        rev_s = (time.perf_counter() - t0) / nrev
        reverse = dict(ms_per_step_vjp=1e3 * rev_s, ratio_to_forward=rev_s / (wall / steps),
                       workspace_bytes=int(ctx.lib.pcexp_step_vjp_workspace_bytes(ctx.ctx, m)),
                       note="recomputes the forward step with both Krylov bases, then the reverse sweep")

    # live per-kernel timing (HIP events on the step's stream) over a second timed region
    _, _, _, prof = run("f64", "tangent", steps, profile=True)
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
                               "DG P2, Roe, m=30, CFL 20 (dt from eq. x3d at u_0), FP64 tangent JVP",
                   "K": K, "n_elem": ctx.nE, "p": cfg["p"], "flux": cfg["flux"], "m": m, "cfl": cfg["cfl"],
                   "dt": dt},
        "jvp_gbs": round(jvp_gbs, 1),
        "roofline": roofline,
        "variants": variants,
        "reverse": reverse,
        "kernels": kern,
        "gpu_event_seconds": gpu_s,
    }
    if args.calibrate_copy:
        # plain copy kernel of known size: 1 GiB read + 1 GiB written per launch
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8, "launches": 3}
        del src, dst
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, cfg, u0.cpu().numpy(), K)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
