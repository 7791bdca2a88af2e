"""Gradient through 40 PCEXP steps at full size (the adjoint workload).

The 128^2 jittered P2 Roe vortex (K = 786 432), m = 30, dt frozen from
eq. (x3d) at u_0 with CFL 20, checkpoints every 8 steps, functional
J(u_0) = sum_{n=1}^{40} dt int (p_h(t_n) - 1)^2 dx.  The gradient comes from
the library's reverse sweep behind torch.autograd; each of 16 seeded
directions d_k (N(0,1) rescaled to |d_k| = |u_0|) is checked against the
central difference of the FP64 GPU forward sweep.

The functional is only piecewise smooth: the Roe flux without an entropy
fix has kinks where a wave speed changes sign (sonic points lie inside the
strength-5 vortex), and a perturbation h d of the whole state crosses the
kinks of every face point within h of one along the 40 steps.  The central
difference therefore converges to the derivative only as h -> 0, roughly
like h rather than h^2 (measured on this workload at 16 steps:
1.5e-2 at h = 1e-7, 2.5e-3 at 1e-8, 2.1e-5 at 1e-9, 1.2e-5 at 1e-10; at
40 steps 6.4e-2, 8.4e-4, 4.1e-6 for one direction), while the rounding of
the forward sweep adds about eps J / h (eps = 2^-52; 2e-5 relative at
h = 1e-10 for another direction, growing as h shrinks).  The gradient is the
same to the last bit for checkpoint intervals 2, 4, 8 and 16.  The
assertion uses h = 1e-10 with the bar 1e-4 |<g, d>| + 4 eps J / h; the
differences with h = 1e-9, 1e-6 and 1e-5 (and the Richardson combination
of the last two) are printed beside it.
"""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_trajectory_gradient_40_steps_full_size():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1801_06300_amd import PCEXP
    from paper_1801_06300_amd.adjoint import Trajectory, objective

    cfg = W.get_config("adjoint_vortex2d_p2_128x128_roe")
    mesh = W.build_mesh(cfg)
    print(f"\n[case] adjoint workload: nE={mesh.n_elem} P{cfg['p']} {cfg['flux']} m={cfg['m']} "
          f"steps={cfg['steps']} every={cfg['checkpoint_every']}", flush=True)
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"])
    xq = ctx.quad_points().cpu().numpy()
    c = cfg["vortex_center"]
    Uq = W.isentropic_vortex(xq.reshape(-1, 2), center=c, period=mesh.period).reshape(ctx.nE, ctx.nq, ctx.nv)
    u0 = ctx.project(torch.as_tensor(Uq, device="cuda"))
    u0 = (u0 + torch.as_tensor(W.perturbation(tuple(u0.shape), cfg["pert_seed"]), device="cuda")).contiguous()
    dt = ctx.stable_dt(u0, cfg["cfl"])
    traj = Trajectory(ctx, dt, nsteps=cfg["steps"], m=cfg["m"], every=cfg["checkpoint_every"])

    x = u0.clone().requires_grad_(True)
    J = objective(traj)(x)
    J.backward()
    g = x.grad.detach()
    val = float(J.detach())
    print(f"[adjoint] J = {val:.15e}", flush=True)
    assert np.isfinite(val) and val > 0.0
    # forward-only value is the same number
    assert traj.value(u0) == val

    nrm = float(torch.linalg.norm(u0))
    dirs = W.random_directions(cfg["n_dirs"], tuple(u0.shape), cfg["dir_seed"], norm=nrm)

    def f(d, e):
        return traj.value((u0 + e * d).contiguous())

    eps = 2.0 ** -52
    worst = 0.0
    for k in range(cfg["n_dirs"]):
        d = torch.as_tensor(dirs[k], device="cuda")
        D = {h: (f(d, h) - f(d, -h)) / (2 * h) for h in (1e-10, 1e-9, 1e-6, 1e-5)}
        rich = (100.0 * D[1e-6] - D[1e-5]) / 99.0
        gd = float(torch.sum(g * d))
        err = abs(gd - D[1e-10])
        bar = 1e-4 * abs(gd) + 4.0 * eps * val / 1e-10
        worst = max(worst, err / bar)
        print(f"[adjoint] dir {k:2d}: <g,d> {gd:.12e}  D(1e-10) {D[1e-10]:.12e} rel err {err / abs(gd):.2e} "
              f"(bar {bar / abs(gd):.1e})  |  D(1e-9) {abs(gd - D[1e-9]) / abs(gd):.1e}  D(1e-6) "
              f"{abs(gd - D[1e-6]) / abs(gd):.1e}  Richardson(1e-5, 1e-6) {abs(gd - rich) / abs(gd):.1e}",
              flush=True)
        assert err <= bar, (k, gd, D[1e-10])
    print(f"[adjoint] worst error / bar over {cfg['n_dirs']} directions at h = 1e-10: {worst:.2f}", flush=True)
