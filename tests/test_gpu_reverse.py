"""Reverse mode on the GPU (pcexp_vjp2, pcexp_step_vjp, the checkpointed
trajectory) against oracle derivatives and difference quotients.

Tolerances: the oracle's second-order and step derivatives come from
Richardson-extrapolated central differences (error ~1e-10 relative on these
states, see tests/test_oracle_adjoint.py); the GPU results are compared at
1e-8.  The dense linear operator has an exact complex-step reference (1e-11).
"""

import numpy as np
import pytest

import workloads as W
from oracle import adjoint
from oracle.dg import DG
from oracle.derivatives import jvp_cs
from oracle.diagnostics import pressure_fluctuation
from oracle.integrators import DenseSplit, ExactJacobian, stable_dt
from tests.helpers import mesh_case, vortex_state, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1801_06300_amd import PCEXP
    return PCEXP


def _pair(name, p, flux, amp=1e-3):
    """Cube meshes get a free stream with w != 0: with w = 0 the z-face normal
    velocity sits on the kink of |v.n| and difference quotients of second
    derivatives straddle it."""
    PCEXP = _dev()
    m, ang = mesh_case(name)
    prim = W.freestream_prim(m.dim, angle_deg=ang)
    print(f"\n[case] mesh={name} p={p} flux={flux} nE={m.n_elem}", flush=True)
    g = DG(m, p, flux, farfield_prim=prim)
    ctx = PCEXP(m, p, flux, farfield_prim=prim)
    u = vortex_state(g, m, amp, uinf=(0.42, 0.42, 0.3) if m.dim == 3 else None)
    return g, ctx, u


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _n(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,p,flux,full", [("sq3", 1, "lf", True), ("sq3", 2, "roe", True),
                                              ("chan", 1, "roe", True), ("cube3", 1, "roe", False),
                                              ("cube3", 2, "roe", False), ("chan", 2, "roe", False)])
def test_vjp2_parity(name, p, flux, full):
    """Value part = pcexp_vjp (pinned against the dense oracle Jacobian in
    test_gpu_parity); second-order part against the oracle: the whole vector
    (dense-Jacobian route) on small 2D meshes, and projections
    <z, d/de J(u+ev)^T w> = <w, d/de J(u+ez) v> (JVP route) everywhere.
    Difference quotients of the second derivative are meaningful only away
    from the flux's non-smooth points; the LF flux's max(a_L, a_R) switches
    sides within the difference step wherever the two speeds nearly agree,
    so LF is checked on the coarse 2D mesh only.  The JVP route uses a
    smaller step (1e-5) than the dense route: on the channel P2 state a step
    of 1e-4 crosses a sign change of a wave speed at some face point."""
    g, ctx, u = _pair(name, p, flux)
    v = W.random_unit_vector(u.shape, 21)
    w = W.random_unit_vector(u.shape, 22)
    JTw, dJTw = ctx.vjp2(_t(u), _t(v), _t(w))
    assert rel(_n(ctx.vjp(_t(u), _t(w))), _n(JTw)) < 1e-14
    k6 = _n(dJTw)
    if full:
        assert rel(k6, adjoint.vjp2_fd(g, u, v, w)) < 1e-7
    for seed in (23, 24):
        z = W.random_unit_vector(u.shape, seed)
        want = float(np.sum(w * adjoint.richardson(lambda e: jvp_cs(g, u + e * z, v), 1e-5)))
        assert abs(float(np.sum(z * k6)) - want) < 1e-7 * max(abs(want), np.linalg.norm(k6) * 1e-3)


@pytest.mark.parametrize("n,m", [(20, 6), (20, 20), (80, 40), (80, 64)])
@pytest.mark.parametrize("scheme", ["pcexp", "exp1"])
def test_step_vjp_dense(n, m, scheme):
    """Linear split operator: <ubar, D d> with D d exact by complex step.
    With n = 80 the Arnoldi runs reach m = 40 and 64 without breakdown, so
    the reverse sweep's dot passes take more than 32 basis vectors (chunks)
    and its coefficient sums more than 32 columns."""
    PCEXP = _dev()
    rng = np.random.default_rng(7)
    A = rng.standard_normal((n, n)) / 2 - 2 * np.eye(n)
    B = rng.standard_normal((n, n)) / 2 - 1.5 * np.eye(n)
    ctx = PCEXP.dense(A, B)
    op = DenseSplit(A, B)
    u = rng.standard_normal(n)
    ub = rng.standard_normal(n)
    gb = _n(ctx.step_vjp(_t(u), _t(ub), 0.35, m=m, scheme=scheme))
    for k in range(3):
        d = rng.standard_normal(n)
        Dd = adjoint.step_derivative_cs(op, u, d, 0.35, m, scheme)
        lhs, rhs = float(ub @ Dd), float(gb @ d)
        assert abs(lhs - rhs) < 1e-11 * np.linalg.norm(ub) * np.linalg.norm(Dd)


@pytest.mark.parametrize("name,p,flux,m", [("sq4j", 1, "roe", 8), ("sq3", 2, "lf", 10), ("chan", 1, "roe", 8),
                                           ("cube3", 1, "roe", 6), ("cube3", 1, "lf", 6), ("cube3", 2, "lf", 6)])
def test_step_vjp_dg(name, p, flux, m):
    """<ubar, D d> against Richardson differences of the oracle's step (the
    3D cases run the second-order kernel's accumulating form on tetrahedra;
    on these states the projected differences with h = 1e-4, 1e-5, 1e-6
    agree to about 1e-10 of |D d|)."""
    g, ctx, u = _pair(name, p, flux)
    dt = stable_dt(g, u, 4.0)
    op = ExactJacobian(g)
    ub = W.random_unit_vector(u.shape, 31)
    gb = _n(ctx.step_vjp(_t(u), _t(ub), dt, m=m))
    for seed in (32, 33):
        d = W.random_unit_vector(u.shape, seed)
        Dd = adjoint.step_derivative_fd(op, u, d, dt, m)
        lhs, rhs = float(np.sum(ub * Dd)), float(np.sum(gb * d))
        assert abs(lhs - rhs) < 1e-8 * np.linalg.norm(Dd), (lhs, rhs)


def test_step_vjp_exp1_dg():
    g, ctx, u = _pair("sq4j", 1, "roe")
    dt = stable_dt(g, u, 4.0)
    op = ExactJacobian(g)
    ub = W.random_unit_vector(u.shape, 41)
    d = W.random_unit_vector(u.shape, 42)
    gb = _n(ctx.step_vjp(_t(u), _t(ub), dt, m=8, scheme="exp1"))
    Dd = adjoint.step_derivative_fd(op, u, d, dt, 8, "exp1")
    assert abs(float(np.sum(ub * Dd)) - float(np.sum(gb * d))) < 1e-8 * np.linalg.norm(Dd)


def test_pressure_functional_parity():
    g, ctx, u = _pair("sq4j", 2, "roe")
    val, grad = ctx.pressure_functional(_t(u), 1.0, grad=True)
    want = pressure_fluctuation(g, u, 1.0)
    assert abs(val - want) < 1e-12 * abs(want)
    d = W.random_unit_vector(u.shape, 51)
    cs = np.imag(pressure_fluctuation(g, u + 1e-30j * d, 1.0)) / 1e-30
    assert abs(float(np.sum(_n(grad) * d)) - cs) < 1e-11 * max(abs(cs), 1e-12)


def test_pressure_functional_acc_parity():
    """value_acc += s P(u) and grad_acc += s dP/du on the device, against the
    oracle's functional and its complex-step derivative; two calls in a row
    accumulate."""
    g, ctx, u = _pair("sq4j", 2, "roe")
    ud = _t(u)
    val = torch.full((), 0.5, dtype=torch.float64, device="cuda")
    r0 = W.random_unit_vector(u.shape, 52)
    grad = _t(r0)
    s = 0.3
    ctx.pressure_functional_acc(ud, s, 1.0, value_acc=val, grad_acc=grad)
    ctx.pressure_functional_acc(ud, -0.1, 1.0, value_acc=val)
    P = pressure_fluctuation(g, u, 1.0)
    assert abs(float(val) - (0.5 + 0.2 * P)) < 1e-12 * abs(0.5 + 0.2 * P)
    d = W.random_unit_vector(u.shape, 51)
    cs = np.imag(pressure_fluctuation(g, u + 1e-30j * d, 1.0)) / 1e-30
    got = float(np.sum((_n(grad) - r0) * d)) / s
    assert abs(got - cs) < 1e-11 * max(abs(cs), 1e-12)
    with pytest.raises(Exception):
        ctx.pressure_functional_acc(ud, s, 1.0)            # nothing to accumulate
    with pytest.raises(Exception):
        ctx.pressure_functional_acc(ud, s, 1.0, grad_acc=ud)  # aliasing


def test_trajectory_gradient_checkpointed():
    """Gradient of sum_n dt int (p - 1)^2 over 5 steps with checkpoints every
    2 steps, against the oracle's Richardson derivative of the same sum."""
    from paper_1801_06300_amd.adjoint import Trajectory, objective
    g, ctx, u = _pair("sq4j", 1, "roe")
    dt = stable_dt(g, u, 4.0)
    traj = Trajectory(ctx, dt, nsteps=5, m=8, every=2)
    val, grad = traj.value_and_grad(_t(u))
    op = ExactJacobian(g)
    want = adjoint.trajectory_functional(g, op, u, dt, 8, 5)
    assert abs(val - want) < 1e-11 * abs(want)
    d = W.random_unit_vector(u.shape, 61)
    fd = adjoint.richardson(lambda e: adjoint.trajectory_functional(g, op, u + e * d, dt, 8, 5), 1e-4)
    assert abs(float(np.sum(_n(grad) * d)) - fd) < 1e-7 * max(abs(fd), 1e-12)
    # the same through torch.autograd
    x = _t(u).requires_grad_(True)
    J = objective(traj)(x)
    J.backward()
    assert rel(_n(x.grad), _n(grad)) < 1e-14


def test_step_vjp_full_size():
    """The 128^2 jittered P2 Roe vortex (m = 30, CFL 20), directions
    scaled to |d| = |u_0|: difference quotients of the GPU step against the
    reverse, for PCEXP and EXP1.  Along such directions the step is strongly
    curved (the central difference with h = 1e-6 is off by ~2e-5 relative,
    converging as h^2 down to h ~ 3e-8), so the assertion uses the
    Richardson-extrapolated central difference with h = 2e-7, 1e-7."""
    PCEXP = _dev()
    cfg = W.get_config("vortex2d_p2_128x128_jitter_roe")
    mesh = W.build_mesh(cfg)
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"])
    xq = _n(ctx.quad_points())
    c = cfg["vortex_center"]
    Uq = W.isentropic_vortex(xq.reshape(-1, 2), center=c, period=mesh.period).reshape(ctx.nE, ctx.nq, ctx.nv)
    u0 = ctx.project(_t(Uq))
    u0 = (u0 + _t(W.perturbation(tuple(u0.shape), cfg["pert_seed"]))).contiguous()
    dt = ctx.stable_dt(u0, cfg["cfl"])
    ub = _t(W.random_unit_vector(tuple(u0.shape), 501))
    for scheme in ("pcexp", "exp1"):
        gb = ctx.step_vjp(u0, ub, dt, m=30, scheme=scheme)
        for seed in (502, 503):
            d = _t(W.random_unit_vector(tuple(u0.shape), seed)) * torch.linalg.norm(u0)

            def f(e):
                x = (u0 + e * d).contiguous()
                ctx.step(x, dt=dt, m=30, scheme=scheme)
                return float(torch.sum(ub * x))

            rich = adjoint.richardson(f, 2e-7)
            rhs = float(torch.sum(gb * d))
            print(f"[full] {scheme} seed {seed}: Richardson {rich:.12e} reverse {rhs:.12e}", flush=True)
            assert abs(rich - rhs) < 1e-6 * abs(rich)
