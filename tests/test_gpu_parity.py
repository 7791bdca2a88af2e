"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 tolerance: 1e-11 relative (2-norm over the whole vector) unless a
derived bound is stated.  Every case prints its name, mesh, degree and flux
before touching the GPU.
"""

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG
from oracle import krylov
from oracle.derivatives import jvp_cs, jvp_fd, dense_jacobian
from oracle.integrators import pcexp_step, heun_step, ExactJacobian, DenseSplit, stable_dt
from oracle.diagnostics import conserved_totals
from tests.helpers import mesh_case, vortex_state, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1801_06300_amd import PCEXP
    return PCEXP


def _pair(name, p, flux, amp=1e-6, uinf=None):
    PCEXP = _dev()
    m, ang = mesh_case(name)
    prim = W.freestream_prim(m.dim, angle_deg=ang)
    print(f"\n[case] mesh={name} p={p} flux={flux} nE={m.n_elem}", flush=True)
    g = DG(m, p, flux, farfield_prim=prim)
    ctx = PCEXP(m, p, flux, farfield_prim=prim)
    u = vortex_state(g, m, amp, uinf=uinf)
    return g, ctx, u


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _n(t):
    return t.detach().cpu().numpy()


CASES = [("sq3", 1, "lf"), ("sq4j", 2, "roe"), ("sq4j", 3, "lf"), ("sq3", 0, "roe"),
         ("cube3", 1, "lf"), ("cube3", 2, "roe"), ("chan", 2, "roe"), ("chan", 1, "lf"),
         ("box3", 1, "roe"), ("box3", 2, "lf"), ("cube3", 0, "lf"), ("box3", 0, "roe")]


@pytest.mark.parametrize("name,p,flux", CASES)
def test_residual_parity(name, p, flux):
    g, ctx, u = _pair(name, p, flux, amp=1e-3)
    R = _n(ctx.residual(_t(u)))
    Ro = g.residual(u)
    assert rel(R, Ro) < 1e-11
    assert np.max(np.abs(R - Ro)) < 1e-11 * np.max(np.abs(Ro))


@pytest.mark.parametrize("name,p,flux", [("sq4j", 2, "roe"), ("cube3", 2, "lf"), ("chan", 2, "roe")])
def test_quadrature_projection_evaluation(name, p, flux):
    g, ctx, u = _pair(name, p, flux)
    xq = _n(ctx.quad_points())
    xo = g.quad_points()
    assert np.max(np.abs(xq - xo)) < 1e-13 * max(1.0, np.abs(xo).max())
    m = g.m
    if m.period[0] > 0:
        f = lambda x: W.isentropic_vortex(x, center=(5.0, 5.0), period=m.period)
    else:
        f = lambda x: W.uniform_state(x, W.freestream_prim(2, angle_deg=0.0)) * (1 + 0.1 * np.sin(x[:, :1]))
    Uq = f(xq.reshape(-1, g.d)).reshape(g.nE, g.Nq, g.nv)
    up = _n(ctx.project(_t(Uq)))
    assert rel(up, g.project(f)) < 1e-12
    Ue = _n(ctx.evaluate(_t(u)))
    assert rel(Ue, g.evaluate(u)) < 1e-12


@pytest.mark.parametrize("name,p,flux", CASES)
def test_tangent_jvp_parity(name, p, flux):
    g, ctx, u = _pair(name, p, flux, amp=1e-3)
    v = W.random_unit_vector(u.shape, 7)
    Jv = _n(ctx.jvp(_t(u), _t(v), "tangent", "f64"))
    assert rel(Jv, jvp_cs(g, u, v)) < 1e-11


@pytest.mark.parametrize("name,p,flux", [("sq4j", 2, "roe"), ("cube3", 1, "lf"), ("chan", 2, "roe"),
                                         ("cube3", 2, "lf"), ("box3", 2, "roe")])
def test_fd_jvp_parity(name, p, flux):
    """FD JVP against the oracle's FD JVP (same eps formula).  The two residual
    evaluations differ by a few ulps of R, amplified by 1/eps:
    |dFD| <~ 8 u_R |R| / eps, bounded here by 1e-7 relative."""
    g, ctx, u = _pair(name, p, flux, amp=1e-3)
    v = W.random_unit_vector(u.shape, 8)
    fd = _n(ctx.jvp(_t(u), _t(v), "fd", "f64"))
    assert rel(fd, jvp_fd(g, u, v)) < 1e-7
    assert rel(fd, jvp_cs(g, u, v)) < 1e-5


@pytest.mark.parametrize("name,p,flux", [("sq4j", 2, "roe"), ("cube3", 2, "lf"), ("chan", 2, "roe"),
                                         ("box3", 2, "roe")])
def test_mixed_jvp_bound(name, p, flux):
    """FP32 tangent JVP against the FP64 oracle: stated bound 1e-5 relative."""
    g, ctx, u = _pair(name, p, flux, amp=1e-3)
    v = W.random_unit_vector(u.shape, 9)
    Jv = _n(ctx.jvp(_t(u), _t(v), "tangent", "mixed"))
    assert rel(Jv, jvp_cs(g, u, v)) < 1e-5


@pytest.mark.parametrize("name,p,flux", [("sq3", 1, "roe"), ("sq3", 2, "lf"), ("cube3", 1, "roe"),
                                         ("chan", 1, "roe"), ("box3", 1, "lf"), ("sq3", 0, "lf"),
                                         ("sq3", 3, "roe"), ("cube3", 0, "roe")])
def test_vjp_parity(name, p, flux):
    g, ctx, u = _pair(name, p, flux, amp=1e-3)
    w = W.random_unit_vector(u.shape, 10)
    v = W.random_unit_vector(u.shape, 11)
    JTw = _n(ctx.vjp(_t(u), _t(w)))
    J = dense_jacobian(g, u)
    assert rel(JTw.ravel(), J.T @ w.ravel()) < 1e-11
    Jv = _n(ctx.jvp(_t(u), _t(v)))
    lhs, rhs = float(np.sum(w * Jv)), float(np.sum(JTw * v))
    assert abs(lhs - rhs) < 1e-12 * max(np.linalg.norm(w) * np.linalg.norm(Jv), 1.0)


@pytest.mark.parametrize("name,p,flux", [("cube3", 2, "lf"), ("box3", 2, "roe")])
def test_vjp_parity_sampled_3d_p2(name, p, flux):
    """J^T w on the 3D P2 meshes (8100 unknowns, where a dense oracle Jacobian
    takes minutes) against the oracle through the adjoint identity on six
    seeded directions: <J^T w, v_k> = <w, J v_k>, with J v_k the oracle's
    complex-step JVP (exact to rounding), at 1e-11 of |J^T w| |v_k|."""
    g, ctx, u = _pair(name, p, flux, amp=1e-3)
    w = W.random_unit_vector(u.shape, 10)
    JTw = _n(ctx.vjp(_t(u), _t(w)))
    scale = np.linalg.norm(JTw)
    for seed in range(30, 36):
        v = W.random_unit_vector(u.shape, seed)
        want = float(np.sum(w * jvp_cs(g, u, v)))
        got = float(np.sum(JTw * v))
        assert abs(got - want) < 1e-11 * scale * np.linalg.norm(v), (seed, got, want)


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("jvp", ["tangent", "fd"])
def test_arnoldi_phi_parity(k, jvp):
    g, ctx, u = _pair("sq4j", 2, "roe")
    b = g.residual(u)
    dt = stable_dt(g, u, 5.0)
    out, info = ctx.arnoldi_phi(_t(u), _t(b), dt, k=k, m=12, jvp=jvp, info=True)
    op = ExactJacobian(g, "exact" if jvp == "tangent" else "fd")
    Rn = g.residual(u)
    want, oinfo = krylov.arnoldi_phi(lambda x: op.jvp(u, x.reshape(u.shape), Rn), b, dt, k, 12,
                                     return_info=True)
    tol = 1e-11 if jvp == "tangent" else 1e-6
    assert rel(_n(out), want) < tol
    assert info["m_eff"] == oinfo["m_eff"] == 12
    assert abs(info["beta"] - oinfo["beta"]) < 1e-13 * oinfo["beta"]


def test_arnoldi_phi_vs_dense_dg():
    """Krylov phi_1 on the tiny-mesh DG Jacobian with m = 40 equals the dense phi_1."""
    g, ctx, u = _pair("sq3", 1, "lf")
    J = dense_jacobian(g, u)
    b = g.residual(u)
    dt = stable_dt(g, u, 2.0)
    out = _n(ctx.arnoldi_phi(_t(u), _t(b), dt, k=1, m=40))
    want = krylov.dense_phi(J, b.ravel(), dt, 1).reshape(u.shape)
    assert rel(out, want) < 1e-11


@pytest.mark.parametrize("m,prec", [(64, "f64"), (48, "mixed"), (33, "f64")])
def test_arnoldi_phi_long_basis(m, prec):
    """Bases beyond one 32-vector chunk of the fused Gram-Schmidt pass."""
    g, ctx, u = _pair("sq4j", 2, "roe")
    b = g.residual(u)
    dt = stable_dt(g, u, 5.0)
    out, info = ctx.arnoldi_phi(_t(u), _t(b), dt, k=1, m=m, prec=prec, info=True)
    want, oinfo = krylov.arnoldi_phi(lambda x: jvp_cs(g, u, x.reshape(u.shape)), b, dt, 1, m,
                                     return_info=True)
    assert info["m_eff"] == oinfo["m_eff"] == m
    assert rel(_n(out), want) < (1e-10 if prec == "f64" else 1e-5)


def test_arnoldi_phi_large_mesh_separate_reduction():
    """Above 4096 tiles the Arnoldi reduction is a pass of its own rather than
    part of the JVP launch: 294 x 294 x 2 jittered triangles, P1 LF (4116 FP64
    tangent tiles), m = 8, against the oracle; the bytes of the reduction
    class show which path ran (the separate pass reads j + 2 vectors per
    iteration, the column sums of the fused path about a megabyte)."""
    PCEXP = _dev()
    m = W.periodic_square(294, 20.0, 0.15, 31)
    print(f"\n[case] mesh=sq294j p=1 flux=lf nE={m.n_elem}", flush=True)
    g = DG(m, 1, "lf")
    ctx = PCEXP(m, 1, "lf")
    u = vortex_state(g, m, 1e-3)
    b = g.residual(u)
    dt = stable_dt(g, u, 5.0)
    ud, bd = _t(u), _t(b)
    ctx.arnoldi_phi(ud, bd, dt, k=1, m=8)
    torch.cuda.synchronize()
    ctx.profile("start")
    out, info = ctx.arnoldi_phi(ud, bd, dt, k=1, m=8, info=True)
    torch.cuda.synchronize()
    prof = ctx.profile("read")
    ctx.profile("stop")
    vec_bytes = 8.0 * u.size
    # separate passes: sum_{j<8} (j + 2) + 9 (closing) = 53 vectors; fused: 9 plus column sums
    assert prof["gs_reduce"][2] > 30 * vec_bytes, prof["gs_reduce"]
    want, oinfo = krylov.arnoldi_phi(lambda x: jvp_cs(g, u, x.reshape(u.shape)), b, dt, 1, 8,
                                     return_info=True)
    assert info["m_eff"] == oinfo["m_eff"] == 8
    assert rel(_n(out), want) < 1e-11


def test_arnoldi_phi_zero_vector_and_mixed():
    g, ctx, u = _pair("sq4j", 2, "roe")
    out, info = ctx.arnoldi_phi(_t(u), _t(np.zeros_like(u)), 0.1, k=1, m=5, info=True)
    assert info["m_eff"] == 0 and np.all(_n(out) == 0)
    b = g.residual(u)
    dt = stable_dt(g, u, 5.0)
    out = _n(ctx.arnoldi_phi(_t(u), _t(b), dt, k=1, m=12, prec="mixed"))
    want = krylov.arnoldi_phi(lambda x: jvp_cs(g, u, x.reshape(u.shape)), b, dt, 1, 12)
    assert rel(out, want) < 1e-5


# ------------------------------------------------------------- dense operators
def test_dense_split_model_growth():
    """1x1 split operator through the device stepper: eq. (grow), eq. (exp1_grow)."""
    PCEXP = _dev()
    for a in (-3.0, -0.7, 0.4):
        for b in (-6.0, -1.3, 0.25, 1.5):
            ctx = PCEXP.dense([[b]], [[a + b]])
            u = torch.ones(1, dtype=torch.float64, device="cuda")
            ctx.step(u, dt=1.0, m=1)
            printed = (a * (a - b) + np.exp(2 * b) * (a + b) * a + 2 * np.exp(b) * (b * b - a * a)) / (2 * b * b)
            assert abs(u.item() - printed) < 1e-12 * max(1, abs(printed))
            u = torch.ones(1, dtype=torch.float64, device="cuda")
            ctx.step(u, dt=1.0, m=1, scheme="exp1")
            assert abs(u.item() - (a * (np.exp(b) - 1) + b * np.exp(b)) / b) < 1e-12 * max(1, abs(u.item()))


@pytest.mark.parametrize("n", [20, 21])
def test_dense_linear_exactness_and_breakdown(n):
    """n = 21: an odd vector length exercises the unpaired last entry of the
    two-entries-per-lane Gram-Schmidt passes."""
    from scipy.linalg import expm
    PCEXP = _dev()
    rng = np.random.default_rng(4)
    A = rng.standard_normal((n, n)) - 4 * np.eye(n)
    u0 = rng.standard_normal(n)
    ctx = PCEXP.dense(A, A)
    u = _t(u0)
    info = ctx.step(u, dt=0.4, m=n, info=True)
    want = expm(0.4 * A) @ u0
    assert rel(_n(u), want) < 1e-12
    # nilpotent shift: the Krylov space of e_6 has dimension 6 -> breakdown, exact result
    N = np.diag(np.ones(5), 1)
    ctx = PCEXP.dense(N, N)
    b = np.zeros(6)
    b[-1] = 1.0
    out, info = ctx.arnoldi_phi(_t(np.zeros(6)), _t(b), 1.0, k=1, m=20, info=True)
    assert info["breakdown"] and info["m_eff"] == 6
    assert np.allclose(_n(out), krylov.dense_phi(N, b, 1.0, 1), atol=1e-14)


def test_dense_overflow_terminates():
    """An operator whose Krylov quantities overflow (|Jv|^2 = inf, so H gets
    infinite entries) still returns from the step: the scaling exponent of
    the small-matrix exponential is bounded for an infinite norm."""
    from paper_1801_06300_amd import PcexpError
    PCEXP = _dev()
    print("\n[case] dense overflow n=6", flush=True)
    rng = np.random.default_rng(7)
    A = 1e300 * rng.standard_normal((6, 6))
    ctx = PCEXP.dense(A, A)
    u = _t(rng.standard_normal(6))
    try:
        ctx.step(u, dt=1.0, m=4)
        torch.cuda.synchronize()
        assert not np.all(np.isfinite(_n(u)))
    except PcexpError:
        pass


def test_dense_phi_closed_forms():
    """Diagonal operator: phi_k closed forms through the device phi kernel."""
    from math import factorial
    PCEXP = _dev()
    z = np.array([-40.0, -7.5, -1.0, -1e-3, 0.5, 2.0])
    b = np.linspace(0.5, 1.5, z.size)
    dt = 0.7
    ctx = PCEXP.dense(np.diag(z / dt), np.diag(z / dt))
    for k in (0, 1, 2, 3):
        out = _n(ctx.arnoldi_phi(_t(np.zeros_like(b)), _t(b), dt, k=k, m=10))
        small = np.abs(z) < 1e-2
        ph = np.where(small, sum(z ** j / factorial(j + k) for j in range(12)),
                      (np.exp(z) - sum(z ** j / factorial(j) for j in range(k))) / np.where(small, 1, z) ** k)
        assert np.all(np.abs(out - ph * b) <= 1e-12 * np.abs(ph * b) + 1e-14)


# ------------------------------------------------------------------- stepping
def test_step_parity_16x16_p1_ten_steps():
    """16x16 periodic mesh, P1, LF, m = 20, CFL 5: 10 PCEXP steps."""
    g, ctx, u0 = _pair("sq16", 1, "lf")
    op = ExactJacobian(g)
    u_o = u0.copy()
    u_d = _t(u0)
    for n in range(10):
        dt = stable_dt(g, u_o, 5.0)
        u_o = pcexp_step(op, u_o, dt, 20)
        info = ctx.step(u_d, cfl=5.0, m=20, info=True)
        assert abs(info["dt"] - dt) < 1e-13 * dt
        assert rel(_n(u_d), u_o) < 1e-11, n
    assert info["k1"]["m_eff"] == 20 and info["flags"] == 0


@pytest.mark.parametrize("scheme,jvp,prec,tol", [("exp1", "tangent", "f64", 1e-11),
                                                  ("pcexp", "fd", "f64", 1e-8),
                                                  ("pcexp", "tangent", "mixed", 1e-5),
                                                  ("pcexp", "zero", "f64", 1e-13)])
def test_step_variants(scheme, jvp, prec, tol):
    """FP64 variants: the state at the FP64 bar (FD: its O(sqrt(eps)) JVP
    error).  Mixed precision: the one-step increment u_{n+1} - u_n at the
    stated 1e-5 relative bound."""
    g, ctx, u0 = _pair("sq4j", 2, "roe")
    dt = stable_dt(g, u0, 5.0)
    if jvp == "zero":
        want = heun_step(ExactJacobian(g), u0, dt)
    else:
        want = pcexp_step(ExactJacobian(g, "exact" if jvp != "fd" else "fd"), u0, dt, 12, scheme=scheme)
    u = _t(u0)
    ctx.step(u, dt=dt, m=12, scheme=scheme, jvp=jvp, prec=prec)
    if prec == "mixed":
        err = rel(_n(u) - u0, want - u0)
        print(f"[mixed] one-step increment rel err {err:.3e} (bound {tol:.0e})", flush=True)
        assert err < tol
    else:
        assert rel(_n(u), want) < tol


def test_mixed_precision_stated_bounds_ten_steps():
    """Mixed precision against the FP64 oracle at the stated bounds, on the
    16x16 P1 LF vortex (m = 20, CFL 5, 10 steps): every one-step increment,
    taken from the oracle's own u_n, within 1e-5 relative of the oracle's;
    the device's own 10-step trajectory within 1e-6 relative of the oracle's
    final state."""
    g, ctx, u0 = _pair("sq16", 1, "lf")
    op = ExactJacobian(g)
    u_o = u0.copy()
    u_d = _t(u0)
    worst_inc = 0.0
    for n in range(10):
        dt = stable_dt(g, u_o, 5.0)
        nxt = pcexp_step(op, u_o, dt, 20)
        one = _t(u_o)
        ctx.step(one, dt=dt, m=20, prec="mixed")
        e_inc = rel(_n(one) - u_o, nxt - u_o)
        worst_inc = max(worst_inc, e_inc)
        ctx.step(u_d, cfl=5.0, m=20, prec="mixed")
        u_o = nxt
    e_state = rel(_n(u_d), u_o)
    print(f"[mixed] worst one-step increment rel err {worst_inc:.3e} (bound 1e-5); "
          f"10-step state rel err {e_state:.3e} (bound 1e-6)", flush=True)
    assert worst_inc < 1e-5
    assert e_state < 1e-6


@pytest.mark.parametrize("p", [1, 2])
def test_supersonic_farfield_parity(p):
    """Both supersonic branches of the Riemann-invariant far field: a Mach 1.5
    stream along x through the 12x4 bump channel whose top is also a far
    field, so the left faces take the exterior state (supersonic inflow),
    the right faces the interior state (supersonic outflow) and the top faces
    the subsonic characteristic state.  Residual and tangent JVP at 1e-11."""
    PCEXP = _dev()
    m = W.channel_bump(12, 4, height=0.1, seed=5, top_bc=W.BC_FARFIELD)
    prim = W.freestream_prim(2, mach=1.5, angle_deg=0.0)
    print(f"\n[case] supersonic far field: 12x4 channel, Mach 1.5, p={p}", flush=True)
    g = DG(m, p, "roe", farfield_prim=prim)
    ctx = PCEXP(m, p, "roe", farfield_prim=prim)
    u = g.project(lambda x: W.uniform_state(x, prim))
    u = u + W.perturbation(u.shape, 17, 1e-3)
    # the branches are exercised: |v.n| > c on the left and right boundary faces
    c_inf = np.sqrt(1.4 * prim[-1] / prim[0])
    assert prim[1] / c_inf > 1.4 and abs(prim[2]) < 1e-15
    R = _n(ctx.residual(_t(u)))
    Ro = g.residual(u)
    print(f"[super] residual rel {rel(R, Ro):.3e}", flush=True)
    assert rel(R, Ro) < 1e-11
    v = W.random_unit_vector(u.shape, 18)
    Jd = _n(ctx.jvp(_t(u), _t(v), "tangent", "f64"))
    Jo = jvp_cs(g, u, v)
    print(f"[super] tangent JVP rel {rel(Jd, Jo):.3e}", flush=True)
    assert rel(Jd, Jo) < 1e-11


def test_step_conservation_and_determinism():
    g, ctx, u0 = _pair("sq8j", 2, "roe")
    q0 = ctx.conserved_totals(_t(u0))
    assert np.allclose(q0, conserved_totals(g, u0), rtol=1e-13, atol=1e-13)
    a, b = _t(u0), _t(u0)
    for _ in range(5):
        ctx.step(a, cfl=10.0, m=15)
        ctx.step(b, cfl=10.0, m=15)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    q1 = ctx.conserved_totals(a)
    assert np.max(np.abs(q1 - q0) / np.abs(q0).max()) < 1e-13


@pytest.mark.parametrize("name,p,flux", [("sq4j", 2, "roe"), ("cube3", 2, "lf"), ("box3", 1, "roe")])
def test_stable_dt_parity(name, p, flux):
    g, ctx, u = _pair(name, p, flux)
    assert abs(ctx.stable_dt(_t(u), 3.0) - stable_dt(g, u, 3.0)) < 1e-14 * stable_dt(g, u, 3.0)


@pytest.mark.parametrize("name,p,flux,scheme", [("cube3", 2, "lf", "pcexp"), ("box3", 2, "roe", "pcexp"),
                                                ("box3", 1, "lf", "pcexp"), ("cube3", 2, "roe", "exp1")])
def test_step_parity_3d(name, p, flux, scheme):
    """One FP64 PCEXP (or EXP1) step (m = 10, CFL 5) on the 3^3 x 6
    tetrahedral meshes, periodic and bounded, against the oracle's step at
    1e-11."""
    g, ctx, u0 = _pair(name, p, flux, amp=1e-3)
    dt = stable_dt(g, u0, 5.0)
    want = pcexp_step(ExactJacobian(g), u0, dt, 10, scheme=scheme)
    u = _t(u0)
    ctx.step(u, dt=dt, m=10, scheme=scheme)
    print(f"[3d step] state rel {rel(_n(u), want):.2e}, increment rel {rel(_n(u) - u0, want - u0):.2e}", flush=True)
    assert rel(_n(u), want) < 1e-11
    assert rel(_n(u) - u0, want - u0) < 1e-10


def test_unphysical_flag():
    """A state with negative pressure is reported by the next synchronising call."""
    from paper_1801_06300_amd import PcexpError
    g, ctx, u = _pair("sq3", 1, "lf")
    bad = u.copy()
    bad[0, -1, :] = -1.0     # negative total energy in element 0
    R = ctx.residual(_t(bad))
    with pytest.raises(PcexpError):
        ctx.step(_t(bad), dt=0.01, m=4, info=True)


def test_advance_parity():
    """pcexp_advance: N steps with one change of basis in and out equal the
    oracle's N steps (fixed dt; dt from eq. (x3d) at every step; EXP1) and N
    calls of pcexp_step up to the rounding of the basis changes."""
    from paper_1801_06300_amd import PcexpError
    g, ctx, u0 = _pair("sq4j", 2, "roe")
    op = ExactJacobian(g)
    dt = stable_dt(g, u0, 5.0)
    want = u0
    for _ in range(3):
        want = pcexp_step(op, want, dt, 12)
    a = _t(u0)
    ctx.advance(a, 3, dt=dt, m=12)
    assert rel(_n(a), want) < 1e-11
    b = _t(u0)
    for _ in range(3):
        ctx.step(b, dt=dt, m=12)
    assert rel(_n(a), _n(b)) < 1e-13
    want = u0
    for _ in range(3):
        want = pcexp_step(op, want, stable_dt(g, want, 5.0), 12)
    c = _t(u0)
    info = ctx.advance(c, 3, cfl=5.0, m=12, info=True)
    assert rel(_n(c), want) < 1e-11 and info["flags"] == 0
    want = u0
    for _ in range(2):
        want = pcexp_step(op, want, dt, 12, scheme="exp1")
    d = _t(u0)
    ctx.advance(d, 2, dt=dt, m=12, scheme="exp1")
    assert rel(_n(d), want) < 1e-11
    with pytest.raises(PcexpError):
        ctx.advance(_t(u0), 0, dt=dt, m=12)


@pytest.mark.parametrize("prec,jvp", [("f64", "fd"), ("mixed", "tangent")])
def test_advance_matches_steps_other_paths(prec, jvp):
    """pcexp_advance with the finite-difference JVP and in mixed precision:
    N steps in one call against N calls of pcexp_step (the same kernels; only
    the per-call changes of basis differ, and their rounding reaches the FD
    quotient amplified by 1/eps and the FP32 copies of the state as a flipped
    last bit), and against the oracle's steps with the same operator.  Bars
    are those of the single-step variant test: FD 1e-8 on the state (a
    rounding of u by the basis change, ~1e-16, moves the FD quotient by about
    1e-16 / eps ~ 1e-8 relative; measured 1.3e-9 between the two forms), mixed
    1e-4 on the increment."""
    g, ctx, u0 = _pair("sq4j", 2, "roe")
    op = ExactJacobian(g, "fd" if jvp == "fd" else "exact")
    dt = stable_dt(g, u0, 5.0)
    want = u0
    for _ in range(3):
        want = pcexp_step(op, want, dt, 12)
    a = _t(u0)
    ctx.advance(a, 3, dt=dt, m=12, prec=prec, jvp=jvp)
    b = _t(u0)
    for _ in range(3):
        ctx.step(b, dt=dt, m=12, prec=prec, jvp=jvp)
    if prec == "mixed":
        assert rel(_n(a) - u0, _n(b) - u0) < 1e-5
        assert rel(_n(a) - u0, want - u0) < 1e-4
    else:
        assert rel(_n(a), _n(b)) < 1e-8
        assert rel(_n(a), want) < 1e-8


def test_step_argument_errors_on_a_live_context():
    """The step entry point's argument checks on a live context: each bad
    request is rejected on the host with its status before anything is
    launched (the state is untouched), and the context keeps working."""
    import ctypes
    from paper_1801_06300_amd import PcexpError
    g, ctx, u = _pair("sq3", 1, "lf")
    ud = _t(u)
    lib, st = ctx.lib, ctx._stream()

    def step(m, prec=0, jvp=0, ws=None, nbytes=None, x=ud):
        if ws is None:
            ws, nb = ctx.workspace(min(max(m, 1), 64), 1, "f64", "tangent")
            nbytes = nb if nbytes is None else nbytes
        return lib.pcexp_step(ctx.ctx, ctypes.c_void_p(x.data_ptr()), ctypes.c_double(0.01), ctypes.c_double(0.0),
                              m, 0, prec, jvp, ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(nbytes), None, st)

    before = ud.clone()
    assert step(0) == -1 and step(65) == -1                     # m outside [1, 64]
    ws, nb = ctx.workspace(8, 1, "f64", "tangent")
    assert step(8, ws=ws, nbytes=nb - 8) == -4                  # workspace too small
    assert step(8, ws=ws[1:], nbytes=nb) == -4                  # misaligned workspace
    assert step(8, prec=1, jvp=1) == -7                         # FD JVP in mixed precision
    assert step(8, prec=5) == -1 and step(8, jvp=9) == -1       # unknown precision / JVP kind
    torch.cuda.synchronize()
    assert torch.equal(ud, before)
    with pytest.raises(PcexpError):
        ctx.step(ud, dt=0.01, m=65)
    want = pcexp_step(ExactJacobian(g), u, 0.01, 8)
    ctx.step(ud, dt=0.01, m=8)
    assert rel(_n(ud), want) < 1e-11


# ------------------------------------------------------------------ ETD2
def _etd2_oracle(op, u0, dt, m, nsteps):
    from oracle.integrators import etd2_step
    u, up, Rp = np.array(u0), None, None
    for _ in range(nsteps):
        unew, Rn = etd2_step(op, u, up, Rp, dt, m)
        up, Rp, u = u, Rn, unew
    return u, up, Rp


def test_step_etd2_parity_dense():
    """Three ETD2 steps (eq. (s7); the first is ETD1) on a split operator whose
    part outside J makes the scheme inexact; the history buffers hold u_n and
    R(u_n) afterwards."""
    PCEXP = _dev()
    print("\n[case] etd2 dense n=24", flush=True)
    rng = np.random.default_rng(31)
    n = 24
    A = rng.standard_normal((n, n)) / np.sqrt(n) - 2.0 * np.eye(n)
    B = 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    u0 = rng.standard_normal(n)
    ctx = PCEXP.dense(A, A + B)
    u, up, rp = _t(u0), _t(np.zeros(n)), _t(np.zeros(n))
    for i in range(3):
        ctx.step_etd2(u, up, rp, i > 0, 0.25, m=20)
    want, wup, wrp = _etd2_oracle(DenseSplit(A, A + B), u0, 0.25, 20, 3)
    assert rel(_n(u), want) < 1e-12
    assert rel(_n(up), wup) < 1e-13 and rel(_n(rp), wrp) < 1e-12


@pytest.mark.parametrize("name,p,flux", [("sq4j", 2, "roe"), ("cube3", 2, "lf")])
def test_step_etd2_parity_dg(name, p, flux):
    """Three ETD2 steps with the tangent JVP on the jittered 4x4 P2 Roe vortex
    and on the 3^3 x 6 tetrahedral P2 LF vortex."""
    from oracle.integrators import stable_dt
    g, ctx, u = _pair(name, p, flux, amp=1e-3)
    dt = stable_dt(g, u, 5.0)
    ud, up, rp = _t(u), _t(np.zeros_like(u)), _t(np.zeros_like(u))
    for i in range(3):
        info = ctx.step_etd2(ud, up, rp, i > 0, dt, m=30, info=True)
    print(f"[etd2] m_eff {info['k1']['m_eff']}/{info['k2']['m_eff']}", flush=True)
    want, wup, wrp = _etd2_oracle(ExactJacobian(g), u, dt, 30, 3)
    assert rel(_n(ud), want) < 1e-10
    assert rel(_n(up), wup) < 1e-12 and rel(_n(rp), wrp) < 1e-10
