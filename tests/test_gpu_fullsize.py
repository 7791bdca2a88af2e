"""Forward parity at the full 2D workload size, in the launch configuration
the throughput benchmark times: isentropic vortex on the 128 x 128 x 2
jittered periodic triangle mesh, DG P2, Roe flux, m = 30, CFL 20, FP64
tangent JVP (the variants: FD JVP and FP32 tangent).

At this size the oracle needs about 1 s per residual and 1.5 s per JVP, so
the residual and JVP are compared over the whole vector, and one PCEXP step
(61 oracle JVPs, about 80 s on one core) is compared over the whole vector
too.  The oracle's initial state is handed to the device, never the other way
round.  Tolerances: 1e-11 relative for FP64 JVPs and the step (the
small-mesh bar).  The residual of this smooth, nearly steady vortex is a small
difference of flux terms, so summation-order rounding is large relative to it:
the residual of the uniform free stream (zero in exact arithmetic, same flux
magnitudes) measures that noise on this mesh (4e-11 of the vortex residual in
the 2-norm), and the residual bar is ten times that ratio.  The FD
and FP32 variants against the exact-Jacobian oracle step use 1e-4 relative on
the increment u_{n+1} - u_n, the bar the small-mesh variant tests use for
FP32, which also bounds the FD JVP's O(sqrt(eps)) error after it passes
through phi_1.
"""

import sys

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG
from oracle.derivatives import jvp_cs, jvp_fd
from oracle.integrators import pcexp_step, ExactJacobian, stable_dt
from oracle.diagnostics import conserved_totals
from tests.helpers import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_CACHE = {}


def _full():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    if "g" not in _CACHE:
        from paper_1801_06300_amd import PCEXP
        cfg = W.get_config("vortex2d_p2_128x128_jitter_roe")
        print(f"\n[case] {cfg['name']} m={cfg['m']} cfl={cfg['cfl']}", flush=True)
        mesh = W.build_mesh(cfg)
        g = DG(mesh, cfg["p"], cfg["flux"])
        c = cfg["vortex_center"]
        u0 = g.project(lambda x: W.isentropic_vortex(x, center=c, period=mesh.period))
        u0 = u0 + W.perturbation(u0.shape, cfg["pert_seed"])
        R0 = g.residual(u0)
        u_fs = g.project(lambda x: W.uniform_state(x, W.freestream_prim(2)))
        R_fs = g.residual(u_fs)
        floor2 = np.linalg.norm(R_fs) / np.linalg.norm(R0)
        floorm = np.abs(R_fs).max() / np.abs(R0).max()
        _CACHE.update(cfg=cfg, g=g, u0=u0, R0=R0, ctx=PCEXP(mesh, cfg["p"], cfg["flux"]),
                      dt=stable_dt(g, u0, cfg["cfl"]), tol_r=max(1e-11, 10 * floor2),
                      tol_rmax=max(1e-11, 10 * floorm))
    return _CACHE


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _n(t):
    return t.detach().cpu().numpy()


class _Progress(ExactJacobian):
    """The oracle's exact-Jacobian operator, printing a line every ten JVPs so
    that the long oracle step shows it is running.  With `capsys` the lines
    bypass pytest's output capture (a long step must not look silent)."""

    def __init__(self, dg, capsys=None):
        super().__init__(dg)
        self.calls = 0
        self.capsys = capsys

    def jvp(self, u_lin, v, R_lin=None):
        self.calls += 1
        if self.calls % 10 == 0:
            if self.capsys is not None:
                with self.capsys.disabled():
                    print(f"[oracle] {self.calls} JVPs", flush=True)
            else:
                print(f"[oracle] {self.calls} JVPs", flush=True)
            sys.stdout.flush()
        return super().jvp(u_lin, v, R_lin)


def _oracle_step():
    c = _full()
    if "step" not in c:
        info = {}
        c["step"] = pcexp_step(_Progress(c["g"]), c["u0"], c["dt"], c["cfg"]["m"], info=info)
        c["step_info"] = info
    return c["step"], c["step_info"]


def test_fullsize_residual_and_jvps():
    c = _full()
    g, ctx, u0 = c["g"], c["ctx"], c["u0"]
    assert ctx.nE == g.nE == 32768
    ud = _t(u0)
    Ro = c["R0"]
    R = _n(ctx.residual(ud))
    print(f"[full] residual rel {rel(R, Ro):.3e} (bar {c['tol_r']:.2e}), max "
          f"{np.max(np.abs(R - Ro)) / np.max(np.abs(Ro)):.3e} (bar {c['tol_rmax']:.2e})", flush=True)
    assert rel(R, Ro) < c["tol_r"]
    assert np.max(np.abs(R - Ro)) < c["tol_rmax"] * np.max(np.abs(Ro))
    v = W.random_unit_vector(u0.shape, 7)
    vd = _t(v)
    Jo = jvp_cs(g, u0, v)
    Jt = _n(ctx.jvp(ud, vd, "tangent", "f64"))
    print(f"[full] tangent JVP rel {rel(Jt, Jo):.3e}", flush=True)
    assert rel(Jt, Jo) < 1e-11
    Jm = _n(ctx.jvp(ud, vd, "tangent", "mixed"))
    print(f"[full] FP32 tangent JVP rel {rel(Jm, Jo):.3e}", flush=True)
    assert rel(Jm, Jo) < 1e-5
    Jf = _n(ctx.jvp(ud, vd, "fd", "f64"))
    Jfo = jvp_fd(g, u0, v)
    print(f"[full] FD JVP rel {rel(Jf, Jfo):.3e} (vs exact {rel(Jf, Jo):.3e})", flush=True)
    assert rel(Jf, Jfo) < 1e-7
    assert rel(Jf, Jo) < 1e-5


def test_fullsize_residual_perturbed_state():
    """The residual of the full-size vortex plus a seeded 1e-3 perturbation of
    every coefficient: the perturbation's flux differences are not small
    against the flux terms, so summation-order rounding stays below the FP64
    bar of 1e-11 here (the bar the smooth state needs is the floor-derived
    one of test_fullsize_residual_and_jvps, printed beside it)."""
    c = _full()
    g, ctx, u0 = c["g"], c["ctx"], c["u0"]
    u1 = u0 + W.perturbation(u0.shape, 7, 1e-3)
    Ro = g.residual(u1)
    R = _n(ctx.residual(_t(u1)))
    e = rel(R, Ro)
    print(f"[full] perturbed-state residual rel {e:.3e} (bar 1e-11; smooth-state floor bar {c['tol_r']:.2e})",
          flush=True)
    assert e < 1e-11


def test_fullsize_stable_dt():
    c = _full()
    dt = c["ctx"].stable_dt(_t(c["u0"]), c["cfg"]["cfl"])
    assert abs(dt - c["dt"]) < 1e-14 * c["dt"]


@pytest.mark.timeout(900)
def test_fullsize_pcexp_step():
    """One PCEXP step, FP64 tangent JVP, m = 30: whole-vector parity, the
    Krylov dimensions and flags, conservation of the totals, and that the
    step took the fused JVP + reduction path."""
    c = _full()
    want, oinfo = _oracle_step()
    ctx, u0 = c["ctx"], c["u0"]
    u = _t(u0)
    torch.cuda.synchronize()
    ctx.profile("start")
    info = ctx.step(u, dt=c["dt"], m=c["cfg"]["m"], info=True)
    torch.cuda.synchronize()
    prof = ctx.profile("read")
    ctx.profile("stop")
    got = _n(u)
    # the Arnoldi reduction ran inside the JVP launches (1171 tiles): the
    # reduction class holds only column sums and the two closing passes
    vec = 8.0 * u0.size
    assert prof["gs_reduce"][2] < 100 * vec and prof["jvp"][2] > 61 * 3 * vec, prof
    print(f"[full] step rel {rel(got, want):.3e}, increment rel {rel(got - u0, want - u0):.3e}", flush=True)
    assert rel(got, want) < 1e-11
    assert rel(got - u0, want - u0) < 1e-9
    assert info["flags"] == 0
    assert info["k1"]["m_eff"] == oinfo["k1"]["m_eff"] == c["cfg"]["m"]
    q0 = conserved_totals(c["g"], u0)
    q1 = conserved_totals(c["g"], got)
    assert np.max(np.abs(q1 - q0)) < 1e-12 * np.abs(q0).max()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("jvp,prec", [("fd", "f64"), ("tangent", "mixed")])
def test_fullsize_step_variants(jvp, prec):
    c = _full()
    want, _ = _oracle_step()
    u0 = c["u0"]
    u = _t(u0)
    c["ctx"].step(u, dt=c["dt"], m=c["cfg"]["m"], prec=prec, jvp=jvp)
    got = _n(u)
    r = rel(got - u0, want - u0)
    print(f"[full] {jvp}/{prec} step: increment rel {r:.3e}", flush=True)
    assert r < 1e-4


def test_fullsize_step_determinism():
    """Two runs of the same step on the device agree bit for bit."""
    c = _full()
    a, b = _t(c["u0"]), _t(c["u0"])
    for x in (a, b):
        c["ctx"].step(x, dt=c["dt"], m=c["cfg"]["m"])
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.timeout(900)
def test_fullsize_channel():
    """The steady bump channel at full size (384 x 128 x 2 jittered triangles,
    P2 Roe, slip walls and Riemann-invariant far field).  Residual, the three
    JVPs and Dt over the whole vector at the free stream plus a 1e-3 seeded
    perturbation (a residual of O(1e3), well above its rounding level); one
    EXP1 step with m = 10 at CFL 5 from the free stream plus a 1e-6
    perturbation, a step that moves the state by 0.2 % and halves the
    residual (its JVP launches, 3511 tiles, carry the fused Arnoldi
    reduction).  That residual, O(10), is a small difference of wall flux
    terms, so its rounding is ~1e-11 of it: the step is compared on the state
    (1e-11) and on the increment with 1e-9."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1801_06300_amd import PCEXP
    cfg = W.get_config("channel_bump_p2_384x128")
    print(f"\n[case] {cfg['name']}", flush=True)
    mesh = W.build_mesh(cfg)
    prim = W.freestream_prim(2, mach=cfg["mach"], angle_deg=cfg["angle_deg"])
    g = DG(mesh, cfg["p"], cfg["flux"], farfield_prim=prim)
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"], farfield_prim=prim)
    ufs = g.project(lambda x: W.uniform_state(x, prim))
    u0 = ufs + W.perturbation(ufs.shape, 307, 1e-3)
    ud = _t(u0)
    Ro = g.residual(u0)
    R = _n(ctx.residual(ud))
    print(f"[full] channel residual rel {rel(R, Ro):.3e}", flush=True)
    assert rel(R, Ro) < 1e-11
    v = W.random_unit_vector(u0.shape, 309)
    vd = _t(v)
    Jo = jvp_cs(g, u0, v)
    Jt = _n(ctx.jvp(ud, vd, "tangent", "f64"))
    Jm = _n(ctx.jvp(ud, vd, "tangent", "mixed"))
    Jf = _n(ctx.jvp(ud, vd, "fd", "f64"))
    print(f"[full] channel JVP rel: tangent {rel(Jt, Jo):.3e}, FP32 {rel(Jm, Jo):.3e}, "
          f"FD {rel(Jf, jvp_fd(g, u0, v)):.3e}", flush=True)
    assert rel(Jt, Jo) < 1e-11
    assert rel(Jm, Jo) < 1e-5
    assert rel(Jf, jvp_fd(g, u0, v)) < 1e-7
    u1 = ufs + W.perturbation(ufs.shape, 311, 1e-6)
    dt = stable_dt(g, u1, 5.0)
    assert abs(ctx.stable_dt(_t(u1), 5.0) - dt) < 1e-14 * dt
    want = pcexp_step(_Progress(g), u1, dt, 10, scheme="exp1")
    u = _t(u1)
    ctx.step(u, dt=dt, m=10, scheme="exp1")
    got = _n(u)
    print(f"[full] channel EXP1 step rel {rel(got, want):.3e}, increment rel {rel(got - u1, want - u1):.3e}",
          flush=True)
    assert rel(got, want) < 1e-11
    assert rel(got - u1, want - u1) < 1e-9


def test_fullsize_3d_properties():
    """The 3D vortex column at full size (48^3 cubes x 6 tetrahedra, P2 LF),
    in the launch configuration of the 3D benchmark, through properties that
    hold at any size (the oracle needs minutes per residual here; parity on
    a 16^3 mesh is test_3d_16cube_parity): free-stream preservation,
    conservation of the residual, of both JVPs and of a mixed-precision PCEXP
    step (m = 30, CFL 10) on the periodic mesh, exact doubling of the FP64
    tangent under a doubled direction, and bitwise determinism of the step."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1801_06300_amd import PCEXP
    cfg = W.get_config("vortex3d_p2_48cube_lf")
    print(f"\n[case] {cfg['name']}", flush=True)
    mesh = W.build_mesh(cfg)
    ctx = PCEXP(mesh, cfg["p"], cfg["flux"])
    xq = _n(ctx.quad_points()).reshape(-1, 3)
    Uq = W.isentropic_vortex(xq, center=cfg["vortex_center"], period=mesh.period).reshape(ctx.nE, ctx.nq, ctx.nv)
    u0 = ctx.project(_t(Uq))
    u0 = (u0 + _t(W.perturbation(tuple(u0.shape), cfg["pert_seed"]))).contiguous()
    ufs = ctx.project(_t(W.uniform_state(xq, W.freestream_prim(3)).reshape(ctx.nE, ctx.nq, ctx.nv))).contiguous()

    def cons(x):
        tot = np.asarray(ctx.conserved_totals(x.contiguous()))
        scale = np.asarray(ctx.conserved_totals(x.abs().contiguous()))
        return np.max(np.abs(tot) / scale)

    R0 = ctx.residual(u0)
    Rfs = ctx.residual(ufs)
    fs = float(torch.linalg.norm(Rfs) / torch.linalg.norm(R0))
    print(f"[full] 3d free stream |R|/|R_vortex| {fs:.2e}, residual conservation {cons(R0):.2e}", flush=True)
    assert fs < 1e-9
    assert cons(R0) < 1e-11
    v = _t(W.random_unit_vector(tuple(u0.shape), 17))
    Jt = ctx.jvp(u0, v, "tangent", "f64")
    Jm = ctx.jvp(u0, v, "tangent", "mixed")
    print(f"[full] 3d JVP conservation: FP64 {cons(Jt):.2e}, FP32 {cons(Jm.double()):.2e}", flush=True)
    assert cons(Jt) < 1e-11
    assert cons(Jm.double()) < 1e-5
    assert rel(_n(Jm.double()), _n(Jt)) < 1e-5
    J2 = ctx.jvp(u0, (2.0 * v).contiguous(), "tangent", "f64")
    assert torch.equal(J2, 2.0 * Jt)
    dt = ctx.stable_dt(u0, cfg["cfl"])
    q0 = np.asarray(ctx.conserved_totals(u0))
    a, b = u0.clone(), u0.clone()
    info = ctx.step(a, dt=dt, m=cfg["m"], prec="mixed", info=True)
    ctx.step(b, dt=dt, m=cfg["m"], prec="mixed")
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert info["flags"] == 0
    q1 = np.asarray(ctx.conserved_totals(a))
    dq = np.max(np.abs(q1 - q0) / np.abs(q0).max())
    print(f"[full] 3d mixed step: conserved totals drift {dq:.2e}, m_eff {info['k1']['m_eff']}", flush=True)
    assert dq < 1e-6


@pytest.mark.timeout(900)
def test_3d_16cube_parity():
    """3D vortex column on 16^3 cubes x 6 tetrahedra (24 576), P2 LF, against
    the oracle over the whole vector: residual, FP64 and FP32 tangent JVPs,
    and Arnoldi phi_1 with m = 5 (its JVP launches carry the fused
    reduction: 3511 FP64 tiles).  The FP32 bar is the small-mesh one (1e-5
    at 3 cubes per side) scaled with 1/h: the JVP is a difference of flux
    terms of size 1/h times its result, and FP32 rounding is relative to
    those terms."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1801_06300_amd import PCEXP
    from tests.helpers import vortex_state
    from oracle import krylov
    mesh = W.periodic_cube(16, 10.0)
    print(f"\n[case] mesh=cube16 p=2 flux=lf nE={mesh.n_elem}", flush=True)
    g = DG(mesh, 2, "lf", cache_limit=1e8)     # tables cached: 3 s per oracle JVP
    ctx = PCEXP(mesh, 2, "lf")
    u = vortex_state(g, mesh, 1e-3)
    ud = _t(u)
    Ro = g.residual(u)
    R = _n(ctx.residual(ud))
    v = W.random_unit_vector(u.shape, 19)
    Jo = jvp_cs(g, u, v)
    Jt = _n(ctx.jvp(ud, _t(v), "tangent", "f64"))
    Jm = _n(ctx.jvp(ud, _t(v), "tangent", "mixed"))
    print(f"[full] cube16 residual {rel(R, Ro):.2e}, JVP FP64 {rel(Jt, Jo):.2e}, FP32 {rel(Jm, Jo):.2e}", flush=True)
    assert rel(R, Ro) < 1e-11
    assert rel(Jt, Jo) < 1e-11
    assert rel(Jm, Jo) < 1e-5 * 16 / 3
    dt = stable_dt(g, u, 5.0)
    out = _n(ctx.arnoldi_phi(ud, _t(Ro), dt, k=1, m=5))
    want = krylov.arnoldi_phi(lambda x: jvp_cs(g, u, x.reshape(u.shape)), Ro, dt, 1, 5)
    print(f"[full] cube16 Arnoldi phi_1 (m = 5) {rel(out, want):.2e}", flush=True)
    assert rel(out, want) < 1e-11


@pytest.mark.timeout(1200)
def test_3d_16cube_mixed_pcexp_step(capsys):
    """One mixed-precision PCEXP step (m = 30, CFL 10) of the 3D vortex column
    on 16^3 cubes x 6 tetrahedra (24 576, P2 LF, K = 1 228 800) against the
    FP64 oracle's step (61 complex-step JVPs on the host) over the whole
    vector: the state at 1e-6 relative and the increment u_{n+1} - u_n at
    the stated 1e-5 relative."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1801_06300_amd import PCEXP
    from tests.helpers import vortex_state
    mesh = W.periodic_cube(16, 10.0)
    print(f"\n[case] mesh=cube16 p=2 flux=lf nE={mesh.n_elem}: mixed PCEXP step, m=30", flush=True)
    g = DG(mesh, 2, "lf", cache_limit=1e8)     # tables cached: 3 s per oracle JVP
    ctx = PCEXP(mesh, 2, "lf")
    u = vortex_state(g, mesh, 1e-6)
    dt = stable_dt(g, u, 10.0)
    ud = _t(u)
    info = ctx.step(ud, dt=dt, m=30, prec="mixed", info=True)
    got = _n(ud)
    want = pcexp_step(_Progress(g, capsys), u, dt, 30)
    e_state, e_inc = rel(got, want), rel(got - u, want - u)
    print(f"[full] cube16 mixed PCEXP step: state rel {e_state:.3e} (bar 1e-6), increment rel {e_inc:.3e} "
          f"(bar 1e-5), m_eff {info['k1']['m_eff']}/{info['k2']['m_eff']}", flush=True)
    assert info["flags"] == 0
    assert e_state < 1e-6
    assert e_inc < 1e-5
