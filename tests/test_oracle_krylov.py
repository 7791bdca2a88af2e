"""Pins of the oracle's JVPs, Krylov phi-functions and PCEXP stepper against
closed forms, library routines on small systems and invariants (Sec. 2, 3, 4.4)."""

from math import factorial

import numpy as np
import pytest
from scipy.linalg import expm

import workloads as W
from oracle import krylov
from oracle.dg import DG
from oracle.derivatives import jvp_cs, jvp_fd, dense_jacobian
from oracle.integrators import (pcexp_step, heun_step, ExactJacobian, DenseSplit,
                                stable_dt, cfl_ramp, res_rho_norm)
from oracle.diagnostics import conserved_totals


def _tiny(flux="roe", p=1, n=3, jitter=0.1, dim=2, amp=1e-6, uinf=None):
    if dim == 2:
        m = W.periodic_square(n, 10.0, jitter, 17)
    else:
        m = W.periodic_cube(n, 10.0)
    g = DG(m, p, flux)
    u = g.project(lambda x: W.isentropic_vortex(x, center=(5.0, 5.0), period=m.period, uinf=uinf))
    u = u + W.perturbation(u.shape, 101, amp)
    return g, u


# ------------------------------------------------------------------ JVP
@pytest.mark.parametrize("flux", ["lf", "roe"])
@pytest.mark.parametrize("dim", [2, 3])
def test_complex_step_vs_central_fd(flux, dim):
    # keep the state away from the kinks of |v.n| and max(): the vortex column
    # has v.n = 0 on z-faces, so give it a z-velocity here
    uinf = (0.42, 0.42, 0.3) if dim == 3 else None
    g, u = _tiny(flux, 1, 3, dim=dim, amp=1e-3, uinf=uinf)
    v = W.random_unit_vector(u.shape, 5)
    Jv = jvp_cs(g, u, v)
    h = 1e-5
    cfd = (g.residual(u + h * v) - g.residual(u - h * v)) / (2 * h)
    assert np.linalg.norm(Jv - cfd) < 1e-7 * np.linalg.norm(Jv)
    # FD-JVP baseline agrees to first order
    fd = jvp_fd(g, u, v)
    assert np.linalg.norm(Jv - fd) < 1e-6 * np.linalg.norm(Jv)


def test_jvp_linear_and_conservative():
    g, u = _tiny("roe", 2, 3)
    v1 = W.random_unit_vector(u.shape, 1)
    v2 = W.random_unit_vector(u.shape, 2)
    J = lambda v: jvp_cs(g, u, v)
    lhs = J(0.3 * v1 - 2.0 * v2)
    assert np.linalg.norm(lhs - (0.3 * J(v1) - 2.0 * J(v2))) < 1e-13 * np.linalg.norm(lhs)
    tot = np.sum(np.sqrt(g.mesh.vol)[:, None] * J(v1)[:, :, 0], axis=0)
    assert np.max(np.abs(tot)) < 1e-12 * np.linalg.norm(J(v1))


def test_dense_jacobian_columns():
    g, u = _tiny("lf", 1, 3)
    J = dense_jacobian(g, u)
    v = W.random_unit_vector(u.shape, 9)
    assert np.allclose(J @ v.ravel(), jvp_cs(g, u, v).ravel(), atol=1e-12)
    # periodic: J is singular (Sec. 2.2): the conserved totals are a left null space
    ell = np.zeros(u.shape)
    ell[:, 0, 0] = np.sqrt(g.mesh.vol)
    assert np.linalg.norm(ell.ravel() @ J) < 1e-12 * np.linalg.norm(J)


# ------------------------------------------------------------ phi closed forms
def _phi_closed(k, z):
    """phi_k(z) = (e^z - sum_{j<k} z^j/j!) / z^k, series near 0."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 1e-2
    zs = z[small]
    out[small] = sum(zs ** j / factorial(j + k) for j in range(12))
    zb = z[~small]
    out[~small] = (np.exp(zb) - sum(zb ** j / factorial(j) for j in range(k))) / zb ** k
    return out


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_phi_diagonal_closed_forms(k):
    """Diagonal J: phi_1 = (e^z-1)/z (eq. (Phi1)), phi_2 = (e^z-1-z)/z^2 (eq.
    (Phi2)), ...; with m >= the number of distinct eigenvalues the Krylov
    result is exact (breakdown)."""
    z = np.array([-40.0, -7.5, -1.0, -1e-3, 0.0, 1e-9, 0.5, 2.0])
    rng = np.random.default_rng(0)
    b = rng.uniform(0.5, 1.5, z.size)
    dt = 0.7
    got, info = krylov.arnoldi_phi(lambda v: (z / dt) * v, b, dt, k, 12, return_info=True)
    want = _phi_closed(k, z) * b
    assert np.all(np.abs(got - want) <= 1e-12 * np.abs(want) + 1e-14 * np.linalg.norm(b))
    # 0 and 1e-9 are distinct but numerically close: breakdown may come one step late
    assert info["breakdown"] and info["m_eff"] <= z.size + 1


def test_phi_recursion():
    """Eq. (s6): phi_{k+1}(z) = (phi_k(z) - 1/k!)/z."""
    for z in (-3.0, -0.25, 0.8):
        A = np.array([[z]])
        ph = [krylov.phi_augmented(A, k)[0] for k in range(5)]
        for k in range(1, 4):
            assert abs(ph[k + 1] - (ph[k] - 1.0 / factorial(k)) / z) < 1e-14 * max(1, abs(ph[k + 1]))


def test_krylov_vs_dense_random():
    """Random 50x50 matrix with a prescribed (complex, left-half-plane) spectrum:
    the Krylov phi_k(dt A) b with m = 50 equals the dense one."""
    rng = np.random.default_rng(3)
    n = 50
    lam = np.concatenate([-rng.uniform(0, 5, 25) + 1j * rng.uniform(0, 8, 25)])
    D = np.zeros((n, n))
    for i, l in enumerate(lam):
        D[2 * i:2 * i + 2, 2 * i:2 * i + 2] = [[l.real, l.imag], [-l.imag, l.real]]
    Q = rng.standard_normal((n, n)) + 3 * np.eye(n)
    A = Q @ D @ np.linalg.inv(Q)
    b = rng.standard_normal(n)
    for k in (0, 1, 2):
        got = krylov.arnoldi_phi(lambda v: A @ v, b, 0.3, k, n)
        want = krylov.dense_phi(A, b, 0.3, k)
        assert np.linalg.norm(got - want) < 1e-11 * np.linalg.norm(want)
    # dense phi_1 itself against its definition A^{-1}(e^{dtA} - I)/dt b  (eq. (Phi1))
    want1 = np.linalg.solve(0.3 * A, (expm(0.3 * A) - np.eye(n)) @ b)
    assert np.linalg.norm(krylov.dense_phi(A, b, 0.3, 1) - want1) < 1e-11 * np.linalg.norm(want1)


@pytest.mark.parametrize("flux", ["lf", "roe"])
def test_krylov_vs_dense_dg_jacobian(flux):
    g, u = _tiny(flux, 1, 3)
    J = dense_jacobian(g, u)
    b = g.residual(u)
    dt = stable_dt(g, u, 2.0)
    got = krylov.arnoldi_phi(lambda v: jvp_cs(g, u, v.reshape(u.shape)), b, dt, 1, 60)
    want = krylov.dense_phi(J, b.ravel(), dt, 1).reshape(u.shape)
    assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want)


def test_zero_vector_and_nilpotent_breakdown():
    out, info = krylov.arnoldi_phi(lambda v: v, np.zeros(7), 1.0, 1, 5, return_info=True)
    assert np.all(out == 0) and info["m_eff"] == 0
    N = np.diag(np.ones(5), 1)     # nilpotent shift: Krylov space of e_6 has dimension 6
    b = np.zeros(6)
    b[-1] = 1.0
    got, info = krylov.arnoldi_phi(lambda v: N @ v, b, 1.0, 1, 20, return_info=True)
    assert info["breakdown"] and info["m_eff"] == 6
    assert np.allclose(got, krylov.dense_phi(N, b, 1.0, 1), atol=1e-14)


# ------------------------------------------------------------- integrators
def test_pcexp_exact_on_linear_systems():
    """Sec. 3.1: with no nonlinear part PCEXP is exact: u_{n+1} = e^{dt A} u_n."""
    rng = np.random.default_rng(4)
    n = 20
    A = rng.standard_normal((n, n)) - 4 * np.eye(n)
    u = rng.standard_normal(n)
    op = DenseSplit(A, A)
    got = pcexp_step(op, u, 0.4, n)
    want = expm(0.4 * A) @ u
    assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want)


def test_pcexp_scalar_split_model_eq_grow():
    """1x1 split operator A_jac = [b], A_res = [a + b] (dt = 1): the stepper's
    growth factor is eq. (grow); EXP1's is eq. (exp1_grow)."""
    for a in (-3.0, -0.7, 0.4):
        for b in (-6.0, -1.3, 0.25, 1.5):
            op = DenseSplit([[b]], [[a + b]])
            r = pcexp_step(op, np.array([1.0]), 1.0, 1)[0]
            printed = (a * (a - b) + np.exp(2 * b) * (a + b) * a + 2 * np.exp(b) * (b * b - a * a)) / (2 * b * b)
            assert abs(r - printed) < 1e-12 * max(1, abs(printed))
            r1 = pcexp_step(op, np.array([1.0]), 1.0, 1, scheme="exp1")[0]
            assert abs(r1 - (a * (np.exp(b) - 1) + b * np.exp(b)) / b) < 1e-12 * max(1, abs(r1))


def test_pcexp_zero_jacobian_is_heun():
    """Eq. (rk2) / Sec. 3.1 item 2: J -> 0 gives Heun's method, on the DG residual."""
    g, u = _tiny("roe", 1, 3)
    dt = stable_dt(g, u, 0.5)
    got = pcexp_step(ExactJacobian(g, "zero"), u, dt, 10)
    want = heun_step(ExactJacobian(g), u, dt)
    assert np.linalg.norm(got - want) < 1e-14 * np.linalg.norm(want)


def test_pcexp_conserves_totals():
    """Periodic: the conserved totals drift by rounding only over 10 steps."""
    g, u = _tiny("lf", 1, 4)
    op = ExactJacobian(g)
    q0 = conserved_totals(g, u)
    for _ in range(10):
        u = pcexp_step(op, u, stable_dt(g, u, 5.0), 20)
    assert np.max(np.abs(conserved_totals(g, u) - q0) / np.abs(q0).max()) < 1e-13


def test_pcexp_temporal_order_two():
    """Sec. 5.1 analogue: CFL = 0.1*2^n; error against the smallest CFL falls
    like dt^2 (second order in time)."""
    m = W.periodic_square(6, 10.0)
    g = DG(m, 1, "lf")
    u0 = g.project(lambda x: W.isentropic_vortex(x, center=(5.0, 5.0), period=m.period))
    op = ExactJacobian(g)
    dt0 = stable_dt(g, u0, 0.1)
    T = 32 * dt0 * 2          # two steps of the largest CFL (3.2)
    def run(cfl_mult):
        u, dt = u0.copy(), dt0 * cfl_mult
        for _ in range(int(round(T / dt))):
            u = pcexp_step(op, u, dt, 20)
        return u
    ref = run(2)               # CFL 0.2 serves as the time-exact solution
    errs = [np.linalg.norm(run(mult) - ref) for mult in (8, 16, 32)]
    rates = np.log2(np.array(errs[1:]) / np.array(errs[:-1]))
    assert np.all(rates > 1.7), (errs, rates)


def test_dt_and_cfl_ramp():
    """Eq. (x3d) on a uniform mesh at the free stream, and eq. (cfl)."""
    m = W.periodic_square(4, 10.0)
    g = DG(m, 2, "lf")
    prim = W.freestream_prim(2)
    u = g.project(lambda x: W.uniform_state(x, prim))
    h_tri = 2 * 2 * (0.5 * 2.5 ** 2) / (2.5 * 2 + 2.5 * np.sqrt(2))   # 2d|E|/|dE|
    speed = np.linalg.norm(prim[1:3]) + np.sqrt(1.4)
    assert abs(stable_dt(g, u, 3.0) - 3.0 * h_tri / (5 * speed)) < 1e-14
    # eq. (x2d) with d = 2: 2/h_2D = 3/h_3D - 1/dz for an extruded prism equals 4|E|/|dE|
    dz = 0.37
    area, perim = 0.5 * 2.5 ** 2, 2.5 * 2 + 2.5 * np.sqrt(2)
    h3 = 2 * 3 * area * dz / (2 * area + perim * dz)
    assert abs(2.0 / (3.0 / h3 - 1.0 / dz) - h_tri) < 1e-14
    assert cfl_ramp(1, 10.0, 2, 1000.0) == 1.0
    assert cfl_ramp(11, 10.0, 2, 1000.0) == 3.0
    assert cfl_ramp(5, 0.05, 2, 1000.0) == 1000.0
    assert abs(cfl_ramp(5, 0.5, 2, 1000.0) - 8.0) < 1e-12
    R = g.residual(u + W.perturbation(u.shape, 1, 1e-3))
    assert abs(res_rho_norm(g, R) - np.sqrt(np.sum(R[:, 0, :] ** 2)) / 100.0) < 1e-15


def test_krylov_error_estimate_tracks_true_error():
    """The a-posteriori estimate dt h_{m+1,m} |[phi_2(dt H) e_1]_m| / |phi_1(dt H) e_1|
    against the true relative error of the Krylov phi_1 (dense phi_1 from
    scipy.linalg.expm of the augmented matrix of the full operator)."""
    from scipy.linalg import expm
    rng = np.random.default_rng(12)
    n = 80
    A = rng.standard_normal((n, n)) / np.sqrt(n) - 1.5 * np.eye(n)
    b = rng.standard_normal(n)
    M = np.zeros((n + 1, n + 1))
    for dt in (0.5, 1.0, 2.0):
        M[:n, :n] = dt * A
        M[:n, n] = b
        exact = expm(M)[:n, n]          # phi_1(dt A) b
        for m in (6, 10, 14):
            V, H, beta, meff, brk = krylov.arnoldi_mgs(lambda v: A @ v, b, m)
            y, est = krylov.phi1_with_error(H[:meff, :meff], beta, H[meff, meff - 1], dt)
            approx = beta * V[:, :meff] @ y
            true = np.linalg.norm(approx - exact) / np.linalg.norm(exact)
            if 1e-13 < true < 1e-2:
                assert 0.1 < est / true < 10.0, (dt, m, est, true)


def test_krylov_dt_control_meets_tolerance():
    from scipy.linalg import expm
    rng = np.random.default_rng(13)
    n = 80
    A = rng.standard_normal((n, n)) / np.sqrt(n) * 3 - 2.0 * np.eye(n)
    b = rng.standard_normal(n)
    x, dt, err, halv, info = krylov.arnoldi_phi1_controlled(lambda v: A @ v, b, 8.0, 8, 1e-6)
    assert halv > 0 and dt == 8.0 / 2 ** halv and err <= 1e-6
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = dt * A
    M[:n, n] = b
    exact = dt * expm(M)[:n, n]
    assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 1e-5


def test_krylov_adaptive_dimension_meets_tolerance():
    """Adaptive dimension: the run stops at the first checked j whose estimate
    meets tol; the stopped approximation is within a small multiple of tol
    of the dense phi_1 (scipy.linalg.expm of the augmented full matrix), and
    a dimension one check earlier is not."""
    from scipy.linalg import expm
    rng = np.random.default_rng(14)
    n = 90
    A = rng.standard_normal((n, n)) / np.sqrt(n) - 1.5 * np.eye(n)
    b = rng.standard_normal(n)
    dt, m, tol, every = 1.0, 40, 1e-8, 3
    x, dt_used, err, halv, info = krylov.arnoldi_phi1_controlled(lambda v: A @ v, b, dt, m, tol,
                                                                 check_every=every)
    meff = info["m_eff"]
    assert halv == 0 and dt_used == dt and err <= tol
    assert meff < m and meff % every == 0 and not info["breakdown"]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = dt * A
    M[:n, n] = b
    exact = dt * expm(M)[:n, n]
    assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 10 * tol
    # one check earlier the approximation misses the tolerance
    V, H, beta, _, _ = krylov.arnoldi_mgs(lambda v: A @ v, b, m)
    j = meff - every
    y, _ = krylov.phi1_with_error(H[:j, :j], beta, H[j, j - 1], dt)
    early = dt * beta * V[:, :j] @ y
    assert np.linalg.norm(early - exact) / np.linalg.norm(exact) > tol


def test_krylov_adaptive_dimension_limits():
    """A tolerance no dimension below m meets leaves the run at m (the fixed-m
    result, bit for bit); check_every = 0 never stops early."""
    rng = np.random.default_rng(15)
    n = 60
    A = rng.standard_normal((n, n)) / np.sqrt(n) - 1.0 * np.eye(n)
    b = rng.standard_normal(n)
    mv = lambda v: A @ v
    fixed, _, _, _, i0 = krylov.arnoldi_phi1_controlled(mv, b, 0.5, 12, 1e-30, dt_control=False)
    for every in (0, 1, 4):
        x, _, _, _, info = krylov.arnoldi_phi1_controlled(mv, b, 0.5, 12, 1e-30, check_every=every,
                                                          dt_control=False)
        assert info["m_eff"] == 12 and np.array_equal(x, fixed)
    # a loose tolerance stops at the first check
    x, _, _, _, info = krylov.arnoldi_phi1_controlled(mv, b, 0.5, 12, 1.0, check_every=2, dt_control=False)
    assert info["m_eff"] == 2


def test_pcexp_step_adaptive_dimension_close_to_fixed():
    """A PCEXP step with the adaptive dimension (tol 1e-9) agrees with the
    fixed-dimension step to about the tolerance on a linear system, where the
    fixed step with m = n is exact."""
    from scipy.linalg import expm
    rng = np.random.default_rng(16)
    n = 50
    A = rng.standard_normal((n, n)) / np.sqrt(n) - 2.0 * np.eye(n)
    op = DenseSplit(A, A)
    u0 = rng.standard_normal(n)
    info = {}
    u1 = pcexp_step(op, u0, 0.3, 45, krylov_tol=1e-9, krylov_every=2, info=info)
    assert info["k1"]["m_eff"] < 45 and info["k2"]["m_eff"] < 45
    exact = expm(0.3 * A) @ u0
    assert np.linalg.norm(u1 - exact) / np.linalg.norm(exact) < 1e-7


class _Quadratic:
    """u' = A u + c * u * u (elementwise) with J = A: the linear part is treated
    exponentially and N = c u * u explicitly (the classical exponential time
    differencing setting, where ETD1 is first order and ETD2 second)."""

    def __init__(self, A, c):
        self.A, self.c = np.asarray(A, float), float(c)

    def residual(self, u):
        return self.A @ u + self.c * u * u

    def jvp(self, u, v, R=None):
        return self.A @ v


def _etd2_run(op, u0, dt, nsteps, m):
    from oracle.integrators import etd2_step
    u, up, Rp = np.array(u0, float), None, None
    for _ in range(nsteps):
        unew, Rn = etd2_step(op, u, up, Rp, dt, m)
        up, Rp, u = u, Rn, unew
    return u


def test_etd2_exact_on_linear_systems():
    """Eq. (s7) with no nonlinear part (N_n - N_{n-1} = 0): ETD2 is exact."""
    rng = np.random.default_rng(21)
    n = 16
    A = rng.standard_normal((n, n)) - 4 * np.eye(n)
    u0 = rng.standard_normal(n)
    got = _etd2_run(DenseSplit(A, A), u0, 0.3, 3, n)
    want = expm(0.9 * A) @ u0
    assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want)


def test_etd2_first_step_is_etd1():
    """Without history the step is ETD1, eq. (s8) (the EXP1 predictor)."""
    from oracle.integrators import etd2_step
    g, u = _tiny("roe", 1, 3)
    op = ExactJacobian(g)
    dt = stable_dt(g, u, 2.0)
    got, _ = etd2_step(op, u, None, None, dt, 12)
    want = pcexp_step(op, u, dt, 12, scheme="exp1")
    assert np.array_equal(got, want)


@pytest.mark.parametrize("case", ["scalar", "system"])
def test_etd2_temporal_order_two(case):
    """With J the linear part and N = c u * u explicit, ETD2 converges like
    dt^2 and ETD1 like dt: u' = -u/2 - u^2 (exact: the logistic solution
    a u0 e^{-at} / (a + u0 (1 - e^{-at})), a = 1/2) and a 4 x 4 system
    (reference: ETD2 at a 32x smaller step).  A missing or sign-flipped
    difference term would leave first order."""
    T = 2.0
    if case == "scalar":
        a = 0.5
        op, u0, m = _Quadratic([[-a]], -1.0), np.array([1.0]), 1
        ref = a * u0 * np.exp(-a * T) / (a + u0 * (1.0 - np.exp(-a * T)))
    else:
        rng = np.random.default_rng(22)
        A = rng.standard_normal((4, 4)) * 0.5 - 1.0 * np.eye(4)
        op, u0, m = _Quadratic(A, 0.3), rng.standard_normal(4), 4
        ref = _etd2_run(op, u0, T / 2048, 2048, m)
    e2, e1 = [], []
    for nsteps in (16, 32, 64):
        dt = T / nsteps
        e2.append(np.linalg.norm(_etd2_run(op, u0, dt, nsteps, m) - ref))
        u = u0.copy()
        for _ in range(nsteps):
            u = pcexp_step(op, u, dt, m, scheme="exp1")
        e1.append(np.linalg.norm(u - ref))
    r2 = np.log2(np.array(e2[:-1]) / np.array(e2[1:]))
    r1 = np.log2(np.array(e1[:-1]) / np.array(e1[1:]))
    assert np.all(r2 > 1.8) and np.all(r1 < 1.3) and np.all(r1 > 0.8), (e2, r2, e1, r1)
