"""Pins of the oracle's reference derivatives for the reverse mode
(oracle/adjoint.py) against facts that do not come from the oracle itself:
closed forms, linearity, symmetry of second derivatives and two independent
difference routes."""

import numpy as np

import workloads as W
from oracle import adjoint
from oracle.derivatives import jvp_cs, dense_jacobian
from oracle.dg import DG
from oracle.integrators import DenseSplit, pcexp_step
from scipy.linalg import expm
from tests.helpers import mesh_case, vortex_state, rel


def test_richardson_closed_form():
    # f(e) = sin(2e) + e^5 exp(e): f'(0) = 2
    f = lambda e: np.sin(2 * e) + e ** 5 * np.exp(e)
    assert abs(adjoint.richardson(f, 1e-3) - 2.0) < 1e-11


def test_step_derivative_linear_full_krylov():
    """With m >= n the Krylov step of a linear operator is the exact linear
    map u -> exp-based propagator, so its derivative along d is step(d)."""
    rng = np.random.default_rng(3)
    n = 8
    A = rng.standard_normal((n, n)) - 3 * np.eye(n)
    op = DenseSplit(A, A)
    u, d = rng.standard_normal(n), rng.standard_normal(n)
    for scheme in ("pcexp", "exp1"):
        der = adjoint.step_derivative_cs(op, u, d, 0.3, n, scheme)
        assert rel(der, pcexp_step(op, d, 0.3, n, scheme)) < 1e-12
    # EXP1 with J = A_res = A is exp(dt A) u
    assert rel(pcexp_step(op, d, 0.3, n, "exp1"), expm(0.3 * A) @ d) < 1e-12


def test_step_derivative_nonlinear_krylov_routes_agree():
    """m < n: the Krylov approximation is nonlinear in b; complex step and
    Richardson central differences of the same step must agree."""
    rng = np.random.default_rng(5)
    n = 12
    A = rng.standard_normal((n, n)) / 2 - 2 * np.eye(n)
    B = rng.standard_normal((n, n)) / 2 - 2 * np.eye(n)
    op = DenseSplit(A, B)
    u, d = rng.standard_normal(n), rng.standard_normal(n)
    cs = adjoint.step_derivative_cs(op, u, d, 0.4, 5)
    fd = adjoint.step_derivative_fd(op, u, d, 0.4, 5, h=1e-3)
    assert rel(fd, cs) < 1e-9
    # and it is not the linear map: step(u + d) - step(u) != derivative
    lin = pcexp_step(op, u + d, 0.4, 5) - pcexp_step(op, u, 0.4, 5)
    assert rel(lin, cs) > 1e-6


def test_second_order_term_two_routes():
    """<z, d/de[J(u+ev)^T w]> = w^T R''(u)[v, z] = <w, d/de[J(u+ez) v]>:
    differentiate J^T along v (oracle route) or J v along z (independent)."""
    m, _ = mesh_case("sq3")
    g = DG(m, 1, "roe")
    u = vortex_state(g, m, 1e-3)
    v = W.random_unit_vector(u.shape, 1)
    w = W.random_unit_vector(u.shape, 2)
    z = W.random_unit_vector(u.shape, 3)
    k6 = adjoint.vjp2_fd(g, u, v, w)
    lhs = float(np.sum(z * k6))
    rhs = float(np.sum(w * adjoint.richardson(lambda e: jvp_cs(g, u + e * z, v), 1e-4)))
    assert abs(lhs - rhs) < 1e-8 * max(abs(rhs), 1e-3)
    # symmetry in (v, z)
    k6z = adjoint.vjp2_fd(g, u, z, w)
    assert abs(float(np.sum(v * k6z)) - lhs) < 1e-8 * max(abs(lhs), 1e-3)


def test_second_order_term_step_consistency():
    """The extrapolated difference is converged: halving h moves it by less
    than the bound used in the GPU comparison (LF flux, with its max() kink
    away from the state)."""
    m, _ = mesh_case("sq3")
    g = DG(m, 1, "lf")
    u = vortex_state(g, m, 1e-3)
    v = W.random_unit_vector(u.shape, 4)
    w = W.random_unit_vector(u.shape, 5)
    a = adjoint.vjp2_fd(g, u, v, w, h=1e-4)
    b = adjoint.vjp2_fd(g, u, v, w, h=5e-5)
    assert rel(a, b) < 1e-7


def test_trajectory_functional_matches_direct_sum():
    m, _ = mesh_case("sq3")
    g = DG(m, 1, "lf")
    from oracle.integrators import ExactJacobian
    from oracle.diagnostics import pressure_fluctuation
    u0 = vortex_state(g, m, 1e-3)
    op = ExactJacobian(g)
    J = adjoint.trajectory_functional(g, op, u0, 0.05, 6, 2)
    u1 = pcexp_step(op, u0, 0.05, 6)
    u2 = pcexp_step(op, u1, 0.05, 6)
    assert abs(J - 0.05 * (pressure_fluctuation(g, u1) + pressure_fluctuation(g, u2))) < 1e-15
