"""Pins of the oracle's diagnostics and step-size rules against closed forms.

Each test builds a field that the P2 space represents exactly (quadratic
conserved variables), so the quantity under test has a value computed here
from the vertex coordinates and the field's formula alone, without the
oracle's basis, coefficients or quadrature.  Each test also checks that the
plausible mistakes it is meant to catch (evaluation at a vertex, the cell
average, a dropped normalisation, a wrong kinetic-energy term) move the
value by far more than the tolerance, so that it has the power to fail them.
"""

from math import factorial

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG
from oracle.diagnostics import entropy_error, pressure_fluctuation
from oracle.integrators import res_rho_norm, stable_dt

GAMMA = 1.4


def _tri_h(X):
    """h_E = 2 d |E| / |dE| of eq. (x3d) for triangles X (E, 3, 2), d = 2."""
    e1, e2 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    perim = (np.linalg.norm(X[:, 1] - X[:, 0], axis=1) + np.linalg.norm(X[:, 2] - X[:, 1], axis=1)
             + np.linalg.norm(X[:, 0] - X[:, 2], axis=1))
    return 2 * 2 * area / perim, area


def _quadratic_field(x):
    """A state with quadratic conserved variables (exact in P2):
    rho = 1 + 0.2 x + 0.1 y^2 / 100, momentum (0.5 + 0.02 x^2, -0.3 + 0.01 x y),
    rho E = 3 + 0.05 y + 0.01 x^2."""
    X, Y = x[..., 0], x[..., 1]
    rho = 1.0 + 0.02 * X + 0.001 * Y * Y
    mx = 0.5 + 0.02 * X * X
    my = -0.3 + 0.01 * X * Y
    rE = 3.0 + 0.05 * Y + 0.01 * X * X
    return np.stack([rho, mx, my, rE], axis=-1)


def _dt_per_element(X, cfl, p, where):
    """Eq. (x3d) per element with v and c taken at the points `where` (E, 2)."""
    h, _ = _tri_h(X)
    U = _quadratic_field(where)
    rho, m, rE = U[:, 0], U[:, 1:3], U[:, 3]
    vel = m / rho[:, None]
    pres = (GAMMA - 1.0) * (rE - 0.5 * np.sum(m * m, axis=1) / rho)
    lam = np.linalg.norm(vel, axis=1) + np.sqrt(GAMMA * pres / rho)
    return cfl * h / ((2 * p + 1) * lam)


def test_stable_dt_centroid_value_on_jittered_mesh():
    """Eq. (x3d): dt = CFL min_E h_E / ((2p+1)(|v| + c)) with v and c the point
    values at the element centroid (reading: "velocity at the cell centre").
    The field is quadratic, so the centroid value differs from the vertex
    values and from the cell average; the mesh is jittered, so h_E varies."""
    m = W.periodic_square(6, 10.0, 0.15, 7)
    g = DG(m, 2, "roe")
    u = g.project(_quadratic_field)
    X = m.vert[m.elem]
    cfl = 7.0
    cen = X.mean(axis=1)
    want = np.min(_dt_per_element(X, cfl, 2, cen))
    got = stable_dt(g, u, cfl)
    assert abs(got - want) <= 1e-13 * want, (got, want)
    # the mistakes this pin must catch move the result far beyond its tolerance
    at_vertex = np.min(_dt_per_element(X, cfl, 2, X[:, 0]))
    assert abs(at_vertex - want) > 1e-6 * want
    # cell average of each conserved variable: exact 3-edge-midpoint rule for quadratics
    mids = [(X[:, a] + X[:, b]) / 2 for a, b in ((0, 1), (1, 2), (2, 0))]
    avg = sum(_quadratic_field(q) for q in mids) / 3.0
    h, _ = _tri_h(X)
    rho, mom, rE = avg[:, 0], avg[:, 1:3], avg[:, 3]
    pres = (GAMMA - 1.0) * (rE - 0.5 * np.sum(mom * mom, axis=1) / rho)
    lam = np.linalg.norm(mom / rho[:, None], axis=1) + np.sqrt(GAMMA * pres / rho)
    with_average = np.min(cfl * h / (5 * lam))
    assert abs(with_average - want) > 1e-9 * want
    # p enters as 2p + 1
    assert abs(stable_dt(DG(m, 1, "roe"), DG(m, 1, "roe").project(lambda x: W.uniform_state(
        x, W.freestream_prim(2))), cfl) * 3 - stable_dt(g, g.project(lambda x: W.uniform_state(
            x, W.freestream_prim(2))), cfl) * 5) < 1e-13


def _p2_density_only(g, f):
    """Coefficient vector whose density component is the projection of f and
    whose other components are zero."""
    u = g.project(lambda x: np.stack([f(x)] + [np.zeros(x.shape[0])] * (g.nv - 1), axis=-1))
    return u


def test_res_rho_norm_constant_field_closed_form():
    """Eq. (cfl): ||R(rho)||_2 = (1/|Omega|) (int_Omega R(rho)^2 dx)^(1/2).  For a
    constant density residual c the integral is c^2 |Omega|, so the norm is
    c / |Omega|^(1/2) exactly (the 1/|Omega| sits outside the square root)."""
    m = W.periodic_square(5, 4.0, 0.15, 3)
    g = DG(m, 2, "lf")
    c = 0.37
    R = _p2_density_only(g, lambda x: np.full(x.shape[0], c))
    R[:, 1:, :] = 5.0          # other variables must not enter
    omega = 16.0
    assert abs(res_rho_norm(g, R) - c / np.sqrt(omega)) < 1e-14
    # the reading with 1/|Omega| inside the root gives c, not c/4
    assert abs(c / np.sqrt(omega) - c) > 0.1


def test_res_rho_norm_equals_quadrature_of_the_field():
    """||R(rho)|| from the coefficients (orthonormal basis) against the integral
    of the squared density field R_h(rho)(x) = sum_i R_i psi_i(x), integrated
    exactly on each triangle from its values at the six P2 nodes (vertices and
    edge midpoints): the field is quadratic, its square quartic, and the
    integral of a quartic is computed here by the closed form
    int_T l1^a l2^b l3^c = 2|T| a! b! c! / (a + b + c + 2)! on the quadratic's
    barycentric (Bernstein) coefficients."""
    m = W.periodic_square(4, 3.0, 0.15, 11)
    g = DG(m, 2, "roe")
    rng = np.random.default_rng(5)
    R = rng.standard_normal((g.nE, g.nv, g.N))
    X = m.vert[m.elem]
    # nodal values of the density field at vertices and edge midpoints of each element
    nodes_bary = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [.5, .5, 0], [0, .5, .5], [.5, 0, .5]])
    ref = nodes_bary[:, 1:]                                  # reference coords (l2, l3)
    vals = np.real(g.evaluate_at(R, ref))[:, :, 0]          # (E, 6)
    # Bernstein coefficients of a quadratic from the six nodal values
    b200, b020, b002 = vals[:, 0], vals[:, 1], vals[:, 2]
    b110 = 2 * vals[:, 3] - 0.5 * (b200 + b020)
    b011 = 2 * vals[:, 4] - 0.5 * (b020 + b002)
    b101 = 2 * vals[:, 5] - 0.5 * (b200 + b002)
    # f = sum_{|a|=2} B_a (2!/a!) l^a ; f^2 = sum over pairs; integrate monomials
    terms = {(2, 0, 0): b200, (0, 2, 0): b020, (0, 0, 2): b002,
             (1, 1, 0): 2 * b110, (0, 1, 1): 2 * b011, (1, 0, 1): 2 * b101}
    _, area = _tri_h(X)
    total = np.zeros(g.nE)
    for ea, ca in terms.items():
        for eb, cb in terms.items():
            a, b, c = (ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2])
            total += ca * cb * 2 * area * factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 2)
    want = np.sqrt(np.sum(total)) / 9.0
    assert abs(res_rho_norm(g, R) - want) < 1e-12 * want


def _barycentric_quadratic_integral(X, f):
    """Exact integral over each triangle of X (E, 3, 2) of the square of a
    quadratic f, from its values at the 6 P2 nodes (closed form above)."""
    V = [X[:, 0], X[:, 1], X[:, 2], (X[:, 0] + X[:, 1]) / 2, (X[:, 1] + X[:, 2]) / 2, (X[:, 0] + X[:, 2]) / 2]
    v = [f(q) for q in V]
    b200, b020, b002 = v[0], v[1], v[2]
    terms = {(2, 0, 0): b200, (0, 2, 0): b020, (0, 0, 2): b002,
             (1, 1, 0): 2 * (2 * v[3] - 0.5 * (b200 + b020)),
             (0, 1, 1): 2 * (2 * v[4] - 0.5 * (b020 + b002)),
             (1, 0, 1): 2 * (2 * v[5] - 0.5 * (b200 + b002))}
    _, area = _tri_h(X)
    total = np.zeros(X.shape[0])
    for ea, ca in terms.items():
        for eb, cb in terms.items():
            a, b, c = (ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2])
            total += ca * cb * 2 * area * factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 2)
    return total


def test_pressure_fluctuation_closed_form():
    """int_Omega (p_h - p_ref)^2 dx for a state with constant density 2,
    linear momentum and rho E = p/(gamma-1) + |m|^2/(2 rho) with p quadratic:
    every conserved variable is exactly in P2 and p_h = p pointwise, so the
    functional is the exact integral of a squared quadratic (closed form on
    barycentric monomials).  A kinetic term without 1/rho or without the 1/2
    changes the value by orders of magnitude more than the tolerance."""
    m = W.periodic_square(4, 3.0, 0.15, 9)
    g = DG(m, 2, "roe")
    rho0 = 2.0

    def mom(x):
        return np.stack([0.3 + 0.1 * x[..., 0], -0.2 + 0.05 * x[..., 1]], axis=-1)

    def pres(x):
        return 1.0 + 0.04 * x[..., 0] * x[..., 1] - 0.03 * x[..., 1] ** 2

    def state(x):
        mm = mom(x)
        rE = pres(x) / (GAMMA - 1) + 0.5 * np.sum(mm * mm, axis=-1) / rho0
        return np.concatenate([np.full(x.shape[:-1] + (1,), rho0), mm, rE[..., None]], axis=-1)

    u = g.project(state)
    X = m.vert[m.elem]
    want = float(np.sum(_barycentric_quadratic_integral(X, lambda q: pres(q) - 1.0)))
    got = pressure_fluctuation(g, u, 1.0)
    assert abs(got - want) < 1e-12 * want, (got, want)
    # a wrong kinetic term (density not divided out) would differ by far more
    def pres_wrong(q):
        mm = mom(q)
        return pres(q) + (GAMMA - 1) * 0.5 * np.sum(mm * mm, axis=-1) * (1 / rho0 - 1)
    wrong = float(np.sum(_barycentric_quadratic_integral(X, lambda q: pres_wrong(q) - 1.0)))
    assert abs(wrong - want) > 1e-6 * want


def test_entropy_error_isentropic_and_closed_form():
    """Entropy error, reading of eq. (entropy_error):
    E = ((1/|Omega|) int (s/s_0 - 1)^2 dx)^(1/2), s = p / rho^gamma.
    (a) Constant rho and p with linear velocity (all conserved variables in
    P2): s is constant, E = 0 to rounding with s_0 = p / rho^gamma.
    (b) rho = 1, v = 0, p = 1 + eps q(x) with q linear: s / s_0 - 1 = eps q,
    so E^2 |Omega| is the exact integral of a squared linear function."""
    m = W.periodic_square(4, 3.0, 0.15, 13)
    g = DG(m, 2, "roe")
    rho0, p0 = 1.7, 0.9

    def isentropic(x):
        vx, vy = 0.2 + 0.05 * x[..., 0], -0.1 + 0.03 * x[..., 1]
        rE = p0 / (GAMMA - 1) + 0.5 * rho0 * (vx * vx + vy * vy)
        return np.stack([np.full_like(vx, rho0), rho0 * vx, rho0 * vy, rE], axis=-1)

    u = g.project(isentropic)
    s0 = p0 / rho0 ** GAMMA
    assert entropy_error(g, u, s0) < 1e-13
    # with a wrong reference entropy the error is |s/s0' - 1| exactly
    assert abs(entropy_error(g, u, 2 * s0) - 0.5) < 1e-13

    eps = 1e-2

    def q(x):
        return 0.3 * x[..., 0] - 0.2 * x[..., 1] + 0.1

    def perturbed(x):
        pr = 1.0 + eps * q(x)
        z = np.zeros_like(pr)
        return np.stack([np.ones_like(pr), z, z, pr / (GAMMA - 1)], axis=-1)

    u = g.project(perturbed)
    X = m.vert[m.elem]
    want = np.sqrt(np.sum(_barycentric_quadratic_integral(X, lambda x: eps * q(x))) / 9.0)
    got = entropy_error(g, u, 1.0)
    assert abs(got - want) < 1e-12 * want, (got, want)
    # the printed (garbled) form int (s/s0)^2 / |Omega| - 1 differs at first order in eps
    garbled = np.sum(_barycentric_quadratic_integral(X, lambda x: 1 + eps * q(x))) / 9.0 - 1.0
    assert abs(np.sqrt(abs(garbled)) - want) > 1e-3 * want
