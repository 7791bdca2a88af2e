"""Time integrators (Sec. 2.1 eqs. (s8), (s9), (s10); Sec. 5 eqs. (x3d), (cfl)).

PCEXP (eqs. (s9)-(s10)), both stages with the Jacobian J_n at u_n:
  x1     = dt Phi_1(dt J_n) R_n
  u*     = u_n + x1
  N* - N_n = R(u*) - R_n - J_n (u* - u_n)
  u_{n+1} = u* + dt/2 Phi_1(dt J_n) (N* - N_n)
EXP1 (first stage alone, eq. (s8)): u_{n+1} = u*.

The operator ``op`` provides residual(u) and jvp(u_lin, v).  With the exact
Jacobian the JVP is the complex-step derivative of the residual; a separate
"split" operator (residual A_res u, jvp A_jac v) reproduces the scalar model
problem of Sec. 3.
"""

import numpy as np

from . import krylov
from .derivatives import jvp_cs, jvp_fd


class ExactJacobian:
    """Residual of a DG operator and its exact JVP by complex step."""

    def __init__(self, dg, jvp="exact"):
        self.dg = dg
        self.kind = jvp

    def residual(self, u):
        return self.dg.residual(u)

    def jvp(self, u_lin, v, R_lin=None):
        if self.kind == "exact":
            return jvp_cs(self.dg, u_lin, v)
        if self.kind == "fd":
            return jvp_fd(self.dg, u_lin, v, R_lin)
        if self.kind == "zero":
            return np.zeros_like(v)
        raise ValueError(self.kind)


class DenseSplit:
    """Linear test operator: R(u) = A_res u, J v = A_jac v (any shape of u)."""

    def __init__(self, A_jac, A_res):
        self.A_jac = np.asarray(A_jac)
        self.A_res = np.asarray(A_res)

    def residual(self, u):
        return (self.A_res @ np.reshape(u, -1)).reshape(np.shape(u))

    def jvp(self, u_lin, v, R_lin=None):
        return (self.A_jac @ np.reshape(v, -1)).reshape(np.shape(v))


def pcexp_step(op, u, dt, m, scheme="pcexp", eta=1e-12, info=None, krylov_tol=0.0, krylov_every=0):
    """One PCEXP (or EXP1) step u_n -> u_{n+1}.  With krylov_tol > 0 the
    predictor's dt is halved until the Krylov error estimate is <= krylov_tol
    (krylov.arnoldi_phi1_controlled) and both stages use that dt; with also
    krylov_every > 0 each stage's Krylov dimension is chosen adaptively
    (krylov.adaptive_dimension) before that."""
    u = np.asarray(u)
    shape = u.shape
    Rn = op.residual(u)
    mv = lambda v: op.jvp(u, np.reshape(v, shape), Rn)
    if krylov_tol > 0.0:
        x1, dt, err, halv, i1 = krylov.arnoldi_phi1_controlled(mv, Rn, dt, m, krylov_tol, eta,
                                                               check_every=krylov_every)
        i1 = dict(i1, dt=dt, err_est=err, dt_halvings=halv)
    else:
        x1, i1 = krylov.arnoldi_phi(mv, Rn, dt, 1, m, eta, return_info=True)
        x1 = dt * x1
    ustar = u + x1
    if info is not None:
        info["k1"] = i1
    if scheme == "exp1":
        return ustar
    Rs = op.residual(ustar)
    d = Rs - Rn - op.jvp(u, x1, Rn)
    if krylov_tol > 0.0 and krylov_every > 0:
        x2, _, err2, _, i2 = krylov.arnoldi_phi1_controlled(mv, d, dt, m, krylov_tol, eta,
                                                            check_every=krylov_every, dt_control=False)
        i2 = dict(i2, err_est=err2)
        unext = ustar + 0.5 * x2
    else:
        x2, i2 = krylov.arnoldi_phi(mv, d, dt, 1, m, eta, return_info=True)
        unext = ustar + 0.5 * dt * x2
    if info is not None:
        info["k2"] = i2
    return unext


def etd2_step(op, u, u_prev, R_prev, dt, m, eta=1e-12, info=None):
    """One ETD2 step, eq. (s7): u_{n+1} = u_n + dt Phi_1(dt J_n) R_n
    + dt Phi_2(dt J_n)(N_n - N_{n-1}) with N = R - J_n u on the step (the
    split of eq. (s3)), so N_n - N_{n-1} = R_n - R_{n-1} - J_n (u_n - u_{n-1}).
    Without history (u_prev None) the step is ETD1, eq. (s8).  Returns
    (u_{n+1}, R_n) so that the caller can pass (u_n, R_n) as the next history."""
    u = np.asarray(u)
    shape = u.shape
    Rn = op.residual(u)
    mv = lambda v: op.jvp(u, np.reshape(v, shape), Rn)
    x1, i1 = krylov.arnoldi_phi(mv, Rn, dt, 1, m, eta, return_info=True)
    unext = u + dt * x1
    if info is not None:
        info["k1"] = i1
    if u_prev is None:
        return unext, Rn
    d = Rn - R_prev - op.jvp(u, u - u_prev, Rn)
    x2, i2 = krylov.arnoldi_phi(mv, d, dt, 2, m, eta, return_info=True)
    if info is not None:
        info["k2"] = i2
    return unext + dt * x2, Rn


def heun_step(op, u, dt):
    """Second-order Runge-Kutta (Heun): the J -> 0 limit of PCEXP (eq. (rk2))."""
    Rn = op.residual(u)
    us = u + dt * Rn
    return us + 0.5 * dt * (op.residual(us) - Rn)


def stable_dt(dg, u, cfl):
    """Eq. (x3d): dt = CFL min_E h_E / ((2p+1)(|v| + c)), with v and c at the
    element centroid (the "cell centre"), global minimum over elements."""
    d = dg.d
    cen = np.full((1, d), 1.0 / (d + 1))
    U = np.real(dg.evaluate_at(u, cen))[:, 0, :]
    rho = U[:, 0]
    vel = U[:, 1:-1] / rho[:, None]
    p = (dg.gamma - 1.0) * (U[:, -1] - 0.5 * rho * np.sum(vel * vel, axis=1))
    c = np.sqrt(dg.gamma * p / rho)
    lam = np.linalg.norm(vel, axis=1) + c
    return float(cfl * np.min(dg.mesh.h / ((2 * dg.p + 1) * lam)))


def res_rho_norm(dg, R):
    """||R(rho)||_2 of eq. (cfl): (1/|Omega|) (int R_rho^2)^{1/2}; with the
    orthonormal basis the integral is the sum of squared coefficients."""
    return float(np.sqrt(np.sum(np.real(R[:, 0, :]) ** 2)) / dg.mesh.volume_total)


def cfl_ramp(n, rnorm, p, cfl_max):
    """Eq. (cfl): CFL(n) = min{CFL_max, max[||R(rho_n)||^-3, 1 + (n-1)/(2p+1)]}."""
    big = np.inf if rnorm == 0.0 else rnorm ** -3
    return float(min(cfl_max, max(big, 1.0 + (n - 1) / (2 * p + 1))))


def steady_iterations(dg, op, u, niter, cfl_max, m, scheme="pcexp", krylov_tol=0.0, krylov_every=0):
    """Pseudo-time stepping toward R(u) = 0 (Sec. 5): at iteration n = 1, 2, ...
    CFL(n) from eq. (cfl) with ||R(rho_n)||, dt from eq. (x3d) at u_n with that
    CFL, then one PCEXP (or EXP1) step.  Returns the state and the list of
    ||R(rho_n)||."""
    hist = []
    for n in range(1, niter + 1):
        R = dg.residual(u)
        r = res_rho_norm(dg, R)
        hist.append(r)
        dt = stable_dt(dg, u, cfl_ramp(n, r, dg.p, cfl_max))
        u = pcexp_step(op, u, dt, m, scheme, krylov_tol=krylov_tol, krylov_every=krylov_every)
    return u, hist
