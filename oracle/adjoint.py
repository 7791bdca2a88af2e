"""Reference derivatives for the reverse mode of the PCEXP step.

The paper has no adjoint; the reverse mode differentiates the discrete step
of Sec. 2.1 (eqs. (s8)-(s10)) with the Krylov evaluation of Sec. 2.2.  The
oracle does not run a reverse sweep: it supplies the exact directional
derivatives the reverse result must reproduce through the identity
<ubar, (du_{n+1}/du_n) d> = <(du_{n+1}/du_n)^T ubar, d>:

* for the linear test operator (DenseSplit) the step is an analytic
  function of u_n and its complex-step derivative is exact to rounding;
* for the DG operator the JVP inside the step is itself a complex-step
  derivative, so the step derivative is taken by central differences with
  one Richardson extrapolation (error O(h^4) + O(eps/h)).

The second-order adjoint term (d_u [J(u) v])^T w is checked the same way,
from central differences of the dense Jacobian transpose.
"""

import numpy as np

from .derivatives import dense_jacobian
from .integrators import pcexp_step

H_CS = 1e-30


def step_derivative_cs(op, u, d, dt, m, scheme="pcexp"):
    """d/de u_{n+1}(u + e d) at e = 0 by complex step (analytic operators only)."""
    u = np.asarray(u, dtype=np.float64)
    out = pcexp_step(op, u + 1j * H_CS * np.asarray(d), dt, m, scheme)
    return np.imag(out) / H_CS


def richardson(f, h):
    """Central difference of f at 0 with step h, extrapolated with h/2:
    D(h) = (f(h) - f(-h)) / 2h, result (4 D(h/2) - D(h)) / 3."""
    d1 = (f(h) - f(-h)) / (2.0 * h)
    d2 = (f(0.5 * h) - f(-0.5 * h)) / h
    return (4.0 * d2 - d1) / 3.0


def step_derivative_fd(op, u, d, dt, m, scheme="pcexp", h=1e-5):
    """d/de u_{n+1}(u + e d) at e = 0 by Richardson-extrapolated central differences."""
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    return richardson(lambda e: pcexp_step(op, u + e * d, dt, m, scheme), h)


def vjp2_fd(dg, u, v, w, h=1e-4):
    """d/de [J(u + e v)^T w] at e = 0 (J dense by complex step, then
    Richardson-extrapolated central differences in e)."""
    u = np.asarray(u, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64).reshape(-1)

    def jtw(e):
        J = dense_jacobian(dg, u + e * np.asarray(v))
        return (J.T @ w).reshape(u.shape)

    return richardson(jtw, h)


def trajectory_functional(dg, op, u0, dt, m, nsteps, p_ref=1.0, scheme="pcexp"):
    """sum_{n=1}^{N} dt int_Omega (p_h(t_n) - p_ref)^2 dx along N steps from u0."""
    from .diagnostics import pressure_fluctuation
    u = np.asarray(u0)
    total = 0.0
    for _ in range(nsteps):
        u = pcexp_step(op, u, dt, m, scheme)
        total = total + dt * pressure_fluctuation(dg, u, p_ref)
    return total
