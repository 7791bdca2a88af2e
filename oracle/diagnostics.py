"""Diagnostics: conserved totals, entropy error (Sec. 5.1 eq. (entropy_error)),
L2 field error and the integrated pressure-fluctuation functional.

Entropy error reading (the printed formula is garbled):
  E(s) = sqrt( (1/|Omega|) int_Omega (s/s_0 - 1)^2 dx ),  s = p / rho^gamma.
"""

import numpy as np

from .euler import primitives


def conserved_totals(dg, u):
    """Q_k = int_Omega U_k dx = sum_E |E|^{1/2} u_{E,k,1} (psi_1 = |E|^{-1/2})."""
    return np.sum(np.sqrt(dg.mesh.vol)[:, None] * u[:, :, 0], axis=0)


def entropy_error(dg, u, s0=1.0):
    U = dg.evaluate(u)
    rho, _, p = primitives(U, dg.gamma)
    s = p / rho ** dg.gamma
    return float(np.sqrt(dg.integrate((s / s0 - 1.0) ** 2) / dg.mesh.volume_total))


def l2_error(dg, u, exact):
    """sqrt(int |U_h - U_exact|^2) over all conserved variables."""
    from .mesh import affine_map
    x = affine_map(dg.mesh, dg.ref_pts)
    Ue = exact(x.reshape(-1, dg.d)).reshape(dg.nE, dg.Nq, dg.nv)
    diff = dg.evaluate(u) - Ue
    return float(np.sqrt(dg.integrate(np.sum(diff * diff, axis=-1))))


def pressure_fluctuation(dg, u, p_inf=1.0):
    """int_Omega (p_h - p_inf)^2 dx (complex-safe)."""
    U = dg.evaluate(u)
    _, _, p = primitives(U, dg.gamma)
    return dg.integrate((p - p_inf) ** 2)
