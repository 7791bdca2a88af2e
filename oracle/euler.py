"""Euler physics and numerical fluxes (Sec. 4.1 eq. (euler) with omega = 0;
Sec. 4.2 eq. (euler3); Sec. 4.4 boundary fluxes).

All functions are complex-safe for the complex-step derivative:
``cabs(x) = x sign(Re x)`` (derivative sign(x), with sign(0) = 0) and
``cmax`` compares real parts and returns the first argument on a tie.

Conserved variables U = (rho, rho v, rho E); p = (gamma-1)(rho E - |rho v|^2/(2 rho)),
H = (rho E + p)/rho, c = sqrt(gamma p / rho).

Readings where the paper leaves the choice open (pinned by their defining
properties, not by values from the paper): Roe's flux is used without
entropy fix; the Lax-Friedrichs flux is the local (Rusanov) form with
alpha = max(|v_L.n| + c_L, |v_R.n| + c_R) per face point; the ghost states
are the mirror state (slip wall) and the Riemann-invariant far field.
"""

import numpy as np


def cabs(x):
    return x * np.sign(np.real(x))


def cmax(a, b):
    return np.where(np.real(a) >= np.real(b), a, b)


def primitives(U, gamma):
    rho = U[..., 0]
    vel = U[..., 1:-1] / rho[..., None]
    rhoE = U[..., -1]
    p = (gamma - 1.0) * (rhoE - 0.5 * rho * np.sum(vel * vel, axis=-1))
    return rho, vel, p


def physical_flux(U, gamma):
    """F(U) with shape (..., nv, d)."""
    rho, vel, p = primitives(U, gamma)
    d = vel.shape[-1]
    rhoE = U[..., -1]
    F = np.empty(U.shape + (d,), dtype=U.dtype)
    F[..., 0, :] = rho[..., None] * vel
    for i in range(d):
        F[..., 1 + i, :] = rho[..., None] * vel[..., i:i + 1] * vel
        F[..., 1 + i, i] += p
    F[..., -1, :] = (rhoE + p)[..., None] * vel
    return F


def normal_flux(U, n, gamma):
    return np.einsum("...kd,...d->...k", physical_flux(U, gamma), n)


def lax_friedrichs(UL, UR, n, gamma):
    rL, vL, pL = primitives(UL, gamma)
    rR, vR, pR = primitives(UR, gamma)
    aL = cabs(np.sum(vL * n, axis=-1)) + np.sqrt(gamma * pL / rL)
    aR = cabs(np.sum(vR * n, axis=-1)) + np.sqrt(gamma * pR / rR)
    alpha = cmax(aL, aR)
    return 0.5 * (normal_flux(UL, n, gamma) + normal_flux(UR, n, gamma)) \
        - 0.5 * alpha[..., None] * (UR - UL)


def roe(UL, UR, n, gamma):
    """Roe's approximate Riemann flux (Roe 1981), no entropy fix."""
    rL, vL, pL = primitives(UL, gamma)
    rR, vR, pR = primitives(UR, gamma)
    HL = (UL[..., -1] + pL) / rL
    HR = (UR[..., -1] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    den = sL + sR
    ut = (sL[..., None] * vL + sR[..., None] * vR) / den[..., None]
    Ht = (sL * HL + sR * HR) / den
    q2 = np.sum(ut * ut, axis=-1)
    c2 = (gamma - 1.0) * (Ht - 0.5 * q2)
    ct = np.sqrt(c2)
    vn = np.sum(ut * n, axis=-1)
    rt = sL * sR
    dr = rR - rL
    dp = pR - pL
    dv = vR - vL
    dvn = np.sum(dv * n, axis=-1)
    a1 = (dp - rt * ct * dvn) / (2.0 * c2)
    a3 = (dp + rt * ct * dvn) / (2.0 * c2)
    a2 = dr - dp / c2
    l1 = cabs(vn - ct)
    l2 = cabs(vn)
    l3 = cabs(vn + ct)
    d = vL.shape[-1]
    D = np.empty(UL.shape, dtype=np.result_type(UL, UR))
    D[..., 0] = l1 * a1 + l2 * a2 + l3 * a3
    for i in range(d):
        D[..., 1 + i] = (l1 * a1 * (ut[..., i] - ct * n[..., i])
                         + l2 * (a2 * ut[..., i] + rt * (dv[..., i] - dvn * n[..., i]))
                         + l3 * a3 * (ut[..., i] + ct * n[..., i]))
    D[..., -1] = (l1 * a1 * (Ht - ct * vn)
                  + l2 * (a2 * 0.5 * q2 + rt * (np.sum(ut * dv, axis=-1) - vn * dvn))
                  + l3 * a3 * (Ht + ct * vn))
    return 0.5 * (normal_flux(UL, n, gamma) + normal_flux(UR, n, gamma)) - 0.5 * D


def slip_wall_ghost(UL, n, gamma):
    """Mirror state: (rho, rho (v - 2 (v.n) n), rho E)."""
    G = UL.copy()
    mn = np.sum(UL[..., 1:-1] * n, axis=-1)
    G[..., 1:-1] = UL[..., 1:-1] - 2.0 * mn[..., None] * n
    return G


def farfield_ghost(UL, n, prim_inf, gamma):
    """Riemann-invariant far field.

    Supersonic outflow (v_L.n >= c_L): interior state; supersonic inflow
    (v_L.n <= -c_L): free stream.  Otherwise R+ = v_L.n + 2 c_L/(gamma-1)
    from inside, R- = v_inf.n - 2 c_inf/(gamma-1) from outside,
    v_n = (R+ + R-)/2, c = (gamma-1)(R+ - R-)/4; entropy p/rho^gamma and
    tangential velocity from the interior if v_n >= 0, else from the free stream.
    """
    rL, vL, pL = primitives(UL, gamma)
    cL = np.sqrt(gamma * pL / rL)
    vnL = np.sum(vL * n, axis=-1)
    rinf = prim_inf[0]
    vinf = np.asarray(prim_inf[1:-1], dtype=np.float64)
    pinf = prim_inf[-1]
    cinf = np.sqrt(gamma * pinf / rinf)
    vninf = np.sum(vinf * n, axis=-1)
    Rp = vnL + 2.0 * cL / (gamma - 1.0)
    Rm = vninf - 2.0 * cinf / (gamma - 1.0)
    vnb = 0.5 * (Rp + Rm)
    cb = 0.25 * (gamma - 1.0) * (Rp - Rm)
    out = np.real(vnb) >= 0
    s_in = pL / rL ** gamma
    s_inf = pinf / rinf ** gamma
    sb = np.where(out, s_in, s_inf)
    vt = np.where(out[..., None], vL - vnL[..., None] * n, vinf - vninf[..., None] * n)
    rb = (cb * cb / (gamma * sb)) ** (1.0 / (gamma - 1.0))
    pb = rb * cb * cb / gamma
    vb = vt + vnb[..., None] * n
    G = np.empty(UL.shape, dtype=np.result_type(UL, vb))
    G[..., 0] = rb
    G[..., 1:-1] = rb[..., None] * vb
    G[..., -1] = pb / (gamma - 1.0) + 0.5 * rb * np.sum(vb * vb, axis=-1)
    Uinf = np.empty_like(G)
    Uinf[..., 0] = rinf
    Uinf[..., 1:-1] = rinf * vinf
    Uinf[..., -1] = pinf / (gamma - 1.0) + 0.5 * rinf * np.sum(vinf * vinf)
    sup_out = np.real(vnL) >= np.real(cL)
    sup_in = np.real(vnL) <= -np.real(cL)
    G = np.where(sup_out[..., None], UL, G)
    G = np.where(sup_in[..., None], Uinf, G)
    return G
