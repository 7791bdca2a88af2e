"""Linear stability and local truncation error on the scalar model problem
(Sec. 3: eqs. (model), (G_m), (grow), (y_poly), (rk2), (pcexp_bd),
(exp1_grow), (exp1_bd), (rkgrow), (taylor), (trun1), (trun2)).

Model: u' = J u + lambda u with J the "linear" part the exponential scheme
treats exactly; a = dt lambda, b = dt J.  Growth factors are derived here by
applying each scheme's stage formulas to the model (not by retyping the
printed closed forms), so that the printed forms can pin them.
"""

from math import factorial

import numpy as np
import mpmath
import sympy as sp


def phi1(b):
    """phi_1(b) = (e^b - 1)/b with phi_1(0) = 1 (numpy, elementwise)."""
    b = np.asarray(b, dtype=np.float64)
    out = np.ones_like(b)
    nz = b != 0
    out[nz] = np.expm1(b[nz]) / b[nz]
    return out


def growth_pcexp(a, b):
    """u_{n+1}/u_n of PCEXP on the model: x1 = phi1(b)(a+b) u, u* = u + x1,
    N* - N_n = lambda x1 (J x1 cancels), u_{n+1} = u* + (1/2) phi1(b) a x1."""
    p = phi1(b)
    x1 = p * (a + b)
    return 1.0 + x1 + 0.5 * a * p * x1


def growth_exp1(a, b):
    """EXP1 = first PCEXP stage: 1 + phi1(b)(a + b)."""
    return 1.0 + phi1(b) * (a + b)


def growth_tvdrk3(a, b):
    """Shu-Osher SSP-RK3 stages on u' = (a+b)/dt u."""
    z = np.asarray(a) + np.asarray(b)
    u1 = 1.0 + z
    u2 = 0.75 + 0.25 * (u1 + z * u1)
    return 1.0 / 3.0 + 2.0 / 3.0 * (u2 + z * u2)


def taylor_G(m, z):
    """G_m(z) = sum_{k=0}^m z^k / k!  (eq. (G_m)), mpmath-capable."""
    s = mpmath.mpf(0) if isinstance(z, mpmath.mpf) else 0.0
    t = 1
    for k in range(m + 1):
        if k > 0:
            t = t * z / k
        s = s + t
    return s


def max_stable_real(m, dps=45, step=0.05):
    """Largest x with |G_m(-y)| <= 1 for all y in [0, x] (Table "timesize")."""
    with mpmath.workdps(dps):
        f = lambda y: abs(taylor_G(m, -mpmath.mpf(y))) - 1
        y = mpmath.mpf(step)
        prev = y
        while f(y) <= 0:
            prev = y
            y += step
            if y > 10 * m + 10:
                raise RuntimeError("no boundary found")
        lo, hi = prev, y
        for _ in range(60):
            mid = (lo + hi) / 2
            if f(mid) <= 0:
                lo = mid
            else:
                hi = mid
        return float(lo)


def complex_region_radius(m, n_angle=64, dps=30):
    """Radius of the stability region of G_m along rays in the left half plane."""
    radii = []
    with mpmath.workdps(dps):
        for th in np.linspace(np.pi / 2 + 0.05, 3 * np.pi / 2 - 0.05, n_angle):
            d = mpmath.exp(1j * mpmath.mpf(th))
            f = lambda r: abs(taylor_G(m, r * d)) - 1
            r = dr = mpmath.mpf(0.1)
            while f(r) <= 0 and r < 10 * m + 10:
                r += dr
            lo, hi = r - dr, r
            for _ in range(30):
                mid = (lo + hi) / 2
                if f(mid) <= 0:
                    lo = mid
                else:
                    hi = mid
            radii.append(float(lo))
    return np.array(radii)


def rk3_strip_constant():
    """Left edge of the real TVDRK3 stability interval: the real root of
    |1 + z + z^2/2 + z^3/6| = 1 with z < 0 (found numerically)."""
    z = sp.Symbol("z", real=True)
    poly = 1 + z + z ** 2 / 2 + z ** 3 / 6 + 1
    roots = [complex(r) for r in sp.Poly(poly, z).nroots(n=30)]
    real = [r.real for r in roots if abs(r.imag) < 1e-20]
    return min(real)


# ----------------------------------------------------------------- symbolic
_a, _b, _h, _J, _lam = sp.symbols("a b h J lambda")


def symbolic_growth(scheme):
    """Growth factor as a sympy expression of (a, b), derived from the stages."""
    ph = (sp.exp(_b) - 1) / _b
    x1 = ph * (_a + _b)
    if scheme == "exp1":
        return 1 + x1
    if scheme == "pcexp":
        return 1 + x1 + sp.Rational(1, 2) * _a * ph * x1
    raise ValueError(scheme)


def series_in_b(scheme, order=3):
    """Taylor coefficients of the growth factor in b (eq. (y_poly))."""
    r = symbolic_growth(scheme)
    ser = sp.series(r, _b, 0, order).removeO()
    return [sp.simplify(ser.coeff(_b, k)) for k in range(order)]


def local_error(scheme, order=4):
    """Leading local error (exact - scheme) per unit u_n, with a = h lambda,
    b = h J, as a polynomial in h up to h^(order-1)."""
    r = symbolic_growth(scheme).subs({_a: _h * _lam, _b: _h * _J})
    exact = sp.exp(_h * (_J + _lam))
    diff = sp.series(exact - r, _h, 0, order).removeO()
    return sp.expand(diff)


SYMBOLS = dict(a=_a, b=_b, h=_h, J=_J, lam=_lam)
