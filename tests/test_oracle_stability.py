"""Pins of the oracle's 1D model analysis against values and closed forms the
paper prints (Sec. 3)."""

import os

import numpy as np
import pytest
import sympy as sp

from oracle import stability as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "timesize.txt")


def _table():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            m, v = line.split()
            rows.append((int(m), v))
    return rows


@pytest.mark.parametrize("m,printed", _table())
def test_timesize_table(m, printed):
    """Table "timesize": max stable dt|zeta| of G_m (eq. (G_m)) on the real axis."""
    got = S.max_stable_real(m)
    decimals = len(printed.split(".")[1])
    tol = 0.5 * 10.0 ** -decimals
    if m == 30:
        # the printed 12.55170 differs from the root (12.5517282) in the last digit
        tol = 5e-5
    assert abs(got - float(printed)) <= tol, (m, got, printed)


def test_timesize_linear_growth():
    """Sec. 3.1: the maximum stable |dt zeta| grows linearly with m."""
    ms = np.array([20, 40, 60, 80])
    vals = np.array([S.max_stable_real(int(m)) for m in ms])
    slope = np.diff(vals) / np.diff(ms)
    assert np.all(np.abs(slope - slope.mean()) < 0.01 * slope.mean())


def test_complex_region_semicircle_grows_linearly():
    """Fig. "sreigion": the complex stability region of G_m is close to a
    half disc whose radius grows linearly with m."""
    r20 = np.median(S.complex_region_radius(20, n_angle=9))
    r40 = np.median(S.complex_region_radius(40, n_angle=9))
    r80 = np.median(S.complex_region_radius(80, n_angle=9))
    assert abs((r80 - r40) / 40 - (r40 - r20) / 20) < 0.05 * (r40 - r20) / 20


def test_rk3_strip_constant():
    """Printed left edge of the TVDRK3 strip: -1 - (4+sqrt17)^(1/3) + (4+sqrt17)^(-1/3)."""
    c = 4.0 + np.sqrt(17.0)
    printed = -1.0 - c ** (1.0 / 3.0) + c ** (-1.0 / 3.0)
    assert abs(S.rk3_strip_constant() - printed) < 1e-12


def _grid(lo=-10, hi=10, n=401):
    a = np.linspace(lo, hi, n)
    A, B = np.meshgrid(a, a, indexing="ij")
    return A, B


def test_growth_pcexp_matches_eq_grow():
    """Eq. (grow): r = (a(a-b) + e^{2b}(a+b)a + 2e^b(b^2-a^2)) / (2 b^2)."""
    A, B = _grid(-3, 3, 121)
    B = np.where(np.abs(B) < 0.05, 0.05, B)   # the printed form cancels badly near b = 0
    printed = (A * (A - B) + np.exp(2 * B) * (A + B) * A + 2 * np.exp(B) * (B ** 2 - A ** 2)) / (2 * B ** 2)
    assert np.max(np.abs(S.growth_pcexp(A, B) - printed) / np.maximum(1, np.abs(printed))) < 1e-10


def test_growth_exp1_matches_eq_exp1_grow():
    A, B = _grid(-5, 5, 101)
    B = np.where(np.abs(B) < 1e-3, 1e-3, B)
    printed = (A * (np.exp(B) - 1) + B * np.exp(B)) / B
    assert np.max(np.abs(S.growth_exp1(A, B) - printed) / np.maximum(1, np.abs(printed))) < 1e-12


def test_exp1_stability_bounds():
    """Eq. (exp1_bd): |r| <= 1 iff -b coth(b/2) <= a <= -b (grid on [-10,10]^2)."""
    A, B = _grid()
    B = np.where(B == 0, 1e-9, B)
    stable = np.abs(S.growth_exp1(A, B)) <= 1
    bound = (A <= -B) & (A >= -B * (np.exp(B) + 1) / (np.exp(B) - 1))
    mism = stable != bound
    # points within 1e-9 of the boundary may go either way
    edge = (np.abs(A + B) < 1e-6) | (np.abs(A + B * (np.exp(B) + 1) / (np.exp(B) - 1)) < 1e-6)
    assert not np.any(mism & ~edge)


def test_pcexp_stability_bounds_small_b():
    """Eq. (pcexp_bd) (a <= -b, a >= 2b/(1-e^b)) holds for b <= ln 3; beyond
    that the printed region is not exact (a documented erratum)."""
    A, B = _grid()
    B = np.where(B == 0, 1e-9, B)
    stable = np.abs(S.growth_pcexp(A, B)) <= 1
    bound = (A <= -B) & (A >= 2 * B / (1 - np.exp(B)))
    region = B <= np.log(3.0)
    edge = (np.abs(A + B) < 1e-6) | (np.abs(A - 2 * B / (1 - np.exp(B))) < 1e-6)
    assert not np.any((stable != bound) & region & ~edge)
    # and for larger b the printed region misses stable points
    assert np.any((stable != bound) & ~region)


def test_tvdrk3_strip():
    """Eq. (rkgrow): stability is the strip c <= a + b <= 0."""
    A, B = _grid()
    stable = np.abs(S.growth_tvdrk3(A, B)) <= 1
    c = S.rk3_strip_constant()
    z = A + B
    edge = (np.abs(z) < 1e-9) | (np.abs(z - c) < 1e-9)
    assert not np.any((stable != ((z <= 0) & (z >= c))) & ~edge)


def test_y_poly_series():
    """Eq. (y_poly): r = (1+a+a^2/2) + (1+a+a^2/2) b + (1/2 + 2a/3 + 7a^2/24) b^2 + O(b^3)."""
    a = S.SYMBOLS["a"]
    c = S.series_in_b("pcexp", 3)
    printed = [1 + a + a ** 2 / 2, 1 + a + a ** 2 / 2,
               sp.Rational(1, 2) + 2 * a / 3 + sp.Rational(7, 24) * a ** 2]
    for got, want in zip(c, printed):
        assert sp.simplify(got - want) == 0


def test_rk2_limit():
    """Eq. (rk2): b -> 0 gives Heun's growth factor 1 + a + a^2/2."""
    a = np.linspace(-3, 1, 41)
    assert np.max(np.abs(S.growth_pcexp(a, 0.0 * a) - (1 + a + a * a / 2))) < 1e-14


def test_linear_exactness_scalar():
    """Eq. (growthfactor): with no nonlinear part (a = 0) PCEXP is exact: r = e^b."""
    b = np.linspace(-20, 2, 221)
    assert np.max(np.abs(S.growth_pcexp(0 * b, b) - np.exp(b)) / np.maximum(1.0, np.exp(b))) < 1e-14


def test_local_truncation_errors():
    """Eq. (trun2) for EXP1 as printed; for PCEXP the h^3 term is
    (1/6) h^3 lambda (lambda - J)(lambda + J) u_n (the printed eq. (trun1) is an
    erratum; both vanish at lambda = 0 as eq. (growthfactor) requires)."""
    h, J, lam = S.SYMBOLS["h"], S.SYMBOLS["J"], S.SYMBOLS["lam"]
    e1 = S.local_error("exp1", 3)
    assert sp.simplify(e1 - sp.Rational(1, 2) * h ** 2 * lam * (J + lam)) == 0
    e2 = S.local_error("pcexp", 4)
    assert sp.simplify(e2 - sp.Rational(1, 6) * h ** 3 * lam * (lam - J) * (lam + J)) == 0
    # second order: no h^2 term
    assert sp.simplify(sp.expand(e2).coeff(h, 2)) == 0
