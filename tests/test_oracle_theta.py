"""Pins for the oracle's θ (forward error bound of §3) against Tables 1 and 2
of §5.1 and the accuracy orderings the paper states in §2, §4.1 and §4.2."""

from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import coefficients as co
from oracle import theta as th

TOLS = [2.0 ** -24, 1e-8, 1e-10, 1e-12]


def test_table1_taylor_thresholds(golden):
    for e in golden["theta_single"]:
        if e["kind"] == "taylor":
            v = th.theta_taylor("exp", e["degree"], 2.0 ** -24)
            assert round(v, 3) == e["theta"], e["cite"]


def test_table2_r5_threshold(golden):
    e = [e for e in golden["theta_single"] if e["kind"] == "set"][0]
    assert round(th.theta_set("exp", 5, 2.0 ** -24), 3) == e["theta"]


def test_bound_is_relative_would_not_match():
    """Dividing eps(x) by e^x (a relative bound) moves Table 1 away from the
    printed values, which fixes the absolute reading."""
    cf = th.bound_coeffs_taylor("exp", 10, 400)
    lo, hi = 0.0, 5.0
    for _ in range(80):
        mid = (lo + hi) / 2
        if th.eps(cf, mid) / np.exp(mid) <= 2.0 ** -24:
            lo = mid
        else:
            hi = mid
    assert round(lo, 3) != 1.073


@pytest.mark.parametrize("tol", TOLS)
def test_orderings_stated_in_paper(golden, tol):
    # §2 / §4.1: R4 (alpha = 5) more accurate than the Padé r22
    assert th.theta_set("exp", 4, tol) > th.theta_set("exp", 1, tol)
    # §4.1: phi1 on alpha = 6 shifts beats the phi1 Padé pair
    e = golden["weights"][4]
    c = [Fr(x) for x in e["shifts"]]
    b = [Fr(x) for x in e["b"]]
    th_a6 = th.theta(th.bound_coeffs_real("phi1", c, b), tol, 3.0)
    assert th_a6 > th.theta_set("phi1", 1, tol)
    # §4.2: R8 more accurate than the degree-8 Taylor polynomial
    assert th.theta_set("exp", 8, tol) > th.theta_taylor("exp", 8, tol)


def test_eps_at_theta_equals_tol():
    cf = th.bound_coeffs_real("exp", *co.real_set("exp", 8))
    t = th.theta_set("exp", 8, 1e-12)
    assert th.eps(cf, t) <= 1e-12
    assert th.eps(cf, t * (1 + 1e-9)) > 1e-12


def test_bound_holds_on_matrices():
    """||e^B - r(B)||_1 <= tol for random B with ||B||_1 just below θ,
    with r evaluated in the plain form of eq. (2) and e^B from scipy."""
    rng = np.random.default_rng(7)
    tol = 1e-8
    c, b = co.real_set("exp", 8)
    t = th.theta_set("exp", 8, tol)
    for _ in range(5):
        B = rng.standard_normal((12, 12))
        B *= 0.999 * t / np.abs(B).sum(0).max()
        I = np.eye(12)
        r = sum(float(bi) * np.linalg.inv(I - float(ci) * B) for ci, bi in zip(c, b))
        err = np.abs(r - sla.expm(B)).sum(0).max()
        assert err <= tol


def test_table2_r10_threshold(golden):
    """§5.1, Table 2: θ_10 = 1.734 for the r_10^(11) scheme at u <= 2^-24."""
    e = [e for e in golden["theta_single"] if e["kind"] == "hybrid"][0]
    c, b, d = co.hybrid_set(e["set"])
    cf = th.bound_coeffs_hybrid("exp", c, b, d, 400)
    v = th.theta(cf, 2.0 ** -24, 0.9 / float(max(abs(x) for x in c)))
    assert round(v, 3) == e["theta"], e["cite"]


# ------------------- the m = 1 Padé pairs: bound coefficients from eqs. 5, 6 --

def _printed_pade(func):
    """The rational forms printed in §2: r22 (eq. 5) and r~22 (eq. 6)."""
    import sympy as sp
    x = sp.symbols("x")
    if func == "exp":
        return x, (1 + x / 2 + x ** 2 / 12) / (1 - x / 2 + x ** 2 / 12)
    return x, (1 + sp.Rational(1, 10) * x + x ** 2 / 60) / (1 - sp.Rational(2, 5) * x + x ** 2 / 20)


def check_pair_bound_against_printed_form(func, K=13):
    """|a_k - alpha_k| of the oracle's pole form equals |a_k - d_k|, where d_k
    are the Taylor coefficients of the printed quotient of quadratics (§3: the
    d_k of the Padé bounds are the series coefficients of r22 / r~22), for
    k < K.  The quotient's series is taken by sympy from the printed
    numerator and denominator, independently of the partial fractions."""
    import sympy as sp
    import mpmath
    x, r = _printed_pade(func)
    ser = sp.series(r, x, 0, K).removeO()
    dk = [sp.Rational(ser.coeff(x, k)) for k in range(K)]
    ak = co.taylor_coeffs(func, K)
    want = [abs(Fr(int(a.numerator), int(a.denominator)) - Fr(int(d.p), int(d.q))) for a, d in zip(ak, dk)]
    got = th.bound_coeffs_pair(func, co.pade22_exp() if func == "exp" else co.pade22_phi1(), K)
    with mpmath.workdps(50):
        for k in range(K):
            w = mpmath.mpf(want[k].numerator) / want[k].denominator
            assert abs(got[k] - w) <= mpmath.mpf(10) ** -40 * max(1, abs(w)), (func, k, got[k], w)
    return want


@pytest.mark.parametrize("func", ["exp", "phi1"])
def test_pair_bound_coefficients_match_printed_pade(func):
    want = check_pair_bound_against_printed_form(func)
    # both are 4th order (eqs. 5, 6): zero through k = 4, nonzero at k = 5
    assert all(w == 0 for w in want[:5]) and want[5] != 0
    if func == "exp":
        # e^x - r22(x): 1/720 x^5 + 1/720 x^6 + 47/60480 x^7 + 19/60480 x^8 ...
        assert want[5:9] == [Fr(1, 720), Fr(1, 720), Fr(47, 60480), Fr(19, 60480)]


def test_planted_pair_factor_error_is_caught(monkeypatch):
    """Drop the factor 2 of the conjugate pair's moments in the oracle: the
    printed-form pin must fail (while theta(R4) > theta(r22) alone would
    still hold)."""
    import mpmath

    def broken(d, b, c, k):
        return d + mpmath.re(b) if k == 0 else mpmath.re(b * c ** k)
    monkeypatch.setattr(th, "pair_moment", broken)
    assert th.theta_set("exp", 4, 1e-12) > th.theta_set("exp", 1, 1e-12)
    with pytest.raises(AssertionError):
        check_pair_bound_against_printed_form("exp")
