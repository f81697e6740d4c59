"""Pins for the oracle's coefficient sets against the numbers the paper prints.

Every printed weight table must come out of the oracle's exact solve of the
Vandermonde system (§2, eq. 4) as the identical rational; the complex Padé
pairs must reproduce the Padé rational functions of §2 (eqs. 5, 6).
"""

import math
from fractions import Fraction as Fr

import pytest
import sympy as sp

from oracle import coefficients as co


def _fr(s):
    return Fr(s)


def test_printed_weight_tables_exact(golden):
    for entry in golden["weights"]:
        c = [_fr(x) for x in entry["shifts"]]
        a = co.taylor_coeffs(entry["func"], len(c))
        b = co.solve_weights(c, a)
        assert b == [_fr(x) for x in entry["b"]], entry["cite"]


@pytest.mark.parametrize("m,idx", [(4, 3), (8, 5), (5, 6)])
def test_registry_sets_are_the_papers(golden, m, idx):
    entry = golden["weights"][idx]
    c, b = co.real_set("exp", m)
    assert c == [_fr(x) for x in entry["shifts"]]
    assert b == [_fr(x) for x in entry["b"]]


@pytest.mark.parametrize("m", [4, 5, 8])
@pytest.mark.parametrize("func", ["exp", "phi1"])
def test_order_conditions(m, func):
    """alpha_k = a_k exactly for k <= P-1 and not for k = P (eq. 3: the error
    is O(x^P) and no better)."""
    c, b = co.real_set(func, m)
    P = len(c)
    a = co.taylor_coeffs(func, P + 1)
    al = co.moments(b, c, P + 1)
    assert al[:P] == a[:P]
    assert al[P] != a[P]
    assert sum(b) == a[0]          # the identity behind the round-off form (§4.3)
    assert co.order_of(m) == P - 1


def test_solver_is_not_trivially_symmetric():
    """A transposed system (sum_k b_k c_i^k) gives a different answer; guard
    against solving V b = a instead of V^T b = a."""
    c = co.shifts_frac4()
    a = co.taylor_coeffs("exp", 5)
    b = co.solve_weights(c, a)
    # check each equation of eq. (4) directly
    for k in range(5):
        assert sum(bi * ci ** k for bi, ci in zip(b, c)) == a[k]


def test_pade_pair_exp_reproduces_r22():
    x = sp.symbols("x")
    pr = co.pade22_exp()
    c, b, d = pr["c"], pr["b"], pr["d"]
    r = d + b / (1 - c * x) + sp.conjugate(b) / (1 - sp.conjugate(c) * x)
    r22 = (1 + x / 2 + x ** 2 / 12) / (1 - x / 2 + x ** 2 / 12)
    assert sp.simplify(sp.expand_complex(r - r22)) == 0
    assert sp.simplify(c - (sp.Rational(1, 4) + sp.sqrt(3) * sp.I / 12)) == 0
    assert sp.simplify(b - (-2 * sp.sqrt(3) * sp.I)) == 0
    assert d == 1


def test_pade_pair_phi1_reproduces_printed_form(golden):
    x = sp.symbols("x")
    pr = co.pade22_phi1()
    c, b, d = pr["c"], pr["b"], pr["d"]
    r = d + b / (1 - c * x) + sp.conjugate(b) / (1 - sp.conjugate(c) * x)
    rt = (1 + x / 10 + x ** 2 / 60) / (1 - sp.Rational(2, 5) * x + x ** 2 / 20)
    assert sp.simplify(sp.expand_complex(r - rt)) == 0
    # the printed pole form of eq. (6)
    printed = sp.Rational(1, 3) + 2 * sp.re((sp.Rational(7, 3) + 8 * sp.I) / (x - (4 - 2 * sp.I)))
    xs = sp.symbols("xs", real=True)
    assert sp.simplify(printed.subs(x, xs) - rt.subs(x, xs)) == 0


def test_printed_r22_pole_form_needs_sqrt3_reading():
    """eq. (5) prints the numerator as 6 + i 6 sqrt(6); only 6 + 6 sqrt(3) i
    makes the pole form equal r_22."""
    xs = sp.symbols("xs", real=True)
    r22 = (1 + xs / 2 + xs ** 2 / 12) / (1 - xs / 2 + xs ** 2 / 12)
    pole = 3 - sp.I * sp.sqrt(3)
    good = 1 + 2 * sp.re((6 + 6 * sp.sqrt(3) * sp.I) / (xs - pole))
    bad = 1 + 2 * sp.re((6 + 6 * sp.sqrt(6) * sp.I) / (xs - pole))
    assert sp.simplify(good - r22) == 0
    assert sp.simplify(bad - r22) != 0


@pytest.mark.parametrize("m", [1, 4, 5, 8])
@pytest.mark.parametrize("func", ["exp", "phi1"])
def test_roundoff_form_equals_plain_form(m, func):
    """a0 + sum w_k x/(1 - c_k x) == sum b_k/(1 - c_k x) (§4.3) at sample x."""
    a0, terms = co.roundoff_terms(func, m)
    for x in (0.013, -0.07, 0.21):
        lhs = a0
        for c, w, pair in terms:
            t = w * x / (1 - c * x)
            lhs += 2 * t.real if pair else t
        if m == 1:
            pr = co.pade22_exp() if func == "exp" else co.pade22_phi1()
            c, b, d = (complex(pr[k].evalf(30)) for k in ("c", "b", "d"))
            rhs = (d + 2 * (b / (1 - c * x)).real).real
        else:
            # plain form evaluated exactly (in floats it cancels: sum|b| ~ 5.8e3 for m = 8)
            cs, bs = co.real_set(func, m)
            xq = Fr(x)
            rhs = float(sum(bi / (1 - ci * xq) for ci, bi in zip(cs, bs)))
        assert abs(lhs.real - rhs) <= 2e-13 * max(1, abs(rhs))


def test_hybrid_sets_are_the_papers(golden):
    """§4.3: both 10th-order hybrid sets, solved from the order conditions
    with b_9, b_10 fixed, equal the printed b_1..b_8 and d_0..d_2 exactly."""
    for e in golden["hybrid"]:
        c, b, d = co.hybrid_set(e["set"])
        assert c == [Fr(x) for x in e["shifts"]], e["cite"]
        assert b[:8] == [Fr(x) for x in e["b"]], e["cite"]
        assert b[8:] == [Fr(x) for x in e["b_free"]], e["cite"]
        assert d == [Fr(x) for x in e["d"]], e["cite"]
        assert d[0] + sum(b) == 1  # a0 = 1: the round-off form's constant


def test_hybrid_set_order_conditions():
    """r(x) = d0 + d1 x + d2 x^2 + sum b_i/(1 - c_i x) matches exp to order 10
    and misses at order 11 (independent of the solver: the moments are summed
    directly)."""
    for v in ("R10", "R10*"):
        c, b, d = co.hybrid_set(v)
        for k in range(12):
            alpha = sum(bi * ci ** k for bi, ci in zip(b, c)) + (d[k] if k < 3 else 0)
            if k <= 10:
                assert alpha == Fr(1, math.factorial(k)), (v, k)
            else:
                assert alpha != Fr(1, math.factorial(k)), (v, k)


def test_log1m_registry_is_the_papers(golden):
    """The log(1 - x) set (m = 5) is the §2 worked example: shifts 1/2..1/6 and
    the printed weights."""
    e = [e for e in golden["weights"] if e["func"] == "log1m"][0]
    c, b = co.real_set("log1m", 5)
    assert c == [Fr(x) for x in e["shifts"]]
    assert b == [Fr(x) for x in e["b"]]
    a0, terms = co.roundoff_terms("log1m", 5)
    assert a0 == 0.0 and len(terms) == 5
