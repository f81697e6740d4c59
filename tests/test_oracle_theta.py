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
