"""Forward error bound and the admissible-norm threshold θ (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

§3: with alpha_k = sum_i b_i c_i^k the Taylor coefficients of the approximant,
    || f(B) - r(B) || <= sum_k |a_k - alpha_k| ||B||^k =: eps(||B||)
for any consistent norm.  For a tolerance tol, θ is the largest x with
eps(x) <= tol; a matrix with ||B|| <= θ then meets tol.  The bound is absolute
(not divided by ||f(B)||): that reading reproduces the printed single-precision
thresholds of Tables 1 and 2 (§5.1).

Evaluation is done with mpmath at 60 significant digits, summing K terms
(default 400) of the series; the differences a_k - alpha_k are exact rationals
for real shift sets.  θ is found by bisection and rounded down to binary64.
"""

from fractions import Fraction as Fr
import mpmath

from . import coefficients as co

DPS = 60


def _mpf(q):
    return mpmath.mpf(q.numerator) / q.denominator


def bound_coeffs_real(func, c, b, K=400):
    """|a_k - alpha_k| for k = 0..K-1, exact (real shift sets)."""
    a = co.taylor_coeffs(func, K)
    al = co.moments(b, c, K)
    return [abs(x - y) for x, y in zip(a, al)]


def bound_coeffs_pair(func, pair, K=400):
    """|a_k - alpha_k| for a complex-conjugate pair set d + b/(1-cx) + conj.

    alpha_0 = d + 2 Re b, alpha_k = 2 Re(b c^k) for k >= 1.  Evaluated in
    mpmath (the pair constants involve sqrt(3))."""
    with mpmath.workdps(DPS):
        c = mpmath.mpc(str(pair["c"].as_real_imag()[0].evalf(DPS)),
                       str(pair["c"].as_real_imag()[1].evalf(DPS)))
        b = mpmath.mpc(str(pair["b"].as_real_imag()[0].evalf(DPS)),
                       str(pair["b"].as_real_imag()[1].evalf(DPS)))
        d = mpmath.mpf(str(pair["d"].evalf(DPS)))
        a = co.taylor_coeffs(func, K)
        return [abs(_mpf(a[k]) - pair_moment(d, b, c, k)) for k in range(K)]


def pair_moment(d, b, c, k):
    """Taylor coefficient k of d + b/(1 - c x) + conj(b)/(1 - conj(c) x):
    the two geometric series add to 2 Re(b c^k); the constant d joins k = 0."""
    return d + 2 * mpmath.re(b) if k == 0 else 2 * mpmath.re(b * c ** k)


def bound_coeffs_taylor(func, degree, K=400):
    """Truncated Taylor polynomial of the given degree: a_k for k > degree."""
    a = co.taylor_coeffs(func, K)
    return [Fr(0) if k <= degree else abs(a[k]) for k in range(K)]


def _as_mpf(coeffs):
    return [_mpf(q) if isinstance(q, Fr) else mpmath.mpf(q) for q in coeffs]


def eps(coeffs, x):
    """eps(x) = sum_k coeffs[k] x^k  (§3), in mpmath (Horner; all terms >= 0)."""
    with mpmath.workdps(DPS):
        cf = coeffs if coeffs and isinstance(coeffs[0], mpmath.mpf) else _as_mpf(coeffs)
        x = mpmath.mpf(x)
        s = mpmath.mpf(0)
        for q in reversed(cf):
            s = s * x + q
        return s


def theta(coeffs, tol, hi):
    """Largest x in [0, hi) with eps(x) <= tol, by bisection (§3).

    ``hi`` must lie inside the radius of convergence of the series.  The
    result is rounded down to a binary64 value."""
    with mpmath.workdps(DPS):
        coeffs = _as_mpf(coeffs)
        tol = mpmath.mpf(tol)
        lo, up = mpmath.mpf(0), mpmath.mpf(hi)
        if eps(coeffs, up) <= tol:
            raise ValueError("bisection interval too small")
        for _ in range(200):
            mid = (lo + up) / 2
            if eps(coeffs, mid) <= tol:
                lo = mid
            else:
                up = mid
        v = float(lo)
        if mpmath.mpf(v) > lo:  # round down
            import math
            v = math.nextafter(v, 0.0)
        return v


def theta_set(func, m, tol, K=400):
    """θ for the oracle's registry entry (func, m)."""
    if m == 1:
        pr = co.pade22_exp() if func == "exp" else co.pade22_phi1()
        cf = bound_coeffs_pair(func, pr, K)
        cmax = abs(complex(pr["c"].evalf(30)))
    elif m in co.HYBRID_SETS:
        c, b, d = co.hybrid_set(co.HYBRID_SETS[m], func)
        cf = bound_coeffs_hybrid(func, c, b, d, K)
        cmax = float(max(abs(x) for x in c))
    else:
        c, b = co.real_set(func, m)
        cf = bound_coeffs_real(func, c, b, K)
        cmax = float(max(abs(x) for x in c))
    return theta(cf, tol, 0.9 / cmax)


def bound_coeffs_hybrid(func, c, b, d, K=400):
    """|a_k - alpha_k| for a hybrid set (§4.3): alpha_k = sum_i b_i c_i^k plus
    d_k for k <= 2, exact."""
    a = co.taylor_coeffs(func, K)
    al = co.moments(b, c, K)
    for k in range(3):
        al[k] += d[k]
    return [abs(x - y) for x, y in zip(a, al)]


def theta_taylor(func, degree, tol, K=400):
    return theta(bound_coeffs_taylor(func, degree, K), tol, 50.0)

