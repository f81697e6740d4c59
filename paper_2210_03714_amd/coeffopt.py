"""Offline optimiser of the free parameters of the paper's shift families.

The parallel method approximates f(x) by r(x) = sum_i b_i / (1 - c_i x) (§2):
the shifts c_i are chosen, and the weights b_i then follow from the order
conditions sum_i b_i c_i^k = a_k, k = 0..P-1 (the Vandermonde system, eq. 4),
where a_k are the Taylor coefficients of f (1/k! for exp, 1/(k+1)! for phi1).
The forward error bound of §3 is

    eps(x) = sum_{k >= P} |a_k - sum_i b_i c_i^k| x^k .

§4.1 and §4.2 write the shifts as one-parameter families and pick the
parameter by a search that minimises eps(x) for small x:

    R4(alpha)  c = (0, 1/alpha, -1/alpha, 1/(2 alpha), -1/(2 alpha))
    R8(alpha)  c = (0, +-1/alpha, +-2/(3 alpha), +-1/(2 alpha), +-2/(5 alpha))

The search here maximises θ(tol), the largest x with eps(x) <= tol (§3),
which is what fixes the number of squarings or steps, over the parameters
whose round-off floor sum_k |w_k| θ 2^-53 (w_k = b_k c_k, the weights of the
round-off form of §4.3) stays a small share of tol.  For x near 0 the bound
is dominated by its first term |e_P(alpha)| x^P, e_P = a_P - sum_i b_i c_i^P,
and the optimum sits near a root of e_P.  It is reported with θ(tol) at it and
at its nearest integer, and the exact weights (rationals) at that integer.

§4.3 adds processors whose weights are free (more shifts than order
conditions).  ``explore_free`` evaluates, for given values of the free
weights, the remaining weights, θ(tol) and the round-off amplification
sum_k |w_k| (w_k = b_k c_k, the weights of the round-off form) that §4.3
warns about, so that candidate sets can be compared on both.

This is an offline tool (exact rationals and mpmath); the library's tables
are generated separately at build time.

    python -m paper_2210_03714_amd.coeffopt R4 exp
"""

import sys
from fractions import Fraction as Fr
from math import factorial

import mpmath as mp

mp.mp.dps = 40


def taylor(func, K):
    """a_0..a_{K-1} of exp (1/k!) or phi1 (1/(k+1)!), exact."""
    if func == "exp":
        return [Fr(1, factorial(k)) for k in range(K)]
    if func == "phi1":
        return [Fr(1, factorial(k + 1)) for k in range(K)]
    raise ValueError(func)


def family(name, alpha):
    """Shifts of a one-parameter family (§4.1, §4.2) at alpha (Fraction or mpf)."""
    one = Fr(1) if isinstance(alpha, Fr) else mp.mpf(1)
    if name == "R4":
        return [0 * one, one / alpha, -one / alpha, one / (2 * alpha), -one / (2 * alpha)]
    if name == "R8":
        out = [0 * one]
        for num, den in ((1, 1), (2, 3), (1, 2), (2, 5)):
            out += [num * one / (den * alpha), -num * one / (den * alpha)]
        return out
    raise ValueError(name)


def weights(c, a):
    """b solving sum_i b_i c_i^k = a_k, k = 0..P-1 (eq. 4), by elimination
    with partial pivoting in the arithmetic of c (exact for Fractions)."""
    P = len(c)
    exact = isinstance(c[0], Fr)
    M = [[(ci ** k if k else (Fr(1) if exact else mp.mpf(1))) for ci in c] +
         [a[k] if exact else mp.mpf(a[k].numerator) / a[k].denominator] for k in range(P)]
    for col in range(P):
        piv = max(range(col, P), key=lambda r: abs(M[r][col]))
        M[col], M[piv] = M[piv], M[col]
        for r in range(col + 1, P):
            f = M[r][col] / M[col][col]
            if f:
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    b = [None] * P
    for r in range(P - 1, -1, -1):
        s = M[r][P] - sum(M[r][j] * b[j] for j in range(r + 1, P))
        b[r] = s / M[r][r]
    return b


def error_coeffs(c, b, a):
    """e_k = a_k - sum_i b_i c_i^k for k = 0..len(a)-1 (signed)."""
    return [a[k] - sum(bi * (ci ** k if k else 1) for bi, ci in zip(b, c)) for k in range(len(a))]


def lead_error(name, func, alpha):
    """e_P(alpha), the first nonzero coefficient of f - r (signed), in mpmath."""
    c = family(name, mp.mpf(alpha))
    a = taylor(func, len(c) + 1)
    b = weights(c, a)
    return error_coeffs(c, b, [mp.mpf(x.numerator) / x.denominator for x in a])[len(c)]


_THETA = {}


def theta(name, func, alpha, tol, K=150):
    """θ(tol): the largest x with eps(x) <= tol (bisection below 0.9 / max|c|)."""
    key = (name, func, float(alpha), tol, K)
    if key not in _THETA:
        _THETA[key] = _theta(name, func, alpha, tol, K)
    return _THETA[key]


def _theta(name, func, alpha, tol, K):
    c = family(name, mp.mpf(alpha))
    a = taylor(func, K)
    b = weights(c, a)
    am = [mp.mpf(x.numerator) / x.denominator for x in a]
    d = [abs(e) for e in error_coeffs(c, b, am)]
    P = len(c)
    eps = lambda x: mp.fsum(d[k] * x ** k for k in range(P, K))
    lo, hi = mp.mpf(0), mp.mpf("0.9") / max(abs(x) for x in c)
    if eps(hi) <= tol:
        return float(hi)
    for _ in range(60):
        mid = (lo + hi) / 2
        if eps(mid) <= tol:
            lo = mid
        else:
            hi = mid
    return float(lo)


def roundoff_floor(name, func, alpha, tol):
    """sum_k |w_k| θ(tol) 2^-53, w_k = b_k c_k: the rounding of the round-off
    form (§4.3) that no tolerance can go under."""
    c = family(name, mp.mpf(alpha))
    b = weights(c, taylor(func, len(c)))
    sw = mp.fsum(abs(bi * ci) for bi, ci in zip(b, c))
    return float(sw * theta(name, func, alpha, tol) * mp.mpf(2) ** -53)


def optimise_alpha(name, func, tol=1e-12, share=0.05, lo=2.0, hi=12.0, grid=21):
    """The alpha in [lo, hi] that maximises θ(tol) -- the largest ||B|| for
    which the bound eps stays below tol, so the fewest squarings or steps --
    among the alphas whose round-off floor (roundoff_floor) is at most
    share * tol: a grid, then golden section around its best feasible point.
    Near an alpha where e_P vanishes the bound's leading term drops out, which
    is what the search finds for the families of §4.1-4.2; the round-off
    condition rules out the larger alphas, whose shifts near 0 need large
    weights of opposite signs."""
    def score(x):
        if roundoff_floor(name, func, x, tol) > share * tol:
            return -1.0
        return theta(name, func, x, tol)
    xs = [lo + (hi - lo) * i / (grid - 1) for i in range(grid)]
    sc = [score(x) for x in xs]
    i = max(range(grid), key=lambda j: sc[j])
    if sc[i] < 0:
        raise ValueError("no alpha in [%g, %g] keeps the round-off floor under %g tol" % (lo, hi, share))
    a = mp.mpf(xs[max(i - 1, 0)])
    b = mp.mpf(xs[min(i + 1, grid - 1)])
    g = (mp.sqrt(5) - 1) / 2
    x1, x2 = b - g * (b - a), a + g * (b - a)
    f1, f2 = score(x1), score(x2)
    for _ in range(30):
        if f1 > f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - g * (b - a)
            f1 = score(x1)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + g * (b - a)
            f2 = score(x2)
    return float((a + b) / 2)


def exact_set(name, func, alpha):
    """Shifts and weights at a rational alpha, exactly (eq. 4)."""
    c = family(name, Fr(alpha))
    b = weights(c, taylor(func, len(c)))
    return c, b


def explore_free(c, free, func, tol, K=200):
    """A set with more shifts than order conditions (§4.3): the last
    len(free) weights take the given values, the others solve the order
    conditions k = 0..P-1-len(free) (exact).  Returns the weights, θ(tol),
    and sum_k |b_k c_k| (the round-off amplification of §4.3)."""
    c = [Fr(x) for x in c]
    nf = len(free)
    P = len(c) - nf
    a = taylor(func, K)
    rhs = [a[k] - sum(Fr(f) * (ci ** k if k else 1) for f, ci in zip(free, c[P:])) for k in range(P)]
    b = weights(c[:P], rhs) + [Fr(f) for f in free]
    e = error_coeffs(c, b, a)
    order = next(k for k in range(K) if e[k] != 0) - 1
    d = [abs(mp.mpf(x.numerator) / x.denominator) for x in e]
    eps = lambda x: mp.fsum(d[k] * x ** k for k in range(order + 1, K))
    lo, hi = mp.mpf(0), mp.mpf("0.9") / max(abs(float(x)) for x in c)
    for _ in range(80):
        mid = (lo + hi) / 2
        if eps(mid) <= tol:
            lo = mid
        else:
            hi = mid
    amp = float(sum(abs(bi * ci) for bi, ci in zip(b, c)))
    return {"b": b, "order": order, "theta": float(lo), "sum_abs_w": amp}


def explore_free_hybrid(c, free, func, tol, K=150):
    """The hybrid form of §4.3, r(x) = d0 + d1 x + d2 x^2 + sum_i b_i / (1 - c_i x):
    the last len(free) weights b_i take the given values, the other b_i solve
    the order conditions k = 3..P+2 (P = len(c) - len(free)), and d_k = a_k -
    sum_i b_i c_i^k for k = 0, 1, 2.  Returns the weights, the polynomial part,
    the order, θ(tol) and sum_k |b_k c_k| + |d1| + |d2| (the round-off
    amplification of the round-off form)."""
    c = [Fr(x) for x in c]
    nf = len(free)
    P = len(c) - nf
    a = taylor(func, K)
    # sum_{i<P} (b_i c_i^3) c_i^j = a_{j+3} - sum_free b c^{j+3}, j = 0..P-1
    rhs = [a[j + 3] - sum(Fr(f) * ci ** (j + 3) for f, ci in zip(free, c[P:])) for j in range(P)]
    e = weights(c[:P], rhs)
    b = [ei / ci ** 3 for ei, ci in zip(e, c[:P])] + [Fr(f) for f in free]
    d = [a[k] - sum(bi * (ci ** k if k else 1) for bi, ci in zip(b, c)) for k in range(3)]
    err = [a[k] - sum(bi * (ci ** k if k else 1) for bi, ci in zip(b, c)) - (d[k] if k < 3 else 0)
           for k in range(K)]
    order = next(k for k in range(K) if err[k] != 0) - 1
    dm = [abs(mp.mpf(x.numerator) / x.denominator) for x in err]
    eps = lambda x: mp.fsum(dm[k] * x ** k for k in range(order + 1, K))
    lo, hi = mp.mpf(0), mp.mpf("0.9") / max(abs(float(x)) for x in c)
    for _ in range(60):
        mid = (lo + hi) / 2
        if eps(mid) <= tol:
            lo = mid
        else:
            hi = mid
    amp = float(sum(abs(bi * ci) for bi, ci in zip(b, c)) + abs(d[1]) + abs(d[2]))
    return {"b": b, "d": d, "order": order, "theta": float(lo), "sum_abs_w": amp}


def main(argv):
    name = argv[1] if len(argv) > 1 else "R4"
    func = argv[2] if len(argv) > 2 else "exp"
    tol = float(argv[3]) if len(argv) > 3 else 1e-12
    al = optimise_alpha(name, func, tol)
    ar = round(al)
    print("%s %s: optimum alpha = %.6f (theta(%g) maximal), nearest integer %d, e_P there %.3e"
          % (name, func, al, tol, ar, float(lead_error(name, func, al))))
    print("  theta(%g) at the optimum %.6f, at %d %.6f" % (tol, theta(name, func, al, tol), ar,
                                                          theta(name, func, ar, tol)))
    c, b = exact_set(name, func, ar)
    for ci, bi in zip(c, b):
        print("  c = %-8s b = %s" % (ci, bi))


if __name__ == "__main__":
    main(sys.argv)
