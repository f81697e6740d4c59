"""Exact coefficient sets of the parallel rational approximations (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method of §2 writes f(x) ~ r(x) = sum_i b_i / (1 - c_i x)  (eq. 2) where the
shifts c_i are chosen freely and the weights b_i solve the transposed
Vandermonde system  sum_i b_i c_i^k = a_k,  k = 0..P-1  (eq. 4), a_k being the
Taylor coefficients of f (eq. 1).  Everything here is done in exact rational
arithmetic (``fractions.Fraction``), by plain Gaussian elimination on that
system, so the printed tables of §2, §4.1, §4.2 and §5.1 can be compared for
exact equality.  Floats appear only when a caller asks for them, and each
constant is then rounded once to the nearest binary64.

The two complex-pole Padé sets of §2 (eqs. 5 and 6) are rebuilt here from the
Padé numerator and denominator with sympy, in the (1 - c x)^{-1} convention
used everywhere else.
"""

from fractions import Fraction as Fr
from math import factorial

import sympy as sp

# --------------------------------------------------------------------------
# Taylor coefficients a_k of the target functions (eq. 1)
# --------------------------------------------------------------------------


def taylor_coeffs(func, K):
    """a_0..a_{K-1} of the power series of ``func`` about 0, as Fractions.

    exp:    a_k = 1/k!
    phiJ:   phi_J(x) = (e^x - sum_{j<J} x^j/j!) / x^J, so a_k = 1/(k+J)!  (§1;
            the subtracted polynomial has degree J-1, otherwise phi_J(0) would
            vanish)
    log1m:  log(1 - x) = -sum_{k>=1} x^k / k                         (§2)
    """
    if func == "exp":
        return [Fr(1, factorial(k)) for k in range(K)]
    if func.startswith("phi"):
        J = int(func[3:])
        return [Fr(1, factorial(k + J)) for k in range(K)]
    if func == "log1m":
        return [Fr(0)] + [Fr(-1, k) for k in range(1, K)]
    raise ValueError(func)


# --------------------------------------------------------------------------
# Shift sets (real)
# --------------------------------------------------------------------------


def shifts_R4(alpha=5):
    """§4.1: four processors, c = (0, 1/a, -1/a, 1/(2a), -1/(2a))."""
    a = Fr(alpha)
    return [Fr(0), 1 / a, -1 / a, 1 / (2 * a), -1 / (2 * a)]


def shifts_R8(alpha=5):
    """§4.2: eight processors, c = (0, ±1/a, ±2/(3a), ±1/(2a), ±2/(5a))."""
    a = Fr(alpha)
    out = [Fr(0)]
    for base in (1 / a, 2 / (3 * a), 1 / (2 * a), 2 / (5 * a)):
        out += [base, -base]
    return out


def shifts_frac4():
    """§2 worked example: five shifts c_i = 1/(i+1), i = 1..5 (no zero shift)."""
    return [Fr(1, i + 1) for i in range(1, 6)]


def shifts_R5():
    """§5.1: c_1 = 0 and c_i = 1/(i+1), i = 2..6."""
    return [Fr(0)] + [Fr(1, i + 1) for i in range(2, 7)]


# --------------------------------------------------------------------------
# The linear system of eq. (4), solved exactly
# --------------------------------------------------------------------------


def solve_weights(c, a):
    """Solve sum_i b_i c_i^k = a_k for k = 0..P-1 (eq. 4) exactly.

    ``c`` are P distinct Fractions, ``a`` at least P Fractions.  Plain Gaussian
    elimination with exact arithmetic on the P x P matrix V[k][i] = c_i^k
    (0^0 = 1, so a zero shift contributes only to the k = 0 row).
    """
    P = len(c)
    if len(set(c)) != P:
        raise ValueError("shifts must be distinct (§2)")
    M = [[ci ** k if not (ci == 0 and k == 0) else Fr(1) for ci in c] + [a[k]]
         for k in range(P)]
    for col in range(P):
        piv = next(r for r in range(col, P) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(P):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[i][P] / M[i][i] for i in range(P)]


def moments(b, c, K):
    """alpha_k = sum_i b_i c_i^k for k = 0..K-1: the Taylor coefficients of the
    rational approximant itself (§3, forward bound)."""
    out = []
    for k in range(K):
        s = Fr(0)
        for bi, ci in zip(b, c):
            s += bi * (Fr(1) if k == 0 else ci ** k)
        out.append(s)
    return out


# --------------------------------------------------------------------------
# Hybrid 10th-order sets (§4.3): r(x) = d0 + d1 x + d2 x^2 + sum_i b_i/(1 - c_i x)
# --------------------------------------------------------------------------


def shifts_R10(variant):
    """The ten shifts of the two 10th-order examples of §4.3, named as in the
    list of methods of the numerical examples (§5):
    'R10*': c_i = 1/(6 + i), i = 1..10 (eqs. Frac10ciNO, Frac10biNO);
    'R10':  c_{2i-1} = -1/(6 + 2i), c_{2i} = 1/(6 + 2i), i = 1..5
            (eqs. Frac10ci, Frac10bi)."""
    if variant == "R10*":
        return [Fr(1, 6 + i) for i in range(1, 11)]
    if variant == "R10":
        out = []
        for i in range(1, 6):
            out += [Fr(-1, 6 + 2 * i), Fr(1, 6 + 2 * i)]
        return out
    raise ValueError(variant)


HYBRID_FREE = {"R10*": (Fr(-50000), Fr(350000)), "R10": (Fr(2000), Fr(-3500))}


def hybrid_set(variant, func="exp"):
    """Exact (c, b, d) of a §4.3 hybrid set: with b_9, b_10 fixed, b_1..b_8
    solve sum_{i=1}^{10} b_i c_i^k = a_k for k = 3..10, and
    d_k = a_k - sum_i b_i c_i^k for k = 0, 1, 2 (so that d_0 + d_1 x + d_2 x^2
    carries the low orders).  Plain Gaussian elimination on the 8 x 8 system
    in exact arithmetic."""
    c = shifts_R10(variant)
    b9, b10 = HYBRID_FREE[variant]
    a = taylor_coeffs(func, 11)
    M = [[c[i] ** k for i in range(8)] + [a[k] - b9 * c[8] ** k - b10 * c[9] ** k] for k in range(3, 11)]
    for col in range(8):
        piv = next(r for r in range(col, 8) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(8):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    b = [M[i][8] / M[i][i] for i in range(8)] + [b9, b10]
    d = [a[k] - sum(bi * ci ** k for bi, ci in zip(b, c)) for k in range(3)]
    return c, b, d


# --------------------------------------------------------------------------
# Complex-conjugate Padé sets (§2, eqs. 5 and 6)
# --------------------------------------------------------------------------


def _pade_pair(num, den):
    """Partial fractions of num(x)/den(x) (both quadratic, den(0) = 1) as
    d + b/(1 - c x) + conj(b)/(1 - conj(c) x), exactly, with sympy.

    den(x) = (1 - c x)(1 - conj(c) x) fixes c from the roots of den: the roots
    are 1/c and 1/conj(c).  d is the limit of num/den at infinity (the
    (1-cx)^{-1} terms vanish there), and b = lim_{x->1/c} (1 - c x) num/den.
    """
    x = sp.symbols("x")
    roots = sp.solve(sp.Eq(den(x), 0), x)
    # pick the root whose reciprocal has positive imaginary part
    cs = [sp.nsimplify(sp.simplify(1 / r)) for r in roots]
    c = [ci for ci in cs if sp.im(ci) > 0][0]
    cc = sp.conjugate(c)
    d = sp.limit(num(x) / den(x), x, sp.oo)
    b = sp.simplify(num(1 / c) / (1 - cc / c))
    return {"d": sp.nsimplify(d), "c": sp.simplify(c), "b": sp.simplify(b)}


def pade22_exp():
    """r_{2,2}(x) = (1 + x/2 + x^2/12) / (1 - x/2 + x^2/12)  (§2, eq. 5)."""
    return _pade_pair(lambda x: 1 + x / 2 + x ** 2 / 12,
                      lambda x: 1 - x / 2 + x ** 2 / 12)


def pade22_phi1():
    """r~_{2,2}(x) = (1 + x/10 + x^2/60) / (1 - 2x/5 + x^2/20)  (§2, eq. 6)."""
    return _pade_pair(lambda x: 1 + sp.Rational(1, 10) * x + x ** 2 / 60,
                      lambda x: 1 - sp.Rational(2, 5) * x + x ** 2 / 20)


# --------------------------------------------------------------------------
# Registry used by the oracle's algorithm: m -> shift set
# --------------------------------------------------------------------------

# m counts the shifted solves ("processors"); a zero shift costs nothing
# (§2: taking c_1 = 0 leaves b_1 as a free constant term).
REAL_SETS = {4: shifts_R4, 5: shifts_R5, 8: shifts_R8}
# log(1 - x) (§2, worked example): the five shifts c_i = 1/(i + 1), with the
# weights of eq. (4) for a_k = -1/k (a_0 = 0); it has no scaling identity,
# so it is evaluated at s = 0 only
LOG1M_SETS = {5: shifts_frac4}
# m = 10: the hybrid set of §4.3 with the smaller coefficients (R10), for
# the exponential (the paper gives no phi1 weights for it)
HYBRID_SETS = {10: "R10", 110: "R10*"}  # registry keys of the two sets (110: R*10)


def real_set(func, m):
    """Exact (c, b) for ``func`` on the m-solve set.  exp uses the paper's
    sets; phi1 re-solves eq. (4) with a_k = 1/(k+1)! on the *same* shifts,
    which §2 allows ("different functions ... just by looking for a new set
    of coefficients b_i")."""
    c = LOG1M_SETS[m]() if func == "log1m" else REAL_SETS[m]()
    a = taylor_coeffs(func, len(c))
    return c, solve_weights(c, a)


def roundoff_terms(func, m):
    """Terms of the round-off form of §4.3.

    Since 1/(1 - c x) = 1 + c x/(1 - c x) and sum_k b_k = a_0, the approximant
    is r(x) = a0 + sum_k b_k c_k x / (1 - c_k x).  On matrices each term is
    w_k (I - c_k B)^{-1} B with w_k = b_k c_k, and zero shifts drop out.

    Returns (a0, [(c_k, w_k, is_pair)]) as Python complex/float values, each
    rounded once from the exact value.  For m = 1 the set is the complex pair
    of the Padé approximant of ``func`` (eq. 5 for exp, eq. 6 for phi1) and
    is_pair marks that the conjugate term is implied.
    """
    if m == 1:
        pr = pade22_exp() if func == "exp" else pade22_phi1()
        c, b, d = pr["c"], pr["b"], pr["d"]
        w = sp.expand(b * c)
        a0 = sp.simplify(d + 2 * sp.re(b))
        return float(a0), [(complex(sp.N(c, 40)), complex(sp.N(w, 40)), True)]
    if m in HYBRID_SETS:
        if func != "exp":
            raise NotImplementedError("the hybrid 10th-order set is given for the exponential only")
        c, b, d = hybrid_set(HYBRID_SETS[m], func)
        a0 = d[0] + sum(b, Fr(0))
        return float(a0), [(float(ci), float(bi * ci), False) for ci, bi in zip(c, b)]
    c, b = real_set(func, m)
    a0 = sum(b, Fr(0))
    terms = [(float(ci), float(bi * ci), False) for ci, bi in zip(c, b) if ci != 0]
    return float(a0), terms


def poly_terms(func, m):
    """(d_1, d_2) of the polynomial part d_1 x + d_2 x^2 of a hybrid set (§4.3),
    each rounded once; (0, 0) for the pure partial-fraction sets."""
    if m not in HYBRID_SETS:
        return 0.0, 0.0
    _, _, d = hybrid_set(HYBRID_SETS[m], func)
    return float(d[1]), float(d[2])


def order_of(m):
    """Order s of the approximation error O(x^{s+1}) (eq. 3): s = P - 1 with
    P = number of shifts including the zero one; 4 for the Padé pair."""
    if m == 1:
        return 4
    if m in HYBRID_SETS:
        return 10  # §4.3: ten shifts and a quadratic, order 10
    return len(REAL_SETS[m]()) - 1


def order_of_log1m(m):
    """Order of the log(1 - x) set: P shifts, none zero, match a_0..a_{P-1}."""
    return len(LOG1M_SETS[m]()) - 1
