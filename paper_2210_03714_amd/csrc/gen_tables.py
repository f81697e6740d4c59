#!/usr/bin/env python3
"""Build-time generator of the library's coefficient tables (pfm_tables.inc).

For every registered solve count m and function f it emits, as binary64
constants each rounded once from an exact value:

* the shifts c_k (complex for the Padé pairs) of the nonzero-shift solves,
* the round-off-form weights w_k = b_k c_k (§4.3) and the constant a0,
* the order of the approximation,
* the forward-bound series coefficients d_k = |a_k - alpha_k| (§3), from
  which the library finds θ(tol) at run time by bisection,
* for the two hybrid 10th-order sets of §4.3 (the exponential: m = 10,
  the one with the smaller coefficients, and m = 110 for the other, R*10),
  the polynomial part d_1 x + d_2 x^2 of r(x) = d_0 + d_1 x + d_2 x^2 +
  sum b_i / (1 - c_i x); its d_0 is in a0 = d_0 + sum b_i.

Weights come from the transposed Vandermonde system of §2 (eq. 4), solved here
through the Lagrange basis: the coefficient of x^k in the Lagrange polynomial
L_i(x) = prod_{j != i} (x - c_j) / (c_i - c_j) is the (i, k) entry of the
inverse, so b_i = sum_k [x^k] L_i(x) * a_k.  All of this is exact
(``fractions.Fraction``).  The Padé pairs of §2 (eqs. 5, 6) are handled in
closed form: for a denominator 1 - beta x + gamma x^2 = (1 - c x)(1 - conj(c) x)
one has c = beta/2 + i sqrt(gamma - beta^2/4) and the residue
b = p(1/c) / (1 - conj(c)/c), evaluated with ``decimal`` at 50 digits.
"""

import decimal
import sys
from fractions import Fraction as Q
from math import factorial

decimal.getcontext().prec = 60
D = decimal.Decimal
KBOUND = 160  # series terms kept for the run-time bound


def series(func, K):
    if func == "exp":
        return [Q(1, factorial(k)) for k in range(K)]
    if func == "phi1":
        return [Q(1, factorial(k + 1)) for k in range(K)]
    if func == "phi2":  # phi2(x) = (e^x - 1 - x) / x^2 (§1, degree-1 polynomial removed)
        return [Q(1, factorial(k + 2)) for k in range(K)]
    if func == "log1m":  # log(1 - x) = -sum_{k >= 1} x^k / k
        return [Q(0)] + [Q(-1, k) for k in range(1, K)]
    raise ValueError(func)


def poly_mul_linear(p, root):
    """p(x) * (x - root), coefficients low to high."""
    out = [Q(0)] * (len(p) + 1)
    for k, a in enumerate(p):
        out[k + 1] += a
        out[k] -= a * root
    return out


def lagrange_weights(c, a):
    P = len(c)
    b = []
    for i in range(P):
        poly = [Q(1)]
        den = Q(1)
        for j in range(P):
            if j != i:
                poly = poly_mul_linear(poly, c[j])
                den *= c[i] - c[j]
        b.append(sum(poly[k] * a[k] for k in range(P)) / den)
    return b


def shifts(m):
    if m == 4:                     # §4.1, alpha = 5
        al = Q(5)
        return [Q(0), 1 / al, -1 / al, 1 / (2 * al), -1 / (2 * al)]
    if m == 8:                     # §4.2, alpha = 5
        al = Q(5)
        out = [Q(0)]
        for num, den in ((1, 1), (2, 3), (1, 2), (2, 5)):
            out += [Q(num) / (den * al), -Q(num) / (den * al)]
        return out
    if m == 5:                     # §5.1
        return [Q(0)] + [Q(1, i + 1) for i in range(2, 7)]
    raise ValueError(m)


def real_entry(func, m):
    # log(1 - x): the five shifts 1/2..1/6 of the §2 example
    c = [Q(1, i + 1) for i in range(1, 6)] if func == "log1m" else shifts(m)
    a = series(func, KBOUND)
    b = lagrange_weights(c, a[:len(c)])
    assert sum(b) == a[0]
    d = []
    for k in range(KBOUND):
        alpha = sum(bi * (ci ** k if k else Q(1)) for bi, ci in zip(b, c))
        d.append(abs(a[k] - alpha))
    terms = [(ci, Q(0), bi * ci, Q(0)) for ci, bi in zip(c, b) if ci != 0]
    return {"a0": a[0], "order": len(c) - 1, "terms": terms, "pair": 0, "d": d}


def hybrid_entry(star=False):
    """§4.3: star = False, the set with c_{2i-1} = -1/(6+2i), c_{2i} = 1/(6+2i)
    and b_9 = 2000, b_10 = -3500; star = True, the set with c_i = 1/(6+i),
    i = 1..10, and b_9 = -5 10^4, b_10 = 3.5 10^5.  b_1..b_8 from
    sum_i b_i c_i^k = 1/k!, k = 3..10, through the Lagrange basis of the first
    eight shifts (x^3 times it gives the rows k = 3..10), then
    d_k = 1/k! - sum_i b_i c_i^k, k = 0..2."""
    c = []
    if star:
        c = [Q(1, 6 + i) for i in range(1, 11)]
        b9, b10 = Q(-50000), Q(350000)
    else:
        for i in range(1, 6):
            c += [Q(-1, 6 + 2 * i), Q(1, 6 + 2 * i)]
        b9, b10 = Q(2000), Q(-3500)
    a = series("exp", KBOUND)
    # sum_{i<8} (b_i c_i^3) c_i^j = a_{j+3} - b9 c9^{j+3} - b10 c10^{j+3}, j = 0..7
    rhs = [a[j + 3] - b9 * c[8] ** (j + 3) - b10 * c[9] ** (j + 3) for j in range(8)]
    e = lagrange_weights(c[:8], rhs)
    b = [ei / ci ** 3 for ei, ci in zip(e, c[:8])] + [b9, b10]
    dpoly = [a[k] - sum(bi * ci ** k for bi, ci in zip(b, c)) for k in range(3)]
    a0 = dpoly[0] + sum(b)
    assert a0 == 1
    d = []
    for k in range(KBOUND):
        alpha = sum(bi * ci ** k for bi, ci in zip(b, c)) + (dpoly[k] if k < 3 else Q(0))
        d.append(abs(a[k] - alpha))
    assert all(x == 0 for x in d[:11])
    terms = [(ci, Q(0), bi * ci, Q(0)) for ci, bi in zip(c, b)]
    return {"a0": a0, "order": 10, "terms": terms, "pair": 0, "d": d, "poly": (dpoly[1], dpoly[2])}


# -- complex pairs in Decimal ------------------------------------------------


def cmul(x, y):
    return (x[0] * y[0] - x[1] * y[1], x[0] * y[1] + x[1] * y[0])


def cdiv(x, y):
    den = y[0] * y[0] + y[1] * y[1]
    return ((x[0] * y[0] + x[1] * y[1]) / den, (x[1] * y[0] - x[0] * y[1]) / den)


def pair_entry(func):
    if func == "exp":     # eq. (5): (1 + x/2 + x^2/12) / (1 - x/2 + x^2/12)
        num = (D(1), D(1) / 2, D(1) / 12)
        beta, gamma = D(1) / 2, D(1) / 12
    else:                 # eq. (6): (1 + x/10 + x^2/60) / (1 - 2x/5 + x^2/20)
        num = (D(1), D(1) / 10, D(1) / 60)
        beta, gamma = D(2) / 5, D(1) / 20
    c = (beta / 2, (gamma - beta * beta / 4).sqrt())
    cc = (c[0], -c[1])
    xinv = cdiv((D(1), D(0)), c)
    p = (num[0], D(0))
    xp = (D(1), D(0))
    for k in (1, 2):
        xp = cmul(xp, xinv)
        p = (p[0] + num[k] * xp[0], p[1] + num[k] * xp[1])
    one_minus = (D(1) - cdiv(cc, c)[0], -cdiv(cc, c)[1])
    b = cdiv(p, one_minus)
    dconst = num[2] / gamma
    a0 = dconst + 2 * b[0]
    w = cmul(b, c)
    a = series(func, KBOUND)
    d = []
    ck = (D(1), D(0))
    for k in range(KBOUND):
        if k == 0:
            alpha = dconst + 2 * b[0]
        else:
            ck = cmul(ck, c)
            alpha = 2 * cmul(b, ck)[0]
        ak = D(a[k].numerator) / D(a[k].denominator)
        d.append(abs(ak - alpha))
    return {"a0": a0, "order": 4, "terms": [(c[0], c[1], w[0], w[1])], "pair": 1, "d": d}


def f64(x):
    if isinstance(x, Q):
        return float(x)
    return float(x)


def emit(path):
    entries = []
    for m in (1, 4, 5, 8):
        for fi, func in enumerate(("exp", "phi1")):
            e = pair_entry(func) if m == 1 else real_entry(func, m)
            entries.append((m, fi, e))
    entries.append((10, 0, hybrid_entry()))  # the exponential only
    entries.append((110, 0, hybrid_entry(star=True)))  # R*10, the exponential only
    entries.append((5, 2, real_entry("log1m", 5)))  # log(1 - x), evaluated at s = 0
    for m in (4, 5, 8):  # phi2 on the exponential's real shift sets (index 3)
        entries.append((m, 3, real_entry("phi2", m)))
    lines = ["/* Generated by gen_tables.py -- do not edit. */",
             "#define PFM_KBOUND %d" % KBOUND,
             "struct PfmSetEntry { int m; int func; int pair; int order; int nterms; double a0;",
             "  double c_re[16]; double c_im[16]; double w_re[16]; double w_im[16]; double poly[2];",
             "  double d[PFM_KBOUND]; };",
             "static const PfmSetEntry kPfmSets[] = {"]
    for m, fi, e in entries:
        t = e["terms"]
        pad = lambda xs: ", ".join(x.hex() for x in (list(xs) + [0.0] * (16 - len(xs))))
        lines.append("  { %d, %d, %d, %d, %d, %s," % (m, fi, e["pair"], e["order"], len(t), f64(e["a0"]).hex()))
        lines.append("    { %s }," % pad([f64(x[0]) for x in t]))
        lines.append("    { %s }," % pad([f64(x[1]) for x in t]))
        lines.append("    { %s }," % pad([f64(x[2]) for x in t]))
        lines.append("    { %s }," % pad([f64(x[3]) for x in t]))
        poly = e.get("poly", (Q(0), Q(0)))
        lines.append("    { %s, %s }," % (f64(poly[0]).hex(), f64(poly[1]).hex()))
        lines.append("    { %s } }," % ", ".join(f64(x).hex() for x in e["d"]))
    lines.append("};")
    lines.append("static const int kPfmNumSets = %d;" % len(entries))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    emit(sys.argv[1])
