"""The parallel rational method, step by step, in plain FP64 (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Full matrix, f in {exp, phi1, phi2} (§1, §2, §4.3):
  1. eta = ||A||_1 (max column sum of |a_ij|; §5 names the 1-norm as the usual
     choice) and θ = θ(f, m, tol) from the forward bound of §3.
  2. s = smallest integer s >= 0 with eta * 2^-s <= θ; B = A * 2^-s (exact).
  3. For each nonzero shift c_k: LU with partial pivoting of M_k = I - c_k B
     (LAPACK getrf) and Z_k = M_k^{-1} B (getrs).  These are the m
     independent "processors" of §2.
  4. Round-off form of §4.3: R = a0 I + sum_k w_k Z_k with w_k = b_k c_k; for
     a complex-conjugate pair on real A the pair contributes 2 Re(w_k Z_k).
     The hybrid set of §4.3 (m = 10) adds its polynomial part d1 B + d2 B^2
     (its constant d0 is part of a0 = d0 + sum_k b_k).
  5. Undo the scaling (§1): s times { Phi <- (R + I) Phi / 2 ; R <- R R }.
     The phi1 step is the doubling identity of §1 written for B:
     phi1(2B) = (e^B + I) phi1(B) / 2 (the form printed in §1 lacks the
     factor t that phi1(tA) carries), and it uses R *before* it is squared.
     phi2 (§1's phi_k with k = 2: (e^x - 1 - x) / x^2, weights for
     a_k = 1/(k+2)! on the same shifts) doubles as
     phi2(2B) = (phi1(B)^2 + 2 phi2(B)) / 4, which follows from
     e^{2x} - 1 - 2x = x^2 phi1(x)^2 + 2 x^2 phi2(x); it uses Phi before
     Phi's own step, so phi2 always carries the phi1 chain.

Action on a block V (n x p) (§1, §2):
  1. eta, θ as above; N = max(1, ceil(eta / θ)) (correctly rounded quotient);
     B = A / N entry by entry.
  2. LU of every M_k once, reused for all N steps (§5.1, first remark).
  3. exp:  v_0 = V, v_j = r(B) v_{j-1} for j = 1..N where
           r(B) y = a0 y + sum_k w_k M_k^{-1} (B y)            (round-off form)
     phi1: u_1 = phi1-approximant(B) V / N, u_{j+1} = r(B) u_j + u_1, and
           u_N = phi1(A) V.  This is the solution u(1) of u' = A u + V,
           u(0) = 0, stepped with h = 1/N (the linear ODE of §1).

All arithmetic is numpy/scipy FP64 (complex128 where A or a shift is complex);
the only library primitives are LAPACK getrf/getrs and matrix products.
"""

import math

import numpy as np
import scipy.linalg as sla

from . import coefficients as co
from . import theta as th

_THETA_CACHE = {}


def norm1(A):
    """||A||_1 = max_j sum_i |a_ij| (|z| for complex entries)."""
    return float(np.abs(np.asarray(A)).sum(axis=0).max())


def theta_for(funcs, m, tol):
    """θ used by the plan.  phi1 always needs the exponential approximant as
    well (its doubling step and its N-step recurrence both apply e^B), so a
    request containing phi1 takes min(θ_exp, θ_phi1); phi2's doubling squares
    phi1, so a request containing phi2 takes min(θ_exp, θ_phi1, θ_phi2)."""
    key = (tuple(sorted(funcs)), m, float(tol))
    if key not in _THETA_CACHE:
        need = set(funcs) if "log1m" in funcs else {"exp"} | set(funcs)
        if "phi2" in need:
            need.add("phi1")
        _THETA_CACHE[key] = min(th.theta_set(f, m, tol) for f in need)
    return _THETA_CACHE[key]


def plan_scaling(eta, theta):
    """Smallest s >= 0 with eta * 2^-s <= θ (§1: N = 2^s, then s squarings)."""
    if not math.isfinite(eta):
        raise FloatingPointError("non-finite norm")
    s = 0
    while math.ldexp(eta, -s) > theta:
        s += 1
    return s


def plan_steps(eta, theta):
    """N = max(1, ceil(eta / θ)) (§1: v_n = e^{A/N} v_{n-1}, n = 1..N)."""
    if not math.isfinite(eta):
        raise FloatingPointError("non-finite norm")
    return max(1, math.ceil(eta / theta))


def build_terms(funcs, m, complex_A):
    """Solve list [(c_k, {func: w_k}, is_pair)] and the constants a0 per func.

    Every requested function shares the same solves (§2: several functions
    from one set of F_i), except m = 1, where exp and phi1 have different
    Padé poles and so need a pair each.  For complex A a conjugate pair cannot
    be folded into 2 Re(.), so it is expanded into its two conjugate terms.
    """
    if "log1m" in funcs:
        # log(1 - x) alone, on its own shift set (§2)
        if tuple(funcs) != ("log1m",):
            raise ValueError("log1m is evaluated on its own")
        a0l, tl = co.roundoff_terms("log1m", m)
        return {"log1m": a0l}, [(c, {"log1m": w}, pair) for c, w, pair in tl]
    need = ["exp"] + (["phi1"] if ("phi1" in funcs or "phi2" in funcs) else []) + \
        (["phi2"] if "phi2" in funcs else [])
    a0 = {}
    terms = []
    if m == 1:
        if "phi2" in funcs:
            raise NotImplementedError("the m = 1 Padé pairs are given for exp and phi1 only")
        for f in need:
            a0[f], tl = co.roundoff_terms(f, 1)
            (c, w, _), = tl
            if complex_A:
                terms.append((c, {f: w}, False))
                terms.append((c.conjugate(), {f: w.conjugate()}, False))
            else:
                terms.append((c, {f: w}, True))
        return a0, terms
    per_f = {}
    for f in need:
        a0[f], per_f[f] = co.roundoff_terms(f, m)
    for k in range(len(per_f["exp"])):
        c = per_f["exp"][k][0]
        ws = {f: per_f[f][k][1] for f in need}
        for f in need:
            assert per_f[f][k][0] == c
        terms.append((c, ws, False))
    return a0, terms


def _accumulate(acc, Z, w, pair):
    if pair:
        acc += 2.0 * (w * Z).real
    else:
        acc += w * Z


def doubling_step(R, Phi, Phi2, I):
    """One undoing of the scaling (§1) for B -> 2B: phi2 from phi1 and phi2,
    phi1 from e^B and phi1 (both before their own step), then R <- R R."""
    if Phi2 is not None:
        Phi2 = 0.25 * (Phi @ Phi) + 0.5 * Phi2
    if Phi is not None:
        Phi = 0.5 * ((R + I) @ Phi)
    return R @ R, Phi, Phi2


def expm_full(A, funcs=("exp",), m=8, tol=1e-12, force_plan=None):
    """f(A) for f in ``funcs`` (subset of {"exp", "phi1", "phi2"}) by the full-matrix
    algorithm in the module docstring.  Returns a dict with the requested
    results and the plan (s, θ, eta)."""
    A = np.asarray(A)
    n = A.shape[0]
    cplx = np.iscomplexobj(A)
    theta = theta_for(funcs, m, tol)
    eta = norm1(A)
    if "log1m" in funcs:
        s = 0  # no scaling identity: r(A) itself (the bound holds for eta <= θ)
    else:
        s = plan_scaling(eta, theta) if force_plan is None else int(force_plan)
    B = np.ldexp(A.real, -s) + (1j * np.ldexp(A.imag, -s) if cplx else 0.0)
    a0, terms = build_terms(funcs, m, cplx)
    I = np.eye(n)
    out_dtype = np.complex128 if cplx else np.float64
    acc = {f: a0[f] * I.astype(out_dtype) for f in a0}
    for f in acc:
        d1, d2 = co.poly_terms(f, m)
        if d1 or d2:
            acc[f] = acc[f] + d1 * B + d2 * (B @ B)
    for c, ws, pair in terms:
        M = I - c * B
        lu = sla.lu_factor(M)
        Z = sla.lu_solve(lu, B.astype(M.dtype))
        for f, w in ws.items():
            _accumulate(acc[f], Z, w, pair and not cplx)
    if "log1m" in funcs:
        return {"plan": 0, "theta": theta, "eta": eta, "log1m": acc["log1m"]}
    R = acc["exp"]
    Phi = acc.get("phi1")
    Phi2 = acc.get("phi2")
    for _ in range(s):
        R, Phi, Phi2 = doubling_step(R, Phi, Phi2, I)
    res = {"plan": s, "theta": theta, "eta": eta}
    if "exp" in funcs:
        res["exp"] = R
    if "phi1" in funcs:
        res["phi1"] = Phi
    if "phi2" in funcs:
        res["phi2"] = Phi2
    return res


def action(A, V, funcs=("exp",), m=8, tol=1e-12, force_plan=None):
    """f(A) V for f in ``funcs`` by the N-step recurrence of the module
    docstring.  V is n x p.  Returns a dict with the results and the plan."""
    A = np.asarray(A)
    V = np.asarray(V)
    n = A.shape[0]
    cplx = np.iscomplexobj(A) or np.iscomplexobj(V)
    theta = theta_for(funcs, m, tol)
    eta = norm1(A)
    N = plan_steps(eta, theta) if force_plan is None else int(force_plan)
    B = A / N
    a0, terms = build_terms(funcs, m, np.iscomplexobj(A))
    I = np.eye(n)
    lus = [sla.lu_factor(I - c * B) for c, _, _ in terms]
    real_out = not cplx

    def apply_r(f, X):
        Y = B @ X
        out = a0[f] * X.astype(np.complex128 if cplx else np.float64)
        d1, d2 = co.poly_terms(f, m)
        if d1 or d2:
            out = out + d1 * Y + d2 * (B @ Y)
        for (c, ws, pair), lu in zip(terms, lus):
            w = ws.get(f, 0.0)
            if w == 0.0:
                continue
            Z = sla.lu_solve(lu, Y.astype(lu[0].dtype))
            _accumulate(out, Z, w, pair and real_out)
        return out

    res = {"plan": N, "theta": theta, "eta": eta}
    if "exp" in funcs:
        v = V
        for _ in range(N):
            v = apply_r("exp", v)
        res["exp"] = v
    if "phi1" in funcs:
        u1 = apply_r("phi1", V) / N
        u = u1
        for _ in range(N - 1):
            u = apply_r("exp", u) + u1
        res["phi1"] = u
    return res


def r_scalar(func, m, x):
    """The approximant of ``func`` on the m-solve set at scalars x (array),
    in the round-off form of §4.3: a0 + sum_k w_k x / (1 - c_k x), plus
    d1 x + d2 x^2 for the hybrid sets of §4.3."""
    x = np.asarray(x, dtype=np.complex128)
    a0, terms = co.roundoff_terms(func, m)
    out = np.full(x.shape, a0, dtype=np.complex128)
    d1, d2 = co.poly_terms(func, m)
    if d1 or d2:
        out += d1 * x + d2 * x * x
    for c, w, pair in terms:
        t = w * x / (1 - c * x)
        out += t + np.conj(w) * x / (1 - np.conj(c) * x) if pair else t
    return out


def _r_mp(func, m, xs, N, geo):
    """r(x)^N (geo=False) or rho(x) / N * sum_{j<N} r(x)^j (geo=True, rho the
    phi1 approximant) at 40 digits, from the binary64 coefficients the
    method uses; returned as complex128."""
    import mpmath
    a0e, te = co.roundoff_terms("exp", m)
    pe = co.poly_terms("exp", m)
    if geo:
        a0p, tp = co.roundoff_terms("phi1", m)
        pp = co.poly_terms("phi1", m)
    out = np.empty(len(xs), dtype=np.complex128)
    with mpmath.workdps(40):
        def rat(a0, terms, poly, x):
            v = mpmath.mpc(a0) + mpmath.mpf(poly[0]) * x + mpmath.mpf(poly[1]) * x * x
            for c, w, pair in terms:
                v += mpmath.mpc(w) * x / (1 - mpmath.mpc(c) * x)
                if pair:
                    v += mpmath.conj(mpmath.mpc(w)) * x / (1 - mpmath.conj(mpmath.mpc(c)) * x)
            return v
        for i, x in enumerate(xs):
            xm = mpmath.mpc(complex(x))
            r = rat(a0e, te, pe, xm)
            if not geo:
                v = r ** N
            else:
                s = mpmath.mpf(N) if r == 1 else (1 - r ** N) / (1 - r)
                v = rat(a0p, tp, pp, xm) / N * s
            out[i] = complex(v)
    return out


def action_normal(mu, U, V, funcs=("exp",), m=8, N=1, exact_scalars=False):
    """The N-step action of ``action`` for a normal A = U diag(mu) U^H
    (U unitary), evaluated per eigenvalue instead of by solves: with
    x = mu / N, the steps act on U^H V as multiplication by r(x), so
      exp:  U diag(r(x)^N) U^H V
      phi1: U diag(rho(x) / N * sum_{j<N} r(x)^j) U^H V,
    rho the phi1 approximant (u_1 = rho(B) V / N, u_{j+1} = r(B) u_j + u_1).
    Exact up to rounding for any n, so it serves as the reference at sizes
    where the step-by-step oracle is too slow.

    With exact_scalars the per-eigenvalue factors are evaluated at 40 digits
    (from the same binary64 coefficients): in binary64 their rounding,
    about sum_k |w_k x / (1 - c_k x)| u, is amplified N times by the power,
    which at N in the hundreds reaches 1e-12."""
    mu = np.asarray(mu)
    x = mu / N
    W = U.conj().T @ V
    res = {}
    if exact_scalars:
        if "exp" in funcs:
            res["exp"] = U @ (_r_mp("exp", m, x, N, False)[:, None] * W)
        if "phi1" in funcs:
            res["phi1"] = U @ (_r_mp("phi1", m, x, N, True)[:, None] * W)
        return res
    r = r_scalar("exp", m, x)
    if "exp" in funcs:
        res["exp"] = U @ ((r ** N)[:, None] * W)
    if "phi1" in funcs:
        geo = np.zeros_like(r)
        for _ in range(N):
            geo = geo * r + 1.0
        res["phi1"] = U @ ((r_scalar("phi1", m, x) / N * geo)[:, None] * W)
    return res


def rational(A, c, w, a0, conj_pairs=True, V=None):
    """A caller-given partial-fraction set (§2, a rational function with simple
    poles 1/c_k), in the round-off form of §4.3 with no scaling:
        r(A) = a0 I + sum_k w_k (I - c_k A)^{-1} A        (V is None), or
        r(A) V = a0 V + sum_k w_k (I - c_k A)^{-1} (A V)  (one step).
    With conj_pairs every term with a complex shift also stands for its
    conjugate (c_k*, w_k*); on real A and V the pair is then 2 Re(w_k Z_k)
    (the conjugate solve is the conjugate of Z_k) and the result is real.  One
    LAPACK getrf/getrs per solve, the terms summed in the listed order."""
    A = np.asarray(A)
    n = A.shape[0]
    c = [complex(x) for x in c]
    w = [complex(x) for x in w]
    real_in = not np.iscomplexobj(A) and (V is None or not np.iscomplexobj(V))
    if real_in and not conj_pairs and any(x.imag != 0.0 for x in c + w):
        raise ValueError("complex terms on real A need the conjugates for a real result")
    out_complex = not real_in
    dt = np.complex128 if (out_complex or any(x.imag != 0.0 for x in c)) else np.float64
    I = np.eye(n)
    rhs = A if V is None else A @ np.asarray(V)
    acc = (a0 * (I if V is None else np.asarray(V))).astype(np.complex128 if out_complex else np.float64)
    for ck, wk in zip(c, w):
        shift = ck if (out_complex or ck.imag != 0.0) else ck.real
        Z = sla.lu_solve(sla.lu_factor(I - shift * A), rhs.astype(dt))
        if out_complex:
            acc = acc + wk * Z
            if conj_pairs and ck.imag != 0.0:
                Zc = sla.lu_solve(sla.lu_factor(I - ck.conjugate() * A), rhs.astype(dt))
                acc = acc + wk.conjugate() * Zc
        elif ck.imag != 0.0:
            acc = acc + 2.0 * (wk * Z).real
        else:
            acc = acc + wk.real * Z.real
    return acc


def rel_fro(X, Xref):
    """Relative Frobenius error ||X - Xref||_F / ||Xref||_F."""
    X = np.asarray(X)
    Xref = np.asarray(Xref)
    return float(np.linalg.norm(X - Xref) / np.linalg.norm(Xref))
