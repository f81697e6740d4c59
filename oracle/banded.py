"""The action f(A)V for a tridiagonal or banded A, step by step, in plain FP64 (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A is given by its three diagonals: dl (A[i+1, i], length d - 1), dd (A[i, i],
length d) and du (A[i, i+1], length d - 1).  The algorithm is the N-step
recurrence of ``method.action`` (§1, §2, §4.3), written for this storage as
the paper does for tridiagonal matrices (§2.1, §5): I - c_k B is again
tridiagonal, so each shifted system is solved by a tridiagonal LU (LAPACK
gttrf once per shift, gttrs per solve; §5.1 reuses the factors across
steps), and B v costs one tridiagonal product.

  1. eta = ||A||_1, the largest column sum |du[j-1]| + |dd[j]| + |dl[j]|;
     θ = θ(f, m, tol); N = max(1, ceil(eta / θ)); B = A / N entry by entry.
  2. For each shift c_k: the LU of M_k = I - c_k B (subdiagonal -c_k dl/N,
     diagonal 1 - c_k dd/N, superdiagonal -c_k du/N).
  3. r(B) y = a0 y + sum_k w_k M_k^{-1} (B y)   (round-off form, §4.3);
     the hybrid set of §4.3 (m = 10, exp) adds d1 B y + d2 B (B y), the
     scheme the numerical examples (§5) apply to a tridiagonal A as R10':
     one product and the tridiagonal solves per step
     exp:  v_0 = V, v_j = r(B) v_{j-1}, j = 1..N
     phi1: u_1 = rho(B) V / N, u_{j+1} = r(B) u_j + u_1 (rho the phi1
           approximant), and u_N = phi1(A) V.

The only library primitives are LAPACK gttrf / gttrs (getrf / getrs for
d <= 2, which scipy's gttrf wrapper does not accept), and gbtrf / gbtrs for
the banded case (``band_action``: pentadiagonal and wider bands, §2.1, §5).
"""

import numpy as np
import scipy.linalg as sla
import scipy.linalg.lapack as lapack

from . import method


def tri_dense(dl, dd, du):
    """The dense d x d matrix with the given diagonals."""
    return np.diag(dd) + np.diag(dl, -1) + np.diag(du, 1)


def tri_norm1(dl, dd, du):
    """||A||_1: the largest column sum of |a_ij| over the three diagonals."""
    s = np.abs(np.asarray(dd, dtype=np.float64)).copy()
    s[1:] += np.abs(du)
    s[:-1] += np.abs(dl)
    return float(s.max())


def tri_matvec(dl, dd, du, X):
    """A X for tridiagonal A (the 5d-flop product of §2.1), X of shape d x p."""
    Y = dd[:, None] * X
    Y[1:] += dl[:, None] * X[:-1]
    Y[:-1] += du[:, None] * X[1:]
    return Y


def tri_action(dl, dd, du, V, funcs=("exp",), m=8, tol=1e-12, force_plan=None):
    """f(A) V for a real tridiagonal A and real V (d x p) by the N-step
    recurrence in the module docstring.  Returns a dict with the results and
    the plan (N, θ, eta)."""
    dl = np.asarray(dl, dtype=np.float64)
    dd = np.asarray(dd, dtype=np.float64)
    du = np.asarray(du, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    theta = method.theta_for(funcs, m, tol)
    eta = tri_norm1(dl, dd, du)
    N = method.plan_steps(eta, theta) if force_plan is None else int(force_plan)
    bl, bd, bu = dl / N, dd / N, du / N
    a0, terms = method.build_terms(funcs, m, False)
    facs = []
    for c, _, pair in terms:
        if pair or complex(c).imag != 0.0:
            raise NotImplementedError("tridiagonal oracle: real shifts only")
        c = float(complex(c).real)
        if len(bd) <= 2:  # scipy's gttrf wrapper needs d >= 3: dense LAPACK LU
            facs.append(sla.lu_factor(tri_dense(-c * bl, 1.0 - c * bd, -c * bu)))
            continue
        f = lapack.dgttrf(-c * bl, 1.0 - c * bd, -c * bu)
        if f[-1] != 0:
            raise FloatingPointError("singular shifted tridiagonal matrix")
        facs.append(f[:5])

    def apply_r(fname, X):
        Y = tri_matvec(bl, bd, bu, X)
        out = a0[fname] * X
        d1, d2 = method.co.poly_terms(fname, m)
        if d1 or d2:  # the hybrid sets: d1 B + d2 B^2
            out = out + d1 * Y + d2 * tri_matvec(bl, bd, bu, Y)
        for (c, ws, _), fac in zip(terms, facs):
            w = float(complex(ws.get(fname, 0.0)).real)
            if w == 0.0:
                continue
            if len(fac) == 2:
                Z = sla.lu_solve(fac, Y)
            else:
                Z, info = lapack.dgttrs(*fac, Y)
                assert info == 0
            out = out + w * Z
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


def laplacian_1d_eig(d):
    """Eigen-decomposition of trid{-1, 2, -1} of size d (Dirichlet): the
    eigenvalues 2 - 2 cos(j pi / (d + 1)) and the orthonormal sine vectors
    sqrt(2 / (d + 1)) sin(i j pi / (d + 1)), i, j = 1..d (a textbook closed
    form; the paper's tridiagonal test matrix of §5)."""
    j = np.arange(1, d + 1)
    lam = 2.0 - 2.0 * np.cos(j * np.pi / (d + 1))
    U = np.sqrt(2.0 / (d + 1)) * np.sin(np.outer(j, j) * np.pi / (d + 1))
    return lam, U


# ---------------------------------------------------------------------------
# Banded A (the pentadiagonal and banded case the paper names beside the
# tridiagonal one in §2.1 and §5): the same N-step recurrence, with A given
# by its 2b + 1 diagonals.  bands has shape (2b + 1, d) and
# bands[b + o, i] = A[i, i + o] for o = -b..b; entries with i + o outside
# [0, d) are not part of A and are never read.  I - c_k B is banded with the
# same b, so each shifted system is one banded LU (LAPACK gbtrf once per
# shift, gbtrs per solve), and B v is one banded product.

def band_dense(bands, b):
    """The dense d x d matrix with the given diagonals."""
    bands = np.asarray(bands, dtype=np.float64)
    d = bands.shape[1]
    A = np.zeros((d, d))
    for o in range(-b, b + 1):
        for i in range(max(0, -o), min(d, d - o)):
            A[i, i + o] = bands[b + o, i]
    return A


def _band_clean(bands, b):
    """bands with the entries outside A set to zero (so that they are never
    read as values)."""
    B = np.array(bands, dtype=np.float64, copy=True)
    d = B.shape[1]
    for o in range(-b, b + 1):
        lo = min(d, max(0, -o))
        hi = max(lo, min(d, d - o))
        B[b + o, :lo] = 0.0
        B[b + o, hi:] = 0.0
    return B


def band_norm1(bands, b):
    """||A||_1: the largest column sum; column j adds |A[i, j]| for rows
    i = j - b .. j + b in increasing order."""
    B = _band_clean(bands, b)
    d = B.shape[1]
    s = np.zeros(d)
    for o in range(b, -b - 1, -1):  # row i = j - o, increasing as o falls
        col = np.zeros(d)
        j = np.arange(d)
        i = j - o
        ok = (i >= 0) & (i < d)
        col[ok] = np.abs(B[b + o, i[ok]])
        s = s + col
    return float(s.max())


def band_matvec(bands, b, X):
    """A X for banded A, X of shape d x p: row i adds A[i, i + o] x_{i+o}
    for o = -b..b in increasing order."""
    B = _band_clean(bands, b)
    X = np.asarray(X)
    d = B.shape[1]
    Y = np.zeros_like(X, dtype=np.float64)
    for o in range(-b, b + 1):
        lo = min(d, max(0, -o))
        hi = max(lo, min(d, d - o))
        Y[lo:hi] += B[b + o, lo:hi, None] * X[lo + o:hi + o]
    return Y


def _gb_storage(M, b):
    """LAPACK gbtrf storage of the band of M with kl = ku = b: ab has
    2 kl + ku + 1 rows, and ab[kl + ku + i - j, j] = M[i, j]."""
    d = M.shape[0]
    ab = np.zeros((3 * b + 1, d))
    for j in range(d):
        for i in range(max(0, j - b), min(d, j + b + 1)):
            ab[2 * b + i - j, j] = M[i, j]
    return ab


def band_action(bands, b, V, funcs=("exp",), m=8, tol=1e-12, force_plan=None):
    """f(A) V for a real banded A (half-bandwidth b) and real V (d x p), by the
    N-step recurrence of ``tri_action`` with banded LU solves.  Returns a dict
    with the results and the plan (N, θ, eta)."""
    bands = _band_clean(bands, b)
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    d = bands.shape[1]
    theta = method.theta_for(funcs, m, tol)
    eta = band_norm1(bands, b)
    N = method.plan_steps(eta, theta) if force_plan is None else int(force_plan)
    Bb = bands / N
    Bd = band_dense(Bb, b)
    a0, terms = method.build_terms(funcs, m, False)
    facs = []
    for c, _, pair in terms:
        if pair or complex(c).imag != 0.0:
            raise NotImplementedError("banded oracle: real shifts only")
        c = float(complex(c).real)
        M = -c * Bd
        M[np.diag_indices(d)] = 1.0 - c * np.diag(Bd)
        lub, piv, info = lapack.dgbtrf(_gb_storage(M, b), b, b)
        if info != 0:
            raise FloatingPointError("singular shifted banded matrix")
        facs.append((lub, piv))

    def apply_r(fname, X):
        Y = band_matvec(Bb, b, X)
        out = a0[fname] * X
        d1, d2 = method.co.poly_terms(fname, m)
        if d1 or d2:  # the hybrid sets: d1 B + d2 B^2
            out = out + d1 * Y + d2 * band_matvec(Bb, b, Y)
        for (c, ws, _), (lub, piv) in zip(terms, facs):
            w = float(complex(ws.get(fname, 0.0)).real)
            if w == 0.0:
                continue
            Z, info = lapack.dgbtrs(lub, b, b, Y, piv)
            assert info == 0
            out = out + w * Z
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


def laplacian_sq_bands(d, tau=1.0):
    """Diagonals (b = 2) of -tau L^2 with L = trid{-1, 2, -1}: rows of L^2 are
    (1, -4, 6, -4, 1) except the first and last diagonal entries, which are 5.
    L^2 has L's sine eigenvectors and the eigenvalues squared."""
    bands = np.zeros((5, d))
    bands[0, :] = 1.0
    bands[1, :] = -4.0
    bands[2, :] = 6.0
    bands[3, :] = -4.0
    bands[4, :] = 1.0
    bands[2, 0] = bands[2, d - 1] = 5.0
    return _band_clean(-tau * bands, 2)
