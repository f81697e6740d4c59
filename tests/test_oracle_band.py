"""Pins for the banded-action oracle (oracle/banded.py, ``band_action``), each
against something other than its own code path:

* the norm and the product against the dense matrix (brute force), with the
  entries outside A filled with NaN to show they are never read;
* the whole N-step recurrence against the dense oracle (dense LAPACK getrf /
  getrs instead of the banded gbtrf / gbtrs), same plan, for b = 1..4;
* b = 1 against the tridiagonal oracle (gttrf / gttrs);
* -tau L^2 (pentadiagonal, L = trid{-1, 2, -1}) against the closed-form sine
  eigen-decomposition with squared eigenvalues: the method's exact result per
  eigenvalue and the exact exponential within the N-step error bound.
"""

import numpy as np
import pytest

from oracle import banded as bd
from oracle import coefficients as co
from oracle import method as me
from paper_2210_03714_amd import workloads as wl

U64 = 2.0 ** -53


def _sum_abs_w(funcs, m):
    s = 0.0
    for f in set(funcs) | {"exp"}:
        _, terms = co.roundoff_terms(f, m)
        s = max(s, sum(abs(complex(w)) * (2 if pair else 1) for _, w, pair in terms))
    return s


def _outside_nan(bands, b):
    """A copy of bands with every entry outside A set to NaN."""
    B = np.array(bands, copy=True)
    d = B.shape[1]
    for o in range(-b, b + 1):
        lo = min(d, max(0, -o))
        B[b + o, :lo] = np.nan
        B[b + o, max(lo, min(d, d - o)):] = np.nan
    return B


@pytest.mark.parametrize("b", [1, 2, 4])
def test_norm_and_product_against_dense(b):
    d = 23
    bands = _outside_nan(np.random.default_rng(b).standard_normal((2 * b + 1, d)), b)
    A = bd.band_dense(bands, b)
    assert np.isfinite(A).all()
    assert bd.band_norm1(bands, b) == np.abs(A).sum(axis=0).max()
    X = np.random.default_rng(1).standard_normal((d, 4))
    assert np.abs(bd.band_matvec(bands, b, X) - A @ X).max() <= 8 * U64 * np.abs(A).sum(1).max() * np.abs(X).max()


@pytest.mark.parametrize("b,d", [(1, 5), (2, 2), (2, 3), (2, 40), (3, 2), (3, 7), (4, 1), (4, 3), (4, 33)])
@pytest.mark.parametrize("funcs", [("exp",), ("phi1",), ("exp", "phi1")])
@pytest.mark.parametrize("m", [4, 8])
def test_banded_equals_dense_oracle(funcs, m, b, d):
    """Same plan as the dense oracle and the same result up to the solvers'
    rounding (a few units times sum |w_k| per step, N steps)."""
    p = 3
    bands = wl.band_gaussian_batch(1, d, b, 0.5, 8.0, wl.SEED_BASE + 800 + 10 * b + m)[0]
    V = np.random.default_rng(m + b).standard_normal((d, p))
    got = bd.band_action(_outside_nan(bands, b), b, V, funcs, m, 1e-12)
    ref = me.action(bd.band_dense(bands, b), V, funcs, m, 1e-12)
    assert got["plan"] == ref["plan"]
    bound = 16 * d * got["plan"] * (1 + _sum_abs_w(funcs, m)) * U64
    for f in funcs:
        assert me.rel_fro(got[f], ref[f]) <= bound, (f, me.rel_fro(got[f], ref[f]), bound)


def test_banded_hybrid_equals_dense_oracle():
    """R10' (the hybrid set of §4.3, exp) on a pentadiagonal A against the
    dense oracle, whose polynomial part is a dense product."""
    d, b, p = 31, 2, 2
    bands = wl.band_gaussian_batch(1, d, b, 0.5, 8.0, wl.SEED_BASE + 830)[0]
    V = np.random.default_rng(3).standard_normal((d, p))
    got = bd.band_action(bands, b, V, ("exp",), 10, 1e-12)
    ref = me.action(bd.band_dense(bands, b), V, ("exp",), 10, 1e-12)
    assert got["plan"] == ref["plan"]
    d1, d2 = co.poly_terms("exp", 10)
    bound = 16 * d * got["plan"] * (1 + _sum_abs_w(("exp",), 10) + abs(d1) + abs(d2)) * U64
    assert me.rel_fro(got["exp"], ref["exp"]) <= bound


def test_b1_equals_tridiagonal_oracle():
    d, p = 50, 3
    dl, dd, du = wl.tri_gaussian_batch(1, d, 0.5, 8.0, wl.SEED_BASE + 840)[0]
    bands = np.zeros((3, d))
    bands[0, 1:] = dl
    bands[1] = dd
    bands[2, :-1] = du
    V = np.random.default_rng(4).standard_normal((d, p))
    got = bd.band_action(bands, 1, V, ("exp", "phi1"), 8, 1e-12)
    ref = bd.tri_action(dl, dd, du, V, ("exp", "phi1"), 8, 1e-12)
    assert got["plan"] == ref["plan"] and got["eta"] == ref["eta"]
    bound = 16 * d * got["plan"] * (1 + _sum_abs_w(("exp", "phi1"), 8)) * U64
    for f in ("exp", "phi1"):
        assert me.rel_fro(got[f], ref[f]) <= bound


@pytest.mark.parametrize("tau", [0.25, 1.0])
def test_laplacian_squared_closed_form(tau):
    """A = -tau L^2 is pentadiagonal and symmetric with L's sine eigenvectors
    and eigenvalues lambda_j^2; per eigenvalue the N steps multiply by r(x)^N
    (exp) or rho(x) / N sum_j r(x)^j (phi1), x = mu / N."""
    d, p = 64, 2
    bands = bd.laplacian_sq_bands(d, tau)
    lam, U = bd.laplacian_1d_eig(d)
    mu = -tau * lam ** 2
    assert np.abs(U @ np.diag(mu) @ U.T - bd.band_dense(bands, 2)).max() <= 1e-12 * 16 * tau
    V = np.random.default_rng(9).standard_normal((d, p))
    got = bd.band_action(bands, 2, V, ("exp", "phi1"), 8, 1e-12)
    N = got["plan"]
    assert got["eta"] == 16.0 * tau
    meth = me.action_normal(mu, U, V, ("exp", "phi1"), 8, N, exact_scalars=True)
    for f in ("exp", "phi1"):
        assert me.rel_fro(got[f], meth[f]) <= 64 * N * U64 * (1 + _sum_abs_w(("exp", "phi1"), 8)), f
    ex = U @ (np.exp(mu)[:, None] * (U.T @ V))
    assert me.rel_fro(got["exp"], ex) <= N * 1e-12 * 10
    ph = U @ ((np.expm1(mu) / mu)[:, None] * (U.T @ V))
    assert me.rel_fro(got["phi1"], ph) <= N * 1e-12 * 10
