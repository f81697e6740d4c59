"""Pins for the tridiagonal-action oracle (oracle/banded.py), each against
something other than its own code path:

* the norm and the product against the dense matrix (brute force);
* the whole N-step recurrence against the dense oracle (dense LAPACK getrf /
  getrs instead of the tridiagonal gttrf / gttrs), same plan, and the two
  agree to rounding;
* -tau trid{-1, 2, -1} against the closed-form sine eigen-decomposition: the
  method's exact result per eigenvalue (40-digit scalars) and the exact
  exponential within the N-step error bound;
* the 1 x 1 case against the scalar rational approximant.
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


def _random_tri(d, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(d - 1), scale * rng.standard_normal(d),
            scale * rng.standard_normal(d - 1))


def test_norm_and_product_against_dense():
    dl, dd, du = _random_tri(37, wl.SEED_BASE + 400)
    A = bd.tri_dense(dl, dd, du)
    assert bd.tri_norm1(dl, dd, du) == np.abs(A).sum(axis=0).max()
    X = np.random.default_rng(1).standard_normal((37, 5))
    assert np.abs(bd.tri_matvec(dl, dd, du, X) - A @ X).max() <= 4 * U64 * np.abs(A).sum(1).max() * np.abs(X).max()


@pytest.mark.parametrize("d", [2, 3, 48])
@pytest.mark.parametrize("funcs", [("exp",), ("phi1",), ("exp", "phi1")])
@pytest.mark.parametrize("m", [4, 5, 8])
def test_tridiagonal_equals_dense_oracle(funcs, m, d):
    """Same plan as the dense oracle, and the same result up to the solvers'
    rounding: each step's difference is at most a few units of rounding times
    sum |w_k| (the round-off form's amplification, §4.3), and N steps add up."""
    p = 3
    dl, dd, du = _random_tri(d, wl.SEED_BASE + 401 + m)
    V = np.random.default_rng(m).standard_normal((d, p))
    got = bd.tri_action(dl, dd, du, V, funcs, m, 1e-12)
    ref = me.action(bd.tri_dense(dl, dd, du), V, funcs, m, 1e-12)
    assert got["plan"] == ref["plan"]
    bound = 16 * d * got["plan"] * (1 + _sum_abs_w(funcs, m)) * U64
    for f in funcs:
        assert me.rel_fro(got[f], ref[f]) <= bound, (f, me.rel_fro(got[f], ref[f]), bound)


@pytest.mark.parametrize("d", [2, 3, 48])
def test_tridiagonal_hybrid_equals_dense_oracle(d):
    """The hybrid set of §4.3 (m = 10, exp; R10' of §5 on a tridiagonal A):
    same plan and result as the dense oracle, whose polynomial part is a
    dense product, to the rounding bound above with the polynomial
    coefficients added to the amplification."""
    p = 3
    dl, dd, du = _random_tri(d, wl.SEED_BASE + 411)
    V = np.random.default_rng(10).standard_normal((d, p))
    got = bd.tri_action(dl, dd, du, V, ("exp",), 10, 1e-12)
    ref = me.action(bd.tri_dense(dl, dd, du), V, ("exp",), 10, 1e-12)
    assert got["plan"] == ref["plan"]
    d1, d2 = co.poly_terms("exp", 10)
    bound = 16 * d * got["plan"] * (1 + _sum_abs_w(("exp",), 10) + abs(d1) + abs(d2)) * U64
    assert me.rel_fro(got["exp"], ref["exp"]) <= bound, (me.rel_fro(got["exp"], ref["exp"]), bound)


def test_laplacian_hybrid_closed_form():
    """R10' on A = -trid{-1, 2, -1}, d = 64: per eigenvalue the N steps
    multiply by r(x)^N, and the result is exp(A) V within the N-step bound."""
    d, p = 64, 2
    dl = np.full(d - 1, 1.0)
    dd = np.full(d, -2.0)
    du = np.full(d - 1, 1.0)
    lam, U = bd.laplacian_1d_eig(d)
    mu = -lam
    V = np.random.default_rng(8).standard_normal((d, p))
    got = bd.tri_action(dl, dd, du, V, ("exp",), 10, 1e-12)
    N = got["plan"]
    meth = me.action_normal(mu, U, V, ("exp",), 10, N, exact_scalars=True)
    d1, d2 = co.poly_terms("exp", 10)
    assert me.rel_fro(got["exp"], meth["exp"]) <= 64 * N * U64 * (1 + _sum_abs_w(("exp",), 10) + abs(d1) + abs(d2))
    ex = U @ (np.exp(mu)[:, None] * (U.T @ V))
    assert me.rel_fro(got["exp"], ex) <= N * 1e-12 * 10


@pytest.mark.parametrize("tau", [1.0, 8.0])
def test_laplacian_closed_form(tau):
    """A = -tau trid{-1, 2, -1} (the test matrix of §5) is symmetric, with the
    textbook sine eigenvectors; per eigenvalue the N steps multiply by
    r(x)^N (exp) or rho(x) / N sum_j r(x)^j (phi1), x = mu / N."""
    d, p = 64, 2
    dl = np.full(d - 1, tau)
    dd = np.full(d, -2.0 * tau)
    du = np.full(d - 1, tau)
    lam, U = bd.laplacian_1d_eig(d)
    mu = -tau * lam
    V = np.random.default_rng(7).standard_normal((d, p))
    got = bd.tri_action(dl, dd, du, V, ("exp", "phi1"), 8, 1e-12)
    N = got["plan"]
    meth = me.action_normal(mu, U, V, ("exp", "phi1"), 8, N, exact_scalars=True)
    for f in ("exp", "phi1"):
        assert me.rel_fro(got[f], meth[f]) <= 64 * N * U64 * (1 + _sum_abs_w(("exp", "phi1"), 8)), f
    ex = U @ (np.exp(mu)[:, None] * (U.T @ V))
    assert me.rel_fro(got["exp"], ex) <= N * 1e-12 * 10
    ph = U @ ((np.expm1(mu) / mu)[:, None] * (U.T @ V))
    assert me.rel_fro(got["phi1"], ph) <= N * 1e-12 * 10


def test_one_by_one_is_the_scalar_approximant():
    a = -3.7
    got = bd.tri_action(np.zeros(0), np.array([a]), np.zeros(0), np.array([[1.5]]), ("exp",), 8, 1e-12)
    N = got["plan"]
    r = me.r_scalar("exp", 8, np.array([a / N]))[0].real
    assert abs(got["exp"][0, 0] - 1.5 * r ** N) <= 4 * N * U64 * abs(got["exp"][0, 0]) * (1 + _sum_abs_w(("exp",), 8))


def test_force_plan_and_complex_shift_rejected():
    dl, dd, du = _random_tri(10, 3)
    V = np.ones((10, 1))
    assert bd.tri_action(dl, dd, du, V, ("exp",), 8, 1e-12, force_plan=5)["plan"] == 5
    with pytest.raises(NotImplementedError):
        bd.tri_action(dl, dd, du, V, ("exp",), 1, 1e-12)
