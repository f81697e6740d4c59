"""Pins of the oracle's phi2 (§1's phi_k with k = 2: (e^x - 1 - x) / x^2) to
things the paper and the mathematics fix, not to the oracle itself:

* the augmented-matrix identity: the top block row of
  exp([[A, I, 0], [0, 0, I], [0, 0, 0]]) is [e^A, phi1(A), phi2(A)]
  (scipy's expm, a different algorithm, on the 3n x 3n matrix);
* scalar closed forms at 50 digits (diagonal A, including s > 0);
* a nilpotent A, where phi2(A) is the finite sum of A^k / (k + 2)!;
* the phi2 weights: eq. (4) with a_k = 1/(k + 2)! makes the approximant's
  Taylor series agree through x^(P-1), checked by expanding the rounded
  round-off form with mpmath (a dropped factor in a weight fails it);
* a planted mistake in the doubling step (phi2 <- (phi1^2 + phi2) / 4) is
  caught by the augmented-matrix pin.
"""

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import coefficients as co
from oracle import method as me
from paper_2210_03714_amd import workloads as wl


def _augmented(A):
    n = A.shape[0]
    Z = np.zeros((3 * n, 3 * n))
    Z[:n, :n] = A
    Z[:n, n:2 * n] = np.eye(n)
    Z[n:2 * n, 2 * n:] = np.eye(n)
    E = sla.expm(Z)
    return E[:n, :n], E[:n, n:2 * n], E[:n, 2 * n:]


@pytest.mark.parametrize("m", [4, 5, 8])
@pytest.mark.parametrize("n, eta", [(6, 0.1), (20, 3.0), (12, 40.0)])
def test_augmented_matrix_identity(m, n, eta):
    G = wl.gaussian(n, 1.0, wl.SEED_BASE + 1300 + n)
    A = G - G.T if eta > 10 else G  # skew-symmetric at the large norm: no growth over the squarings
    A = A * (eta / np.abs(A).sum(axis=0).max())
    r = me.expm_full(A, ("exp", "phi1", "phi2"), m, 1e-12)
    e, p1, p2 = _augmented(A)
    bar = 1e-12 * max(1.0, 2.0 ** (r["plan"] - 5))
    assert me.rel_fro(r["phi2"], p2) <= bar, (r["plan"], me.rel_fro(r["phi2"], p2))
    assert me.rel_fro(r["phi1"], p1) <= bar
    assert me.rel_fro(r["exp"], e) <= bar
    # phi2 alone gives the same phi2 (the phi1 chain is carried either way)
    r2 = me.expm_full(A, ("phi2",), m, 1e-12)
    assert np.array_equal(r2["phi2"], r["phi2"]) and r2["plan"] == r["plan"]


def test_scalar_closed_form():
    mpmath.mp.dps = 50
    lam = [-30.0, -2.5, -1e-3, 0.0, 1e-3, 0.7, 5.0, 20.0]
    r = me.expm_full(np.diag(lam), ("phi2",), 8, 1e-12)
    assert r["plan"] > 0
    for i, x in enumerate(lam):
        xm = mpmath.mpf(x)
        ref = mpmath.mpf(1) / 2 if x == 0 else (mpmath.exp(xm) - 1 - xm) / xm ** 2
        got = r["phi2"][i, i]
        assert abs(got - float(ref)) <= 1e-12 * abs(float(ref)) * max(1.0, 2.0 ** (r["plan"] - 5)), (x, got, ref)


def test_nilpotent_finite_sum():
    n = 5
    N = 0.3 * np.eye(n, k=1) + 0.2 * np.eye(n, k=2)
    ref = sum(np.linalg.matrix_power(N, k) / mpmath.factorial(k + 2) for k in range(n)).astype(float)
    r = me.expm_full(N, ("phi2",), 8, 1e-12)
    assert np.abs(r["phi2"] - ref).max() <= 1e-15


@pytest.mark.parametrize("m", [4, 5, 8])
def test_phi2_weights_match_taylor(m):
    """r(x) = a0 + sum_k w_k x / (1 - c_k x) from the rounded weights agrees
    with sum_k x^k / (k + 2)! through the order of the set (eq. 4), up to the
    rounding of the weights; the next coefficient does not."""
    mpmath.mp.dps = 40
    a0, terms = co.roundoff_terms("phi2", m)
    P = co.order_of(m) + 1
    w = [mpmath.mpf(t[1]) for t in terms]
    c = [mpmath.mpf(t[0]) for t in terms]
    coef = [mpmath.mpf(a0)] + [sum(wi * ci ** (k - 1) for wi, ci in zip(w, c)) for k in range(1, P + 2)]
    scale = sum(abs(wi) for wi in w) + 1
    for k in range(P):
        assert abs(coef[k] - 1 / mpmath.factorial(k + 2)) <= 1e-14 * scale, (m, k)
    assert abs(coef[P] - 1 / mpmath.factorial(P + 2)) > 1e-10 / mpmath.factorial(P + 2)


def test_planted_doubling_error_is_caught(monkeypatch):
    """phi2 <- (phi1^2 + phi2) / 4 (a dropped factor 2) must fail the pin."""
    def broken(R, Phi, Phi2, I):
        if Phi2 is not None:
            Phi2 = 0.25 * (Phi @ Phi) + 0.25 * Phi2
        if Phi is not None:
            Phi = 0.5 * ((R + I) @ Phi)
        return R @ R, Phi, Phi2

    A = wl.gaussian(20, 3.0, wl.SEED_BASE + 1320)
    monkeypatch.setattr(me, "doubling_step", broken)
    r = me.expm_full(A, ("phi2",), 8, 1e-12)
    assert r["plan"] > 0
    assert me.rel_fro(r["phi2"], _augmented(A)[2]) > 1e-6
