"""Pins for the oracle's algorithm against closed forms, exact scalar
reductions and high-precision evaluations -- none of which re-use the
oracle's own code path.

* diagonal reduction: for A = diag(l) the method returns diag(r(l 2^-s)^(2^s))
  exactly; r is evaluated in mpmath from the weights the paper prints, in the
  plain form of eq. (2), so the round-off rewrite of §4.3, the weights, the
  plan and the squaring are all checked at once;
* the whole pipeline against exact functions within the error the bound of §3
  allows: exp of diagonal, Jordan and rotation-generator matrices,
  exp(A) exp(-A) = I, phi1 through the augmented-matrix identity, phi1 of a
  diagonal via expm1;
* the action path against the -tau*L eigen-decomposition (discrete sine
  transform) and the i*H eigen-decomposition, and against the full-matrix
  result for small n.
"""

import math
from fractions import Fraction as Fr

import mpmath
import numpy as np
import pytest
import scipy.fft
import scipy.linalg as sla

from oracle import coefficients as co
from oracle import method as me
from paper_2210_03714_amd import workloads as wl

mpmath.mp.dps = 40


def _printed_r(golden, idx):
    e = golden["weights"][idx]
    c = [mpmath.mpf(Fr(x).numerator) / Fr(x).denominator for x in e["shifts"]]
    b = [mpmath.mpf(Fr(x).numerator) / Fr(x).denominator for x in e["b"]]
    return lambda z: sum(bi / (1 - ci * z) for ci, bi in zip(c, b))


def _r22(z):
    # eq. (5), pole form with the sqrt(3) reading
    return 1 + 2 * mpmath.re((6 + 6 * mpmath.sqrt(3) * 1j) / (z - (3 - mpmath.sqrt(3) * 1j)))


@pytest.mark.parametrize("m,idx", [(8, 5), (4, 3), (5, 6), (1, None)])
def test_diagonal_reduction_exact(golden, m, idx):
    lam = np.array([-8.0, -3.25, -0.5, 0.0, 0.125, 1.75, 4.0, 7.9])
    r = _r22 if idx is None else _printed_r(golden, idx)
    res = me.expm_full(np.diag(lam), ("exp",), m, 1e-12)
    s = res["plan"]
    # plan: smallest s with max|l| 2^-s <= θ, written with log2 here
    q = 8.0 / res["theta"]
    assert s == max(0, math.ceil(math.log2(q)))
    for i, l in enumerate(lam):
        want = r(mpmath.mpf(l) * mpmath.mpf(2) ** -s) ** (2 ** s)
        got = res["exp"][i, i]
        # round-off of the combination (~sum|w| |x| eps, §4.3) grows 2^s-fold
        # through the squarings: 2e-12 relative covers s <= 6 with margin
        assert abs(got - float(want)) <= 2e-12 * abs(float(want))
    off = res["exp"] - np.diag(np.diag(res["exp"]))
    assert np.all(off == 0)


def test_similarity_invariance():
    rng = np.random.default_rng(3)
    n = 16
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(-6, 6, n)
    A = Q @ np.diag(lam) @ Q.T
    ra = me.expm_full(A, ("exp",), 8, 1e-12)
    rd = me.expm_full(np.diag(lam), ("exp",), 8, 1e-12, force_plan=ra["plan"])
    assert me.rel_fro(ra["exp"], Q @ rd["exp"] @ Q.T) < 1e-12


@pytest.mark.parametrize("m", [4, 8])
def test_same_approximant_high_precision(golden, m):
    """n <= 8: evaluate the plain form of eq. (2) with the printed weights in
    mpmath (50 digits), then square s times; the FP64 oracle must agree to
    round-off, which isolates round-off from truncation."""
    idx = {4: 3, 8: 5}[m]
    e = golden["weights"][idx]
    rng = np.random.default_rng(11 + m)
    A = rng.standard_normal((6, 6))
    A *= 3.0 / np.abs(A).sum(0).max()
    res = me.expm_full(A, ("exp",), m, 1e-12)
    s = res["plan"]
    with mpmath.workdps(50):
        B = mpmath.matrix(A.tolist()) * mpmath.mpf(2) ** -s
        I = mpmath.eye(6)
        R = mpmath.zeros(6, 6)
        for cs, bs in zip(e["shifts"], e["b"]):
            c, b = Fr(cs), Fr(bs)
            cm = mpmath.mpf(c.numerator) / c.denominator
            bm = mpmath.mpf(b.numerator) / b.denominator
            R += bm * mpmath.inverse(I - cm * B)
        for _ in range(s):
            R = R * R
        Rn = np.array(R.tolist(), dtype=float)
    # round-off of the combination (sum|w| ||B|| eps) amplified by 2^s squarings
    assert me.rel_fro(res["exp"], Rn) < 2e-13


@pytest.mark.parametrize("lam", [-8.0, -1.0, 0.5, 3.0])
def test_jordan_block(lam):
    n = 6
    J = lam * np.eye(n) + np.eye(n, k=1)
    Nil = np.eye(n, k=1)
    want = math.exp(lam) * sum(np.linalg.matrix_power(Nil, k) / math.factorial(k) for k in range(n))
    res = me.expm_full(J, ("exp",), 8, 1e-12)
    # the bound of §3 holds per scaled step; s squarings multiply it by ~2^s
    assert me.rel_fro(res["exp"], want) < 2 ** res["plan"] * 1e-12


@pytest.mark.parametrize("t", [0.1, 1.0, 3.0, 10.0])
def test_rotation_generator(t):
    G = np.array([[0.0, -t], [t, 0.0]])
    want = np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
    res = me.expm_full(G, ("exp",), 8, 1e-12)
    # ||e^B|| = 1 here, so the truncation error after s squarings is ~2^s tol
    assert np.abs(res["exp"] - want).max() < 2 ** res["plan"] * 1e-12


@pytest.mark.parametrize("m,tol", [(8, 1e-12), (4, 1e-8), (1, 1e-8)])
def test_diagonal_vs_exact_exp_and_phi1(m, tol):
    """Norm-wise error (the bound of §3 is a norm bound) within 2^s tol."""
    lam = np.linspace(-8, 8, 17)
    res = me.expm_full(np.diag(lam), ("exp", "phi1"), m, tol)
    bound = 2.0 * 2 ** res["plan"] * tol
    want_e = np.exp(lam)
    want_p = np.array([math.expm1(l) / l if l != 0 else 1.0 for l in lam])
    assert np.max(np.abs(np.diag(res["exp"]) - want_e)) / want_e.max() < bound
    assert np.max(np.abs(np.diag(res["phi1"]) - want_p)) / want_p.max() < bound


def test_inverse_pair_identity():
    A = wl.gaussian(64, 6.0, 5)
    E = me.expm_full(A, ("exp",), 8, 1e-12)["exp"]
    Em = me.expm_full(-A, ("exp",), 8, 1e-12)["exp"]
    assert np.linalg.norm(E @ Em - np.eye(64)) / 8.0 < 1e-12


@pytest.mark.parametrize("n,eta", [(32, 1.0), (96, 8.0)])
def test_exp_and_phi1_vs_augmented_expm(n, eta):
    """exp([[A, I], [0, 0]]) = [[e^A, phi1(A)], [0, I]]."""
    A = wl.gaussian(n, eta, 17 + n)
    res = me.expm_full(A, ("exp", "phi1"), 8, 1e-12)
    aug = np.zeros((2 * n, 2 * n))
    aug[:n, :n] = A
    aug[:n, n:] = np.eye(n)
    X = sla.expm(aug)
    assert me.rel_fro(res["exp"], X[:n, :n]) < 1e-12
    assert me.rel_fro(res["phi1"], X[:n, n:]) < 1e-12


def test_phi1_doubling_uses_r_before_squaring():
    """Using R after it has been squared breaks the identity of §1; the
    oracle's order is pinned by the augmented-matrix check, restated here on a
    scalar where the two orders differ visibly."""
    A = np.array([[4.0]])
    res = me.expm_full(A, ("exp", "phi1"), 8, 1e-12)
    want = math.expm1(4.0) / 4.0
    assert abs(res["phi1"][0, 0] - want) < 2 ** res["plan"] * 1e-12 * want
    # the wrong order (square first) on the same scalar is off by far more
    s = res["plan"]
    r0 = me.expm_full(np.ldexp(A, -s), ("exp", "phi1"), 8, 1e-12, force_plan=0)
    R, P = r0["exp"][0, 0], r0["phi1"][0, 0]
    for _ in range(s):
        R = R * R
        P = 0.5 * (R + 1) * P
    assert abs(P - want) > 1e-2 * want


def test_paper_toeplitz_matrix():
    A = wl.toeplitz_cauchy(100) * 0.05
    res = me.expm_full(A, ("exp",), 8, 1e-12)
    assert me.rel_fro(res["exp"], sla.expm(A)) < 1e-12


# ---------------------------------------------------------------- action ---


def _dst_laplacian(n, tau):
    j = np.arange(1, n + 1)
    lam = 2 - 2 * np.cos(j * np.pi / (n + 1))
    return -tau * lam


def _r_scalar_float(m, func):
    a0, terms = co.roundoff_terms(func, m)

    def r(z):
        out = a0 + 0j
        for c, w, pair in terms:
            t = w * z / (1 - c * z)
            out += t + (np.conj(w) * z / (1 - np.conj(c) * z) if pair else 0)
        return out
    return r


@pytest.mark.parametrize("n,tau", [(64, 1.0), (256, 2.0)])
def test_action_laplacian_closed_form(n, tau):
    """-tau L = U diag(mu) U^T with U the orthonormal DST-I basis; the method's
    own result is U diag(r(mu/N)^N) U^T V and the exact one U diag(e^mu) U^T V."""
    A = wl.neg_laplacian(n, tau)
    V = wl.vectors(n, 3, 99)
    res = me.action(A, V, ("exp",), 8, 1e-12)
    N = res["plan"]
    assert N == max(1, math.ceil(4 * tau / res["theta"]))
    mu = _dst_laplacian(n, tau)
    dst = lambda X: scipy.fft.dst(X, type=1, axis=0, norm="ortho")
    r = _r_scalar_float(8, "exp")
    method = dst(np.real(r(mu / N) ** N)[:, None] * dst(V))
    exact = dst(np.exp(mu)[:, None] * dst(V))
    assert me.rel_fro(res["exp"], method) < 1e-12
    assert me.rel_fro(res["exp"], exact) < 1e-10


def test_action_ih_eigen_and_norm():
    n = 48
    A = wl.ih_matrix(n, 4)
    V = wl.vectors(n, 4, 5, complex_=True)
    res = me.action(A, V, ("exp",), 8, 1e-12)
    N = res["plan"]
    lam, U = np.linalg.eigh(-1j * A)
    r = _r_scalar_float(8, "exp")
    method = U @ ((r(1j * lam / N) ** N)[:, None] * (U.conj().T @ V))
    assert me.rel_fro(res["exp"], method) < 1e-12
    assert abs(np.linalg.norm(res["exp"]) / np.linalg.norm(V) - 1) < 1e-10


@pytest.mark.parametrize("kind", ["gauss", "lap"])
def test_action_phi1_vs_augmented(kind):
    n = 40
    A = wl.gaussian(n, 5.0, 8) if kind == "gauss" else wl.neg_laplacian(n, 1.0)
    V = wl.vectors(n, 2, 9)
    res = me.action(A, V, ("exp", "phi1"), 8, 1e-12)
    aug = np.zeros((n + 2, n + 2))
    aug[:n, :n] = A
    aug[:n, n:] = V
    X = sla.expm(aug)
    assert me.rel_fro(res["phi1"], X[:n, n:]) < 1e-11
    assert me.rel_fro(res["exp"], sla.expm(A) @ V) < 1e-11


def test_action_pair_set_on_real_matrix():
    A = wl.gaussian(24, 1.0, 12)
    V = wl.vectors(24, 2, 13)
    res = me.action(A, V, ("exp",), 1, 1e-8)
    assert np.isrealobj(res["exp"])
    assert me.rel_fro(res["exp"], sla.expm(A) @ V) < 1e-7


def test_config_small_plan():
    """32 x 32 with ||A||_1 = 1 and R4 at 1e-12: θ ~ 0.0189 gives s = 6, N = 53."""
    A, v = wl.config_small()
    rf = me.expm_full(A, ("exp",), 4, 1e-12)
    ra = me.action(A, v, ("exp",), 4, 1e-12)
    assert rf["plan"] == 6 and ra["plan"] == 53
    assert me.rel_fro(rf["exp"], sla.expm(A)) < 1e-12
    assert me.rel_fro(ra["exp"], sla.expm(A) @ v) < 1e-11


# --------------------------------------------- planted mistakes (on the CPU) --


def test_planted_weight_error_is_caught(golden, monkeypatch):
    """Flip one weight in the oracle: the diagonal-reduction pin must fail."""
    orig = co.roundoff_terms

    def broken(func, m):
        a0, t = orig(func, m)
        t = list(t)
        c, w, p = t[2]
        t[2] = (c, -w, p)
        return a0, t
    monkeypatch.setattr(co, "roundoff_terms", broken)
    with pytest.raises(AssertionError):
        test_diagonal_reduction_exact(golden, 8, 5)


def test_planted_squaring_order_error_is_caught(monkeypatch):
    """Square R before the phi1 doubling step: the augmented check must fail."""
    A = wl.gaussian(32, 8.0, 21)
    good = me.expm_full(A, ("exp", "phi1"), 8, 1e-12)
    s = good["plan"]
    n = 32
    res = me.expm_full(A, ("exp", "phi1"), 8, 1e-12, force_plan=0)
    # replay the undo-scaling loop with the wrong order from the s=0 state
    B = np.ldexp(A, -s)
    r0 = me.expm_full(B, ("exp", "phi1"), 8, 1e-12, force_plan=0)
    R, Phi = r0["exp"], r0["phi1"]
    for _ in range(s):
        R = R @ R
        Phi = 0.5 * ((R + np.eye(n)) @ Phi)
    aug = np.zeros((2 * n, 2 * n))
    aug[:n, :n] = A
    aug[:n, n:] = np.eye(n)
    want = sla.expm(aug)[:n, n:]
    assert me.rel_fro(good["phi1"], want) < 1e-12
    assert me.rel_fro(Phi, want) > 1e-3
    del res


@pytest.mark.parametrize("kind", ["iH", "negL"])
def test_action_normal_matches_step_by_step(kind):
    """The per-eigenvalue form of the N-step action equals the step-by-step
    oracle (LU solves every step) for normal A: iH (complex) and -L (real)."""
    n, p = 40, 3
    if kind == "iH":
        H = wl.ih_matrix(n, wl.SEED_BASE + 300) / 1j
        lam, U = np.linalg.eigh(H)
        mu, A = 1j * lam, 1j * H
        V = wl.vectors(n, p, wl.SEED_BASE + 301, complex_=True)
    else:
        A = wl.neg_laplacian(n, 1.0)
        mu, U = np.linalg.eigh(A)
        V = wl.vectors(n, p, wl.SEED_BASE + 302)
    ref = me.action(A, V, ("exp", "phi1"), 8, 1e-12)
    got = me.action_normal(mu, U, V, ("exp", "phi1"), 8, ref["plan"])
    got_x = me.action_normal(mu, U, V, ("exp", "phi1"), 8, ref["plan"], exact_scalars=True)
    for f in ("exp", "phi1"):
        assert me.rel_fro(got[f], ref[f]) <= 1e-13, (kind, f)
        assert me.rel_fro(got_x[f], ref[f]) <= 1e-13, (kind, f)
    # and both meet the exact functions within the bound (N steps, each <= tol)
    ex = U @ (np.exp(mu)[:, None] * (U.conj().T @ V))
    assert me.rel_fro(got["exp"], ex) <= ref["plan"] * 1e-12 * 10


def test_r_scalar_hybrid_is_the_rational():
    """For the hybrid set (m = 10, §4.3) r_scalar equals
    d0 + d1 x + d2 x^2 + sum b_i / (1 - c_i x) summed exactly at rational
    points, and so meets exp to the order-11 truncation at small x."""
    from fractions import Fraction as Fr
    c, b, d = co.hybrid_set(co.HYBRID_SETS[10])
    a0, terms = co.roundoff_terms("exp", 10)
    d1, d2 = co.poly_terms("exp", 10)
    u = 2.0 ** -53
    for xq in (Fr(1, 7), Fr(-3, 10), Fr(1, 20)):
        exact = d[0] + d[1] * xq + d[2] * xq * xq + sum((bi / (1 - ci * xq) for ci, bi in zip(c, b)), Fr(0))
        got = me.r_scalar("exp", 10, np.array([float(xq)]))[0]
        x = float(xq)
        mag = abs(a0) + abs(d1 * x) + abs(d2 * x * x) + sum(abs(w * x / (1 - cc * x)) for cc, w, _ in terms)
        assert abs(got - float(exact)) <= (len(terms) + 6) * u * mag, (xq, got, float(exact))
    # at x = 0.05 the truncation (order 11) is far below the rounding of the
    # round-off form, which the cancellation in sum |w_k| ~ 1e4 dominates
    x = 0.05
    mag = abs(a0) + abs(d1 * x) + abs(d2 * x * x) + sum(abs(w * x / (1 - cc * x)) for cc, w, _ in terms)
    assert abs(me.r_scalar("exp", 10, np.array([x]))[0] - np.exp(x)) <= (len(terms) + 6) * u * mag + x ** 11


def test_r_scalar_is_the_rational():
    """r_scalar in the round-off form equals sum b_k / (1 - c_k x) summed
    exactly at rational points (the partial-fraction form of eq. 2)."""
    from fractions import Fraction as Fr
    c, b = co.real_set("exp", 8)
    for xq in (Fr(1, 7), Fr(-3, 10), Fr(1, 4)):
        exact = sum((bi / (1 - ci * xq) for ci, bi in zip(c, b)), Fr(0))
        got = me.r_scalar("exp", 8, np.array([float(xq)]))[0]
        # rounding bound of the round-off form: each term w x / (1 - c x)
        # within ~3u, their sum within m u, scaled by sum_k |term_k|
        a0, terms = co.roundoff_terms("exp", 8)
        mag = sum(abs(w * float(xq) / (1 - c * float(xq))) for c, w, _ in terms)
        u = 2.0 ** -53
        assert abs(got - float(exact)) <= (len(terms) + 4) * u * (mag + abs(a0))


def test_hybrid_diagonal_reduction(golden):
    """m = 10 (R10, §4.3) on a diagonal matrix: the oracle's round-off form
    with the polynomial part equals the printed plain form
    d0 + d1 x + d2 x^2 + sum b_i / (1 - c_i x), raised to 2^s, at 40 digits."""
    e = [e for e in golden["hybrid"] if e["set"] == "R10"][0]
    q = lambda x: mpmath.mpf(Fr(x).numerator) / Fr(x).denominator
    c = [q(x) for x in e["shifts"]]
    b = [q(x) for x in e["b"]] + [q(x) for x in e["b_free"]]
    d = [q(x) for x in e["d"]]
    r = lambda z: d[0] + d[1] * z + d[2] * z ** 2 + sum(bi / (1 - ci * z) for ci, bi in zip(c, b))
    lam = np.array([-8.0, -3.25, -0.5, 0.0, 0.125, 1.75, 4.0, 7.9])
    res = me.expm_full(np.diag(lam), ("exp",), 10, 1e-12)
    s = res["plan"]
    assert s == max(0, math.ceil(math.log2(8.0 / res["theta"])))
    sw = sum(abs(float(bi * ci)) for bi, ci in zip(b, c))  # the round-off form's amplification
    for i, l in enumerate(lam):
        want = float(r(mpmath.mpf(l) * mpmath.mpf(2) ** -s) ** (2 ** s))
        got = res["exp"][i, i]
        # each scaled evaluation rounds to ~sum|w| |x| eps; 2^s squarings amplify it
        assert abs(got - want) <= 8 * sw * 2.0 ** -53 * 2 ** s * abs(want) + 1e-300, (l, got, want)


def test_log1m_diagonal_and_logm(golden):
    """log(1 - x) (§2 worked example) has no scaling identity: s = 0.  On a
    diagonal matrix the round-off form equals the printed plain form
    sum b_i / (1 - c_i x) at 40 digits; on a dense matrix with ||A||_1 = θ/2
    the result meets logm(I - A) within the absolute bound of §3."""
    e = [e for e in golden["weights"] if e["func"] == "log1m"][0]
    q = lambda x: mpmath.mpf(Fr(x).numerator) / Fr(x).denominator
    c = [q(x) for x in e["shifts"]]
    b = [q(x) for x in e["b"]]
    th_ = me.theta_for(("log1m",), 5, 1e-12)
    lam = np.array([-1.0, -0.5, 0.0, 0.25, 0.9]) * th_
    res = me.expm_full(np.diag(lam), ("log1m",), 5, 1e-12)
    assert res["plan"] == 0
    for i, l in enumerate(lam):
        want = float(sum(bi / (1 - ci * mpmath.mpf(l)) for ci, bi in zip(c, b)))
        # round-off form: sum |w_k| |x| / (1 - c_k x) eps, about 100 |x| eps here
        assert abs(res["log1m"][i, i] - want) <= 1e3 * 2.0 ** -53 * max(abs(l), 1e-300)
    A = wl.gaussian(24, th_ / 2, 11)
    got = me.expm_full(A, ("log1m",), 5, 1e-12)["log1m"]
    exact = sla.logm(np.eye(24) - A).real
    assert np.abs(got - exact).sum(axis=0).max() <= 1e-12 + 1e-14
