"""Pins of the oracle's caller-given partial-fraction sets (oracle.method.rational):
with the Padé pair of §2 eq. (5) it is the closed-form r22 quotient; on a
diagonalisable A it is Q diag(r(lambda_i)) Q^-1 with r evaluated at each
eigenvalue in 30-digit arithmetic, for real and complex shifts, with and
without the conjugate terms; a planted mistake (the conjugate terms dropped)
fails that pin."""

import mpmath as mp
import numpy as np

from oracle import coefficients as co
from oracle import method as me


def _r_scalar(x, c, w, a0, conj_pairs):
    mp.mp.dps = 30
    x = mp.mpc(x)
    out = mp.mpc(a0)
    for ck, wk in zip(c, w):
        ck, wk = mp.mpc(complex(ck)), mp.mpc(complex(wk))
        out += wk * x / (1 - ck * x)
        if conj_pairs and ck.imag != 0:
            out += mp.conj(wk) * x / (1 - mp.conj(ck) * x)
    return complex(out)


def _by_eigen(A, c, w, a0, conj_pairs):
    lam, Q = np.linalg.eig(A)
    r = np.array([_r_scalar(x, c, w, a0, conj_pairs) for x in lam])
    return Q @ np.diag(r) @ np.linalg.inv(Q)


def test_pade_pair_is_r22():
    """The round-off terms of the exp Padé pair (§2 eq. 5) give
    (I - A/2 + A^2/12)^{-1} (I + A/2 + A^2/12)."""
    rng = np.random.default_rng(11)
    A = rng.standard_normal((12, 12))
    A *= 0.6 / np.abs(A).sum(axis=0).max()
    a0, terms = co.roundoff_terms("exp", 1)
    (c, w, _), = terms
    got = me.rational(A, [c], [w], a0, conj_pairs=True)
    I = np.eye(12)
    ref = np.linalg.solve(I - A / 2 + A @ A / 12, I + A / 2 + A @ A / 12)
    assert np.isrealobj(got)
    assert me.rel_fro(got, ref) <= 1e-14


def test_eigen_form_real_and_complex():
    rng = np.random.default_rng(12)
    n = 10
    c = [0.3 + 0.2j, -0.25, 0.1 - 0.4j]
    w = [1.5 - 0.5j, 2.0, -0.7 + 0.3j]
    a0 = 0.75
    # real A, conjugate pairs: a real result equal to the eigen form
    A = rng.standard_normal((n, n))
    A *= 1.2 / np.abs(A).sum(axis=0).max()
    got = me.rational(A, c, w, a0, conj_pairs=True)
    ref = _by_eigen(A, c, w, a0, True)
    assert np.isrealobj(got) and np.abs(ref.imag).max() <= 1e-12
    assert me.rel_fro(got, ref.real) <= 1e-13
    # complex A, no conjugates
    Ac = A + 1j * rng.standard_normal((n, n)) * 0.1
    gotc = me.rational(Ac, c, w, a0, conj_pairs=False)
    assert me.rel_fro(gotc, _by_eigen(Ac, c, w, a0, False)) <= 1e-13
    # the action form is the full form times V
    V = rng.standard_normal((n, 3))
    assert me.rel_fro(me.rational(A, c, w, a0, True, V=V), got @ V) <= 1e-13


def test_planted_mistake_dropped_conjugates_fails():
    rng = np.random.default_rng(13)
    A = rng.standard_normal((8, 8))
    A *= 0.8 / np.abs(A).sum(axis=0).max()
    c, w, a0 = [0.2 + 0.3j], [1.0 + 2.0j], 1.0
    wrong = me.rational(A.astype(complex), c, w, a0, conj_pairs=False)
    assert me.rel_fro(wrong, _by_eigen(A, c, w, a0, True)) > 1e-3
