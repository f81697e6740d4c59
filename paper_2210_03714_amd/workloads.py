"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws and shapes input matrices and vectors; it holds none of
the method's arithmetic.  It is the one piece of code that both the GPU
library's tests/benchmark and the CPU oracle's tests use, so that both sides
see bit-identical inputs.

Matrix families
---------------
* Gaussian: entries i.i.d. N(0,1) as in the ``randn`` experiments of §5, then
  rescaled so that ||A||_1 takes a prescribed value (drawn per instance).
* i*H with H Hermitian: H = (G + G^H) / sqrt(2n), G_ij = (x + i y)/sqrt(2),
  x, y ~ N(0,1), so E|H_ij|^2 = 1/n and the spectrum of H lies near [-2, 2];
  A = i H has its spectrum on the imaginary axis (unitary evolution).
* -tau * trid{-1, 2, -1}: the tridiagonal matrix of the sparse experiment of
  §5 with the sign flipped so that e^A is dissipative, stored dense.
* A_ij = 1 / (1 + (i - j)^2): the symmetric dense test matrix of §5.
* Tridiagonal (the sparse case of §2.1 and §5), stored as three diagonals:
  N(0,1) diagonals rescaled to a prescribed ||A||_1, and -tau trid{-1, 2, -1}.

All generators take an explicit seed and use numpy's PCG64 default_rng.
"""

import numpy as np

SEED_BASE = 2210037140


def _rescale_norm1(A, target):
    return A * (target / np.abs(A).sum(axis=0).max())


def gaussian(n, norm1, seed):
    """One n x n N(0,1) matrix rescaled to ||A||_1 = norm1."""
    rng = np.random.default_rng(seed)
    return _rescale_norm1(rng.standard_normal((n, n)), norm1)


def gaussian_batch(batch, n, norm_lo, norm_hi, seed):
    """``batch`` Gaussian n x n matrices, ||A||_1 ~ U[norm_lo, norm_hi] each.
    Returns (A[batch, n, n] float64 C-contiguous, targets[batch])."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((batch, n, n))
    t = rng.uniform(norm_lo, norm_hi, size=batch)
    scale = t / np.abs(A).sum(axis=1).max(axis=1)
    A *= scale[:, None, None]
    return np.ascontiguousarray(A), t


def gaussian_uneven(batch, sizes, norm_lo, norm_hi, seed):
    """List of Gaussian matrices with n drawn uniformly from ``sizes``."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=batch)
    out = []
    for n in ns:
        A = rng.standard_normal((int(n), int(n)))
        out.append(_rescale_norm1(A, rng.uniform(norm_lo, norm_hi)))
    return out


def vectors(n, p, seed, complex_=False):
    """Block of p right-hand sides, N(0,1) (complex: (x + i y)/sqrt(2))."""
    rng = np.random.default_rng(seed)
    if complex_:
        return (rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))) / np.sqrt(2)
    return rng.standard_normal((n, p))


def ih_matrix(n, seed):
    """A = i H with H Hermitian, E|H_ij|^2 = 1/n (complex128)."""
    rng = np.random.default_rng(seed)
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2)
    H = (G + G.conj().T) / np.sqrt(2 * n)
    return 1j * H


def neg_laplacian(n, tau=1.0):
    """A = -tau * trid{-1, 2, -1}, dense float64."""
    A = np.zeros((n, n))
    i = np.arange(n)
    A[i, i] = -2.0 * tau
    A[i[:-1], i[:-1] + 1] = tau
    A[i[1:], i[1:] - 1] = tau
    return A


def toeplitz_cauchy(n):
    """A_ij = 1 / (1 + (i - j)^2)."""
    i = np.arange(n)
    return 1.0 / (1.0 + (i[:, None] - i[None, :]) ** 2.0)


def config_small(seed=SEED_BASE + 0):
    """One 32 x 32 N(0,1) matrix with ||A||_1 = 1 and a vector v ~ N(0,1)^32."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((32, 32))
    A = _rescale_norm1(A, 1.0)
    v = rng.standard_normal((32, 1))
    return A, v


def serving_requests(rate, duration, seed, n_lo=16, n_hi=1024):
    """Open-loop Poisson request stream.  Each request is a dict with arrival
    time, n (log-uniform in [n_lo, n_hi]), function, mode, p, tol, matrix
    type and a per-request seed for its matrix."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        reqs.append({
            "t": t,
            "n": n,
            "func": ("exp", "phi1")[rng.integers(2)],
            "mode": ("full", "action")[rng.integers(2)],
            "p": int(rng.integers(1, 33)),
            "tol": (1e-8, 1e-12)[rng.integers(2)],
            "kind": ("gauss", "ih", "lap")[rng.integers(3)],
            "norm1": float(rng.uniform(0.5, 8.0)),
            "seed": int(rng.integers(2**62)),
        })
    return reqs


def request_inputs(req):
    """Materialise the matrix (and block) of a serving request."""
    n, kind = req["n"], req["kind"]
    if kind == "gauss":
        A = gaussian(n, req["norm1"], req["seed"])
    elif kind == "ih":
        A = ih_matrix(n, req["seed"])
    else:
        A = neg_laplacian(n, 1.0)
    V = None
    if req["mode"] == "action":
        V = vectors(n, req["p"], req["seed"] + 1, complex_=np.iscomplexobj(A))
    return A, V


def serving_pool(seed, per_kind=64, n_lo=16, n_hi=1024):
    """Matrices the serving stream draws from: per matrix type, ``per_kind``
    matrices with n log-uniform in [n_lo, n_hi] (Gaussian: ||A||_1 uniform in
    [0.5, 8]; iH; -L with tau = 1), and per type one n_hi x 32 block of
    right-hand sides (complex for iH)."""
    rng = np.random.default_rng(seed)
    pool, vpool = {}, {}
    for kind in ("gauss", "ih", "lap"):
        mats = []
        for _ in range(per_kind):
            n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
            s = int(rng.integers(2**62))
            if kind == "gauss":
                mats.append(gaussian(n, float(rng.uniform(0.5, 8.0)), s))
            elif kind == "ih":
                mats.append(ih_matrix(n, s))
            else:
                mats.append(neg_laplacian(n, 1.0))
        pool[kind] = mats
        vpool[kind] = vectors(n_hi, 32, int(rng.integers(2**62)), complex_=(kind == "ih"))
    return pool, vpool


def serving_stream(rate, duration, seed, pool):
    """Open-loop Poisson arrivals at ``rate`` per second for ``duration``
    seconds over a ``serving_pool``: each request draws a matrix type, a pool
    matrix of that type, a function (exp or phi1), a mode (full matrix, or
    action on the first p in [1, 32] columns of the type's block) and a
    tolerance (1e-8 or 1e-12), all uniformly."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    kinds = ("gauss", "ih", "lap")
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        kind = kinds[rng.integers(3)]
        idx = int(rng.integers(len(pool[kind])))
        reqs.append({"t": t, "kind": kind, "idx": idx, "n": pool[kind][idx].shape[0],
                     "func": ("exp", "phi1")[rng.integers(2)],
                     "mode": ("full", "action")[rng.integers(2)],
                     "p": int(rng.integers(1, 33)),
                     "tol": (1e-8, 1e-12)[rng.integers(2)]})
    return reqs


def _tri_rescale(dl, dd, du, target):
    col = np.abs(dd).copy()
    col[1:] += np.abs(du)
    col[:-1] += np.abs(dl)
    f = target / col.max()
    return dl * f, dd * f, du * f


def tri_gaussian_batch(batch, d, norm_lo, norm_hi, seed):
    """``batch`` tridiagonal d x d matrices with N(0,1) diagonals, each
    rescaled to ||A||_1 ~ U[norm_lo, norm_hi].  Returns a list of
    (dl, dd, du) float64 arrays (lengths d - 1, d, d - 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(batch):
        dl = rng.standard_normal(d - 1)
        dd = rng.standard_normal(d)
        du = rng.standard_normal(d - 1)
        out.append(_tri_rescale(dl, dd, du, rng.uniform(norm_lo, norm_hi)))
    return out


def tri_neg_laplacian(d, tau=1.0):
    """Diagonals of -tau trid{-1, 2, -1} (the test matrix of §5, dissipative sign)."""
    return np.full(d - 1, tau), np.full(d, -2.0 * tau), np.full(d - 1, tau)


def band_gaussian_batch(batch, d, b, norm_lo, norm_hi, seed):
    """``batch`` banded d x d matrices (half-bandwidth b) with N(0,1)
    diagonals, each rescaled to ||A||_1 ~ U[norm_lo, norm_hi].  Returns a
    list of float64 arrays of shape (2b + 1, d), bands[b + o, i] = A[i, i + o];
    entries outside A are zero."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(batch):
        bands = rng.standard_normal((2 * b + 1, d))
        col = np.zeros(d)
        for o in range(-b, b + 1):
            lo = min(d, max(0, -o))
            hi = max(lo, min(d, d - o))
            bands[b + o, :lo] = 0.0
            bands[b + o, hi:] = 0.0
            col[lo + o:hi + o] += np.abs(bands[b + o, lo:hi])
        out.append(bands * (rng.uniform(norm_lo, norm_hi) / col.max()))
    return out
