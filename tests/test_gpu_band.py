"""GPU parity of the banded action (pfm_band_action; §2.1 and §5 name the
pentadiagonal case beside the tridiagonal one) against the banded oracle
(oracle/banded.py, LAPACK gbtrf / gbtrs), element by element on the same
seeded inputs: relative Frobenius error <= 1e-12 per instance and function,
the same N, the same ||A||_1 bit for bit, and route 4.  Half-bandwidths
b = 1..4, uneven batches with ragged 64-column waves, d below and above b,
and the entries of ``bands`` outside A set to NaN on the device (they must
never be read)."""

import ctypes
import sys

import numpy as np
import pytest

from oracle import banded as bd
from oracle import coefficients as co
from oracle import method as me
from paper_2210_03714_amd import workloads as wl

pytestmark = pytest.mark.gpu

BAR = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2210_03714_amd import pfm
    pfm.lib()
    return torch, torch.device("cuda:0")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _outside_nan(bands, b):
    B = np.array(bands, copy=True)
    d = B.shape[1]
    for o in range(-b, b + 1):
        lo = min(d, max(0, -o))
        B[b + o, :lo] = np.nan
        B[b + o, max(lo, min(d, d - o)):] = np.nan
    return B


def _run(torch, dev, bands, vecs, b, funcs, m, tol, force_plan=-1):
    from paper_2210_03714_amd import pfm
    Bt = [torch.from_numpy(np.ascontiguousarray(_outside_nan(x, b))).to(dev) for x in bands]
    V = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in vecs]
    res, info = pfm.band_action(Bt, V, b, funcs, m=m, tol=tol, force_plan=force_plan)
    torch.cuda.synchronize()
    return res, info


def _own(bands, b, V, funcs, m, tol, N):
    own = bd.band_action(bands, b, V, funcs, m, tol)
    q = own["eta"] / own["theta"]
    if abs(q - round(q)) < 1e-12 * q:
        return bd.band_action(bands, b, V, funcs, m, tol, force_plan=N)
    assert N == own["plan"], (N, own["plan"])
    return own


def _check(res, info, bands, vecs, b, funcs, m, tol, bar=BAR, cols=None, idx=None):
    worst = 0.0
    idx = list(range(len(bands))) if idx is None else idx
    for j, i in enumerate(idx):
        V = vecs[i] if cols is None else vecs[i][:, cols]
        N = int(info[i]["plan"])
        own = _own(bands[i], b, V, funcs, m, tol, N)
        assert info[i]["norm1"] == own["eta"], (i, info[i]["norm1"], own["eta"])
        assert info[i]["route"] == 4 and info[i]["status"] == 0 and info[i]["bad_shift"] == -1
        for f in funcs:
            got = res[f][i].cpu().numpy()
            if cols is not None:
                got = got[:, cols]
            err = me.rel_fro(got, own[f])
            worst = max(worst, err)
            assert err <= bar, (i, f, V.shape, N, err, bar)
    return worst


SHAPES = [(1, 1), (2, 3), (5, 64), (37, 65), (130, 7)]


@pytest.mark.parametrize("b", [1, 2, 3, 4])
@pytest.mark.parametrize("funcs,m", [(("exp", "phi1"), 8), (("exp",), 4), (("phi1",), 5)])
def test_uneven_batch(torch_dev, b, funcs, m):
    torch, dev = torch_dev
    bands = [wl.band_gaussian_batch(1, d, b, 0.5, 8.0, wl.SEED_BASE + 900 + 7 * j + b)[0]
             for j, (d, p) in enumerate(SHAPES)]
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 940 + j) for j, (d, p) in enumerate(SHAPES)]
    _say("case band b=%d funcs=%s m=%d" % (b, funcs, m))
    res, info = _run(torch, dev, bands, vecs, b, funcs, m, 1e-12)
    _say("  worst %.2e" % _check(res, info, bands, vecs, b, funcs, m, 1e-12))


def test_pentadiagonal_laplacian_squared(torch_dev):
    """-L^2 (pentadiagonal, ||A||_1 = 16) at d = 1000, the size of the
    paper's tridiagonal example, and tol 1e-8."""
    torch, dev = torch_dev
    bands = [bd.laplacian_sq_bands(1000, 1.0), bd.laplacian_sq_bands(257, 0.25)]
    vecs = [wl.vectors(1000, 3, wl.SEED_BASE + 960), wl.vectors(257, 66, wl.SEED_BASE + 961)]
    for tol in (1e-12, 1e-8):
        _say("case band -L^2 tol=%g" % tol)
        res, info = _run(torch, dev, bands, vecs, 2, ("exp", "phi1"), 8, tol)
        _say("  worst %.2e" % _check(res, info, bands, vecs, 2, ("exp", "phi1"), 8, tol))


def test_b1_matches_tridiagonal_path(torch_dev):
    """b = 1 through the banded entry point and the same matrices through
    pfm_tri_action: the same N and ||A||_1, results within the bar."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    d, p = 300, 70
    tris = wl.tri_gaussian_batch(3, d, 0.5, 8.0, wl.SEED_BASE + 970)
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 971 + i) for i in range(3)]
    bands = []
    for dl, dd, du in tris:
        x = np.zeros((3, d))
        x[0, 1:], x[1], x[2, :-1] = dl, dd, du
        bands.append(x)
    _say("case band b=1 vs tridiagonal path")
    res, info = _run(torch, dev, bands, vecs, 1, ("exp", "phi1"), 8, 1e-12)
    tl = [[torch.from_numpy(t[k]).to(dev) for t in tris] for k in range(3)]
    tres, tinfo = pfm.tri_action(tl[0], tl[1], tl[2], [torch.from_numpy(v).to(dev) for v in vecs],
                                 ("exp", "phi1"), m=8, tol=1e-12)
    torch.cuda.synchronize()
    for i in range(3):
        assert info[i]["plan"] == tinfo[i]["plan"] and info[i]["norm1"] == tinfo[i]["norm1"]
        for f in ("exp", "phi1"):
            assert me.rel_fro(res[f][i].cpu().numpy(), tres[f][i].cpu().numpy()) <= BAR


def test_headline_shape_sampled(torch_dev):
    """The banded leg's shape (pentadiagonal, d = 1024, p = 64,
    ||A||_1 in [0.5, 8]); sampled columns of sampled instances against the
    oracle (columns are independent)."""
    torch, dev = torch_dev
    batch, d, p, b = 64, 1024, 64, 2
    bands = wl.band_gaussian_batch(batch, d, b, 0.5, 8.0, wl.SEED_BASE + 980)
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 981 + i) for i in range(batch)]
    _say("case band headline shape batch=%d d=%d p=%d b=%d" % (batch, d, p, b))
    res, info = _run(torch, dev, bands, vecs, b, ("exp",), 8, 1e-12)
    w = _check(res, info, bands, vecs, b, ("exp",), 8, 1e-12, cols=[0, 31, 63], idx=[0, 17, 63])
    _say("  worst %.2e" % w)


def _hybrid_bar(N):
    """As for the tridiagonal path: a few units of rounding (16) times
    1 + sum_k |w_k| + |d1| + |d2| per step, N steps, both sides."""
    _, terms = co.roundoff_terms("exp", 10)
    d1, d2 = co.poly_terms("exp", 10)
    amp = 1 + sum(abs(w) for _, w, _ in terms) + abs(d1) + abs(d2)
    return 2 * 16 * N * amp * 2.0 ** -53


@pytest.mark.parametrize("b", [2, 3])
def test_hybrid_r10_prime(torch_dev, b):
    """R10' (the hybrid set of §4.3, exp) on banded A: P = d1 B y + d2 B^2 y
    formed in the forward pass, against the banded oracle."""
    torch, dev = torch_dev
    shapes = [(1, 1), (4, 2), (9, 5), (64, 65), (200, 3)]
    bands = [wl.band_gaussian_batch(1, d, b, 0.5, 8.0, wl.SEED_BASE + 990 + j)[0] for j, (d, p) in enumerate(shapes)]
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 995 + j) for j, (d, p) in enumerate(shapes)]
    _say("case band hybrid m=10 b=%d" % b)
    res, info = _run(torch, dev, bands, vecs, b, ("exp",), 10, 1e-12)
    for i in range(len(shapes)):
        N = int(info[i]["plan"])
        own = _own(bands[i], b, vecs[i], ("exp",), 10, 1e-12, N)
        assert info[i]["route"] == 4 and info[i]["status"] == 0 and info[i]["order"] == 10
        err = me.rel_fro(res["exp"][i].cpu().numpy(), own["exp"])
        assert err <= _hybrid_bar(N), (i, N, err)


def test_errors(torch_dev):
    """Refused on the host before anything is enqueued: b outside [1, 4],
    φ1 with the hybrid set, a misaligned array."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    d, p = 16, 4
    bands = torch.from_numpy(wl.band_gaussian_batch(1, d, 2, 0.5, 8.0, wl.SEED_BASE + 999)[0]).to(dev)
    V = torch.from_numpy(wl.vectors(d, p, wl.SEED_BASE + 998)).to(dev)
    F = torch.empty_like(V)
    ctx = pfm.Context(0)
    info = torch.empty(pfm.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    _say("case band errors")
    for bb in (0, 5):
        pr = [pfm.BandProblem(d, p, p, p, bands.data_ptr(), V.data_ptr(), F.data_ptr(), None)]
        assert ctx.band_action(pr, pfm.EXP, 8, 1e-12, bb, info) == pfm.ERR_INVALID
    pr = [pfm.BandProblem(d, p, p, p, bands.data_ptr(), V.data_ptr(), None, F.data_ptr())]
    assert ctx.band_action(pr, pfm.PHI1, 10, 1e-12, 2, info) == pfm.ERR_UNSUPPORTED
    pr = [pfm.BandProblem(d, p, p, p, bands.data_ptr() + 4, V.data_ptr(), F.data_ptr(), None)]
    assert ctx.band_action(pr, pfm.EXP, 8, 1e-12, 2, info) == pfm.ERR_INVALID
    ctx.close()
    with pytest.raises(ValueError):
        pfm.band_action([bands], [V], 1)
