"""GPU parity of the banded action (pfm_band_action; §2.1 and §5 name the
pentadiagonal case beside the tridiagonal one) against the banded oracle
(oracle/banded.py, LAPACK gbtrf / gbtrs), element by element on the same
seeded inputs: relative Frobenius error <= 1e-12 per instance and function,
the same N, the same ||A||_1 bit for bit, and route 4.  Half-bandwidths
b = 1..4, uneven batches with ragged 64-column waves, d below and above b,
and the entries of ``bands`` outside A set to NaN on the device (they must
never be read).  At b = 2 with up to 8 shifts and d <= 1024 the steps run
in the wave-per-shift scan kernel (ragged 16-column workgroups, d = 1024 at
its limit); the uneven batch also holds d = 1100, which the lane-per-column
kernel takes in the same call."""

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


SHAPES = [(1, 1), (2, 3), (5, 64), (37, 65), (1100, 2), (130, 7), (1024, 17)]


@pytest.mark.parametrize("b", [1, 2, 3, 4])
@pytest.mark.parametrize("funcs,m", [(("exp", "phi1"), 8), (("exp",), 8), (("exp",), 4), (("phi1",), 5)])
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


@pytest.mark.parametrize("funcs", [("exp", "phi1"), ("exp",)])
def test_full_scan_path(torch_dev, funcs):
    """A forced N = 1 on a pentadiagonal A with off-diagonals ~1.6 and ~0.4
    (|c_k| ||B||_1 up to 0.88: still diagonally dominant) makes the 16-row
    lane maps of the scan kernel reach 3e-4, so it composes them lane by lane
    instead of over two lanes; against the oracle on the same forced plan,
    in the kernel with phi1 and in the exp-only one."""
    torch, dev = torch_dev
    rng = np.random.default_rng(wl.SEED_BASE + 985)
    bands, vecs = [], []
    for j, d in enumerate((300, 1024, 77)):
        x = np.zeros((5, d))
        x[1] = 1.6 * (1 + 0.05 * rng.standard_normal(d))
        x[3] = 1.6 * (1 + 0.05 * rng.standard_normal(d))
        x[0] = 0.4 * (1 + 0.05 * rng.standard_normal(d))
        x[4] = 0.4 * (1 + 0.05 * rng.standard_normal(d))
        x[2] = 0.05 * rng.standard_normal(d)
        bands.append(x)
        vecs.append(wl.vectors(d, 5 + 13 * j, wl.SEED_BASE + 986 + j))
    _say("case band full scan path funcs=%s" % (funcs,))
    res, info = _run(torch, dev, bands, vecs, 2, funcs, 8, 1e-12, force_plan=1)
    for i in range(len(bands)):
        assert info[i]["plan"] == 1 and info[i]["status"] == 0
        own = bd.band_action(bands[i], 2, vecs[i], funcs, 8, 1e-12, force_plan=1)
        for f in funcs:
            err = me.rel_fro(res[f][i].cpu().numpy(), own[f])
            assert err <= BAR, (i, f, err)


def _hybrid_bar(N):
    """As for the tridiagonal path: a few units of rounding (16) times
    1 + sum_k |w_k| + |d1| + |d2| per step, N steps, both sides."""
    _, terms = co.roundoff_terms("exp", 10)
    d1, d2 = co.poly_terms("exp", 10)
    amp = 1 + sum(abs(w) for _, w, _ in terms) + abs(d1) + abs(d2)
    return 2 * 16 * N * amp * 2.0 ** -53


@pytest.mark.parametrize("b", [1, 2, 3, 4])
def test_hybrid_r10_prime(torch_dev, b):
    """R10' (the hybrid set of §4.3, exp) on banded A: P = d1 B y + d2 B^2 y
    formed in the forward pass, against the banded oracle."""
    torch, dev = torch_dev
    shapes = [(1, 1), (4, 2), (9, 5), (64, 65), (200, 3)]
    bands = [wl.band_gaussian_batch(1, d, b, 0.5, 8.0, wl.SEED_BASE + 990 + j)[0] for j, (d, p) in enumerate(shapes)]
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 995 + j) for j, (d, p) in enumerate(shapes)]
    _say("case band hybrid m=10 b=%d" % b)
    res, info = _run(torch, dev, bands, vecs, b, ("exp",), 10, 1e-12)
    worst, worst_rel = 0.0, 0.0
    for i in range(len(shapes)):
        N = int(info[i]["plan"])
        own = _own(bands[i], b, vecs[i], ("exp",), 10, 1e-12, N)
        assert info[i]["route"] == 4 and info[i]["status"] == 0 and info[i]["order"] == 10
        err = me.rel_fro(res["exp"][i].cpu().numpy(), own["exp"])
        worst, worst_rel = max(worst, err), max(worst_rel, err / _hybrid_bar(N))
        assert err <= _hybrid_bar(N), (i, N, err)
    _say("  worst rel. error %.3e (%.2e of the bar)" % (worst, worst_rel))


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


def test_force_plan(torch_dev):
    """A forced N (more steps than planned) against the oracle at that N."""
    torch, dev = torch_dev
    b = 2
    bands = wl.band_gaussian_batch(2, 40, b, 1.0, 2.0, wl.SEED_BASE + 1010)
    vecs = [wl.vectors(40, 4, wl.SEED_BASE + 1011), wl.vectors(40, 70, wl.SEED_BASE + 1012)]
    _say("case band force_plan")
    res, info = _run(torch, dev, bands, vecs, b, ("exp", "phi1"), 8, 1e-12, force_plan=37)
    for i in range(2):
        assert info[i]["plan"] == 37
        own = bd.band_action(bands[i], b, vecs[i], ("exp", "phi1"), 8, 1e-12, force_plan=37)
        for f in ("exp", "phi1"):
            assert me.rel_fro(res[f][i].cpu().numpy(), own[f]) <= BAR


def test_strided_vectors(torch_dev):
    """V and the results as column slices of wider matrices (row strides 80
    and 72 for p = 64 columns), d = 130 (a ragged last block): the library
    reads and writes only the slices."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    d, p, b = 130, 64, 3
    bands = wl.band_gaussian_batch(2, d, b, 0.5, 8.0, wl.SEED_BASE + 1020)
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 1021 + i) for i in range(2)]
    wideV = [torch.zeros((d, 80), dtype=torch.float64, device=dev) for _ in vecs]
    for w, v in zip(wideV, vecs):
        w[:, 5:5 + p] = torch.from_numpy(v).to(dev)
    sentinel = 12345.0
    wide = {f: [torch.full((d, 72), sentinel, dtype=torch.float64, device=dev) for _ in vecs]
            for f in ("exp", "phi1")}
    out = {f: [w[:, 3:3 + p] for w in wide[f]] for f in ("exp", "phi1")}
    Bt = [torch.from_numpy(np.ascontiguousarray(_outside_nan(x, b))).to(dev) for x in bands]
    _say("case band strided V and outputs d=%d p=%d b=%d" % (d, p, b))
    res, info = pfm.band_action(Bt, [w[:, 5:5 + p] for w in wideV], b, ("exp", "phi1"), m=8, tol=1e-12, out=out)
    torch.cuda.synchronize()
    for f in ("exp", "phi1"):
        for w in wide[f]:
            h = w.cpu().numpy()
            assert (h[:, :3] == sentinel).all() and (h[:, 3 + p:] == sentinel).all()
    _check(res, info, bands, vecs, b, ("exp", "phi1"), 8, 1e-12)


def test_nonfinite_and_singular(torch_dev):
    """A NaN inside A sets PFM_NONFINITE (and ||A||_1 NaN); an exactly zero
    pivot sets PFM_SINGULAR_SHIFT with that shift's index: A[0][0] = 8 with N
    forced to 1 and the shift 1/8 of the m = 10 set, where 1 - c A[0][0] is 0
    exactly whether or not the product and difference are fused (c is a
    power of two).  Both calls complete; the status says the results are not
    valid."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    b, d = 2, 20
    x = wl.band_gaussian_batch(1, d, b, 1.0, 2.0, wl.SEED_BASE + 1030)[0].copy()
    x[b, 7] = np.nan
    V = wl.vectors(d, 2, wl.SEED_BASE + 1031)
    _say("case band nonfinite")
    res, info = _run(torch, dev, [x], [V], b, ("exp",), 8, 1e-12)
    assert info[0]["status"] & pfm.NONFINITE
    assert np.isnan(info[0]["norm1"])
    y = np.zeros((2 * b + 1, 6))
    y[b] = [8.0, 0.5, 0.5, 0.5, 0.5, 0.5]
    c = list(pfm.coeffs(pfm.EXP, 10)[0])
    k = [i for i, ci in enumerate(c) if complex(ci) == 0.125]
    assert len(k) == 1
    _say("case band singular shift")
    res, info = _run(torch, dev, [y], [wl.vectors(6, 1, wl.SEED_BASE + 1032)], b, ("exp",), 10, 1e-12, force_plan=1)
    assert info[0]["status"] & pfm.SINGULAR_SHIFT
    assert info[0]["bad_shift"] == k[0]


def test_step_cap_not_computed(torch_dev):
    """A forced N above PFM_MAX_STEPS: PFM_NOT_COMPUTED from the plan kernel,
    outputs untouched."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    bands = wl.band_gaussian_batch(1, 30, 2, 1.0, 2.0, wl.SEED_BASE + 690)[0]
    V = torch.from_numpy(wl.vectors(30, 2, wl.SEED_BASE + 691)).to(dev)
    out = {"exp": [torch.full_like(V, 7.25)]}
    _say("case band step cap")
    res, info = pfm.band_action([torch.from_numpy(bands).to(dev)], [V], 2, ("exp",), m=8, tol=1e-12,
                                force_plan=pfm.MAX_STEPS + 1, out=out)
    torch.cuda.synchronize()
    assert info[0]["status"] & pfm.NOT_COMPUTED and info[0]["plan"] == pfm.MAX_STEPS + 1
    assert torch.all(res["exp"][0] == 7.25)
