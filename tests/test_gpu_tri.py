"""GPU parity of the tridiagonal action path (pfm_tri_action) against the
tridiagonal oracle (oracle/banded.py), through the C ABI.

Bar: relative Frobenius error per instance and function <= 1e-12, with the
oracle's own plan equal to the GPU's (N = ceil(eta / θ); the GPU's N is
handed to the oracle only when eta / θ sits within 1e-12 of an integer), the
same ||A||_1 bit for bit, and route 3.  Sizes up to d = 1024 run in the
wave-per-column scan kernel (one and many 16-row lane blocks, ragged tails,
ragged last workgroups of 8 columns); larger d in the lane-per-column kernel
(8-row checkpoint chunks, 64-column waves); the uneven batch mixes both in
one call."""

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


def _to(torch, dev, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _run(torch, dev, tris, vecs, funcs, m, tol, force_plan=-1):
    from paper_2210_03714_amd import pfm
    dl = [_to(torch, dev, t[0]) for t in tris]
    dd = [_to(torch, dev, t[1]) for t in tris]
    du = [_to(torch, dev, t[2]) for t in tris]
    V = [_to(torch, dev, v) for v in vecs]
    res, info = pfm.tri_action(dl, dd, du, V, funcs, m=m, tol=tol, force_plan=force_plan)
    torch.cuda.synchronize()
    return res, info


def _check(res, info, tris, vecs, funcs, m, tol, cols=None):
    worst = 0.0
    for i, ((dl, dd, du), V) in enumerate(zip(tris, vecs)):
        Vc = V if cols is None else V[:, cols]
        own = bd.tri_action(dl, dd, du, Vc, funcs, m, tol)
        q = own["eta"] / own["theta"]
        N = int(info[i]["plan"])
        if abs(q - round(q)) < 1e-12 * q:
            own = bd.tri_action(dl, dd, du, Vc, funcs, m, tol, force_plan=N)
        else:
            assert N == own["plan"], (i, N, own["plan"])
        assert info[i]["norm1"] == own["eta"], (i, info[i]["norm1"], own["eta"])
        assert info[i]["route"] == 3 and info[i]["status"] == 0 and info[i]["bad_shift"] == -1
        for f in funcs:
            got = res[f][i].cpu().numpy()
            if cols is not None:
                got = got[:, cols]
            err = me.rel_fro(got, own[f])
            worst = max(worst, err)
            assert err <= BAR, (i, f, V.shape, N, err)
    return worst


@pytest.mark.parametrize("m", [4, 5, 8])
@pytest.mark.parametrize("funcs", [("exp",), ("phi1",), ("exp", "phi1")])
def test_uneven_batch(torch_dev, m, funcs):
    """Several instances of different d and p in one call."""
    torch, dev = torch_dev
    shapes = [(1, 1), (2, 3), (15, 2), (16, 1), (17, 5), (33, 64), (1025, 2), (100, 65), (257, 7), (1500, 3)]
    tris = []
    vecs = []
    for j, (d, p) in enumerate(shapes):
        tris += wl.tri_gaussian_batch(1, d, 0.5, 8.0, wl.SEED_BASE + 500 + 10 * m + j)
        vecs.append(wl.vectors(d, p, wl.SEED_BASE + 550 + 10 * m + j))
    _say("case tri uneven m=%d funcs=%s" % (m, "+".join(funcs)))
    res, info = _run(torch, dev, tris, vecs, funcs, m, 1e-12)
    w = _check(res, info, tris, vecs, funcs, m, 1e-12)
    _say("  worst %.2e" % w)


@pytest.mark.parametrize("tol", [1e-8, 1e-12])
def test_laplacian_and_many_columns(torch_dev, tol):
    """-tau trid{-1, 2, -1} (the test matrix of §5) at d = 1000 with 130
    columns (three waves, the last ragged), exp and phi1."""
    torch, dev = torch_dev
    tris = [wl.tri_neg_laplacian(1000, 1.0), wl.tri_neg_laplacian(1000, 0.25)]
    vecs = [wl.vectors(1000, 130, wl.SEED_BASE + 600), wl.vectors(1000, 3, wl.SEED_BASE + 601)]
    _say("case tri laplacian d=1000 tol=%g" % tol)
    res, info = _run(torch, dev, tris, vecs, ("exp", "phi1"), 8, tol)
    w = _check(res, info, tris, vecs, ("exp", "phi1"), 8, tol)
    _say("  worst %.2e N=%d" % (w, int(info[0]["plan"])))


def test_force_plan(torch_dev):
    torch, dev = torch_dev
    tris = wl.tri_gaussian_batch(2, 40, 1.0, 2.0, wl.SEED_BASE + 610)
    vecs = [wl.vectors(40, 4, wl.SEED_BASE + 611), wl.vectors(40, 4, wl.SEED_BASE + 612)]
    _say("case tri force_plan")
    res, info = _run(torch, dev, tris, vecs, ("exp", "phi1"), 8, 1e-12, force_plan=37)
    for i, ((dl, dd, du), V) in enumerate(zip(tris, vecs)):
        assert info[i]["plan"] == 37
        own = bd.tri_action(dl, dd, du, V, ("exp", "phi1"), 8, 1e-12, force_plan=37)
        for f in ("exp", "phi1"):
            assert me.rel_fro(res[f][i].cpu().numpy(), own[f]) <= BAR


def _lane_products(dl, dd, du, N, cs, rows=16):
    """Largest |prod (-l_r)| and |prod (-em_r)| over 16-row lane blocks of
    the LU of every I - c B, B = A / N (the multipliers of the scan kernel's
    lane maps)."""
    d = len(dd)
    sub = np.concatenate([[0.0], dl / N]); dia = dd / N; sup = np.concatenate([du / N, [0.0]])
    big = 0.0
    for c in cs:
        u = np.empty(d); l = np.zeros(d); em = np.zeros(d)
        u[0] = 1.0 - c * dia[0]
        for r in range(1, d):
            l[r] = -c * sub[r] / u[r - 1]
            u[r] = 1.0 - c * dia[r] - l[r] * (-c * sup[r - 1])
        em[:] = -c * sup / u
        for b0 in range(0, d, rows):
            big = max(big, abs(np.prod(-l[b0:b0 + rows])), abs(np.prod(-em[b0:b0 + rows])))
    return big


def test_full_scan_path(torch_dev):
    """A forced N = 1 on trid{a, eps, a} with a ~ 2 (|c_k| ||B||_1 up to
    0.85: still diagonally dominant, |l_r| ~ 0.5 on every row) makes the
    16-row lane products exceed 2^-30, so the scan kernel composes the lane
    maps over the whole wave instead of two lanes; both functions against
    the oracle on the same forced plan."""
    torch, dev = torch_dev
    rng = np.random.default_rng(wl.SEED_BASE + 615)
    tris = []
    for d in (300, 1024, 77):
        dl = 2.0 * (1.0 + 0.05 * rng.standard_normal(d - 1))
        du = 2.0 * (1.0 + 0.05 * rng.standard_normal(d - 1))
        tris.append((dl, 0.05 * rng.standard_normal(d), du))
    vecs = [wl.vectors(len(t[1]), 5, wl.SEED_BASE + 616 + i) for i, t in enumerate(tris)]
    a0, terms = me.build_terms(("exp",), 8, False)
    cs = [complex(c).real for c, _, _ in terms]
    assert max(_lane_products(*t, 1, cs) for t in tris) > 2.0 ** -30
    _say("case tri full scan path")
    res, info = _run(torch, dev, tris, vecs, ("exp", "phi1"), 8, 1e-12, force_plan=1)
    for i, ((dl, dd, du), V) in enumerate(zip(tris, vecs)):
        assert info[i]["plan"] == 1 and info[i]["status"] == 0
        own = bd.tri_action(dl, dd, du, V, ("exp", "phi1"), 8, 1e-12, force_plan=1)
        for f in ("exp", "phi1"):
            err = me.rel_fro(res[f][i].cpu().numpy(), own[f])
            assert err <= BAR, (i, f, err)
    # the hybrid set (m = 10, |c_k| <= 1/8): a ~ 2.2 gives |l_r| ~ 0.3
    a0, terms = me.build_terms(("exp",), 10, False)
    cs = [complex(c).real for c, _, _ in terms]
    tris = [(1.1 * x[0], 1.1 * x[1], 1.1 * x[2]) for x in tris]
    assert max(_lane_products(*t, 1, cs) for t in tris) > 2.0 ** -30
    res, info = _run(torch, dev, tris, vecs, ("exp",), 10, 1e-12, force_plan=1)
    for i, ((dl, dd, du), V) in enumerate(zip(tris, vecs)):
        assert info[i]["plan"] == 1 and info[i]["status"] == 0
        own = bd.tri_action(dl, dd, du, V, ("exp",), 10, 1e-12, force_plan=1)
        err = me.rel_fro(res["exp"][i].cpu().numpy(), own["exp"])
        assert err <= _hybrid_bar(1), (i, err)


def test_headline_shape_sampled(torch_dev):
    """The benchmark's workload shape (d = 1024, p = 64, ||A||_1 in [0.5, 8]);
    sampled columns of sampled instances against the oracle (columns are
    independent, so the oracle runs on those columns alone)."""
    torch, dev = torch_dev
    batch, d, p = 64, 1024, 64
    tris = wl.tri_gaussian_batch(batch, d, 0.5, 8.0, wl.SEED_BASE + 620)
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 621 + i) for i in range(batch)]
    _say("case tri headline shape batch=%d d=%d p=%d" % (batch, d, p))
    res, info = _run(torch, dev, tris, vecs, ("exp",), 8, 1e-12)
    pick = [0, 17, 63]
    cols = [0, 31, 63]
    w = _check({"exp": [res["exp"][i] for i in pick]}, info[pick], [tris[i] for i in pick],
               [vecs[i] for i in pick], ("exp",), 8, 1e-12, cols=cols)
    _say("  worst %.2e" % w)


def test_strided_vectors(torch_dev):
    """V and the results as column slices of wider matrices (row strides 80
    and 72 for p = 64 columns), d = 130 (three blocks, a ragged last chunk):
    the library reads and writes only the slices."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    d, p = 130, 64
    tris = wl.tri_gaussian_batch(2, d, 0.5, 8.0, wl.SEED_BASE + 640)
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 641 + i) for i in range(2)]
    wideV = [torch.zeros((d, 80), dtype=torch.float64, device=dev) for _ in vecs]
    for w, v in zip(wideV, vecs):
        w[:, 5:5 + p] = torch.from_numpy(v).to(dev)
    sentinel = 12345.0
    wide = {f: [torch.full((d, 72), sentinel, dtype=torch.float64, device=dev) for _ in vecs]
            for f in ("exp", "phi1")}
    out = {f: [w[:, 3:3 + p] for w in wide[f]] for f in ("exp", "phi1")}
    dl = [torch.from_numpy(t[0]).to(dev) for t in tris]
    dd = [torch.from_numpy(t[1]).to(dev) for t in tris]
    du = [torch.from_numpy(t[2]).to(dev) for t in tris]
    _say("case tri strided V and outputs d=%d p=%d" % (d, p))
    res, info = pfm.tri_action(dl, dd, du, [w[:, 5:5 + p] for w in wideV], ("exp", "phi1"), m=8,
                               tol=1e-12, out=out)
    torch.cuda.synchronize()
    for f in ("exp", "phi1"):
        for w in wide[f]:
            wc = w.cpu().numpy()
            assert np.all(wc[:, :3] == sentinel) and np.all(wc[:, 3 + p:] == sentinel)
    w = _check(res, info, tris, vecs, ("exp", "phi1"), 8, 1e-12)
    _say("  worst %.2e" % w)
    bad = {"exp": out["exp"], "phi1": [torch.empty((d, p), dtype=torch.float64, device=dev) for _ in vecs]}
    with pytest.raises(ValueError):
        pfm.tri_action(dl, dd, du, [w[:, 5:5 + p] for w in wideV], ("exp", "phi1"), m=8, out=bad)


def test_nonfinite_and_errors(torch_dev):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    dl, dd, du = wl.tri_gaussian_batch(1, 20, 1.0, 2.0, wl.SEED_BASE + 630)[0]
    dd = dd.copy()
    dd[7] = np.nan
    V = wl.vectors(20, 2, wl.SEED_BASE + 631)
    _say("case tri nonfinite")
    res, info = _run(torch, dev, [(dl, dd, du)], [V], ("exp",), 8, 1e-12)
    assert info[0]["status"] & pfm.NONFINITE
    assert np.isnan(info[0]["norm1"])
    with pytest.raises(pfm.PfmError) as e:
        _run(torch, dev, [(dl, np.abs(dd), du)], [V], ("exp",), 1, 1e-12)
    assert e.value.code == pfm.ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        _run(torch, dev, [(dl[:-1], dd, du)], [V], ("exp",), 8, 1e-12)


def test_misaligned_pointers_rejected(torch_dev):
    """An array whose address is not a multiple of 8 is refused on the host
    (PFM_ERR_INVALID) before anything is enqueued; the pointers are never
    dereferenced."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    d, p = 16, 4
    dl, dd, du = [torch.from_numpy(x).to(dev) for x in wl.tri_gaussian_batch(1, d, 1.0, 2.0, wl.SEED_BASE + 650)[0]]
    V = torch.from_numpy(wl.vectors(d, p, wl.SEED_BASE + 651)).to(dev)
    F = torch.empty_like(V)
    ctx = pfm.Context(0)
    info = torch.empty(pfm.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    L = pfm.lib()
    _say("case tri misaligned pointers")
    for field in ("dl", "dd", "du", "V", "F"):
        ptr = {"dl": dl.data_ptr(), "dd": dd.data_ptr(), "du": du.data_ptr(), "V": V.data_ptr(), "F": F.data_ptr()}
        ptr[field] += 4
        probs = (pfm.TriProblem * 1)()
        probs[0] = pfm.TriProblem(d, p, p, p, ptr["dl"], ptr["dd"], ptr["du"], ptr["V"], ptr["F"], None)
        rc = L.pfm_tri_action(ctx.handle, pfm.EXP, 8, 1e-12, 1, probs, ctypes.c_void_p(info.data_ptr()), -1, None)
        assert rc == pfm.ERR_INVALID, field
    A = torch.from_numpy(wl.gaussian(8, 2.0, wl.SEED_BASE + 652)).to(dev)
    FA = torch.empty_like(A)
    for field in ("A", "F"):
        pa, pf = A.data_ptr() + (4 if field == "A" else 0), FA.data_ptr() + (4 if field == "F" else 0)
        probs = (pfm.Problem * 1)()
        probs[0] = pfm.Problem(8, 0, 8, 0, 8, pa, None, pf, None)
        rc = L.pfm_eval_batched(ctx.handle, pfm.EXP, 8, 1e-12, pfm.FP64, pfm.R64, 1, probs,
                                ctypes.c_void_p(info.data_ptr()), -1, None)
        assert rc == pfm.ERR_INVALID, field
    ctx.close()


def _hybrid_bar(N):
    """Derived from the arithmetic: per step each side's rounding is a few
    units (16 here) times 1 + sum_k |w_k| + |d1| + |d2| (about 1e4 for this
    set: the cancellation the paper notes), over N steps, on both sides."""
    _, terms = co.roundoff_terms("exp", 10)
    d1, d2 = co.poly_terms("exp", 10)
    amp = 1 + sum(abs(w) for _, w, _ in terms) + abs(d1) + abs(d2)
    return 2 * 16 * N * amp * 2.0 ** -53


def test_hybrid_r10_prime(torch_dev):
    """R10' of §5: the hybrid set of §4.3 (m = 10, exp) in the round-off form
    on tridiagonal A, P = d1 B y + d2 B^2 y formed in the forward pass.
    Uneven shapes (d a multiple of 8 or not, ragged column groups) and the
    paper's trid{-1, 2, -1} at d = 1000, against the tridiagonal oracle."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    shapes = [(1, 1), (3, 2), (16, 5), (17, 64), (100, 65)]
    tris = [wl.tri_gaussian_batch(1, d, 0.5, 8.0, wl.SEED_BASE + 700 + j)[0] for j, (d, p) in enumerate(shapes)]
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 720 + j) for j, (d, p) in enumerate(shapes)]
    tris.append(wl.tri_neg_laplacian(1000, 1.0))
    vecs.append(wl.vectors(1000, 3, wl.SEED_BASE + 730))
    _say("case tri hybrid m=10")
    res, info = _run(torch, dev, tris, vecs, ("exp",), 10, 1e-12)
    worst, worst_abs = 0.0, 0.0
    for i, ((dl, dd, du), V) in enumerate(zip(tris, vecs)):
        N = int(info[i]["plan"])
        own = bd.tri_action(dl, dd, du, V, ("exp",), 10, 1e-12)
        q = own["eta"] / own["theta"]
        if abs(q - round(q)) < 1e-12 * q:
            own = bd.tri_action(dl, dd, du, V, ("exp",), 10, 1e-12, force_plan=N)
        else:
            assert N == own["plan"], (i, N, own["plan"])
        assert info[i]["route"] == 3 and info[i]["status"] == 0 and info[i]["order"] == 10
        err = me.rel_fro(res["exp"][i].cpu().numpy(), own["exp"])
        bar = _hybrid_bar(N)
        worst = max(worst, err / bar)
        worst_abs = max(worst_abs, err)
        assert err <= bar, (i, V.shape, N, err, bar)
    _say("  worst err / bar %.2e, worst rel. error %.3e" % (worst, worst_abs))
    dl, dd, du = [_to(torch, dev, x) for x in tris[0]]
    V = _to(torch, dev, vecs[0])
    with pytest.raises(pfm.PfmError) as e:
        pfm.tri_action([dl], [dd], [du], [V], ("phi1",), m=10)
    assert e.value.code == pfm.ERR_UNSUPPORTED


def test_step_cap_not_computed(torch_dev):
    """A forced N above PFM_MAX_STEPS: the plan kernel flags the instance
    PFM_NOT_COMPUTED on the device (nothing is read back) and no kernel
    writes its outputs; the other instance of the call is computed."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    tris = wl.tri_gaussian_batch(2, 24, 1.0, 2.0, wl.SEED_BASE + 660)
    vecs = [wl.vectors(24, 3, wl.SEED_BASE + 661 + i) for i in range(2)]
    dl = [_to(torch, dev, t[0]) for t in tris]
    dd = [_to(torch, dev, t[1]) for t in tris]
    du = [_to(torch, dev, t[2]) for t in tris]
    V = [_to(torch, dev, v) for v in vecs]
    out = {"exp": [torch.full_like(v, 7.25) for v in V]}
    _say("case tri step cap")
    res, info = pfm.tri_action(dl, dd, du, V, ("exp",), m=8, tol=1e-12, force_plan=pfm.MAX_STEPS + 1, out=out)
    torch.cuda.synchronize()
    for i in range(2):
        assert info[i]["status"] & pfm.NOT_COMPUTED and info[i]["plan"] == pfm.MAX_STEPS + 1
        assert torch.all(res["exp"][i] == 7.25)
