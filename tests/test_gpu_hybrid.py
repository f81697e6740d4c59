"""GPU parity of the hybrid 10th-order set of §4.3 (m = 10, the set with
c = -+1/8 .. -+1/16, b_9 = 2000, b_10 = -3500) on the full-matrix path,
against the oracle, through the C ABI.

Bar, derived from the arithmetic: both sides evaluate the same r(B) in
binary64 in different orders.  Per scaled step the round-off form's result
carries rounding of about sum_k |w_k| ||(I - c_k B)^{-1} B|| u
<= sum_k |w_k| θ / (1 - max|c_k| θ) u, times sqrt(n) for the length-n inner
products (rounding errors of independent signs add like a random walk: the
probabilistic bound of Higham and Mary, 2019), and the s squarings amplify a
relative error at most 2^s-fold; the two sides' errors add.  With sum |w_k| ~ 9.7e3 (the cancellation the paper warns of for this
set) this is far above the 1e-12 bar of the partial-fraction sets, which is
why it is stated here; a wrong term (a dropped d1 B or d2 B^2, a wrong sign)
misses it by many orders of magnitude."""

import math
import sys

import numpy as np
import pytest

from oracle import coefficients as co
from oracle import method as me
from paper_2210_03714_amd import workloads as wl

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2210_03714_amd import pfm
    pfm.lib()
    return torch, torch.device("cuda:0")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _bar(n, s, theta):
    _, terms = co.roundoff_terms("exp", 10)
    sw = sum(abs(w) for _, w, _ in terms)
    cmax = max(abs(c) for c, _, _ in terms)
    return 2 * 2 ** s * math.sqrt(n) * sw * theta / (1 - cmax * theta) * U


def _run(torch, dev, mats, tol=1e-12, force_plan=-1, route=None):
    from paper_2210_03714_amd import pfm
    At = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in mats]
    return pfm.expm(At, ("exp",), m=10, tol=tol, force_plan=force_plan)


def _check(mats, res, info, tol=1e-12):
    worst = 0.0
    for i, A in enumerate(mats):
        s = int(info[i]["plan"])
        own = me.expm_full(A, ("exp",), 10, tol)
        q = own["eta"] / own["theta"]
        if q > 0 and abs(math.log2(q) - round(math.log2(q))) < 1e-12:
            own = me.expm_full(A, ("exp",), 10, tol, force_plan=s)
        else:
            assert s == own["plan"], (i, s, own["plan"])
        assert info[i]["status"] == 0 and info[i]["order"] == 10
        err = me.rel_fro(res["exp"][i].cpu().numpy(), own["exp"])
        bar = _bar(A.shape[0], s, own["theta"])
        worst = max(worst, err / bar)
        assert err <= bar, (i, A.shape[0], s, err, bar)
    return worst


def test_uneven_batch_gauss_jordan_route(torch_dev):
    torch, dev = torch_dev
    mats = wl.gaussian_uneven(10, [40, 64, 130, 256, 300], 0.5, 8.0, wl.SEED_BASE + 700)
    _say("case hybrid m=10 uneven batch")
    res, info = _run(torch, dev, mats)
    for i in range(len(mats)):
        assert info[i]["route"] == 1
    w = _check(mats, res, info)
    _say("  worst err / bar %.2e" % w)


def test_large_instance_route(torch_dev):
    """n = 600 takes the multi-workgroup route, whose R = a0 I +
    (alpha1 + d1) B + B (T + d2 I) B carries the polynomial part."""
    torch, dev = torch_dev
    mats = [wl.gaussian(600, 6.0, wl.SEED_BASE + 701)]
    _say("case hybrid m=10 n=600")
    res, info = _run(torch, dev, mats)
    assert info[0]["route"] == 2
    w = _check(mats, res, info)
    _say("  worst err / bar %.2e" % w)


def test_headline_shape_sampled(torch_dev):
    torch, dev = torch_dev
    A, _ = wl.gaussian_batch(64, 256, 0.5, 8.0, wl.SEED_BASE + 702)
    _say("case hybrid m=10 64 x n=256")
    from paper_2210_03714_amd import pfm
    At = torch.from_numpy(A).to(dev)
    res, info = pfm.expm(At, ("exp",), m=10, tol=1e-12)
    torch.cuda.synchronize()
    pick = [0, 31, 63]
    w = _check([A[i] for i in pick], {"exp": [res["exp"][i] for i in pick]}, info[pick])
    _say("  worst err / bar %.2e" % w)


def test_action_against_oracle(torch_dev):
    """exp(A) V with the hybrid set on every action route: n = 17 and 100 on
    the single-workgroup LU-factor route (the step adds d1 Y + d2 B Y to the
    shifted solves), n = 200 and 600 on the multi-workgroup route (the
    explicit r(B) = a0 I + (alpha1 + d1) B + B (T + d2 I) B).  Bar as for the
    full matrix with the N steps' errors adding (N in place of 2^s)."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    sizes, ps, norms = [17, 100, 200, 600], [1, 5, 16, 33], [1.0, 2.5, 3.0, 2.0]
    mats = [wl.gaussian(n, t, wl.SEED_BASE + 740 + n) for n, t in zip(sizes, norms)]
    vecs = [wl.vectors(n, p, wl.SEED_BASE + 750 + n) for n, p in zip(sizes, ps)]
    At = [torch.from_numpy(a).to(dev) for a in mats]
    Vt = [torch.from_numpy(v).to(dev) for v in vecs]
    _say("case hybrid m=10 action")
    res, info = pfm.action(At, Vt, ("exp",), m=10)
    torch.cuda.synchronize()
    worst = 0.0
    for i, (A, V) in enumerate(zip(mats, vecs)):
        N = int(info[i]["plan"])
        own = me.action(A, V, ("exp",), 10, 1e-12, force_plan=N)
        assert info[i]["status"] == 0 and info[i]["order"] == 10
        assert info[i]["route"] == (0 if sizes[i] <= 128 else 2), (i, info[i]["route"])
        err = me.rel_fro(res["exp"][i].cpu().numpy(), own["exp"])
        bar = _bar(A.shape[0], 0, own["theta"]) * N
        worst = max(worst, err / bar)
        assert err <= bar, (i, sizes[i], N, err, bar)
    _say("  worst err / bar %.2e" % worst)


def test_unsupported_combinations(torch_dev):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    A = wl.gaussian(64, 8.0, wl.SEED_BASE + 703)
    At = torch.from_numpy(A).to(dev)
    V = torch.ones((64, 2), dtype=torch.float64, device=dev)
    _say("case hybrid m=10 unsupported")
    with pytest.raises(pfm.PfmError) as e:
        pfm.expm([At], ("phi1",), m=10)
    assert e.value.code == pfm.ERR_UNSUPPORTED
    with pytest.raises(pfm.PfmError) as e:
        pfm.action([At], [V], ("phi1",), m=10)
    assert e.value.code == pfm.ERR_UNSUPPORTED
    with pytest.raises(pfm.PfmError) as e:
        pfm.expm([At.to(torch.complex128)], ("exp",), m=10)
    assert e.value.code == pfm.ERR_UNSUPPORTED
    # a forced s = 0 leaves |c_k| ||B||_1 = 1 > 1/2: no Gauss-Jordan route;
    # the device finds that after the plan and does not compute the instance
    out = {"exp": [torch.full_like(At, 7.25)]}
    res, info = pfm.expm([At], ("exp",), m=10, force_plan=0, out=out)
    torch.cuda.synchronize()
    assert info[0]["status"] & pfm.NOT_COMPUTED
    assert torch.all(res["exp"][0] == 7.25)
    ctx = pfm.Context(0)
    ctx.set_route(pfm.ROUTE_LU)
    with pytest.raises(pfm.PfmError) as e:
        pfm.expm([At], ("exp",), m=10, ctx=ctx)
    assert e.value.code == pfm.ERR_UNSUPPORTED
    ctx.close()


def _bar_set(m, n, s, theta):
    """The bar of this module for set m (10 or 110)."""
    _, terms = co.roundoff_terms("exp", m)
    sw = sum(abs(w) for _, w, _ in terms)
    cmax = max(abs(c) for c, _, _ in terms)
    return 2 * 2 ** s * math.sqrt(n) * sw * theta / (1 - cmax * theta) * U


def test_r10star_full_and_tridiagonal(torch_dev):
    """R*10 (m = PFM_R10STAR, §4.3 eqs. Frac10ciNO-Frac10biNO) at tol 1e-8:
    full matrices on the Gauss-Jordan route, the dense action on both of its
    routes and the tridiagonal action (R*10' of §5), against the oracle at the same plan, within the bars of
    this module and of the tridiagonal tests (its weights, sum |w| ~ 1.3e6,
    set the rounding).  Below its rounding floor (tol 1e-12) it is refused."""
    torch, dev = torch_dev
    from oracle import banded as bd
    from paper_2210_03714_amd import pfm
    m, tol = pfm.R10STAR, 1e-8
    mats = wl.gaussian_uneven(6, [40, 64, 130, 256], 0.5, 8.0, wl.SEED_BASE + 710)
    _say("case R*10 full matrices")
    res, info = pfm.expm([torch.from_numpy(a).to(dev) for a in mats], ("exp",), m=m, tol=tol)
    torch.cuda.synchronize()
    worst = 0.0
    for i, A in enumerate(mats):
        s = int(info[i]["plan"])
        own = me.expm_full(A, ("exp",), 110, tol, force_plan=s)
        assert info[i]["status"] == 0 and info[i]["order"] == 10 and info[i]["route"] == 1
        err = me.rel_fro(res["exp"][i].cpu().numpy(), own["exp"])
        bar = _bar_set(110, A.shape[0], s, own["theta"])
        worst = max(worst, err / bar)
        assert err <= bar, (i, A.shape[0], s, err, bar)
    _say("  worst err / bar %.2e" % worst)
    tris = [wl.tri_gaussian_batch(1, d, 0.5, 8.0, wl.SEED_BASE + 720 + d)[0] for d in (17, 300)]
    vecs = [wl.vectors(d, p, wl.SEED_BASE + 730 + d) for d, p in ((17, 3), (300, 70))]
    _say("case R*10' tridiagonal")
    dl = [torch.from_numpy(np.ascontiguousarray(t[0])).to(dev) for t in tris]
    dd = [torch.from_numpy(np.ascontiguousarray(t[1])).to(dev) for t in tris]
    du = [torch.from_numpy(np.ascontiguousarray(t[2])).to(dev) for t in tris]
    Vt = [torch.from_numpy(v).to(dev) for v in vecs]
    rt, it = pfm.tri_action(dl, dd, du, Vt, ("exp",), m=m, tol=tol)
    torch.cuda.synchronize()
    _, terms = co.roundoff_terms("exp", 110)
    d1, d2 = co.poly_terms("exp", 110)
    amp = 1 + sum(abs(w) for _, w, _ in terms) + abs(d1) + abs(d2)
    for i, ((a, b, c), V) in enumerate(zip(tris, vecs)):
        N = int(it[i]["plan"])
        own = bd.tri_action(a, b, c, V, ("exp",), 110, tol, force_plan=N)
        err = me.rel_fro(rt["exp"][i].cpu().numpy(), own["exp"])
        assert err <= 2 * 16 * N * amp * U, (i, N, err)
    # the dense action on both routes (n = 60 single-workgroup, n = 200 multi-workgroup)
    amats = [wl.gaussian(n, 2.0, wl.SEED_BASE + 740 + n) for n in (60, 200)]
    avecs = [wl.vectors(n, p, wl.SEED_BASE + 750 + n) for n, p in ((60, 4), (200, 9))]
    _say("case R*10 dense action")
    ra, ia = pfm.action([torch.from_numpy(a).to(dev) for a in amats], [torch.from_numpy(v).to(dev) for v in avecs],
                        ("exp",), m=m, tol=tol)
    torch.cuda.synchronize()
    for i, (A, V) in enumerate(zip(amats, avecs)):
        N = int(ia[i]["plan"])
        own = me.action(A, V, ("exp",), 110, tol, force_plan=N)
        assert ia[i]["status"] == 0 and ia[i]["route"] == (0 if A.shape[0] <= 128 else 2)
        err = me.rel_fro(ra["exp"][i].cpu().numpy(), own["exp"])
        bar = _bar_set(110, A.shape[0], 0, own["theta"]) * N
        assert err <= bar, (i, A.shape[0], N, err, bar)
    A0 = torch.from_numpy(mats[0]).to(dev)
    for t in (1e-12, 1e-10):
        with pytest.raises(pfm.PfmError) as e:
            pfm.expm([A0], ("exp",), m=m, tol=t)
        assert e.value.code == pfm.ERR_UNSUPPORTED
        with pytest.raises(pfm.PfmError) as e:
            pfm.tri_action(dl[:1], dd[:1], du[:1], Vt[:1], ("exp",), m=m, tol=t)
        assert e.value.code == pfm.ERR_UNSUPPORTED
