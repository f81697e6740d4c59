"""GPU parity of log(1 - A) (the §2 example's set, m = 5, s = 0) against the
oracle, through the C ABI.  Bar: relative Frobenius error <= 1e-12 (the
weights' sum |w_k| is about 94, so the round-off form's rounding stays near
1e-14 relative to ||log(1 - A)|| ~ ||A||)."""

import sys

import numpy as np
import pytest

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


def _run_check(torch, dev, mats, tol, ctx=None, route=1, status=0):
    from paper_2210_03714_amd import pfm
    At = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in mats]
    res, info = pfm.expm(At, ("log1m",), m=5, tol=tol, ctx=ctx)
    torch.cuda.synchronize()
    worst = 0.0
    for i, A in enumerate(mats):
        own = me.expm_full(A, ("log1m",), 5, tol)
        assert info[i]["plan"] == 0 and info[i]["route"] == route
        assert info[i]["status"] == status, (i, info[i]["status"])
        assert abs(info[i]["theta"] - own["theta"]) <= 1e-15 * own["theta"]
        err = me.rel_fro(res["log1m"][i].cpu().numpy(), own["log1m"])
        worst = max(worst, err)
        assert err <= BAR, (i, A.shape[0], err)
    return worst


@pytest.mark.parametrize("tol", [1e-8, 1e-12])
def test_in_range_gauss_jordan_route(torch_dev, tol):
    torch, dev = torch_dev
    th_ = me.theta_for(("log1m",), 5, tol)
    mats = wl.gaussian_uneven(8, [32, 64, 130, 256], th_ / 4, th_, wl.SEED_BASE + 800)
    _say("case log1m tol=%g" % tol)
    w = _run_check(torch, dev, mats, tol)
    _say("  worst %.2e" % w)


def test_lu_route_and_out_of_range(torch_dev):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    th_ = me.theta_for(("log1m",), 5, 1e-12)
    mats = wl.gaussian_uneven(4, [48, 100], th_ / 2, th_, wl.SEED_BASE + 801)
    ctx = pfm.Context(0)
    ctx.set_route(pfm.ROUTE_LU)
    _say("case log1m LU route")
    _run_check(torch, dev, mats, 1e-12, ctx=ctx, route=0)
    ctx.close()
    # ||A||_1 = 0.2 > θ: computed at s = 0 all the same, and flagged
    big = [wl.gaussian(64, 0.2, wl.SEED_BASE + 802)]
    _say("case log1m out of range")
    _run_check(torch, dev, big, 1e-12, status=pfm.OUT_OF_RANGE)


def test_rejected(torch_dev):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    A = torch.from_numpy(wl.gaussian(32, 0.005, 3)).to(dev)
    V = torch.ones((32, 2), dtype=torch.float64, device=dev)
    _say("case log1m rejected")
    with pytest.raises(pfm.PfmError) as e:
        pfm.expm([A], ("log1m",), m=8)
    assert e.value.code == pfm.ERR_UNSUPPORTED
    with pytest.raises(pfm.PfmError) as e:
        pfm.action([A], [V], ("log1m",), m=5)
    assert e.value.code == pfm.ERR_UNSUPPORTED
    with pytest.raises(pfm.PfmError) as e:
        pfm.expm([A.to(torch.complex128)], ("log1m",), m=5)
    assert e.value.code == pfm.ERR_UNSUPPORTED
