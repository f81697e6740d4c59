"""GPU parity of the large-instance route (n > 512 real, n > 256 complex):
shifted inverses by block Gauss-Jordan over many workgroups, the explicit
approximant R = a0 I + S B, squarings (full matrix) or N steps U <- R U
(action).  Reference: the step-by-step oracle where it finishes in seconds,
and, at n = 4096, the oracle's per-eigenvalue form of the same N-step
recurrence for normal A (iH and -L)."""

import sys

import numpy as np
import pytest

from oracle import method as me
from paper_2210_03714_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2210_03714_amd import pfm
    pfm.lib()
    return torch, torch.device("cuda:0")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_large_full_real_ragged(torch_dev):
    """n in {513, 600, 700} plus a small instance in the same call (both
    routes at once), exp and phi1, every instance against the oracle."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    sizes = [513, 100, 600, 700]
    rng = np.random.default_rng(wl.SEED_BASE + 400)
    mats = [wl.gaussian(n, float(rng.uniform(0.5, 8.0)), wl.SEED_BASE + 401 + n) for n in sizes]
    _say("case large full real", sizes)
    res, info = pfm.expm([torch.from_numpy(a).to(dev) for a in mats], ("exp", "phi1"), m=8, tol=1e-12)
    torch.cuda.synchronize()
    for i, (a, n) in enumerate(zip(mats, sizes)):
        ref = me.expm_full(a, ("exp", "phi1"), 8, 1e-12, force_plan=int(info[i]["plan"]))
        own = me.expm_full(a, ("exp",), 8, 1e-12)
        assert info[i]["status"] == 0
        assert info[i]["route"] == (2 if n > 512 else 1)
        for f in ("exp", "phi1"):
            err = me.rel_fro(res[f][i].cpu().numpy(), ref[f])
            _say("  n=%d %s s=%d err %.2e" % (n, f, info[i]["plan"], err))
            assert err <= 1e-12, (n, f, err)
        assert abs(me.plan_scaling(own["eta"], me.theta_for(("exp", "phi1"), 8, 1e-12)) - info[i]["plan"]) == 0


def test_large_full_complex(torch_dev):
    """Complex A (n = 300, embedded size 600) with R4 and R8."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    n = 300
    rng = np.random.default_rng(wl.SEED_BASE + 410)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    A *= 3.0 / np.abs(A).sum(0).max()
    for m in (4, 8):
        _say("case large full complex m=%d" % m)
        res, info = pfm.expm([torch.from_numpy(A).to(dev)], ("exp", "phi1"), m=m, tol=1e-12)
        torch.cuda.synchronize()
        assert info[0]["route"] == 2 and info[0]["status"] == 0
        ref = me.expm_full(A, ("exp", "phi1"), m, 1e-12)
        assert int(info[0]["plan"]) == ref["plan"]
        for f in ("exp", "phi1"):
            err = me.rel_fro(res[f][0].cpu().numpy(), ref[f])
            _say("  %s err %.2e" % (f, err))
            assert err <= 1e-12, (m, f, err)


@pytest.mark.parametrize("kind", ["gauss", "iH"])
def test_large_action_vs_oracle(torch_dev, kind):
    """Action at n = 640 real (p = 7) and complex iH n = 300 (p = 5), exp
    and phi1, against the step-by-step oracle."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    if kind == "gauss":
        n, p = 640, 7
        A = wl.gaussian(n, 6.0, wl.SEED_BASE + 420)
        V = wl.vectors(n, p, wl.SEED_BASE + 421)
    else:
        n, p = 300, 5
        A = wl.ih_matrix(n, wl.SEED_BASE + 422)
        V = wl.vectors(n, p, wl.SEED_BASE + 423, complex_=True)
    _say("case large action", kind, n, p)
    res, info = pfm.action([torch.from_numpy(A).to(dev)], [torch.from_numpy(V).to(dev)], ("exp", "phi1"),
                           m=8, tol=1e-12)
    torch.cuda.synchronize()
    ref = me.action(A, V, ("exp", "phi1"), 8, 1e-12)
    assert info[0]["route"] == 2 and info[0]["status"] == 0
    assert int(info[0]["plan"]) == ref["plan"]
    for f in ("exp", "phi1"):
        err = me.rel_fro(res[f][0].cpu().numpy(), ref[f])
        _say("  %s N=%d err %.2e" % (f, ref["plan"], err))
        assert err <= 1e-12, (kind, f, err)


def test_large_forced_plan_not_computed(torch_dev):
    """A forced plan that leaves I - c_k B far from diagonally dominant: the
    large instance is reported NOT_COMPUTED and its output is untouched; the
    small instance in the same call is computed (LU route)."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    big = wl.gaussian(600, 40.0, wl.SEED_BASE + 430)
    small = wl.gaussian(50, 40.0, wl.SEED_BASE + 431)
    At = [torch.from_numpy(big).to(dev), torch.from_numpy(small).to(dev)]
    out = {"exp": [torch.full_like(a, 7.0) for a in At]}
    _say("case large forced plan")
    res, info = pfm.expm(At, ("exp",), m=8, tol=1e-12, force_plan=0, out=out)
    torch.cuda.synchronize()
    assert info[0]["status"] & pfm.NOT_COMPUTED
    assert bool((res["exp"][0] == 7.0).all())
    assert info[1]["status"] == 0 and info[1]["route"] == 0
    ref = me.expm_full(small, ("exp",), 8, 1e-12, force_plan=0)
    assert me.rel_fro(res["exp"][1].cpu().numpy(), ref["exp"]) <= 1e-11


@pytest.mark.parametrize("kind", ["negL", "iH"])
def test_config3_n4096_action(torch_dev, kind):
    """n = 4096, V n x 64: A = -L (real, tau = 1) and A = iH (complex128),
    exp(A)V and phi1(A)V with m = 8 at tol 1e-12, against the oracle's
    per-eigenvalue form of the same N-step recurrence."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    n, p = 4096, 64
    if kind == "negL":
        A = wl.neg_laplacian(n, 1.0)
        mu, U = np.linalg.eigh(A)
        V = wl.vectors(n, p, wl.SEED_BASE + 3)
    else:
        A = wl.ih_matrix(n, wl.SEED_BASE + 3)
        lam, U = np.linalg.eigh(A / 1j)
        mu = 1j * lam
        V = wl.vectors(n, p, wl.SEED_BASE + 4, complex_=True)
    _say("case config3", kind)
    res, info = pfm.action([torch.from_numpy(A).to(dev)], [torch.from_numpy(V).to(dev)], ("exp", "phi1"),
                           m=8, tol=1e-12)
    torch.cuda.synchronize()
    N = int(info[0]["plan"])
    eta = me.norm1(A)
    assert N == me.plan_steps(eta, me.theta_for(("exp", "phi1"), 8, 1e-12))
    assert info[0]["route"] == 2 and info[0]["status"] == 0
    ref = me.action_normal(mu, U, V, ("exp", "phi1"), 8, N, exact_scalars=True)
    for f in ("exp", "phi1"):
        got = res[f][0].cpu().numpy()
        err = me.rel_fro(got, ref[f])
        _say("  %s N=%d err %.2e" % (f, N, err))
        assert err <= 1e-12, (kind, f, err)
    if kind == "iH":
        # e^{iH} is unitary: column norms of V are preserved
        g = res["exp"][0].cpu().numpy()
        assert np.allclose(np.linalg.norm(g, axis=0), np.linalg.norm(V, axis=0), rtol=1e-11)
