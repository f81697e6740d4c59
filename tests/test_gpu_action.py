"""GPU parity of the action path f(A) V (N-step recurrence) against the oracle.

Relative Frobenius error per instance <= 1e-12 with the same N (the GPU's N
is handed to the oracle only when eta/θ sits within 1e-12 of an integer)."""

import math
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


def _run_and_check(torch, dev, mats, vecs, funcs, m, tol, bar=1e-12):
    from paper_2210_03714_amd import pfm
    At = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in mats]
    Vt = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in vecs]
    res, info = pfm.action(At, Vt, funcs, m=m, tol=tol)
    torch.cuda.synchronize()
    worst = 0.0
    for i, (A, V) in enumerate(zip(mats, vecs)):
        own = me.action(A, V, funcs, m, tol)
        q = own["eta"] / own["theta"]
        tie = abs(q - round(q)) < 1e-12 * q
        N = int(info[i]["plan"])
        if tie:
            own = me.action(A, V, funcs, m, tol, force_plan=N)
        else:
            assert N == own["plan"], (i, N, own["plan"])
        for f in funcs:
            err = me.rel_fro(res[f][i].cpu().numpy(), own[f])
            worst = max(worst, err)
            assert err <= bar, (i, f, A.shape, V.shape, err)
    return res, info, worst


def test_config_small_action(torch_dev):
    torch, dev = torch_dev
    A, v = wl.config_small()
    _say("case config_small action m=4")
    res, info, w = _run_and_check(torch, dev, [A], [v], ("exp", "phi1"), 4, 1e-12)
    # exp+phi1 plans with min(θ_exp, θ_phi1) = 0.0182 -> N = 55
    assert info[0]["plan"] == 55
    res, info, w2 = _run_and_check(torch, dev, [A], [v], ("exp",), 4, 1e-12)
    assert info[0]["plan"] == 53   # exp alone: θ = 0.0189
    _say("worst %.3e %.3e" % (w, w2))


def test_neg_laplacian_action_and_closed_form(torch_dev):
    import scipy.fft
    torch, dev = torch_dev
    n = 256
    A = wl.neg_laplacian(n, 1.0)
    V = wl.vectors(n, 16, wl.SEED_BASE + 3)
    _say("case -L n=256 p=16")
    res, info, w = _run_and_check(torch, dev, [A], [V], ("exp", "phi1"), 8, 1e-12)
    N = int(info[0]["plan"])
    assert N == 16
    j = np.arange(1, n + 1)
    mu = -(2 - 2 * np.cos(j * np.pi / (n + 1)))
    dst = lambda X: scipy.fft.dst(X, type=1, axis=0, norm="ortho")
    exact = dst(np.exp(mu)[:, None] * dst(V))
    assert me.rel_fro(res["exp"][0].cpu().numpy(), exact) < 1e-10
    _say("worst %.3e" % w)


def test_gaussian_ragged_p(torch_dev):
    torch, dev = torch_dev
    mats = [wl.gaussian(n, 5.0, wl.SEED_BASE + 200 + n) for n in (17, 100, 200, 333)]
    vecs = [wl.vectors(a.shape[0], p, wl.SEED_BASE + 300 + p) for a, p in zip(mats, (1, 20, 33, 7))]
    _say("case gaussian ragged n/p")
    _run_and_check(torch, dev, mats, vecs, ("exp", "phi1"), 8, 1e-12)


def test_action_pivoting_forced_N(torch_dev):
    """N forced to 1 on ||A||_1 = 40: the shifted matrices need row swaps."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    A = wl.gaussian(80, 40.0, wl.SEED_BASE + 400)
    V = wl.vectors(80, 5, wl.SEED_BASE + 401)
    res, info = pfm.action([torch.from_numpy(A).to(dev)], [torch.from_numpy(V).to(dev)], ("exp",),
                           m=8, tol=1e-12, force_plan=1)
    torch.cuda.synchronize()
    ref = me.action(A, V, ("exp",), 8, 1e-12, force_plan=1)
    assert me.rel_fro(res["exp"][0].cpu().numpy(), ref["exp"]) <= 1e-11


def test_binding_rejects_mismatched_tensors(torch_dev):
    """Shapes, element types and strides the library cannot address safely
    are refused by the binding before anything is enqueued."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    A = torch.from_numpy(wl.gaussian(32, 4.0, wl.SEED_BASE + 660)).to(dev)
    V = torch.from_numpy(wl.vectors(32, 3, wl.SEED_BASE + 661)).to(dev)
    _say("case binding validation")
    bad_outs = [
        {"exp": [torch.empty((32, 31), dtype=torch.float64, device=dev)]},      # wrong shape
        {"exp": [torch.empty((32, 32), dtype=torch.complex128, device=dev)]},   # wrong type
        {"exp": [torch.empty((32, 64), dtype=torch.float64, device=dev)[:, ::2]]},  # column stride 2
        {"exp": [torch.empty((32, 40), dtype=torch.float64, device=dev)[:, :32]],   # row strides differ
         "phi1": [torch.empty((32, 32), dtype=torch.float64, device=dev)]},
    ]
    for out in bad_outs:
        with pytest.raises(ValueError):
            pfm.expm([A], tuple(out), m=8, out=out)
    with pytest.raises(ValueError):  # one element type per call
        pfm.expm([A, A.to(torch.complex128)], ("exp",), m=8)
    with pytest.raises(ValueError):  # V rows != n
        pfm.action([A], [V[:31]], ("exp",), m=8)
    with pytest.raises(ValueError):  # non-square A
        pfm.action([A[:, :31]], [V], ("exp",), m=8)
    with pytest.raises(ValueError):  # complex A: the results are complex
        pfm.action([A.to(torch.complex128)], [V], ("exp",), m=8,
                   out={"exp": [torch.empty_like(V)]})
    # the same call with matching tensors runs
    res, info = pfm.action([A], [V], ("exp",), m=8, out={"exp": [torch.empty_like(V)]})
    torch.cuda.synchronize()
    assert info[0]["status"] == 0
