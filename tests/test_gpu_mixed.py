"""Mixed-precision path (binary32 LU/solves on MFMA + binary64 refinement,
binary64 combination and squaring): per-instance error against the FP64
oracle <= the requested tolerance, with the refinement report checked."""

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


def test_mixed_uneven_sizes(torch_dev):
    """A sample of the uneven-size batch: n in {64, 96, ..., 512}, ||A||_1 in
    [0.5, 4], exp and phi1 at tol 1e-10."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    mats = wl.gaussian_uneven(15, list(range(64, 513, 32)), 0.5, 4.0, wl.SEED_BASE + 3)
    _say("case mixed uneven", [a.shape[0] for a in mats])
    tol = 1e-10
    res, info = pfm.expm([torch.from_numpy(a).to(dev) for a in mats], ("exp", "phi1"), m=8, tol=tol,
                         prec="mixed")
    torch.cuda.synchronize()
    worst = 0.0
    for i, A in enumerate(mats):
        ref = me.expm_full(A, ("exp", "phi1"), 8, tol, force_plan=int(info[i]["plan"]))
        for f in ("exp", "phi1"):
            err = me.rel_fro(res[f][i].cpu().numpy(), ref[f])
            worst = max(worst, err)
            assert err <= tol, (i, f, A.shape[0], err)
        assert info[i]["status"] == 0
        assert 1 <= info[i]["ir_iters"] <= 3
    _say("mixed worst %.3e, ir iters %s" % (worst, sorted(set(int(x) for x in info.get()["ir_iters"]))))


def test_mixed_headline_vs_fp64(torch_dev):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    A, _ = wl.gaussian_batch(512, 256, 0.5, 8.0, wl.SEED_BASE + 10)
    At = torch.from_numpy(A).to(dev)
    _say("case mixed headline")
    rm, im = pfm.expm(At, ("exp",), m=8, tol=1e-10, prec="mixed")
    rd, idd = pfm.expm(At, ("exp",), m=8, tol=1e-10, prec="fp64")
    torch.cuda.synchronize()
    d = (rm["exp"] - rd["exp"]).flatten(1).norm(dim=1) / rd["exp"].flatten(1).norm(dim=1)
    assert float(d.max()) <= 1e-10
    for i in np.random.default_rng(1).choice(512, 6, replace=False):
        ref = me.expm_full(A[i], ("exp",), 8, 1e-10, force_plan=int(im[i]["plan"]))
        assert me.rel_fro(rm["exp"][i].cpu().numpy(), ref["exp"]) <= 1e-10
    _say("mixed vs fp64 GPU max %.3e" % float(d.max()))
