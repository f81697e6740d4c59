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


def test_config4_full_size(torch_dev):
    """The uneven mixed-precision batch at its stated size: 2048 Gaussian
    instances, n uniform over {64, 96, ..., 512}, ||A||_1 ~ U[0.5, 4], exp and
    phi1 with m = 8.  The mixed path at tol 1e-10 is held, on every instance,
    to the binary64 GPU path at the same tolerance (same plan, so the two
    differ only by rounding and refinement), and on a stratified sample (the
    smallest- and largest-norm instance of every size) to the oracle; the
    binary64 path at 1e-12 is held to the oracle on the same sample.  The
    difference between the mixed result and the 1e-12 result is reported."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    sizes = list(range(64, 513, 32))
    mats = wl.gaussian_uneven(2048, sizes, 0.5, 4.0, wl.SEED_BASE + 4)
    norms = np.array([np.abs(a).sum(axis=0).max() for a in mats])
    ns = np.array([a.shape[0] for a in mats])
    _say("case config4: 2048 instances, n histogram %s" % np.bincount(ns // 32 - 2).tolist())
    At = [torch.from_numpy(a).to(dev) for a in mats]
    funcs = ("exp", "phi1")
    rm, im = pfm.expm(At, funcs, m=8, tol=1e-10, prec="mixed")
    torch.cuda.synchronize()
    _say("  mixed done")
    rd, idd = pfm.expm(At, funcs, m=8, tol=1e-10, prec="fp64")
    r12, i12 = pfm.expm(At, funcs, m=8, tol=1e-12, prec="fp64")
    torch.cuda.synchronize()
    _say("  fp64 done")
    imm, idn, i12n = im.get(), idd.get(), i12.get()
    assert np.array_equal(imm["plan"], idn["plan"])
    assert np.all(imm["status"] == 0) and np.all(idn["status"] == 0) and np.all(i12n["status"] == 0)
    assert np.all((imm["ir_iters"] >= 1) & (imm["ir_iters"] <= 3))
    worst_same, worst_12 = 0.0, 0.0
    for f in funcs:
        for i in range(len(mats)):
            ref = rd[f][i]
            d = float((rm[f][i] - ref).norm() / ref.norm())
            worst_same = max(worst_same, d)
            assert d <= 1e-10, (f, i, ns[i], d)
            worst_12 = max(worst_12, float((rm[f][i] - r12[f][i]).norm() / r12[f][i].norm()))
    _say("  mixed vs fp64 (1e-10, same plan) worst %.3e; vs fp64 at 1e-12 worst %.3e; ir iters %s"
         % (worst_same, worst_12, np.bincount(imm["ir_iters"]).tolist()))
    pick = []
    for n in sizes:
        idx = np.nonzero(ns == n)[0]
        pick += [int(idx[np.argmin(norms[idx])]), int(idx[np.argmax(norms[idx])])]
    worst_o = 0.0
    for i in pick:
        ref = me.expm_full(mats[i], funcs, 8, 1e-10, force_plan=int(imm["plan"][i]))
        ref12 = me.expm_full(mats[i], funcs, 8, 1e-12, force_plan=int(i12n["plan"][i]))
        for f in funcs:
            e = me.rel_fro(rm[f][i].cpu().numpy(), ref[f])
            worst_o = max(worst_o, e)
            assert e <= 1e-10, (f, i, ns[i], e)
            assert me.rel_fro(r12[f][i].cpu().numpy(), ref12[f]) <= 1e-12, (f, i, ns[i])
    _say("  stratified sample (%d instances) mixed vs oracle worst %.3e" % (len(pick), worst_o))
