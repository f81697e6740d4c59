"""GPU tests of the autotuner (pfm_tune): it picks one of the candidate
route policies by measurement, later calls of the same batch key use it,
results stay within parity of the oracle under every policy, and the
tuned table survives export / import."""

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


def test_tune_full_small_and_apply(torch_dev):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    A, _ = wl.gaussian_batch(32, 40, 0.5, 8.0, wl.SEED_BASE + 620)
    mats = [torch.from_numpy(a).to(dev) for a in A]
    ctx = pfm.Context(0)
    pol, ms = pfm.tune(mats, None, ("exp",), ctx=ctx)
    _say("  tuned full n=40 x32: policy %d, %.3f ms" % (pol, ms))
    # route policy 0 or 1, either squaring schedule; the tile choice is not
    # tried below a padded size of 256
    assert pol % 4 in (0, 1) and pol < 8 and ms > 0
    res, info = pfm.expm(mats, ("exp",), m=8, tol=1e-12, ctx=ctx)
    torch.cuda.synchronize()
    want_route = 1 if pol % 4 == 0 else 0
    for i in range(len(mats)):
        assert info[i]["route"] == want_route
        ref = me.expm_full(A[i], ("exp",), 8, 1e-12)
        assert me.rel_fro(res["exp"][i].cpu().numpy(), ref["exp"]) <= 1e-12
    text = ctx.tune_export()
    assert text.strip() and len(text.strip().splitlines()) == 1
    ctx2 = pfm.Context(0)
    ctx2.tune_import(text)
    assert ctx2.tune_export() == text
    with pytest.raises(pfm.PfmError):
        ctx2.tune_import("12 99\n")  # no such policy


def test_tune_action_complex(torch_dev):
    """iH n = 150 (embedded 300) action: multi-workgroup route vs LU route;
    both policies give the oracle's result, the tuned one is then used."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    n, p = 150, 6
    mats = [wl.ih_matrix(n, wl.SEED_BASE + 630 + i) for i in range(3)]
    vecs = [wl.vectors(n, p, wl.SEED_BASE + 640 + i, complex_=True) for i in range(3)]
    Am = [torch.from_numpy(a).to(dev) for a in mats]
    Vm = [torch.from_numpy(v).to(dev) for v in vecs]
    ctx = pfm.Context(0)
    pol, ms = pfm.tune(Am, Vm, ("exp",), ctx=ctx)
    _say("  tuned iH action n=150 x3: policy %d, %.3f ms" % (pol, ms))
    assert pol in (0, 2)
    res, info = pfm.action(Am, Vm, ("exp",), m=8, tol=1e-12, ctx=ctx)
    torch.cuda.synchronize()
    for i in range(3):
        assert info[i]["route"] == (2 if pol == 0 else 0)
        ref = me.action(mats[i], vecs[i], ("exp",), 8, 1e-12)
        assert me.rel_fro(res["exp"][i].cpu().numpy(), ref["exp"]) <= 1e-12


def test_tune_full_256_every_policy(torch_dev):
    """n = 256 and 300 (padded sizes 256 and 320, where the product tile
    and the Gauss-Jordan pivot block choices matter): the tuner tries routes x
    squaring schedules x tiles x pivot blocks; then every full-matrix policy
    is imported for the same key and gives the oracle's result."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    mats_np = [wl.gaussian(n, t, wl.SEED_BASE + 650 + i) for i, (n, t) in enumerate([(256, 7.5), (300, 3.0),
                                                                                      (256, 0.7), (300, 60.0)])]
    mats = [torch.from_numpy(a).to(dev) for a in mats_np]
    ctx = pfm.Context(0)
    pol, ms = pfm.tune(mats, None, ("exp", "phi1"), ctx=ctx)
    _say("  tuned full n=256/300 x4: policy %d, %.3f ms" % (pol, ms))
    assert pol % 4 in (0, 1) and 0 <= pol < 32
    key = ctx.tune_export().split()[0]
    refs = [me.expm_full(a, ("exp", "phi1"), 8, 1e-12) for a in mats_np]
    for p in range(32):
        if p % 4 not in (0, 1):
            continue
        ctx.tune_import("%s %d\n" % (key, p))
        res, info = pfm.expm(mats, ("exp", "phi1"), m=8, tol=1e-12, ctx=ctx)
        torch.cuda.synchronize()
        for i, ref in enumerate(refs):
            assert info[i]["route"] == (1 if p % 4 == 0 else 0), (p, i)
            assert info[i]["plan"] == ref["plan"]
            for f in ("exp", "phi1"):
                assert me.rel_fro(res[f][i].cpu().numpy(), ref[f]) <= 1e-12, (p, i, f)
    ctx.check()
