"""pfm_eval_batched without host synchronisation, through the C ABI.

* The call returns while the stream is still busy with earlier work: the
  plan, the routes and the number of squarings are decided on the device.
* A whole call recorded into the caller's stream capture replays bit for bit
  equal to the eager call, several times, with other work in between.
* Squaring levels beyond the directly launched ones run from the persistent
  queue (kern_sched.h): large s, uneven sizes, exp and phi1, every level from
  the queue, against the oracle at the same plan.
"""

import sys
import time

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


def _probs(pfm, At, outs):
    probs = []
    for i, a in enumerate(At):
        probs.append(pfm.Problem(a.shape[0], 0, a.stride(0), 0, outs[i].stride(0), a.data_ptr(), None,
                                 outs[i].data_ptr(), None))
    return probs


def test_call_returns_while_stream_busy(torch_dev):
    """With the stream held by a long kernel, the call returns (all of its
    work enqueued) before that kernel ends; the results are then correct."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    if not hasattr(torch.cuda, "_sleep"):
        pytest.skip("torch.cuda._sleep is not available")
    A, _ = wl.gaussian_batch(16, 96, 0.5, 8.0, wl.SEED_BASE + 1100)
    At = [torch.from_numpy(a).to(dev) for a in A]
    outs = [torch.empty_like(a) for a in At]
    ctx = pfm.Context(0)
    probs = _probs(pfm, At, outs)
    info = torch.empty(len(At) * pfm.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    assert ctx.eval_batched(probs, pfm.EXP, 8, 1e-12, info=info) == pfm.OK  # sizes the workspace
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    for o in outs:
        o.fill_(7.25)
    torch.cuda.synchronize()
    # about 0.5 s of spinning at 2.4 GHz
    _say("case async: call behind a busy stream")
    t0 = time.perf_counter()
    torch.cuda._sleep(int(1.2e9))
    t1 = time.perf_counter()
    rc = ctx.eval_batched(probs, pfm.EXP, 8, 1e-12, info=info)
    t2 = time.perf_counter()
    assert rc == pfm.OK
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    _say("  sleep enqueue %.1f ms, call %.1f ms, until idle %.1f ms" % ((t1 - t0) * 1e3, (t2 - t1) * 1e3,
                                                                          (t3 - t2) * 1e3))
    # the call came back long before the stream drained
    assert (t2 - t1) < 0.5 * (t3 - t1), (t2 - t1, t3 - t1)
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)
    ctx.close()


@pytest.mark.parametrize("funcs", [("exp",), ("exp", "phi1")])
def test_stream_capture_replays(torch_dev, funcs):
    """Record one whole pfm_eval_batched call into a CUDA graph (after the
    same call ran eagerly), replay it three times with the outputs reset and
    unrelated work between the replays, and compare every replay bit for bit
    with the eager result.  Uneven sizes (both product tile sizes)."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    mats = wl.gaussian_uneven(12, [40, 64, 130, 256, 300], 0.5, 8.0, wl.SEED_BASE + 1110)
    At = [torch.from_numpy(a).to(dev) for a in mats]
    fm = pfm.EXP | (pfm.PHI1 if "phi1" in funcs else 0)
    oe = [torch.empty_like(a) for a in At]
    op = [torch.empty_like(a) for a in At]
    probs = []
    for i, a in enumerate(At):
        probs.append(pfm.Problem(a.shape[0], 0, a.stride(0), 0, a.shape[0], a.data_ptr(), None, oe[i].data_ptr(),
                                 op[i].data_ptr() if "phi1" in funcs else None))
    info = torch.empty(len(At) * pfm.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    ctx = pfm.Context(0)
    ctx.set_graphs(False)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        assert ctx.eval_batched(probs, fm, 8, 1e-12, info=info, stream=s) == pfm.OK
    torch.cuda.synchronize()
    ref_e = [o.clone() for o in oe]
    ref_p = [o.clone() for o in op]
    ref_info = info.clone()
    _say("case capture %s" % "+".join(funcs))
    g = torch.cuda.CUDAGraph()
    rcs = []
    with torch.cuda.graph(g, stream=s):
        rcs.append(ctx.eval_batched(probs, fm, 8, 1e-12, info=info, stream=s))
    assert rcs == [pfm.OK], (rcs, ctx.last_error())
    other = torch.randn(512, 512, dtype=torch.float64, device=dev)
    for rep in range(3):
        for o in oe + op:
            o.fill_(7.25)
        info.zero_()
        other = other @ other.T / 512.0  # unrelated work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(At)):
            assert torch.equal(oe[i], ref_e[i]), (rep, i)
            if "phi1" in funcs:
                assert torch.equal(op[i], ref_p[i]), (rep, i)
        assert torch.equal(info, ref_info), rep
    ctx.check()
    # a capture of a call that does not repeat the previous one is refused
    # with nothing recorded
    probs2 = probs[:-1]
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=s):
        rc2 = ctx.eval_batched(probs2, fm, 8, 1e-12, info=info, stream=s)
    assert rc2 == pfm.ERR_INVALID
    ctx.close()


@pytest.mark.parametrize("direct", [8, 0, 2])
def test_squaring_queue_large_s(torch_dev, direct):
    """Norms up to 1e4 (s up to 16 at tol 1e-12) on uneven sizes, exp and
    phi1: the levels beyond `direct` come from the persistent queue.  Every
    instance against the oracle at the GPU's plan."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    sizes = [16, 70, 128, 200, 256, 300, 64, 512]
    norms = [1e4, 3.0, 900.0, 0.3, 40.0, 2e3, 1.0, 150.0]
    mats = []
    for n, t in zip(sizes, norms):
        # skew-symmetric: exp(A) is orthogonal and phi1(A) has norm <= 1, so
        # large norms neither overflow nor lose the relative error
        G = wl.gaussian(n, 1.0, wl.SEED_BASE + 1120 + n)
        S = G - G.T
        mats.append(S * (t / np.abs(S).sum(axis=0).max()))
    ctx = pfm.Context(0)
    ctx.set_schedule(direct)
    _say("case squaring queue, %d levels launched directly" % direct)
    res, info = pfm.expm([torch.from_numpy(a).to(dev) for a in mats], ("exp", "phi1"), m=8, tol=1e-12, ctx=ctx)
    torch.cuda.synchronize()
    ctx.check()
    worst = 0.0
    svals = []
    for i, A in enumerate(mats):
        s = int(info[i]["plan"])
        svals.append(s)
        own = me.expm_full(A, ("exp", "phi1"), 8, 1e-12)
        q = np.log2(own["eta"] / own["theta"])
        assert s == own["plan"] or abs(q - round(q)) < 1e-12, (i, s, own["plan"])
        ref = me.expm_full(A, ("exp", "phi1"), 8, 1e-12, force_plan=s)
        assert info[i]["status"] == 0
        for f in ("exp", "phi1"):
            err = me.rel_fro(res[f][i].cpu().numpy(), ref[f])
            worst = max(worst, err)
            # the s squarings amplify the rounding of r(B) up to 2^s-fold
            assert err <= 1e-12 * max(1.0, 2.0 ** (s - 5)), (i, f, sizes[i], s, err)
    _say("  s = %s, worst %.3e" % (svals, worst))
    assert max(svals) > 8
    ctx.close()


def test_squaring_cap_not_computed(torch_dev):
    """A forced s above PFM_MAX_SQUARINGS: flagged on the device, outputs
    untouched; the other instance of the call is computed."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    A = wl.gaussian(32, 2.0, wl.SEED_BASE + 1130)
    At = torch.from_numpy(A).to(dev)
    out = {"exp": [torch.full_like(At, 7.25)]}
    _say("case squaring cap")
    res, info = pfm.expm([At], ("exp",), m=8, force_plan=1001, out=out)
    torch.cuda.synchronize()
    assert info[0]["status"] & pfm.NOT_COMPUTED and info[0]["plan"] == 1001
    assert torch.all(res["exp"][0] == 7.25)
