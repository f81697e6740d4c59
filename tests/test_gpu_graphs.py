"""GPU tests of launch-sequence reuse (pfm_set_graphs): repeated identical
calls are captured once and replayed; every replay, with eager work and
synchronisations in between, equals the eager result bit for bit."""

import sys
import time

import numpy as np
import pytest

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


@pytest.mark.parametrize("case", ["full_small", "full_large", "action_large"])
def test_graph_replays_equal_eager(torch_dev, case):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    if case == "full_small":
        A, _ = wl.gaussian_batch(24, 100, 0.5, 8.0, wl.SEED_BASE + 600)
        mats, vecs = [torch.from_numpy(a).to(dev) for a in A], None
        funcs = ("exp", "phi1")
    elif case == "full_large":
        mats, vecs = [torch.from_numpy(wl.gaussian(600, 4.0, wl.SEED_BASE + 601)).to(dev)], None
        funcs = ("exp",)
    else:
        mats = [torch.from_numpy(wl.ih_matrix(300, wl.SEED_BASE + 602)).to(dev)]
        vecs = [torch.from_numpy(wl.vectors(300, 8, wl.SEED_BASE + 603, complex_=True)).to(dev)]
        funcs = ("exp", "phi1")
    stream = torch.cuda.Stream()
    like = mats if vecs is None else vecs
    bufs = {}

    def call(ctx, key):
        # fixed output and info buffers per context: a repeated call then
        # repeats its launch sequence exactly
        if key not in bufs:
            bufs[key] = ({f: [torch.empty_like(x) for x in like] for f in funcs},
                         torch.empty(len(mats) * pfm.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev))
        out, ib = bufs[key]
        with torch.cuda.stream(stream):
            if vecs is None:
                res, info = pfm.expm(mats, funcs, m=8, tol=1e-12, ctx=ctx, stream=stream, out=out, info_out=ib)
            else:
                res, info = pfm.action(mats, vecs, funcs, m=8, tol=1e-12, ctx=ctx, stream=stream, out=out,
                                       info_out=ib)
        stream.synchronize()
        return {f: [x.clone() for x in res[f]] for f in funcs}, info

    eager_ctx = pfm.Context(0)
    eager_ctx.set_graphs(False)
    ref, _ = call(eager_ctx, "eager")
    ctx = pfm.Context(0)
    _say("case graphs", case)
    for it in range(5):
        res, info = call(ctx, "graph")
        for f in funcs:
            for a, b in zip(res[f], ref[f]):
                assert torch.equal(a, b), (case, it, f)
        # eager work on the same stream between replays
        with torch.cuda.stream(stream):
            junk = torch.randn(256, 256, device=dev, dtype=torch.float64) @ torch.randn(256, 256, device=dev,
                                                                                     dtype=torch.float64)
        stream.synchronize()
        del junk
    caps, reps = ctx.graph_stats()
    assert (caps, reps) == (1, 3), (caps, reps)
    # timing: eager vs replay
    for label, c in (("eager", eager_ctx), ("graph", ctx)):
        call(c, label)
        t0 = time.perf_counter()
        for _ in range(5):
            call(c, label)
        _say("  %s %.3f ms/call" % (label, (time.perf_counter() - t0) / 5 * 1e3))


def test_graph_new_sequence_runs_eagerly(torch_dev):
    """A different batch invalidates the cached sequence: results follow
    the new inputs, and the old graph is not replayed for them."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    stream = torch.cuda.Stream()
    ctx = pfm.Context(0)
    A1 = torch.from_numpy(wl.gaussian(64, 2.0, wl.SEED_BASE + 610)).to(dev)
    A2 = torch.from_numpy(wl.gaussian(64, 6.0, wl.SEED_BASE + 611)).to(dev)  # other plan
    outs = []
    out = {"exp": [torch.empty_like(A1)]}
    ib = torch.empty(pfm.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    for A in (A1, A1, A1, A2):
        res, _ = pfm.expm([A], ("exp",), m=8, tol=1e-12, ctx=ctx, stream=stream, out=out, info_out=ib)
        stream.synchronize()
        outs.append(res["exp"][0].clone())
    ref2, _ = pfm.expm([A2], ("exp",), m=8, tol=1e-12, stream=stream)
    stream.synchronize()
    assert torch.equal(outs[0], outs[2]) and torch.equal(outs[3], ref2["exp"][0])
    assert ctx.graph_stats() == (1, 1)
