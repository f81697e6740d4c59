"""The allocation-free tridiagonal action (pfm_tri_action_noalloc) against
pfm_tri_action, through the C ABI.

Both run the same kernels on the same inputs, so the bar is bit-for-bit
equality of every output and info record.  Two calls in a row, the second
on a smaller input, check that the shared scratch array carries nothing
from one call into the next; a call over the limits is refused before
anything is enqueued."""

import sys

import numpy as np
import pytest

from paper_2210_03714_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2210_03714_amd import pfm
    pfm.lib()
    return torch, torch.device("cuda:0")


def _inputs(torch, dev, shapes, seed):
    dl, dd, du, V = [], [], [], []
    for i, (d, p) in enumerate(shapes):
        a, b, c = wl.tri_gaussian_batch(1, d, 0.5, 8.0, seed + 1 + i)[0]
        dl.append(torch.from_numpy(np.ascontiguousarray(a)).to(dev))
        dd.append(torch.from_numpy(np.ascontiguousarray(b)).to(dev))
        du.append(torch.from_numpy(np.ascontiguousarray(c)).to(dev))
        V.append(torch.from_numpy(wl.vectors(d, p, seed + 100 + i)).to(dev))
    return dl, dd, du, V


def _outputs(torch, V, funcs):
    # sentinel-filled, so that a missing write shows
    return {f: [torch.full_like(v, 7.25) for v in V] for f in funcs}


def _compare(torch, ra, ia, rb, ib, funcs, n):
    for f in funcs:
        for i in range(n):
            assert torch.equal(ra[f][i], rb[f][i]), (f, i)
            assert not torch.isnan(ra[f][i]).any(), (f, i)
    assert ia.get().tobytes() == ib.get().tobytes()


@pytest.mark.parametrize("case", ["call1_exp_phi1_m8", "call2_smaller_exp_m4"])
def test_noalloc_matches_tri_action(torch_dev, case):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    if case == "call1_exp_phi1_m8":
        shapes, funcs, m, seed = [(1, 3), (37, 70), (300, 1), (1025, 65), (8, 64), (129, 130)], ("exp", "phi1"), 8, 0
    else:
        shapes, funcs, m, seed = [(17, 5), (64, 2)], ("exp",), 4, 50
    _say("case %s: shapes %s funcs %s m %d" % (case, shapes, funcs, m))
    dl, dd, du, V = _inputs(torch, dev, shapes, wl.SEED_BASE + 700 + seed)
    ctx = pfm.Context(0)
    ref_out = _outputs(torch, V, funcs)
    ref, iref = pfm.tri_action(dl, dd, du, V, funcs, m=m, tol=1e-12, ctx=ctx, out=ref_out)
    torch.cuda.synchronize()
    out = _outputs(torch, V, funcs)
    info_buf = torch.zeros(len(V) * pfm.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    res, inf = pfm.tri_action(dl, dd, du, V, funcs, m=m, tol=1e-12, ctx=ctx, out=out, info_out=info_buf,
                              noalloc=True)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    _compare(torch, res, inf, ref, iref, funcs, len(V))
    assert all(inf[i]["route"] == 3 and inf[i]["status"] == 0 for i in range(len(V)))
    if case == "call2_smaller_exp_m4":
        # the first call has loaded every code path; this one must not take
        # device memory
        assert free1 == free0, (free0, free1)


def test_noalloc_two_calls_in_a_row(torch_dev):
    """A large call and then a smaller one, back to back on one stream with
    no synchronisation between them: the second must not see the first's
    leftovers (plans, factors, vectors and checkpoints in the scratch)."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    ctx = pfm.Context(0)
    big = _inputs(torch, dev, [(513, 64), (77, 9), (1000, 3)], wl.SEED_BASE + 760)
    small = _inputs(torch, dev, [(33, 4)], wl.SEED_BASE + 770)
    funcs = ("exp", "phi1")
    rb = pfm.tri_action(*big, funcs, m=5, tol=1e-10, ctx=ctx, out=_outputs(torch, big[3], funcs))
    rs = pfm.tri_action(*small, funcs, m=5, tol=1e-10, ctx=ctx, out=_outputs(torch, small[3], funcs))
    torch.cuda.synchronize()
    _say("case two calls: noalloc big then small")
    nb = pfm.tri_action(*big, funcs, m=5, tol=1e-10, ctx=ctx, out=_outputs(torch, big[3], funcs), noalloc=True)
    ns = pfm.tri_action(*small, funcs, m=5, tol=1e-10, ctx=ctx, out=_outputs(torch, small[3], funcs),
                        noalloc=True)
    torch.cuda.synchronize()
    _compare(torch, nb[0], nb[1], rb[0], rb[1], funcs, 3)
    _compare(torch, ns[0], ns[1], rs[0], rs[1], funcs, 1)


def test_noalloc_limits(torch_dev):
    """Over the batch or byte limit: PFM_ERR_BUDGET and the outputs untouched."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    ctx = pfm.Context(0)
    # bytes: d = 4096, p = 512 needs about 8 d (3 + 3 m + 3 p + m p / 8) > 64 MiB
    d, p = 4096, 512
    dl, dd, du, V = _inputs(torch, dev, [(d, p)], wl.SEED_BASE + 780)
    out = _outputs(torch, V, ("exp",))
    _say("case limits: bytes")
    with pytest.raises(pfm.PfmError) as e:
        pfm.tri_action(dl, dd, du, V, ("exp",), m=8, ctx=ctx, out=out, noalloc=True)
    assert e.value.code == pfm.ERR_BUDGET
    # batch: NOALLOC_MAX_BATCH + 1 tiny instances
    n = pfm.NOALLOC_MAX_BATCH + 1
    a = torch.zeros(1, dtype=torch.float64, device=dev)
    b = torch.full((2,), 0.5, dtype=torch.float64, device=dev)
    v = torch.ones((2, 1), dtype=torch.float64, device=dev)
    outs = {"exp": [torch.full_like(v, 7.25) for _ in range(n)]}
    _say("case limits: batch")
    with pytest.raises(pfm.PfmError) as e:
        pfm.tri_action([a] * n, [b] * n, [a] * n, [v] * n, ("exp",), m=8, ctx=ctx, out=outs, noalloc=True)
    assert e.value.code == pfm.ERR_BUDGET
    torch.cuda.synchronize()
    assert torch.all(out["exp"][0] == 7.25)
    assert all(torch.all(o == 7.25) for o in outs["exp"])
