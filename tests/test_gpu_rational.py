"""GPU parity of caller-given partial-fraction sets (pfm_eval_rational; §2,
a rational function with simple poles, in the round-off form of §4.3, no
scaling) against the oracle (oracle.method.rational), through the C ABI.

Bar: 1e-12 relative Frobenius error per instance; the sets below have
sum |w_k| of a few units and |c_k| ||A||_1 < 1, so both sides' rounding is a
few units of 2^-53 times sqrt(n).  The exp Padé pair passed as a caller set
on real A gives the same terms as the library's m = 1 set at s = 0, so the
two results must agree bit for bit."""

import sys

import numpy as np
import pytest

from oracle import coefficients as co
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


REAL_SET = ([0.25, -0.2, 0.125, -0.1], [1.5, -0.75, 2.0, 0.5], 1.0)
COMPLEX_SET = ([0.3 + 0.2j, -0.25, 0.1 - 0.4j], [1.5 - 0.5j, 2.0, -0.7 + 0.3j], 0.75)


@pytest.mark.parametrize("case", ["real_gj", "real_lu", "conj_pairs_real_A", "complex_A", "action_real",
                                  "action_complex"])
def test_rational_against_oracle(torch_dev, case):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    sizes = [17, 64, 100, 200]
    if case in ("real_gj", "action_real"):
        c, w, a0 = REAL_SET
        norms = [1.0, 1.5, 0.5, 2.0]          # |c| ||A|| <= 1/2: Gauss-Jordan route
    elif case == "real_lu":
        c, w, a0 = REAL_SET
        norms = [3.0, 3.5, 2.5, 3.2]          # |c| ||A|| > 1/2: the pivoting LU route
    else:
        c, w, a0 = COMPLEX_SET
        norms = [0.8, 1.2, 0.5, 1.0]
    mats = [wl.gaussian(n, t, wl.SEED_BASE + 800 + n) for n, t in zip(sizes, norms)]
    if case in ("complex_A", "action_complex"):
        rng = np.random.default_rng(wl.SEED_BASE + 810)
        mats = [a + 0.3j * rng.standard_normal(a.shape) * np.abs(a).mean() for a in mats]
    vecs = None
    if case.startswith("action"):
        vecs = [wl.vectors(n, p, wl.SEED_BASE + 820 + n, complex_=case == "action_complex")
                for n, p in zip(sizes, (1, 5, 16, 33))]
    conj = case != "complex_A" and case != "action_complex"
    _say("case rational %s" % case)
    At = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in mats]
    Vt = None if vecs is None else [torch.from_numpy(v).to(dev) for v in vecs]
    res, info = pfm.rational(At, c, w, a0, conj_pairs=conj, V=Vt)
    torch.cuda.synchronize()
    worst = 0.0
    for i, A in enumerate(mats):
        ref = me.rational(A, c, w, a0, conj_pairs=conj, V=None if vecs is None else vecs[i])
        got = res[i].cpu().numpy()
        err = me.rel_fro(got, ref)
        worst = max(worst, err)
        assert err <= BAR, (case, i, err)
        assert info[i]["status"] == 0 and info[i]["plan"] == (1 if vecs is not None else 0)
        if case == "real_gj":
            assert info[i]["route"] == 1
        if case == "real_lu":
            assert info[i]["route"] == 0
    _say("  worst %.2e" % worst)


def test_pade_pair_as_caller_set_equals_m1(torch_dev):
    """The exp Padé pair (§2 eq. 5) as a caller set equals the library's m = 1
    set at s = 0 bit for bit (the same terms reach the same kernels)."""
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    a0, terms = co.roundoff_terms("exp", 1)
    (c, w, _), = terms
    mats = [wl.gaussian(n, 0.4, wl.SEED_BASE + 830 + n) for n in (20, 90, 150)]
    At = [torch.from_numpy(a).to(dev) for a in mats]
    _say("case rational pade pair")
    r1, _ = pfm.rational(At, [c], [w], a0, conj_pairs=True)
    r2, _ = pfm.expm(At, ("exp",), m=1, force_plan=0)
    torch.cuda.synchronize()
    for i in range(len(mats)):
        assert torch.equal(r1[i], r2["exp"][i]), i


def test_rational_errors(torch_dev):
    torch, dev = torch_dev
    from paper_2210_03714_amd import pfm
    A = [torch.from_numpy(wl.gaussian(16, 1.0, wl.SEED_BASE + 840)).to(dev)]
    _say("case rational errors")
    with pytest.raises(pfm.PfmError) as e:
        pfm.rational(A, [0.2 + 0.1j], [1.0], 1.0, conj_pairs=False)   # complex shift, real A, no conjugates
    assert e.value.code == pfm.ERR_UNSUPPORTED
    with pytest.raises(pfm.PfmError) as e:
        pfm.rational(A, [0.2], [1.0 + 1.0j], 1.0)                   # real shift, complex weight, real A
    assert e.value.code == pfm.ERR_INVALID
    with pytest.raises(pfm.PfmError) as e:
        pfm.rational(A, [float("nan")], [1.0], 1.0)
    assert e.value.code == pfm.ERR_INVALID
    with pytest.raises(pfm.PfmError) as e:
        pfm.rational(A, [0.1] * 17, [1.0] * 17, 1.0)
    assert e.value.code == pfm.ERR_INVALID
