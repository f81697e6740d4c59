"""Thin ctypes binding of libpfm (include/pfm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libpfm.so.  PyTorch supplies device memory and the stream.  There
is no fallback: if the library is missing, or a tensor is not on the GPU, the
call raises.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfm.so")

EXP = 1
PHI1 = 2
LOG1M = 4  # log(1 - A), on its own (its result goes to F_exp)
PHI2 = 8   # phi2(A) (full real matrices up to n = 512, binary64, m = 4, 5, 8)
R64 = 0
C128 = 1
FP64 = 0
MIXED = 1
ROUTE_AUTO = 0
ROUTE_LU = 1

OK = 0
ERR_INVALID = -1
ERR_UNSUPPORTED = -2
ERR_BUDGET = -3
ERR_HIP = -4
ERR_DEVICE = -5

R10STAR = 110                       # PFM_R10STAR: the hybrid set R*10 of §4.3
MAX_STEPS = 1 << 20                 # PFM_MAX_STEPS: more action steps are PFM_NOT_COMPUTED
NOALLOC_MAX_BYTES = 64 << 20        # PFM_NOALLOC_MAX_BYTES
NOALLOC_MAX_BATCH = 1024            # PFM_NOALLOC_MAX_BATCH

SINGULAR_SHIFT = 1
NONFINITE = 2
IR_STALL = 4
NOT_COMPUTED = 8
OUT_OF_RANGE = 16


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.c_int32),
                ("lda", ctypes.c_int64), ("ldv", ctypes.c_int64), ("ldf", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("F_exp", ctypes.c_void_p), ("F_phi1", ctypes.c_void_p), ("F_phi2", ctypes.c_void_p)]


class TriProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("p", ctypes.c_int32),
                ("ldv", ctypes.c_int64), ("ldf", ctypes.c_int64),
                ("dl", ctypes.c_void_p), ("dd", ctypes.c_void_p), ("du", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("F_exp", ctypes.c_void_p), ("F_phi1", ctypes.c_void_p)]


class BandProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("p", ctypes.c_int32),
                ("ldv", ctypes.c_int64), ("ldf", ctypes.c_int64),
                ("bands", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("F_exp", ctypes.c_void_p), ("F_phi1", ctypes.c_void_p)]


INFO_DTYPE = np.dtype([("status", "<i4"), ("plan", "<i4"), ("order", "<i4"), ("ir_iters", "<i4"),
                       ("bad_shift", "<i4"), ("route", "<i4"), ("norm1", "<f8"),
                       ("theta", "<f8"), ("resid", "<f8")])
assert INFO_DTYPE.itemsize == 48

_lib = None


def lib():
    """Load libpfm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpfm.so is not built: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        L.pfm_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_size_t]
        L.pfm_destroy.argtypes = [vp]
        L.pfm_last_error.argtypes = [vp]
        L.pfm_last_error.restype = ctypes.c_char_p
        L.pfm_coeffs.argtypes = [i32, i32, ip, dp, dp, dp, dp, dp, ip, ip]
        L.pfm_theta.argtypes = [i32, i32, dbl, dp]
        L.pfm_poly.argtypes = [i32, i32, dp, dp]
        L.pfm_eval_batched.argtypes = [vp, i32, i32, dbl, i32, i32, i32, ctypes.POINTER(Problem),
                                       vp, i32, vp]
        L.pfm_check.argtypes = [vp, vp]
        L.pfm_version.restype = ctypes.c_char_p
        L.pfm_selftest_mfma.argtypes = [i32, dp]
        L.pfm_profile.argtypes = [vp, i32]
        L.pfm_set_route.argtypes = [vp, i32]
        L.pfm_set_schedule.argtypes = [vp, i32]
        L.pfm_set_graphs.argtypes = [vp, i32]
        L.pfm_eval_batched_tols.argtypes = [vp, i32, i32, dp, dbl, i32, i32, i32, ctypes.POINTER(Problem), vp,
                                            i32, vp]
        L.pfm_tune.argtypes = [vp, i32, i32, dbl, i32, i32, i32, ctypes.POINTER(Problem), i32, vp, ip, dp]
        L.pfm_tune_export.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
        L.pfm_tune_import.argtypes = [vp, ctypes.c_char_p]
        L.pfm_lu_factors.argtypes = [vp, i32, i32, dp, ctypes.c_int64, ip, ip]
        L.pfm_graph_stats.argtypes = [vp, ip, ip]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.pfm_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(Problem)]
        L.pfm_workspace_bytes.restype = ctypes.c_size_t
        L.pfm_srv_start.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.c_size_t, i32]
        L.pfm_srv_stop.argtypes = [vp]
        L.pfm_srv_submit.argtypes = [vp, ctypes.POINTER(Problem), i32, i32, dbl, i32, i32, u64p]
        L.pfm_srv_poll.argtypes = [vp, ctypes.c_uint64, vp, dp]
        L.pfm_srv_drain.argtypes = [vp, i32, u64p, dp, ip]
        L.pfm_srv_fetch.argtypes = [vp, ctypes.c_uint64, i32, vp, ctypes.c_int64]
        L.pfm_srv_timing.argtypes = [vp, ctypes.c_uint64, dp]
        L.pfm_srv_release.argtypes = [vp, ctypes.c_uint64]
        L.pfm_srv_stats.argtypes = [vp, u64p, u64p, u64p, u64p, u64p, dp]
        L.pfm_profile_read.argtypes = [vp, dp, ip, ip]
        L.pfm_tri_action.argtypes = [vp, i32, i32, dbl, i32, ctypes.POINTER(TriProblem), vp, i32, vp]
        L.pfm_eval_rational.argtypes = [vp, i32, dp, dp, dp, dp, dbl, i32, i32, i32, ctypes.POINTER(Problem), vp,
                                        vp]
        L.pfm_tri_action_noalloc.argtypes = [vp, i32, i32, dbl, i32, ctypes.POINTER(TriProblem), vp, i32, vp]
        L.pfm_band_action.argtypes = [vp, i32, i32, dbl, i32, i32, ctypes.POINTER(BandProblem), vp, i32, vp]
        _lib = L
    return _lib


def version():
    return lib().pfm_version().decode()


def coeffs(f, m):
    """(c, w, a0, order, is_pair) of the library's set for f (EXP or PHI1)."""
    L = lib()
    n = ctypes.c_int()
    arrs = [(ctypes.c_double * 16)() for _ in range(4)]
    a0 = ctypes.c_double()
    order = ctypes.c_int()
    pair = ctypes.c_int()
    rc = L.pfm_coeffs(f, m, ctypes.byref(n), *[ctypes.cast(a, ctypes.POINTER(ctypes.c_double)) for a in arrs],
                      ctypes.byref(a0), ctypes.byref(order), ctypes.byref(pair))
    if rc:
        raise ValueError("pfm_coeffs(%d, %d) -> %d" % (f, m, rc))
    k = n.value
    c = np.array(arrs[0][:k]) + 1j * np.array(arrs[1][:k])
    w = np.array(arrs[2][:k]) + 1j * np.array(arrs[3][:k])
    return c, w, a0.value, order.value, bool(pair.value)


def poly(f, m):
    """(d1, d2) of the polynomial part of the library's set for f (0 unless hybrid)."""
    d1, d2 = ctypes.c_double(), ctypes.c_double()
    rc = lib().pfm_poly(f, m, ctypes.byref(d1), ctypes.byref(d2))
    if rc:
        raise ValueError("pfm_poly(%d, %d) -> %d" % (f, m, rc))
    return d1.value, d2.value


def theta(f, m, tol):
    out = ctypes.c_double()
    rc = lib().pfm_theta(f, m, tol, ctypes.byref(out))
    if rc:
        raise ValueError("pfm_theta(%d, %d, %g) -> %d" % (f, m, tol, rc))
    return out.value


def selftest_mfma(device=0):
    """(f64 accumulators, f32 accumulators), each 64 lanes x 4."""
    out = (ctypes.c_double * 512)()
    rc = lib().pfm_selftest_mfma(device, ctypes.cast(out, ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise RuntimeError("pfm_selftest_mfma -> %d" % rc)
    a = np.array(out[:])
    return a[:256].reshape(64, 4), a[256:].reshape(64, 4)


class PfmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pfm error %d: %s" % (code, msg))
        self.code = code


class Context:
    """Owns one pfm_ctx (workspace) on a device."""

    def __init__(self, device=0, budget=0):
        self._h = ctypes.c_void_p()
        rc = lib().pfm_create(ctypes.byref(self._h), device, budget)
        if rc:
            raise PfmError(rc, "pfm_create failed")
        self.device = device

    def close(self):
        if self._h:
            lib().pfm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_route(self, route):
        """ROUTE_AUTO (Gauss-Jordan where pivoting provably never swaps) or
        ROUTE_LU (pivoting LU for every instance)."""
        rc = lib().pfm_set_route(self._h, int(route))
        if rc:
            raise PfmError(rc, self.last_error())

    def set_schedule(self, direct_levels):
        """Squaring levels launched one by one before the persistent queue
        takes the rest (0: all from the queue)."""
        rc = lib().pfm_set_schedule(self._h, int(direct_levels))
        if rc:
            raise PfmError(rc, self.last_error())

    def tune_raw(self, probs, f, m, tol, prec=FP64, dtype=R64, reps=3, stream=None):
        """pfm_tune on a list of Problem: returns (policy, ms per call)."""
        arr = (Problem * len(probs))(*probs)
        pol, ms = ctypes.c_int(), ctypes.c_double()
        rc = lib().pfm_tune(self._h, f, m, tol, prec, dtype, len(probs), arr, reps, _stream_ptr(stream),
                            ctypes.byref(pol), ctypes.byref(ms))
        if rc:
            raise PfmError(rc, self.last_error())
        return pol.value, ms.value

    def tune_export(self):
        """The tuned policy table as text ("key policy" lines)."""
        n = lib().pfm_tune_export(self._h, None, 0)
        buf = ctypes.create_string_buffer(n)
        lib().pfm_tune_export(self._h, buf, n)
        return buf.value.decode()

    def tune_import(self, text):
        rc = lib().pfm_tune_import(self._h, text.encode())
        if rc:
            raise PfmError(rc, self.last_error())

    def lu_factors(self, instance, shift):
        """(lu, ipiv): the stored pivoting-LU factors of one (instance, shift)
        of the last eval call, npad x npad (row index first; off-diagonal
        16 x 16 blocks multiplied by the inverse of their column's diagonal
        block, as pfm_lu_factors documents) and the 0-based LAPACK pivots."""
        npad = ctypes.c_int32(0)
        rc = lib().pfm_lu_factors(self._h, instance, shift, None, 0, None, ctypes.byref(npad))
        if rc:
            raise PfmError(rc, self.last_error())
        np_ = npad.value
        lu = np.zeros(np_ * np_, dtype=np.float64)
        ipiv = np.zeros(np_, dtype=np.int32)
        rc = lib().pfm_lu_factors(self._h, instance, shift, lu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), np_,
                                  ipiv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None)
        if rc:
            raise PfmError(rc, self.last_error())
        return lu.reshape(np_, np_).T.copy(), ipiv

    def set_graphs(self, enable):
        """Capture and replay repeated launch sequences as hipGraphs."""
        rc = lib().pfm_set_graphs(self._h, 1 if enable else 0)
        if rc:
            raise PfmError(rc, self.last_error())

    def graph_stats(self):
        """(captures, replays) since the context was created."""
        c, r = ctypes.c_int(), ctypes.c_int()
        lib().pfm_graph_stats(self._h, ctypes.byref(c), ctypes.byref(r))
        return c.value, r.value

    def profile(self, enable=True):
        rc = lib().pfm_profile(self._h, 1 if enable else 0)
        if rc:
            raise PfmError(rc, self.last_error())

    PHASES = ("lu", "solve_combine", "square", "store")

    def profile_read(self):
        """{phase: (total_ms, launches)} and the number of timed calls."""
        ms = (ctypes.c_double * 4)()
        ln = (ctypes.c_int * 4)()
        calls = ctypes.c_int()
        rc = lib().pfm_profile_read(self._h, ctypes.cast(ms, ctypes.POINTER(ctypes.c_double)),
                                    ctypes.cast(ln, ctypes.POINTER(ctypes.c_int)), ctypes.byref(calls))
        if rc:
            raise PfmError(rc, self.last_error())
        return {p: (ms[i], ln[i]) for i, p in enumerate(self.PHASES)}, calls.value

    def last_error(self):
        return lib().pfm_last_error(self._h).decode()

    def check(self, stream=None):
        rc = lib().pfm_check(self._h, _stream_ptr(stream))
        if rc:
            raise PfmError(rc, self.last_error())

    def eval_batched(self, probs, f, m, tol, prec=FP64, dtype=R64, info=None, force_plan=-1,
                     stream=None):
        """Raw call: ``probs`` is a list of Problem; ``info`` a device tensor of
        len(probs) * 48 bytes or None; ``tol`` a float, or one per problem.
        Returns the C return code."""
        arr = (Problem * len(probs))(*probs)
        iptr = ctypes.c_void_p(info.data_ptr()) if info is not None else ctypes.c_void_p()
        if isinstance(tol, (list, tuple, np.ndarray)):
            tarr = (ctypes.c_double * len(probs))(*[float(x) for x in tol])
            return lib().pfm_eval_batched_tols(self._h, f, m, tarr, 0.5, prec, dtype, len(probs), arr, iptr,
                                               force_plan, _stream_ptr(stream))
        return lib().pfm_eval_batched(self._h, f, m, tol, prec, dtype, len(probs), arr, iptr,
                                      force_plan, _stream_ptr(stream))


    def tri_action(self, probs, f, m, tol, info=None, force_plan=-1, stream=None, noalloc=False):
        """Raw call of pfm_tri_action (``noalloc``: pfm_tri_action_noalloc):
        ``probs`` is a list of TriProblem.  Returns the C return code."""
        arr = (TriProblem * len(probs))(*probs)
        iptr = ctypes.c_void_p(info.data_ptr()) if info is not None else ctypes.c_void_p()
        fn = lib().pfm_tri_action_noalloc if noalloc else lib().pfm_tri_action
        return fn(self._h, f, m, tol, len(probs), arr, iptr, force_plan, _stream_ptr(stream))

    def band_action(self, probs, f, m, tol, b, info=None, force_plan=-1, stream=None):
        """Raw call of pfm_band_action: ``probs`` is a list of BandProblem.
        Returns the C return code."""
        arr = (BandProblem * len(probs))(*probs)
        iptr = ctypes.c_void_p(info.data_ptr()) if info is not None else ctypes.c_void_p()
        return lib().pfm_band_action(self._h, f, m, tol, b, len(probs), arr, iptr, force_plan,
                                     _stream_ptr(stream))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _fmask(funcs):
    m = 0
    for f in funcs:
        m |= {"exp": EXP, "phi1": PHI1, "log1m": LOG1M, "phi2": PHI2}[f]
    return m


_default_ctx = {}


def default_context(device=0):
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def _require_gpu(t):
    if not t.is_cuda:
        raise ValueError("pfm operates on GPU tensors only (no CPU path)")


def expm(A, funcs=("exp",), m=8, tol=1e-12, prec="fp64", force_plan=-1, ctx=None, stream=None,
         out=None, info_out=None):
    """f(A) for every matrix of ``A``.

    ``A`` is a CUDA tensor (batch, n, n) or a list of CUDA tensors (n_i, n_i),
    float64 or complex128, rows contiguous.  Returns (results, info) where
    results maps each requested function to a tensor (or list) like ``A`` and
    info is a numpy structured array (after a stream synchronisation)."""
    import torch
    mats = list(A) if isinstance(A, (list, tuple)) else [A[i] for i in range(A.shape[0])]
    for a in mats:
        _require_gpu(a)
        if a.dim() != 2 or a.shape[0] != a.shape[1] or a.stride(1) != 1:
            raise ValueError("each A must be square with unit column stride")
        if a.dtype != mats[0].dtype or a.dtype not in (torch.float64, torch.complex128):
            raise ValueError("every A must be float64, or every A complex128")
    cplx = mats[0].is_complex()
    fm = _fmask(funcs)
    if out is None:
        out = {}
        for f in funcs:
            if isinstance(A, (list, tuple)):
                out[f] = [torch.empty_like(a) for a in mats]
            else:
                out[f] = torch.empty_like(A)
    outs = {f: (list(out[f]) if isinstance(out[f], (list, tuple)) else [out[f][i] for i in range(len(mats))])
            for f in funcs}
    probs = []
    for i, a in enumerate(mats):
        # log(1 - A) is written to the F_exp slot
        fe = outs["exp"][i] if "exp" in funcs else (outs["log1m"][i] if "log1m" in funcs else None)
        fp = outs["phi1"][i] if "phi1" in funcs else None
        fq = outs["phi2"][i] if "phi2" in funcs else None
        _check_outputs(fe, fp, a.shape, a.dtype, fq)
        ldf = next(o for o in (fe, fp, fq) if o is not None).stride(0)
        probs.append(Problem(a.shape[0], 0, a.stride(0), 0, ldf, a.data_ptr(), None,
                             fe.data_ptr() if fe is not None else None,
                             fp.data_ptr() if fp is not None else None,
                             fq.data_ptr() if fq is not None else None))
    ctx = ctx or default_context(mats[0].device.index or 0)
    info = _info_buffer(info_out, len(mats), mats[0].device)
    rc = ctx.eval_batched(probs, fm, m, tol, {"fp64": FP64, "mixed": MIXED}[prec],
                          C128 if cplx else R64, info, force_plan, stream)
    if rc:
        raise PfmError(rc, ctx.last_error())
    return out, _Info(info)


def _check_outputs(fe, fp, shape, dtype, fq=None):
    """The result tensors of one instance: on the GPU, of the instance's shape
    and element type, unit column stride, and one row stride for all
    functions (the library writes them with the same leading dimension)."""
    present = [o for o in (fe, fp, fq) if o is not None]
    for o in present:
        _require_gpu(o)
        if o.dtype != dtype or tuple(o.shape) != tuple(shape) or o.stride(1) != 1:
            raise ValueError("each output must be a %s tensor of shape %s with unit column stride"
                             % (dtype, tuple(shape)))
    if len({o.stride(0) for o in present}) > 1:
        raise ValueError("the outputs of one instance must share their row stride")


def _info_buffer(info_out, count, device):
    import torch
    nbytes = count * INFO_DTYPE.itemsize
    if info_out is None:
        return torch.empty(nbytes, dtype=torch.uint8, device=device)
    if info_out.dtype != torch.uint8 or info_out.numel() < nbytes or not info_out.is_cuda:
        raise ValueError("info_out must be a CUDA uint8 tensor of at least %d bytes" % nbytes)
    return info_out


def action(A, V, funcs=("exp",), m=8, tol=1e-12, prec="fp64", force_plan=-1, ctx=None, stream=None,
           out=None, info_out=None):
    """f(A) V for every (A, V) pair (lists or batched tensors).  ``out`` may
    map each function to a list of output tensors shaped like the V's."""
    import torch
    mats = list(A) if isinstance(A, (list, tuple)) else [A[i] for i in range(A.shape[0])]
    vecs = list(V) if isinstance(V, (list, tuple)) else [V[i] for i in range(V.shape[0])]
    if len(mats) != len(vecs):
        raise ValueError("one V per A")
    for a, v in zip(mats, vecs):
        _require_gpu(a)
        _require_gpu(v)
        if a.dim() != 2 or a.shape[0] != a.shape[1] or a.stride(1) != 1:
            raise ValueError("each A must be square with unit column stride")
        if v.dim() != 2 or v.shape[0] != a.shape[0] or v.stride(1) != 1:
            raise ValueError("each V must be (n, p) with unit column stride")
        if a.dtype not in (torch.float64, torch.complex128) or v.dtype not in (torch.float64, torch.complex128):
            raise ValueError("A and V must be float64 or complex128")
    cplx = mats[0].is_complex() or vecs[0].is_complex()
    if cplx:  # one element type per call: complex A and V (interleaved)
        mats = [a if a.is_complex() else a.to(torch.complex128) for a in mats]
        vecs = [v if v.is_complex() else v.to(torch.complex128) for v in vecs]
    fm = _fmask(funcs)
    if out is None:
        out = {f: [torch.empty_like(v) for v in vecs] for f in funcs}
    probs = []
    for i, (a, v) in enumerate(zip(mats, vecs)):
        fe = out["exp"][i] if "exp" in funcs else (out["log1m"][i] if "log1m" in funcs else None)
        fp = out["phi1"][i] if "phi1" in funcs else None
        _check_outputs(fe, fp, v.shape, v.dtype)
        ldf = (fe if fe is not None else fp).stride(0)
        probs.append(Problem(a.shape[0], v.shape[1], a.stride(0), v.stride(0), ldf, a.data_ptr(),
                             v.data_ptr(), fe.data_ptr() if fe is not None else None,
                             fp.data_ptr() if fp is not None else None))
    ctx = ctx or default_context(mats[0].device.index or 0)
    info = _info_buffer(info_out, len(mats), mats[0].device)
    rc = ctx.eval_batched(probs, fm, m, tol, {"fp64": FP64, "mixed": MIXED}[prec],
                          C128 if cplx else R64, info, force_plan, stream)
    if rc:
        raise PfmError(rc, ctx.last_error())
    return out, _Info(info)


def rational(A, c, w, a0, conj_pairs=True, V=None, ctx=None, stream=None, out=None, info_out=None):
    """r(A) (V None) or r(A) V for a caller-given partial-fraction set
    (pfm_eval_rational): r(x) = a0 + sum_k w_k x / (1 - c_k x), with c and w
    sequences of (complex) numbers; with ``conj_pairs`` each complex shift
    also stands for its conjugate.  ``A`` (and ``V``) are lists of CUDA
    tensors, float64 or complex128.  Returns (list of results, info)."""
    import torch
    mats = list(A)
    vecs = None if V is None else list(V)
    for a in mats + (vecs or []):
        _require_gpu(a)
        if a.dtype not in (torch.float64, torch.complex128) or a.stride(-1) != 1:
            raise ValueError("A and V must be float64 or complex128 with unit column stride")
    cplx = any(t.is_complex() for t in mats + (vecs or []))
    if cplx:
        mats = [a.to(torch.complex128) for a in mats]
        vecs = None if vecs is None else [v.to(torch.complex128) for v in vecs]
    like = mats if vecs is None else vecs
    if out is None:
        out = [torch.empty_like(x) for x in like]
    probs = []
    for i, a in enumerate(mats):
        if a.dim() != 2 or a.shape[0] != a.shape[1]:
            raise ValueError("each A must be square")
        v = None if vecs is None else vecs[i]
        if v is not None and (v.dim() != 2 or v.shape[0] != a.shape[0]):
            raise ValueError("each V must be (n, p)")
        o = out[i]
        if o.shape != like[i].shape or o.dtype != like[i].dtype or o.stride(-1) != 1:
            raise ValueError("outputs must match A (or V) in shape and dtype")
        probs.append(Problem(a.shape[0], 0 if v is None else v.shape[1], a.stride(0), 0 if v is None else v.stride(0),
                             o.stride(0), a.data_ptr(), None if v is None else v.data_ptr(), o.data_ptr(), None))
    k = len(c)
    if k != len(w):
        raise ValueError("one weight per shift")
    arr = lambda xs: (ctypes.c_double * max(1, k))(*xs)
    cr, ci = arr([complex(x).real for x in c]), arr([complex(x).imag for x in c])
    wr, wi = arr([complex(x).real for x in w]), arr([complex(x).imag for x in w])
    ctx = ctx or default_context(mats[0].device.index or 0)
    info = _info_buffer(info_out, len(mats), mats[0].device)
    pa = (Problem * len(probs))(*probs)
    cast = lambda a: ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
    rc = lib().pfm_eval_rational(ctx.handle, k, cast(cr), cast(ci), cast(wr), cast(wi), float(a0),
                                 1 if conj_pairs else 0, C128 if cplx else R64, len(probs), pa,
                                 ctypes.c_void_p(info.data_ptr()), _stream_ptr(stream))
    if rc:
        raise PfmError(rc, ctx.last_error())
    return out, _Info(info)


def tri_action(dl, dd, du, V, funcs=("exp",), m=8, tol=1e-12, force_plan=-1, ctx=None, stream=None,
               out=None, info_out=None, noalloc=False):
    """f(A) V for tridiagonal A (float64): ``dl``, ``dd``, ``du`` are lists of
    CUDA tensors (sub-, main and superdiagonal of each instance, lengths
    d - 1, d, d - 1) and ``V`` a list of (d, p) CUDA tensors with unit
    column stride.  Returns (results, info) like ``action``.  ``noalloc``
    calls the allocation-free entry point (the library's fixed scratch
    array; pass ``out`` and ``info_out`` as well for a call in which nothing
    is allocated)."""
    import torch
    dls, dds, dus, vecs = list(dl), list(dd), list(du), list(V)
    if not (len(dls) == len(dds) == len(dus) == len(vecs)):
        raise ValueError("one set of diagonals per V")
    for t in dls + dds + dus + vecs:
        _require_gpu(t)
        if t.dtype != torch.float64:
            raise ValueError("the tridiagonal path is float64")
    for a, b, c, v in zip(dls, dds, dus, vecs):
        dlen = b.numel()
        if a.numel() != dlen - 1 or c.numel() != dlen - 1 or not (a.is_contiguous() and b.is_contiguous()
                                                                 and c.is_contiguous()):
            raise ValueError("diagonals must be contiguous with lengths d - 1, d, d - 1")
        if v.dim() != 2 or v.shape[0] != dlen or v.stride(1) != 1:
            raise ValueError("each V must be (d, p) with unit column stride")
    fm = _fmask(funcs)
    if out is None:
        out = {f: [torch.empty_like(v) for v in vecs] for f in funcs}
    probs = []
    for i, (a, b, c, v) in enumerate(zip(dls, dds, dus, vecs)):
        fe = out["exp"][i] if "exp" in funcs else None
        fp = out["phi1"][i] if "phi1" in funcs else None
        _check_outputs(fe, fp, v.shape, torch.float64)
        ldf = (fe if fe is not None else fp).stride(0)
        probs.append(TriProblem(b.numel(), v.shape[1], v.stride(0), ldf,
                                a.data_ptr() if a.numel() else None, b.data_ptr(),
                                c.data_ptr() if c.numel() else None, v.data_ptr(),
                                fe.data_ptr() if fe is not None else None,
                                fp.data_ptr() if fp is not None else None))
    ctx = ctx or default_context(vecs[0].device.index or 0)
    info = _info_buffer(info_out, len(vecs), vecs[0].device)
    rc = ctx.tri_action(probs, fm, m, tol, info, force_plan, stream, noalloc=noalloc)
    if rc:
        raise PfmError(rc, ctx.last_error())
    return out, _Info(info)


def band_action(bands, V, b, funcs=("exp",), m=8, tol=1e-12, force_plan=-1, ctx=None, stream=None,
                out=None, info_out=None):
    """f(A) V for banded A (float64, half-bandwidth b; b = 2 is pentadiagonal):
    ``bands`` is a list of contiguous (2b + 1, d) CUDA tensors with
    bands[b + o, i] = A[i, i + o] (entries outside A are never read) and ``V``
    a list of (d, p) CUDA tensors with unit column stride.  Returns
    (results, info) like ``action``."""
    import torch
    bl, vecs = list(bands), list(V)
    if len(bl) != len(vecs):
        raise ValueError("one set of bands per V")
    for t in bl + vecs:
        _require_gpu(t)
        if t.dtype != torch.float64:
            raise ValueError("the banded path is float64")
    for a, v in zip(bl, vecs):
        if a.dim() != 2 or a.shape[0] != 2 * b + 1 or not a.is_contiguous():
            raise ValueError("bands must be contiguous (2b + 1, d)")
        if v.dim() != 2 or v.shape[0] != a.shape[1] or v.stride(1) != 1:
            raise ValueError("each V must be (d, p) with unit column stride")
    fm = _fmask(funcs)
    if out is None:
        out = {f: [torch.empty_like(v) for v in vecs] for f in funcs}
    probs = []
    for i, (a, v) in enumerate(zip(bl, vecs)):
        fe = out["exp"][i] if "exp" in funcs else None
        fp = out["phi1"][i] if "phi1" in funcs else None
        _check_outputs(fe, fp, v.shape, torch.float64)
        ldf = (fe if fe is not None else fp).stride(0)
        probs.append(BandProblem(v.shape[0], v.shape[1], v.stride(0), ldf, a.data_ptr(), v.data_ptr(),
                                 fe.data_ptr() if fe is not None else None,
                                 fp.data_ptr() if fp is not None else None))
    ctx = ctx or default_context(vecs[0].device.index or 0)
    info = _info_buffer(info_out, len(vecs), vecs[0].device)
    rc = ctx.band_action(probs, fm, m, tol, b, info, force_plan, stream)
    if rc:
        raise PfmError(rc, ctx.last_error())
    return out, _Info(info)


class _Info:
    """Lazily decoded per-instance info (reading it synchronises)."""

    def __init__(self, buf):
        self._buf = buf
        self._arr = None

    def get(self):
        if self._arr is None:
            self._arr = np.frombuffer(self._buf.cpu().numpy().tobytes(), dtype=INFO_DTYPE)
        return self._arr

    def __getitem__(self, k):
        return self.get()[k]


def workspace_bytes(funcs, m, prec, dtype, probs):
    """Upper bound of the workspace bytes a pfm_eval_batched call would use
    (host only; 0 for an unsupported batch)."""
    arr = (Problem * len(probs))(*probs)
    return lib().pfm_workspace_bytes(_fmask(funcs), m, {"fp64": FP64, "mixed": MIXED}[prec], dtype,
                                     len(probs), arr)


class Server:
    """Continuous-batching server (pfm_srv_* in pfm.h) on one device.

    submit() queues one request and returns its ticket; the library's
    scheduler thread admits, batches and runs requests on ``lanes``
    concurrent streams.  Inputs must stay alive until the request is done
    (the server keeps a reference); results live in library memory until
    fetch() or release()."""

    def __init__(self, device=0, lanes=4, budget_bytes=32 << 30, max_batch=256):
        h = ctypes.c_void_p()
        rc = lib().pfm_srv_start(ctypes.byref(h), device, lanes, budget_bytes, max_batch)
        if rc:
            raise PfmError(rc, "pfm_srv_start failed")
        self._h = h
        self._keep = {}
        self._meta = {}

    def submit(self, A, V=None, func="exp", m=8, tol=1e-12, prec="fp64"):
        import torch
        _require_gpu(A)
        cplx = A.is_complex() or (V is not None and V.is_complex())
        if cplx:
            A = A if A.is_complex() else A.to(torch.complex128)
            if V is not None and not V.is_complex():
                V = V.to(torch.complex128)
        n = A.shape[0]
        p = 0 if V is None else V.shape[1]
        pr = Problem(n, p, A.stride(0), 0 if V is None else V.stride(0), 0, A.data_ptr(),
                     None if V is None else V.data_ptr(), None, None)
        t = ctypes.c_uint64()
        fm = _fmask((func,) if isinstance(func, str) else func)
        rc = lib().pfm_srv_submit(self._h, ctypes.byref(pr), fm, m, tol, {"fp64": FP64, "mixed": MIXED}[prec],
                                  C128 if cplx else R64, ctypes.byref(t))
        if rc:
            raise PfmError(rc, "pfm_srv_submit rejected the request")
        self._keep[t.value] = (A, V)
        self._meta[t.value] = (n, p, cplx, fm)
        return t.value

    def poll(self, ticket):
        """(state, info, latency_s): state 0 done, 1 pending."""
        inf = np.zeros(1, dtype=INFO_DTYPE)
        lat = ctypes.c_double()
        rc = lib().pfm_srv_poll(self._h, ticket, inf.ctypes.data, ctypes.byref(lat))
        if rc < 0:
            raise PfmError(rc, "pfm_srv_poll")
        return rc, (inf[0] if rc == 0 else None), (lat.value if rc == 0 else None)

    def drain(self, max_items=4096):
        """Completed requests not reported before: list of (ticket, latency_s, status)."""
        tk = (ctypes.c_uint64 * max_items)()
        lat = (ctypes.c_double * max_items)()
        st = (ctypes.c_int * max_items)()
        k = lib().pfm_srv_drain(self._h, max_items, tk, lat, st)
        if k < 0:
            raise PfmError(k, "pfm_srv_drain")
        out = [(tk[i], lat[i], st[i]) for i in range(k)]
        for t, _, _ in out:
            self._keep.pop(t, None)
        return out

    def timing(self, ticket):
        """Where a finished request's latency went, in seconds: (admission wait,
        wait for a lane, host enqueue, enqueue end to completion seen); None
        while it runs."""
        parts = (ctypes.c_double * 4)()
        rc = lib().pfm_srv_timing(self._h, ticket, parts)
        if rc < 0:
            raise PfmError(rc, "pfm_srv_timing")
        return None if rc == 1 else tuple(parts)

    def fetch(self, ticket, func="exp"):
        """The result as a new CUDA tensor (the request keeps it until release)."""
        import torch
        n, p, cplx, _ = self._meta[ticket]
        out = torch.empty((n, p if p else n), dtype=torch.complex128 if cplx else torch.float64, device="cuda")
        rc = lib().pfm_srv_fetch(self._h, ticket, {"exp": EXP, "phi1": PHI1}[func], out.data_ptr(), out.stride(0))
        if rc:
            raise PfmError(rc, "pfm_srv_fetch")
        return out

    def release(self, ticket):
        rc = lib().pfm_srv_release(self._h, ticket)
        if rc:
            raise PfmError(rc, "pfm_srv_release")
        self._keep.pop(ticket, None)
        self._meta.pop(ticket, None)

    def stats(self):
        v = [ctypes.c_uint64() for _ in range(5)]
        ls = ctypes.c_double()
        rc = lib().pfm_srv_stats(self._h, *[ctypes.byref(x) for x in v], ctypes.byref(ls))
        keys = ("submitted", "done", "batches", "resident_bytes", "peak_resident_bytes")
        d = {k: x.value for k, x in zip(keys, v)}
        d["launch_s"] = ls.value
        d["error"] = rc
        return d

    def stop(self):
        if self._h:
            lib().pfm_srv_stop(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def tune(A, V=None, funcs=("exp",), m=8, tol=1e-12, prec="fp64", reps=3, ctx=None, stream=None):
    """Autotune the route policy for batches like (A, V) (lists of CUDA
    tensors; V None for f(A)).  Returns (policy, ms per call); later calls
    on ``ctx`` with batches of the same key use the chosen policy."""
    import torch
    mats = list(A)
    cplx = mats[0].is_complex() or (V is not None and V[0].is_complex())
    outs, probs = [], []
    for i, a in enumerate(mats):
        v = None if V is None else V[i]
        like = a if v is None else v
        fe = torch.empty_like(like) if "exp" in funcs else None
        fp = torch.empty_like(like) if "phi1" in funcs else None
        outs.append((fe, fp))
        probs.append(Problem(a.shape[0], 0 if v is None else v.shape[1], a.stride(0),
                             0 if v is None else v.stride(0), like.stride(0), a.data_ptr(),
                             None if v is None else v.data_ptr(),
                             fe.data_ptr() if fe is not None else None,
                             fp.data_ptr() if fp is not None else None))
    ctx = ctx or default_context(mats[0].device.index or 0)
    return ctx.tune_raw(probs, _fmask(funcs), m, tol, {"fp64": FP64, "mixed": MIXED}[prec],
                        C128 if cplx else R64, reps, stream)
