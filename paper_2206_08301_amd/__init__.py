"""MI355X (gfx950) MTTKRP / TTMc library -- the local multilinear kernels of
Deinsum (Ziogas et al., arXiv 2206.08301), behind the C ABI of
include/deinsum.h.

This module marshals torch device tensors to that ABI; every arithmetic step
runs in the library's HIP kernels.  torch provides device memory and streams
only.

    import paper_2206_08301_amd as dn
    M = dn.einsum("ijk,ja,ka->ia", X, B, C)                 # MTTKRP (Tab. IV)
    Y = dn.einsum("ijk,jb,kc->ibc", X, B, C)                # TTMc
    M32 = dn.einsum("ijk,ja,ka->ia", X32, B32, C32, precision="fp32")
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import DeinsumError, Report, Spec  # noqa: F401

MTTKRP = 1
TTMC = 2
MTTKRP_MM = 3
F64, F32, BF16, FX20_STORAGE = 0, 1, 2, 3
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "fx20": 4, "auto": 5}
PRECISION_NAMES = {v: k for k, v in PRECISIONS.items()}
STORAGE_NAMES = {F64: "f64", F32: "f32", BF16: "bf16", FX20_STORAGE: "fx20"}
_X_DTYPE = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.bfloat16, "bf16x3": torch.float32,
            "fx20": None}
_U_DTYPE = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.float32, "bf16x3": torch.float32,
            "fx20": torch.float32}
_DT_CODE = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
DIST = {"uniform": 0, "int5": 1, "int3": 2}


def version() -> str:
    return _lib.load().deinsum_version().decode()


def parse(spec: str) -> Spec:
    """Parse an MTTKRP / TTMc einsum (host only)."""
    s = Spec()
    _lib.check(_lib.load().deinsum_parse(spec.encode(), ctypes.byref(s)))
    return s


def _spec(spec) -> Spec:
    return parse(spec) if isinstance(spec, str) else spec


def _i64(vals):
    return (ctypes.c_int64 * max(1, len(vals)))(*[int(v) for v in vals])


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _opts(precision, out_dtype, workspace, plan_hint, split_hint, report, tol=None, x_dtype=None, u_dtype=None):
    o = _lib.Opts()
    _lib.load().deinsum_opts_init(ctypes.byref(o))
    o.precision = PRECISIONS[precision]
    o.out_dtype = _DT_CODE[out_dtype]
    if tol is not None:
        o.tol = float(tol)
    if x_dtype is not None:
        o.x_dtype = int(x_dtype)
    if u_dtype is not None:
        o.u_dtype = int(u_dtype)
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.plan_hint = int(plan_hint)
    o.split_hint = int(split_hint)
    if report is not None:
        o.report = ctypes.pointer(report)
    return o


class FX20:
    """X in FX20 storage (20-bit fixed point in an FP16 and an int8 plane, one power-of-two
    scale; layout in include/deinsum.h): ``buf`` is the uint8 device buffer, ``shape`` the
    tensor's shape."""

    def __init__(self, buf: torch.Tensor, shape):
        self.buf = buf
        self.shape = tuple(int(d) for d in shape)

    def dim(self):
        return len(self.shape)

    def numel(self):
        n = 1
        for d in self.shape:
            n *= d
        return n

    @property
    def device(self):
        return self.buf.device

    def header(self) -> dict:
        """Header fields (copies 40 bytes to the host), with the storage error
        ||X - X_fx20|| / ||X|| and rms(X) derived from the recorded sums."""
        import math
        import struct
        raw = bytes(self.buf[:40].cpu().numpy().tobytes())
        magic, e, count, mx, ssq, esq = struct.unpack("<IiqdQQ", raw)
        rel = math.sqrt(esq / ssq) * 2.0 ** -21 if ssq else 0.0
        rms = math.sqrt(ssq * 2.0 ** -24 / count) * 2.0 ** (e + 19) if count else 0.0
        return {"magic": magic, "exp2": e, "count": count, "max_abs": mx, "sumsq_q": ssq, "errsq_q": esq,
                "storage_rel_err": rel, "rms": rms}


def fx20_size(count: int) -> int:
    n = ctypes.c_size_t(0)
    _lib.check(_lib.load().deinsum_fx20_size(int(count), ctypes.byref(n)))
    return n.value


def to_fx20(X: torch.Tensor, stream=None) -> FX20:
    """Encode an FP64 or FP32 device tensor into FX20 storage (on the device)."""
    if X.device.type != "cuda" or not X.is_contiguous() or X.dtype not in (torch.float64, torch.float32):
        raise TypeError("to_fx20 needs a contiguous FP64 or FP32 device tensor")
    nbytes = fx20_size(X.numel())
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=X.device)
    off = (-buf.data_ptr()) % 256  # the caching allocator aligns to 512; kept general
    buf = buf[off:off + nbytes]
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_fx20_encode(ctypes.c_void_p(X.data_ptr()), _DT_CODE[X.dtype], X.numel(),
                                                   ctypes.c_void_p(buf.data_ptr()), nbytes, _stream(stream)))
    return FX20(buf, X.shape)


def _storage_code(X):
    """opts.x_dtype of X: its dtype, or FX20 for an FX20 buffer."""
    if isinstance(X, FX20):
        return FX20_STORAGE
    if not isinstance(X, torch.Tensor) or X.dtype not in _DT_CODE:
        raise TypeError("X must be a float64 / float32 / bfloat16 device tensor or an FX20 buffer")
    return _DT_CODE[X.dtype]


def _x_check(X, precision):
    if precision == "fx20":
        if not isinstance(X, FX20):
            raise TypeError("the fx20 form takes X from to_fx20()")
    elif precision == "auto":
        if not isinstance(X, FX20):
            if not isinstance(X, torch.Tensor) or X.device.type != "cuda" or not X.is_contiguous():
                raise TypeError("X must be a contiguous CUDA (HIP) tensor or an FX20 buffer")
            _storage_code(X)
    else:
        _check_tensor(X, _X_DTYPE[precision], "X")


def _u_dtype_for(precision, U):
    if precision != "auto":
        return _U_DTYPE[precision]
    dt = U[0].dtype
    if dt not in (torch.float64, torch.float32):
        raise TypeError("factors must be float64 or float32")
    return dt


def _check_tensor(t, dtype, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} for this precision, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")


def _default_out_dtype(precision):
    return torch.float64 if precision in ("fp64", "auto") else torch.float32


def workspace_size(spec, dims, ranks, precision="fp64", out_dtype=None, plan_hint=0, split_hint=0) -> int:
    sp = _spec(spec)
    out_dtype = out_dtype or _default_out_dtype(precision)
    o = _opts(precision, out_dtype, None, plan_hint, split_hint, None)
    n = ctypes.c_size_t(0)
    _lib.check(_lib.load().deinsum_workspace_size(ctypes.byref(sp), _i64(dims), _i64(ranks),
                                                  ctypes.byref(o), ctypes.byref(n)))
    return int(n.value)


def mttkrp(spec, X, U, precision="fp64", out=None, out_dtype=None, workspace=None, plan_hint=0,
           split_hint=0, report=None, stream=None, tol=None, _entry="deinsum_mttkrp"):
    """Mode-n MTTKRP.  ``U`` lists the factor operands in the spec's operand order.
    ``precision="auto"`` with ``tol`` lets the library pick the cheapest form that reads
    X's storage (its dtype, or an FX20 buffer) within the tolerance; ``report`` then
    names the form (``report.precision``) and its estimated error (``report.est_err``).
    ``workspace=None`` takes the library pool's buffer for the device and ``stream``
    (calls on different streams never share one); a caller workspace is the caller's
    to order across streams."""
    sp = _spec(spec)
    if sp.kind != MTTKRP:
        raise ValueError("spec is not an MTTKRP")
    _x_check(X, precision)
    udt = _u_dtype_for(precision, U)
    if X.dim() != sp.order:
        raise ValueError(f"X has {X.dim()} modes, spec has {sp.order}")
    if len(U) != sp.n_factors:
        raise ValueError(f"expected {sp.n_factors} factors, got {len(U)}")
    R = None
    for k, u in enumerate(U):
        _check_tensor(u, udt, f"U[{k}]")
        m = sp.factor_mode[k]
        if u.dim() != 2 or u.shape[0] != X.shape[m]:
            raise ValueError(f"factor {k} must be {X.shape[m]} x R")
        R = u.shape[1] if R is None else R
        if u.shape[1] != R:
            raise ValueError("MTTKRP factors must share one rank")
    out_dtype = out_dtype or (out.dtype if out is not None else _default_out_dtype(precision))
    n = sp.free_mode
    if out is None:
        out = torch.empty((X.shape[n], R), dtype=out_dtype, device=X.device)
    else:
        _check_tensor(out, out_dtype, "out")
        if tuple(out.shape) != (X.shape[n], R):
            raise ValueError("out has the wrong shape")
    ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
    o = _opts(precision, out_dtype, workspace, plan_hint, split_hint, report, tol=tol,
              x_dtype=_storage_code(X), u_dtype=_DT_CODE[udt])
    xptr = X.buf.data_ptr() if isinstance(X, FX20) else X.data_ptr()
    with torch.cuda.device(X.device):
        _lib.check(getattr(_lib.load(), _entry)(ctypes.byref(sp), _i64(X.shape), R, ctypes.c_void_p(xptr),
                                                ptrs, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o),
                                                _stream(stream)))
    return out


def mttkrp_noalloc(spec, X, U, precision="fp64", out=None, out_dtype=None, plan_hint=0, split_hint=0,
                   report=None, stream=None, tol=None):
    """deinsum_mttkrp_noalloc: the MTTKRP with its workspace in the library's fixed
    per-device scratch array (no device allocation by the library; ``out`` is allocated
    here by torch when not given).  Problems whose plan needs more than
    NOALLOC_SCRATCH_BYTES of workspace raise DeinsumError (NO_MEMORY)."""
    return mttkrp(spec, X, U, precision=precision, out=out, out_dtype=out_dtype, workspace=None,
                  plan_hint=plan_hint, split_hint=split_hint, report=report, stream=stream, tol=tol,
                  _entry="deinsum_mttkrp_noalloc")


NOALLOC_SCRATCH_BYTES = 64 << 20


def tune_mttkrp(spec, X, U, precision="fp64", out=None, out_dtype=None, reps=5, batched=False, stream=None,
                tol=None):
    """Autotune the MTTKRP plan for this problem (runs it; ``out`` is overwritten) and
    cache the fastest; later calls with the same shape use it.  Returns the winner's Report."""
    sp = _spec(spec)
    if sp.kind != MTTKRP:
        raise ValueError("spec is not an MTTKRP")
    _x_check(X, precision)
    udt = _u_dtype_for(precision, U)
    R = U[0].shape[1]
    for k, u in enumerate(U):
        _check_tensor(u, udt, f"U[{k}]")
    out_dtype = out_dtype or (out.dtype if out is not None else _default_out_dtype(precision))
    if out is None:
        out = torch.empty((X.shape[sp.free_mode], R), dtype=out_dtype, device=X.device)
    ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
    o = _opts(precision, out_dtype, None, 0, 0, None, tol=tol, x_dtype=_storage_code(X), u_dtype=_DT_CODE[udt])
    rep = Report()
    fn = _lib.load().deinsum_tune_batch_mttkrp if batched else _lib.load().deinsum_tune_mttkrp
    xptr = X.buf.data_ptr() if isinstance(X, FX20) else X.data_ptr()
    with torch.cuda.device(X.device):
        _lib.check(fn(ctypes.byref(sp), _i64(X.shape), R, ctypes.c_void_p(xptr), ptrs,
                      ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), int(reps), ctypes.byref(rep),
                      _stream(stream)))
    return rep


def tune_load(path: str):
    _lib.check(_lib.load().deinsum_tune_load(str(path).encode()))


def tune_save(path: str):
    _lib.check(_lib.load().deinsum_tune_save(str(path).encode()))


def tune_clear():
    _lib.check(_lib.load().deinsum_tune_clear())


def tune_entries() -> int:
    n = ctypes.c_int64(0)
    _lib.check(_lib.load().deinsum_tune_entries(ctypes.byref(n)))
    return n.value


def ttmc(spec, X, U, precision="fp64", out=None, out_dtype=None, workspace=None, report=None, stream=None,
         variant=None, tune_reps=0, tol=None):
    """Mode-n TTMc.  ``U`` lists the factor operands in the spec's operand order.
    ``variant`` picks a compiled fused kernel for the ranks (None = the autotuned one if
    cached, else the default); ``tune_reps`` > 0 autotunes first (``out`` is overwritten).
    ``workspace=None`` takes the library pool's buffer for the device and ``stream``
    (calls on different streams never share one); a caller workspace is the caller's
    to order across streams."""
    sp = _spec(spec)
    if sp.kind != TTMC:
        raise ValueError("spec is not a TTMc")
    _x_check(X, precision)
    udt = _u_dtype_for(precision, U)
    if X.dim() != sp.order or len(U) != sp.n_factors:
        raise ValueError("operand count or order does not match the spec")
    ranks = []
    shape = list(X.shape)
    for k, u in enumerate(U):
        _check_tensor(u, udt, f"U[{k}]")
        m = sp.factor_mode[k]
        if u.dim() != 2 or u.shape[0] != X.shape[m]:
            raise ValueError(f"factor {k} must be {X.shape[m]} x R_{m}")
        ranks.append(u.shape[1])
        shape[m] = u.shape[1]
    out_dtype = out_dtype or (out.dtype if out is not None else _default_out_dtype(precision))
    if out is None:
        out = torch.empty(shape, dtype=out_dtype, device=X.device)
    else:
        _check_tensor(out, out_dtype, "out")
        if list(out.shape) != shape:
            raise ValueError("out has the wrong shape")
    ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
    o = _opts(precision, out_dtype, workspace, 0 if variant is None else int(variant) + 1, 0, report, tol=tol,
              x_dtype=_storage_code(X), u_dtype=_DT_CODE[udt])
    xptr = X.buf.data_ptr() if isinstance(X, FX20) else X.data_ptr()
    if tune_reps:
        rep = Report()
        with torch.cuda.device(X.device):
            _lib.check(_lib.load().deinsum_tune_ttmc(ctypes.byref(sp), _i64(X.shape), _i64(ranks),
                                                     ctypes.c_void_p(xptr), ptrs, ctypes.c_void_p(out.data_ptr()),
                                                     ctypes.byref(o), int(tune_reps), ctypes.byref(rep), _stream(stream)))
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_ttmc(ctypes.byref(sp), _i64(X.shape), _i64(ranks), ctypes.c_void_p(xptr),
                                            ptrs, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), _stream(stream)))
    return out


def mttkrp_mm(spec, X, U, C, precision="fp64", out=None, out_dtype=None, workspace=None, report=None, stream=None,
              tol=None):
    """MTTKRP followed by a matrix product, e.g. "ijk,ja,ka,al->il" (the paper's running
    example): ``U`` lists the MTTKRP factor operands, ``C`` is the R x L matrix.
    ``workspace=None`` takes the library pool's buffer for the device and ``stream``
    (calls on different streams never share one); a caller workspace is the caller's
    to order across streams."""
    sp = _spec(spec)
    if sp.kind != MTTKRP_MM:
        raise ValueError("spec is not an MTTKRP-GEMM chain")
    _x_check(X, precision)
    udt = _u_dtype_for(precision, U)
    if X.dim() != sp.order or len(U) != sp.n_factors:
        raise ValueError("operand count or order does not match the spec")
    R = None
    for k, u in enumerate(U):
        _check_tensor(u, udt, f"U[{k}]")
        m = sp.factor_mode[k]
        if u.dim() != 2 or u.shape[0] != X.shape[m] or (R is not None and u.shape[1] != R):
            raise ValueError(f"factor {k} must be {X.shape[m]} x R with one shared R")
        R = u.shape[1]
    _check_tensor(C, udt, "C")
    if C.dim() != 2 or C.shape[0] != R:
        raise ValueError("C must be R x L")
    L = C.shape[1]
    out_dtype = out_dtype or (out.dtype if out is not None else _default_out_dtype(precision))
    n = sp.free_mode
    if out is None:
        out = torch.empty((X.shape[n], L), dtype=out_dtype, device=X.device)
    else:
        _check_tensor(out, out_dtype, "out")
        if tuple(out.shape) != (X.shape[n], L):
            raise ValueError("out has the wrong shape")
    ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
    o = _opts(precision, out_dtype, workspace, 0, 0, report, tol=tol, x_dtype=_storage_code(X),
              u_dtype=_DT_CODE[udt])
    xptr = X.buf.data_ptr() if isinstance(X, FX20) else X.data_ptr()
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_mttkrp_mm(ctypes.byref(sp), _i64(X.shape), int(R), int(L),
                                                 ctypes.c_void_p(xptr), ptrs, ctypes.c_void_p(C.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), _stream(stream)))
    return out


def einsum(spec: str, X, *U, precision="fp64", out=None, **kw):
    """Dispatch an MTTKRP, TTMc or MTTKRP-GEMM einsum string (Tab. IV forms and the
    chain of Sec. II-A) to the library."""
    sp = parse(spec)
    if sp.kind == MTTKRP:
        return mttkrp(sp, X, list(U), precision=precision, out=out, **kw)
    if sp.kind == MTTKRP_MM:
        return mttkrp_mm(sp, X, list(U[:-1]), U[-1], precision=precision, out=out, **kw)
    return ttmc(sp, X, list(U), precision=precision, out=out, **kw)


def estimate_error(spec, dims, ranks, precision="fp64", X=None, tol=None, x_dtype=None, u_dtype=None, stream=None):
    """deinsum_estimate_error: (form, estimated normwise relative error).  With
    precision="auto" the form is the one AUTO picks for ``tol`` and the storage codes
    ``x_dtype`` / ``u_dtype`` (F64, F32, BF16, FX20_STORAGE); X (an FX20 buffer) is
    needed only for the FX20 form, whose header holds its storage error."""
    sp = _spec(spec)
    o = _opts(precision, torch.float64 if precision in ("fp64", "auto") else torch.float32, None, 0, 0, None,
              tol=tol, x_dtype=x_dtype, u_dtype=u_dtype)
    p = ctypes.c_int32(-1)
    e = ctypes.c_double(0)
    xptr = None
    if X is not None:
        xptr = X.buf.data_ptr() if isinstance(X, FX20) else X.data_ptr()
    _lib.check(_lib.load().deinsum_estimate_error(ctypes.byref(sp), _i64(dims), _i64(ranks), xptr, ctypes.byref(o),
                                                  ctypes.byref(p), ctypes.byref(e),
                                                  _stream(stream) if X is not None else None))
    return PRECISION_NAMES[p.value], e.value


def choose_storage(spec, dims, ranks, tol, max_abs=0.0, rms=0.0):
    """deinsum_choose_storage: (storage, form, estimate) -- the cheapest storage of X
    ("bf16", "fx20", "f32", "f64") with a form whose estimated error is within ``tol``.
    FX20 is considered only given max_abs and rms of X (tensor_stats)."""
    sp = _spec(spec)
    x = ctypes.c_int32(-1)
    p = ctypes.c_int32(-1)
    e = ctypes.c_double(0)
    _lib.check(_lib.load().deinsum_choose_storage(ctypes.byref(sp), _i64(dims), _i64(ranks), float(tol),
                                                  float(max_abs), float(rms), ctypes.byref(x), ctypes.byref(p),
                                                  ctypes.byref(e)))
    return STORAGE_NAMES[x.value], PRECISION_NAMES[p.value], e.value


def tensor_stats(X: torch.Tensor, stream=None):
    """(max |x|, rms) of a device tensor, computed on the device (synchronising)."""
    if X.device.type != "cuda" or not X.is_contiguous() or X.dtype not in _DT_CODE:
        raise TypeError("tensor_stats needs a contiguous float64 / float32 / bfloat16 device tensor")
    mx = ctypes.c_double(0)
    rms = ctypes.c_double(0)
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_tensor_stats(ctypes.c_void_p(X.data_ptr()), _DT_CODE[X.dtype], X.numel(),
                                                    ctypes.byref(mx), ctypes.byref(rms), _stream(stream)))
    return mx.value, rms.value


def prepare(X: torch.Tensor, spec, ranks, tol, stream=None):
    """Store an FP64 device tensor for a tolerance: measures max |x| and rms, asks
    choose_storage for the cheapest storage whose form meets ``tol`` on this problem,
    and returns X in it (X itself for F64; a new BF16 / FP32 tensor or FX20 buffer
    otherwise) with the storage name.  Pass the result with precision="auto", tol=tol."""
    if X.dtype != torch.float64:
        raise TypeError("prepare takes the FP64 tensor")
    mx, rms = tensor_stats(X, stream)
    storage, _, _ = choose_storage(spec, X.shape, ranks, tol, mx, rms)
    if storage == "f64":
        return X, storage
    if storage == "fx20":
        return to_fx20(X, stream), storage
    dst = torch.empty(X.shape, dtype=torch.float32 if storage == "f32" else torch.bfloat16, device=X.device)
    return convert(X, dst, stream), storage


def _decomp_opts(precision, max_sweeps, tol, max_iters, iter_tol, trace):
    o = _lib.DecompOpts()
    _lib.load().deinsum_decomp_opts_init(ctypes.byref(o))
    o.precision = PRECISIONS[precision]
    o.max_sweeps = int(max_sweeps)
    o.tol = float(tol)
    if max_iters is not None:
        o.max_iters = int(max_iters)
    if iter_tol is not None:
        o.iter_tol = float(iter_tol)
    o.fit_trace = ctypes.cast(trace, ctypes.POINTER(ctypes.c_double))
    return o


def cp_als(X, U, precision="fp64", max_sweeps=25, tol=1e-10, stream=None):
    """CP-ALS on the device (deinsum_cp_als).  ``U`` (one dims[m] x R factor per mode) is
    the starting point and is overwritten with the result.  Returns (lambda, info) with
    info = {"sweeps", "fit", "fits" (per sweep), "regularised"}."""
    _check_tensor(X, _X_DTYPE[precision], "X")
    if len(U) != X.dim():
        raise ValueError("one factor per mode is required")
    R = U[0].shape[1]
    for m, u in enumerate(U):
        _check_tensor(u, _U_DTYPE[precision], f"U[{m}]")
        if u.dim() != 2 or u.shape[0] != X.shape[m] or u.shape[1] != R:
            raise ValueError(f"factor {m} must be {X.shape[m]} x {R}")
    lam = torch.empty(R, dtype=torch.float64, device=X.device)
    trace = (ctypes.c_double * int(max_sweeps))()
    o = _decomp_opts(precision, max_sweeps, tol, None, None, trace)
    res = _lib.DecompResult()
    ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_cp_als(X.dim(), _i64(X.shape), R, ctypes.c_void_p(X.data_ptr()), ptrs,
                                              ctypes.c_void_p(lam.data_ptr()), ctypes.byref(o), ctypes.byref(res),
                                              _stream(stream)))
    return lam, {"sweeps": res.sweeps, "fit": res.fit, "fits": list(trace[:res.sweeps]),
                 "regularised": bool(res.flags & 1)}


def tucker_hooi(X, U, precision="fp64", max_sweeps=25, tol=1e-10, max_iters=None, iter_tol=None, stream=None):
    """Tucker decomposition by HOOI on the device (deinsum_tucker_hooi).  ``U`` (one
    dims[m] x R_m factor with orthonormal columns per mode) is the start and is
    overwritten.  Returns (core, info) with info = {"sweeps", "fit", "fits", "iters",
    "max_iters_hit", "rank_deficient"}."""
    _check_tensor(X, _X_DTYPE[precision], "X")
    if len(U) != X.dim():
        raise ValueError("one factor per mode is required")
    ranks = []
    for m, u in enumerate(U):
        _check_tensor(u, _U_DTYPE[precision], f"U[{m}]")
        if u.dim() != 2 or u.shape[0] != X.shape[m]:
            raise ValueError(f"factor {m} must be {X.shape[m]} x R_{m}")
        ranks.append(u.shape[1])
    core = torch.empty(ranks, dtype=torch.float64, device=X.device)
    trace = (ctypes.c_double * int(max_sweeps))()
    o = _decomp_opts(precision, max_sweeps, tol, max_iters, iter_tol, trace)
    res = _lib.DecompResult()
    ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_tucker_hooi(X.dim(), _i64(X.shape), _i64(ranks),
                                                   ctypes.c_void_p(X.data_ptr()), ptrs,
                                                   ctypes.c_void_p(core.data_ptr()), ctypes.byref(o),
                                                   ctypes.byref(res), _stream(stream)))
    return core, {"sweeps": res.sweeps, "fit": res.fit, "fits": list(trace[:res.sweeps]), "iters": res.iters,
                  "max_iters_hit": bool(res.flags & 2), "rank_deficient": bool(res.flags & 4)}


def synth_fill(t: torch.Tensor, seed: int, dist: str = "uniform", offset: int = 0, stream=None):
    """Fill ``t`` with the counter-based SplitMix64 input stream (see include/deinsum.h)."""
    if t.device.type != "cuda" or not t.is_contiguous():
        raise TypeError("synth_fill needs a contiguous device tensor")
    with torch.cuda.device(t.device):
        _lib.check(_lib.load().deinsum_synth_fill(ctypes.c_void_p(t.data_ptr()), _DT_CODE[t.dtype], t.numel(),
                                                  int(seed) & (2 ** 64 - 1), int(offset), DIST[dist],
                                                  _stream(stream)))
    return t


def convert(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Round ``src`` into ``dst`` (f64 -> f32 / bf16, f32 -> bf16; nearest even)."""
    if src.numel() != dst.numel():
        raise ValueError("size mismatch")
    with torch.cuda.device(src.device):
        _lib.check(_lib.load().deinsum_convert(ctypes.c_void_p(src.data_ptr()), _DT_CODE[src.dtype],
                                               ctypes.c_void_p(dst.data_ptr()), _DT_CODE[dst.dtype], src.numel(),
                                               _stream(stream)))
    return dst


KERNEL_KINDS = {1: "mttkrp_stream_kernel", 2: "ttmc_fused_kernel"}


def kernel_timing(enable: bool, capacity: int = 4096):
    """Start (or stop) HIP-event timing of each call's main kernel (deinsum_kernel_timing)."""
    _lib.check(_lib.load().deinsum_kernel_timing(int(bool(enable)), int(capacity)))


def kernel_times(max_n: int = 1 << 16):
    """[(kernel kind name, ms)] of the recorded launches, in launch order (synchronising)."""
    kinds = (ctypes.c_int32 * max_n)()
    ms = (ctypes.c_double * max_n)()
    n = ctypes.c_int64(0)
    _lib.check(_lib.load().deinsum_kernel_times(int(max_n), kinds, ms, ctypes.byref(n)))
    return [(KERNEL_KINDS.get(kinds[i], str(kinds[i])), ms[i]) for i in range(n.value)]


def shutdown():
    _lib.check(_lib.load().deinsum_shutdown())


def last_error() -> str:
    return _lib.load().deinsum_last_error().decode()


class Batch:
    """Many MTTKRP jobs in one persistent, graph-replayed launch (deinsum_batch_*)."""

    def __init__(self, max_jobs: int = 64):
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().deinsum_batch_create(int(max_jobs), ctypes.byref(self._h)))
        self._keep = []

    def add(self, spec, X, U, out=None, precision="fp64", out_dtype=None, split_hint=0):
        """Queue M = MTTKRP(spec, X, U); returns (job_id, M).  Nothing runs until launch()."""
        sp = _spec(spec)
        if sp.kind != MTTKRP:
            raise ValueError("spec is not an MTTKRP")
        _check_tensor(X, _X_DTYPE[precision], "X")
        R = U[0].shape[1]
        for k, u in enumerate(U):
            _check_tensor(u, _U_DTYPE[precision], f"U[{k}]")
        out_dtype = out_dtype or (out.dtype if out is not None else _default_out_dtype(precision))
        n = sp.free_mode
        if out is None:
            out = torch.empty((X.shape[n], R), dtype=out_dtype, device=X.device)
        else:
            _check_tensor(out, out_dtype, "out")
        ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
        o = _opts(precision, out_dtype, None, 0, split_hint, None)
        jid = ctypes.c_int32(-1)
        _lib.check(_lib.load().deinsum_batch_add_mttkrp(self._h, ctypes.byref(sp), _i64(X.shape), R,
                                                        ctypes.c_void_p(X.data_ptr()), ptrs,
                                                        ctypes.c_void_p(out.data_ptr()), ctypes.byref(o),
                                                        ctypes.byref(jid)))
        self._keep.append((X, tuple(U), out))
        return jid.value, out

    def launch(self, stream=None):
        _lib.check(_lib.load().deinsum_batch_launch(self._h, _stream(stream)))

    def reset(self):
        _lib.check(_lib.load().deinsum_batch_reset(self._h))
        self._keep = []

    def info(self) -> dict:
        j, u, c, l_ = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _lib.check(_lib.load().deinsum_batch_info(self._h, ctypes.byref(j), ctypes.byref(u), ctypes.byref(c),
                                                  ctypes.byref(l_)))
        return {"jobs": j.value, "units": u.value, "graph_captures": c.value, "launches": l_.value}

    def close(self):
        if self._h:
            _lib.load().deinsum_batch_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """CP-ALS request server on resident tensors (deinsum_server_*).

    Each request (tensor, mode) runs the mode's MTTKRP and the factor update
    in the library; the factors registered with ``add_tensor`` are updated in
    place.  ``batched=True`` runs continuous batching, ``False`` one launch
    per request.  ``direct_max_jobs=k`` runs an epoch of at most k requests with the
    per-request launches (lower latency; results match the batched ones within the
    form's tolerance); ``0`` keeps every result bitwise the same alone and in any mix.
    """

    def __init__(self, batched=True, max_jobs_per_epoch=256, epochs_in_flight=2, als_update=True,
                 max_requests=1 << 20, hbm_budget_bytes=4 << 30, direct_max_jobs=4):
        cfg = _lib.ServerConfig()
        _lib.load().deinsum_server_config_init(ctypes.byref(cfg))
        cfg.batched = int(bool(batched))
        cfg.max_jobs_per_epoch = int(max_jobs_per_epoch)
        cfg.epochs_in_flight = int(epochs_in_flight)
        cfg.als_update = int(bool(als_update))
        cfg.max_requests = int(max_requests)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.direct_max_jobs = int(direct_max_jobs)
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().deinsum_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._keep = []
        self._n = 0

    def add_tensor(self, X, U, precision="fp64") -> int:
        """Register X (order N) and its N factors (one per mode, dims[m] x R)."""
        if precision not in ("fp64", "fp32"):
            raise ValueError("the server takes fp64 or fp32 tensors")
        dt = torch.float64 if precision == "fp64" else torch.float32
        _check_tensor(X, dt, "X")
        if len(U) != X.dim():
            raise ValueError("one factor per mode is required")
        R = U[0].shape[1]
        for m, u in enumerate(U):
            _check_tensor(u, dt, f"U[{m}]")
            if u.dim() != 2 or u.shape[0] != X.shape[m] or u.shape[1] != R:
                raise ValueError(f"factor {m} must be {X.shape[m]} x {R}")
        ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
        tid = ctypes.c_int32(-1)
        _lib.check(_lib.load().deinsum_server_add_tensor(self._h, X.dim(), _i64(X.shape), R, PRECISIONS[precision],
                                                         ctypes.c_void_p(X.data_ptr()), ptrs, ctypes.byref(tid)))
        self._keep.append((X, tuple(U)))
        return tid.value

    def start(self):
        _lib.check(_lib.load().deinsum_server_start(self._h))

    def submit(self, tensor: int, mode: int, arrival: float = -1.0) -> int:
        rid = ctypes.c_int64(-1)
        _lib.check(_lib.load().deinsum_server_submit(self._h, int(tensor), int(mode), float(arrival),
                                                     ctypes.byref(rid)))
        self._n = max(self._n, rid.value + 1)
        return rid.value

    def replay(self, arrivals, tensors, modes):
        """Open-loop submission at the given arrival times (seconds since start)."""
        import numpy as np
        a = np.ascontiguousarray(arrivals, dtype=np.float64)
        t = np.ascontiguousarray(tensors, dtype=np.int32)
        m = np.ascontiguousarray(modes, dtype=np.int32)
        if not (len(a) == len(t) == len(m)):
            raise ValueError("arrivals, tensors and modes must have one length")
        _lib.check(_lib.load().deinsum_server_replay(
            self._h, len(a), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        self._n += len(a)

    def drain(self, check=True):
        """Wait until every submitted request has finished.  With check=True a failed
        request raises DeinsumError (after all have finished); poll() gives each one's state."""
        st = _lib.load().deinsum_server_drain(self._h)
        if check:
            _lib.check(st)
        return st

    def results(self):
        """(arrival, done, epoch) numpy arrays over all submitted requests (after drain)."""
        import numpy as np
        n = self.stats()["completed"] if self._n == 0 else self._n
        arr, done = np.zeros(n), np.zeros(n)
        ep = np.zeros(n, dtype=np.int64)
        _lib.check(_lib.load().deinsum_server_results(
            self._h, n, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            done.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ep.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return arr, done, ep

    REQUEST_STATES = {0: "done", 1: "pending", 2: "running"}

    def poll(self, request_id: int) -> dict:
        """State of one request: status ("done", "pending", "running", or the name of the
        error it failed with), its raw code, flags ({"regularised"} when the factor update
        needed the pivot floor) and completion time (seconds since start, -1 before)."""
        st, fl, done = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _lib.check(_lib.load().deinsum_server_poll(self._h, int(request_id), ctypes.byref(st), ctypes.byref(fl),
                                                   ctypes.byref(done)))
        name = self.REQUEST_STATES.get(st.value) or _lib.STATUS_NAMES.get(st.value, str(st.value))
        flags = {"regularised"} if fl.value & 1 else set()
        return {"status": name, "code": st.value, "flags": flags, "done": done.value}

    def stats(self) -> dict:
        c, e, mb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(_lib.load().deinsum_server_stats(self._h, ctypes.byref(c), ctypes.byref(e), ctypes.byref(mb)))
        return {"completed": c.value, "epochs": e.value, "max_batch": mb.value}

    def close(self):
        if self._h:
            _lib.load().deinsum_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
