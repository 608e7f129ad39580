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
F64, F32, BF16 = 0, 1, 2
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
_X_DTYPE = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.bfloat16, "bf16x3": torch.float32}
_U_DTYPE = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.float32, "bf16x3": torch.float32}
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


def _opts(precision, out_dtype, workspace, plan_hint, split_hint, report):
    o = _lib.Opts()
    _lib.load().deinsum_opts_init(ctypes.byref(o))
    o.precision = PRECISIONS[precision]
    o.out_dtype = _DT_CODE[out_dtype]
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.plan_hint = int(plan_hint)
    o.split_hint = int(split_hint)
    if report is not None:
        o.report = ctypes.pointer(report)
    return o


def _check_tensor(t, dtype, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} for this precision, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")


def _default_out_dtype(precision):
    return torch.float64 if precision == "fp64" else torch.float32


def workspace_size(spec, dims, ranks, precision="fp64", out_dtype=None, plan_hint=0, split_hint=0) -> int:
    sp = _spec(spec)
    out_dtype = out_dtype or _default_out_dtype(precision)
    o = _opts(precision, out_dtype, None, plan_hint, split_hint, None)
    n = ctypes.c_size_t(0)
    _lib.check(_lib.load().deinsum_workspace_size(ctypes.byref(sp), _i64(dims), _i64(ranks),
                                                  ctypes.byref(o), ctypes.byref(n)))
    return int(n.value)


def mttkrp(spec, X, U, precision="fp64", out=None, out_dtype=None, workspace=None, plan_hint=0,
           split_hint=0, report=None, stream=None):
    """Mode-n MTTKRP.  ``U`` lists the factor operands in the spec's operand order."""
    sp = _spec(spec)
    if sp.kind != MTTKRP:
        raise ValueError("spec is not an MTTKRP")
    _check_tensor(X, _X_DTYPE[precision], "X")
    if X.dim() != sp.order:
        raise ValueError(f"X has {X.dim()} modes, spec has {sp.order}")
    if len(U) != sp.n_factors:
        raise ValueError(f"expected {sp.n_factors} factors, got {len(U)}")
    R = None
    for k, u in enumerate(U):
        _check_tensor(u, _U_DTYPE[precision], f"U[{k}]")
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
    o = _opts(precision, out_dtype, workspace, plan_hint, split_hint, report)
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_mttkrp(ctypes.byref(sp), _i64(X.shape), R, ctypes.c_void_p(X.data_ptr()),
                                              ptrs, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o),
                                              _stream(stream)))
    return out


def ttmc(spec, X, U, precision="fp64", out=None, out_dtype=None, workspace=None, report=None, stream=None):
    """Mode-n TTMc.  ``U`` lists the factor operands in the spec's operand order."""
    sp = _spec(spec)
    if sp.kind != TTMC:
        raise ValueError("spec is not a TTMc")
    _check_tensor(X, _X_DTYPE[precision], "X")
    if X.dim() != sp.order or len(U) != sp.n_factors:
        raise ValueError("operand count or order does not match the spec")
    ranks = []
    shape = list(X.shape)
    for k, u in enumerate(U):
        _check_tensor(u, _U_DTYPE[precision], f"U[{k}]")
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
    o = _opts(precision, out_dtype, workspace, 0, 0, report)
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_ttmc(ctypes.byref(sp), _i64(X.shape), _i64(ranks), ctypes.c_void_p(X.data_ptr()),
                                            ptrs, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), _stream(stream)))
    return out


def einsum(spec: str, X, *U, precision="fp64", out=None, **kw):
    """Dispatch an MTTKRP or TTMc einsum string (Tab. IV forms) to the library."""
    sp = parse(spec)
    if sp.kind == MTTKRP:
        return mttkrp(sp, X, list(U), precision=precision, out=out, **kw)
    return ttmc(sp, X, list(U), precision=precision, out=out, **kw)


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


def shutdown():
    _lib.check(_lib.load().deinsum_shutdown())


def last_error() -> str:
    return _lib.load().deinsum_last_error().decode()
