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
F64, F32, BF16 = 0, 1, 2
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "fx20": 4}
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
        """Header fields (copies 24 bytes to the host)."""
        import struct
        raw = bytes(self.buf[:24].cpu().numpy().tobytes())
        magic, e, count, mx = struct.unpack("<Iiqd", raw)
        return {"magic": magic, "exp2": e, "count": count, "max_abs": mx}


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
           split_hint=0, report=None, stream=None, _entry="deinsum_mttkrp"):
    """Mode-n MTTKRP.  ``U`` lists the factor operands in the spec's operand order."""
    sp = _spec(spec)
    if sp.kind != MTTKRP:
        raise ValueError("spec is not an MTTKRP")
    if precision == "fx20":
        if not isinstance(X, FX20):
            raise TypeError("the fx20 form takes X from to_fx20()")
    else:
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
    xptr = X.buf.data_ptr() if isinstance(X, FX20) else X.data_ptr()
    with torch.cuda.device(X.device):
        _lib.check(getattr(_lib.load(), _entry)(ctypes.byref(sp), _i64(X.shape), R, ctypes.c_void_p(xptr),
                                                ptrs, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o),
                                                _stream(stream)))
    return out


def mttkrp_noalloc(spec, X, U, precision="fp64", out=None, out_dtype=None, plan_hint=0, split_hint=0,
                   report=None, stream=None):
    """deinsum_mttkrp_noalloc: the MTTKRP with its workspace in the library's fixed
    per-device scratch array (no device allocation by the library; ``out`` is allocated
    here by torch when not given).  Problems whose plan needs more than
    NOALLOC_SCRATCH_BYTES of workspace raise DeinsumError (NO_MEMORY)."""
    return mttkrp(spec, X, U, precision=precision, out=out, out_dtype=out_dtype, workspace=None,
                  plan_hint=plan_hint, split_hint=split_hint, report=report, stream=stream,
                  _entry="deinsum_mttkrp_noalloc")


NOALLOC_SCRATCH_BYTES = 64 << 20


def tune_mttkrp(spec, X, U, precision="fp64", out=None, out_dtype=None, reps=5, batched=False, stream=None):
    """Autotune the MTTKRP plan for this problem (runs it; ``out`` is overwritten) and
    cache the fastest; later calls with the same shape use it.  Returns the winner's Report."""
    sp = _spec(spec)
    if sp.kind != MTTKRP:
        raise ValueError("spec is not an MTTKRP")
    if precision == "fx20":
        if not isinstance(X, FX20):
            raise TypeError("the fx20 form takes X from to_fx20()")
    else:
        _check_tensor(X, _X_DTYPE[precision], "X")
    R = U[0].shape[1]
    for k, u in enumerate(U):
        _check_tensor(u, _U_DTYPE[precision], f"U[{k}]")
    out_dtype = out_dtype or (out.dtype if out is not None else _default_out_dtype(precision))
    if out is None:
        out = torch.empty((X.shape[sp.free_mode], R), dtype=out_dtype, device=X.device)
    ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
    o = _opts(precision, out_dtype, None, 0, 0, None)
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
         variant=None, tune_reps=0):
    """Mode-n TTMc.  ``U`` lists the factor operands in the spec's operand order.
    ``variant`` picks a compiled fused kernel for the ranks (None = the autotuned one if
    cached, else the default); ``tune_reps`` > 0 autotunes first (``out`` is overwritten)."""
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
    o = _opts(precision, out_dtype, workspace, 0 if variant is None else int(variant) + 1, 0, report)
    if tune_reps:
        rep = Report()
        with torch.cuda.device(X.device):
            _lib.check(_lib.load().deinsum_tune_ttmc(ctypes.byref(sp), _i64(X.shape), _i64(ranks),
                                                     ctypes.c_void_p(X.data_ptr()), ptrs, ctypes.c_void_p(out.data_ptr()),
                                                     ctypes.byref(o), int(tune_reps), ctypes.byref(rep), _stream(stream)))
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().deinsum_ttmc(ctypes.byref(sp), _i64(X.shape), _i64(ranks), ctypes.c_void_p(X.data_ptr()),
                                            ptrs, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), _stream(stream)))
    return out


def mttkrp_mm(spec, X, U, C, precision="fp64", out=None, out_dtype=None, workspace=None, report=None, stream=None):
    """MTTKRP followed by a matrix product, e.g. "ijk,ja,ka,al->il" (the paper's running
    example): ``U`` lists the MTTKRP factor operands, ``C`` is the R x L matrix."""
    sp = _spec(spec)
    if sp.kind != MTTKRP_MM:
        raise ValueError("spec is not an MTTKRP-GEMM chain")
    if precision == "fx20":
        if not isinstance(X, FX20):
            raise TypeError("the fx20 form takes X from to_fx20()")
    else:
        _check_tensor(X, _X_DTYPE[precision], "X")
    if X.dim() != sp.order or len(U) != sp.n_factors:
        raise ValueError("operand count or order does not match the spec")
    R = None
    for k, u in enumerate(U):
        _check_tensor(u, _U_DTYPE[precision], f"U[{k}]")
        m = sp.factor_mode[k]
        if u.dim() != 2 or u.shape[0] != X.shape[m] or (R is not None and u.shape[1] != R):
            raise ValueError(f"factor {k} must be {X.shape[m]} x R with one shared R")
        R = u.shape[1]
    _check_tensor(C, _U_DTYPE[precision], "C")
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
    o = _opts(precision, out_dtype, workspace, 0, 0, report)
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
    per request.
    """

    def __init__(self, batched=True, max_jobs_per_epoch=256, epochs_in_flight=2, als_update=True,
                 max_requests=1 << 20, hbm_budget_bytes=4 << 30):
        cfg = _lib.ServerConfig()
        _lib.load().deinsum_server_config_init(ctypes.byref(cfg))
        cfg.batched = int(bool(batched))
        cfg.max_jobs_per_epoch = int(max_jobs_per_epoch)
        cfg.epochs_in_flight = int(epochs_in_flight)
        cfg.als_update = int(bool(als_update))
        cfg.max_requests = int(max_requests)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
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

    def drain(self):
        _lib.check(_lib.load().deinsum_server_drain(self._h))

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
