"""ctypes declarations of libdeinsum.so (argument marshalling only).

torch is imported before the library is loaded so that libdeinsum.so binds
to the HIP runtime torch already mapped (same soname): device pointers and
stream handles then belong to one runtime.  A missing library is an error;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading libdeinsum.so)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdeinsum.so")
MAX_ORDER = 8

OK = 0
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "PARSE", -3: "UNSUPPORTED", -4: "SHAPE",
                -5: "NO_MEMORY", -6: "DEVICE", -7: "BUSY"}


class DeinsumError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"deinsum {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Spec(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("free_mode", ctypes.c_int32),
        ("n_factors", ctypes.c_int32),
        ("factor_mode", ctypes.c_int32 * MAX_ORDER),
        ("operand_of_mode", ctypes.c_int32 * MAX_ORDER),
        ("tensor_idx", ctypes.c_char * (MAX_ORDER + 1)),
        ("rank_idx", ctypes.c_char * (MAX_ORDER + 1)),
        ("out_idx", ctypes.c_char * (MAX_ORDER + 2)),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("plan_id", ctypes.c_int32),
        ("tile_m", ctypes.c_int32),
        ("tile_k", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
        ("groups", ctypes.c_int64),
        ("partials", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_size_t),
        ("alg_bytes", ctypes.c_double),
        ("alg_flops", ctypes.c_double),
        ("plan_name", ctypes.c_char * 48),
        ("tuned_us", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("est_err", ctypes.c_double),
    ]


class DecompOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("max_iters", ctypes.c_int32),
        ("iter_tol", ctypes.c_double),
        ("fit_trace", ctypes.POINTER(ctypes.c_double)),
    ]


class DecompResult(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("fit", ctypes.c_double),
        ("iters", ctypes.c_int64),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("batched", ctypes.c_int32),
        ("max_jobs_per_epoch", ctypes.c_int32),
        ("epochs_in_flight", ctypes.c_int32),
        ("als_update", ctypes.c_int32),
        ("max_requests", ctypes.c_int64),
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("direct_max_jobs", ctypes.c_int32),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("out_dtype", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("plan_hint", ctypes.c_int32),
        ("split_hint", ctypes.c_int32),
        ("report", ctypes.POINTER(Report)),
        ("tol", ctypes.c_double),
        ("x_dtype", ctypes.c_int32),
        ("u_dtype", ctypes.c_int32),
        ("deterministic", ctypes.c_int32),
    ]


# Every extern "C" symbol declared in include/deinsum.h.
EXPORTS = (
    "deinsum_opts_init", "deinsum_parse", "deinsum_workspace_size", "deinsum_mttkrp",
    "deinsum_ttmc", "deinsum_last_error", "deinsum_synth_fill", "deinsum_convert",
    "deinsum_shutdown", "deinsum_version", "deinsum_batch_create", "deinsum_batch_add_mttkrp",
    "deinsum_batch_launch", "deinsum_batch_reset", "deinsum_batch_info", "deinsum_batch_destroy",
    "deinsum_server_config_init", "deinsum_server_create", "deinsum_server_add_tensor", "deinsum_server_start",
    "deinsum_server_submit", "deinsum_server_replay", "deinsum_server_drain", "deinsum_server_results",
    "deinsum_server_stats", "deinsum_server_destroy", "deinsum_tune_mttkrp", "deinsum_tune_batch_mttkrp",
    "deinsum_tune_load", "deinsum_tune_save", "deinsum_tune_clear", "deinsum_tune_entries",
    "deinsum_fx20_size", "deinsum_fx20_encode", "deinsum_tune_ttmc", "deinsum_mttkrp_mm",
    "deinsum_mttkrp_noalloc", "deinsum_estimate_error", "deinsum_choose_storage", "deinsum_tensor_stats",
    "deinsum_server_poll", "deinsum_decomp_opts_init", "deinsum_cp_als", "deinsum_tucker_hooi",
    "deinsum_kernel_timing", "deinsum_kernel_times",
)

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_2206_08301_amd/build.py` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp = ctypes.c_void_p
    lib.deinsum_opts_init.argtypes = [ctypes.POINTER(Opts)]
    lib.deinsum_opts_init.restype = None
    lib.deinsum_parse.argtypes = [ctypes.c_char_p, ctypes.POINTER(Spec)]
    lib.deinsum_parse.restype = ctypes.c_int
    lib.deinsum_workspace_size.argtypes = [ctypes.POINTER(Spec), i64p, i64p, ctypes.POINTER(Opts),
                                           ctypes.POINTER(ctypes.c_size_t)]
    lib.deinsum_workspace_size.restype = ctypes.c_int
    lib.deinsum_mttkrp.argtypes = [ctypes.POINTER(Spec), i64p, ctypes.c_int64, vp,
                                   ctypes.POINTER(vp), vp, ctypes.POINTER(Opts), vp]
    lib.deinsum_mttkrp.restype = ctypes.c_int
    lib.deinsum_mttkrp_noalloc.argtypes = lib.deinsum_mttkrp.argtypes
    lib.deinsum_mttkrp_noalloc.restype = ctypes.c_int
    lib.deinsum_ttmc.argtypes = [ctypes.POINTER(Spec), i64p, i64p, vp, ctypes.POINTER(vp), vp,
                                 ctypes.POINTER(Opts), vp]
    lib.deinsum_ttmc.restype = ctypes.c_int
    lib.deinsum_mttkrp_mm.argtypes = [ctypes.POINTER(Spec), i64p, ctypes.c_int64, ctypes.c_int64, vp,
                                      ctypes.POINTER(vp), vp, vp, ctypes.POINTER(Opts), vp]
    lib.deinsum_mttkrp_mm.restype = ctypes.c_int
    lib.deinsum_last_error.argtypes = []
    lib.deinsum_last_error.restype = ctypes.c_char_p
    lib.deinsum_synth_fill.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.c_int64, ctypes.c_int32, vp]
    lib.deinsum_synth_fill.restype = ctypes.c_int
    lib.deinsum_convert.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int64, vp]
    lib.deinsum_convert.restype = ctypes.c_int
    lib.deinsum_shutdown.argtypes = []
    lib.deinsum_shutdown.restype = ctypes.c_int
    lib.deinsum_version.argtypes = []
    lib.deinsum_version.restype = ctypes.c_char_p
    lib.deinsum_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(vp)]
    lib.deinsum_batch_create.restype = ctypes.c_int
    lib.deinsum_batch_add_mttkrp.argtypes = [vp, ctypes.POINTER(Spec), i64p, ctypes.c_int64, vp,
                                             ctypes.POINTER(vp), vp, ctypes.POINTER(Opts),
                                             ctypes.POINTER(ctypes.c_int32)]
    lib.deinsum_batch_add_mttkrp.restype = ctypes.c_int
    lib.deinsum_batch_launch.argtypes = [vp, vp]
    lib.deinsum_batch_launch.restype = ctypes.c_int
    lib.deinsum_batch_reset.argtypes = [vp]
    lib.deinsum_batch_reset.restype = ctypes.c_int
    lib.deinsum_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.deinsum_batch_info.restype = ctypes.c_int
    lib.deinsum_batch_destroy.argtypes = [vp]
    lib.deinsum_batch_destroy.restype = ctypes.c_int
    i32p = ctypes.POINTER(ctypes.c_int32)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.deinsum_server_config_init.argtypes = [ctypes.POINTER(ServerConfig)]
    lib.deinsum_server_config_init.restype = None
    lib.deinsum_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.deinsum_server_create.restype = ctypes.c_int
    lib.deinsum_server_add_tensor.argtypes = [vp, ctypes.c_int32, i64p, ctypes.c_int64, ctypes.c_int32, vp,
                                              ctypes.POINTER(vp), i32p]
    lib.deinsum_server_add_tensor.restype = ctypes.c_int
    lib.deinsum_server_start.argtypes = [vp]
    lib.deinsum_server_start.restype = ctypes.c_int
    lib.deinsum_server_submit.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, i64p]
    lib.deinsum_server_submit.restype = ctypes.c_int
    lib.deinsum_server_replay.argtypes = [vp, ctypes.c_int64, f64p, i32p, i32p]
    lib.deinsum_server_replay.restype = ctypes.c_int
    lib.deinsum_server_drain.argtypes = [vp]
    lib.deinsum_server_drain.restype = ctypes.c_int
    lib.deinsum_server_results.argtypes = [vp, ctypes.c_int64, f64p, f64p, i64p]
    lib.deinsum_server_results.restype = ctypes.c_int
    lib.deinsum_kernel_timing.argtypes = [ctypes.c_int32, ctypes.c_int64]
    lib.deinsum_kernel_timing.restype = ctypes.c_int
    lib.deinsum_kernel_times.argtypes = [ctypes.c_int64, i32p, f64p, i64p]
    lib.deinsum_kernel_times.restype = ctypes.c_int
    lib.deinsum_decomp_opts_init.argtypes = [ctypes.POINTER(DecompOpts)]
    lib.deinsum_decomp_opts_init.restype = None
    lib.deinsum_cp_als.argtypes = [ctypes.c_int32, i64p, ctypes.c_int64, vp, ctypes.POINTER(vp), vp,
                                   ctypes.POINTER(DecompOpts), ctypes.POINTER(DecompResult), vp]
    lib.deinsum_cp_als.restype = ctypes.c_int
    lib.deinsum_tucker_hooi.argtypes = [ctypes.c_int32, i64p, i64p, vp, ctypes.POINTER(vp), vp,
                                        ctypes.POINTER(DecompOpts), ctypes.POINTER(DecompResult), vp]
    lib.deinsum_tucker_hooi.restype = ctypes.c_int
    lib.deinsum_server_poll.argtypes = [vp, ctypes.c_int64, i32p, i32p, f64p]
    lib.deinsum_server_poll.restype = ctypes.c_int
    lib.deinsum_server_stats.argtypes = [vp, i64p, i64p, i64p]
    lib.deinsum_server_stats.restype = ctypes.c_int
    lib.deinsum_server_destroy.argtypes = [vp]
    lib.deinsum_server_destroy.restype = ctypes.c_int
    for name in ("deinsum_tune_mttkrp", "deinsum_tune_batch_mttkrp"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.POINTER(Spec), i64p, ctypes.c_int64, vp, ctypes.POINTER(vp), vp, ctypes.POINTER(Opts),
                      ctypes.c_int32, ctypes.POINTER(Report), vp]
        f.restype = ctypes.c_int
    for name in ("deinsum_tune_load", "deinsum_tune_save"):
        getattr(lib, name).argtypes = [ctypes.c_char_p]
        getattr(lib, name).restype = ctypes.c_int
    lib.deinsum_tune_clear.argtypes = []
    lib.deinsum_tune_clear.restype = ctypes.c_int
    lib.deinsum_tune_entries.argtypes = [i64p]
    lib.deinsum_tune_entries.restype = ctypes.c_int
    lib.deinsum_tune_ttmc.argtypes = [ctypes.POINTER(Spec), i64p, i64p, vp, ctypes.POINTER(vp), vp,
                                      ctypes.POINTER(Opts), ctypes.c_int32, ctypes.POINTER(Report), vp]
    lib.deinsum_tune_ttmc.restype = ctypes.c_int
    lib.deinsum_fx20_size.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    lib.deinsum_fx20_size.restype = ctypes.c_int
    lib.deinsum_fx20_encode.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, vp, ctypes.c_size_t, vp]
    lib.deinsum_fx20_encode.restype = ctypes.c_int
    lib.deinsum_estimate_error.argtypes = [ctypes.POINTER(Spec), i64p, i64p, vp, ctypes.POINTER(Opts),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), vp]
    lib.deinsum_estimate_error.restype = ctypes.c_int
    lib.deinsum_choose_storage.argtypes = [ctypes.POINTER(Spec), i64p, i64p, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.deinsum_choose_storage.restype = ctypes.c_int
    lib.deinsum_tensor_stats.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), vp]
    lib.deinsum_tensor_stats.restype = ctypes.c_int
    _lib = lib
    return lib


def check(status: int):
    if status != OK:
        msg = load().deinsum_last_error()
        raise DeinsumError(status, msg.decode() if msg else "")
