"""Seeded synthetic inputs (host side) for MTTKRP / TTMc workloads.

This module holds the input recipe and none of the method's arithmetic.  It
serves both the HIP path (through ``synth_fill`` in the binding, whose
device generator implements the same counter-based stream) and the CPU
oracle (through the numpy functions here).

Tensor entries -- counter-based SplitMix64 (Steele, Lea & Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): the value at
linear (row-major) index ``i`` of a tensor with seed ``s`` is derived from
``z = mix64(s + (i + 1) * 0x9E3779B97F4A7C15)``, i.e. the (i+1)-th output of
a SplitMix64 stream seeded with ``s``:

  * ``uniform``: ``2 * ((z >> 11) * 2**-53) - 1``   -- exact FP64, in [-1, 1)
  * ``int5``   : ``((z >> 32) % 5) - 2``            -- integers in {-2..2}
  * ``int3``   : ``((z >> 32) % 3) - 1``            -- integers in {-1, 0, 1}

Factor matrices -- numpy's PCG64 ``default_rng(seed)``: N(0,1) entries,
optionally orthonormalised by Householder QR (first R columns of Q), or
integers in a small range for exact-arithmetic tests.
"""
from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

DIST_UNIFORM = 0
DIST_INT5 = 1
DIST_INT3 = 2
DIST_NAMES = {"uniform": DIST_UNIFORM, "int5": DIST_INT5, "int3": DIST_INT3}

SEED_BASE = 2206083010


def config_seed(config: int, operand: int) -> int:
    """Seed of operand ``operand`` (0 = X, 1 + m = factor of mode m) of config 1..5."""
    return SEED_BASE + 100 * int(config) + int(operand)


def splitmix64_at(seed: int, index) -> np.ndarray:
    """Counter-mode SplitMix64: output number ``index`` (0-based) of the stream seeded ``seed``."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def x_values(seed: int, index, dist: str = "uniform") -> np.ndarray:
    """Tensor entries at the given linear indices (FP64)."""
    z = splitmix64_at(seed, index)
    d = DIST_NAMES[dist]
    if d == DIST_UNIFORM:
        return 2.0 * ((z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53) - 1.0
    if d == DIST_INT5:
        return ((z >> np.uint64(32)) % np.uint64(5)).astype(np.float64) - 2.0
    if d == DIST_INT3:
        return ((z >> np.uint64(32)) % np.uint64(3)).astype(np.float64) - 1.0
    raise ValueError(dist)


def x_tensor(seed: int, dims, dist: str = "uniform") -> np.ndarray:
    """The whole tensor (host RAM), row-major."""
    n = int(np.prod(dims))
    return x_values(seed, np.arange(n, dtype=np.uint64), dist).reshape(dims)


def _threads() -> int:
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def x_range(seed: int, start: int, count: int, dist: str = "uniform", chunk: int = 1 << 22,
            out: np.ndarray | None = None) -> np.ndarray:
    """Entries at linear indices [start, start + count), generated in chunks (numpy
    releases the GIL inside its ufuncs, so the chunks run on a thread pool)."""
    if out is None:
        out = np.empty(count, dtype=np.float64)
    starts = list(range(0, count, chunk))

    def one(c0):
        c1 = min(count, c0 + chunk)
        out[c0:c1] = x_values(seed, np.arange(start + c0, start + c1, dtype=np.uint64), dist)

    if len(starts) <= 1:
        for c0 in starts:
            one(c0)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(_threads(), len(starts))) as ex:
            list(ex.map(one, starts))
    return out


def x_slab(seed: int, dims, mode: int, index: int, dist: str = "uniform") -> np.ndarray:
    """The sub-tensor with ``i_mode == index`` (shape: dims with dims[mode] = 1)."""
    dims = [int(d) for d in dims]
    if mode == 0:
        inner = int(np.prod(dims[1:]))
        return x_range(seed, index * inner, inner, dist).reshape([1] + dims[1:])
    strides = np.ones(len(dims), dtype=np.uint64)
    for m in range(len(dims) - 2, -1, -1):
        strides[m] = strides[m + 1] * np.uint64(dims[m + 1])
    sub = list(dims)
    sub[mode] = 1
    grids = np.indices(sub, dtype=np.uint64)
    lin = np.zeros(sub, dtype=np.uint64)
    for m in range(len(dims)):
        g = grids[m] + (np.uint64(index) if m == mode else np.uint64(0))
        lin += g * strides[m]
    return x_values(seed, lin, dist)


def x_rows(seed: int, dims, mode: int, indices, dist: str = "uniform") -> np.ndarray:
    """The sub-tensor whose mode-``mode`` index runs over ``indices`` (in that order):
    shape = dims with dims[mode] = len(indices)."""
    dims = [int(d) for d in dims]
    idx = [int(i) for i in indices]
    outer = int(np.prod(dims[:mode])) if mode else 1
    inner = int(np.prod(dims[mode + 1:])) if mode + 1 < len(dims) else 1
    sub = list(dims)
    sub[mode] = len(idx)
    out = np.empty((outer, len(idx), inner), dtype=np.float64)
    if inner >= (1 << 20):  # long contiguous runs: generate each run directly
        for a in range(outer):
            for p, i in enumerate(idx):
                x_range(seed, (a * dims[mode] + i) * inner, inner, dist, out=out[a, p])
        return out.reshape(sub)
    b = np.arange(inner, dtype=np.uint64)
    rows_per = max(1, (1 << 22) // max(1, inner))

    def one(a0):
        a1 = min(outer, a0 + rows_per)
        a = np.arange(a0, a1, dtype=np.uint64)
        for p, i in enumerate(idx):
            lin = ((a * np.uint64(dims[mode]) + np.uint64(i)) * np.uint64(inner))[:, None] + b[None, :]
            out[a0:a1, p, :] = x_values(seed, lin, dist)

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(one, range(0, outer, rows_per)))
    return out.reshape(sub)


def normal_factor(seed: int, rows: int, cols: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((rows, cols))


def orthonormal_factor(seed: int, rows: int, cols: int) -> np.ndarray:
    """First ``cols`` columns of Q from a Householder QR of an N(0,1) matrix."""
    a = normal_factor(seed, rows, cols)
    q, _ = np.linalg.qr(a, mode="reduced")
    return np.ascontiguousarray(q)


def int_factor(seed: int, rows: int, cols: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    return np.random.default_rng(seed).integers(lo, hi + 1, size=(rows, cols)).astype(np.float64)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    return (u & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
