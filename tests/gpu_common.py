"""Shared helpers for the GPU parity tests (inputs come from the synth module;
expected values from the CPU oracle only)."""
import numpy as np
import torch

SPEC3 = {0: "ijk,ja,ka->ia", 1: "ijk,ia,ka->ja", 2: "ijk,ia,ja->ka"}
LETTERS = "ijklmnop"


def mttkrp_spec(N, n, rank_letter="z"):
    t = LETTERS[:N]
    facs = [t[m] + rank_letter for m in range(N) if m != n]
    return f"{t}," + ",".join(facs) + f"->{t[n]}{rank_letter}"


def ttmc_spec(N, n):
    t = LETTERS[:N]
    ranks = "abcdefgh"
    facs = [t[m] + ranks[m] for m in range(N) if m != n]
    out = "".join(t[m] if m == n else ranks[m] for m in range(N))
    return f"{t}," + ",".join(facs) + f"->{out}"


def nrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.linalg.norm(b.ravel())
    d = np.linalg.norm((a - b).ravel())
    return d / s if s > 0 else d


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def flush(msg):
    print(msg, flush=True)
