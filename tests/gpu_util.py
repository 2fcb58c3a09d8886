"""GPU-test plumbing: numpy <-> torch device tensors and library contexts built
from oracle parameter sets (the oracle only supplies parameters and inputs)."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O


def dev(a: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def ctx_for(F, prm: O.Params):
    return F.fhelin_ctx_create(prm.log_n, prm.q, prm.p, prm.dnum)


def keys_at(prm: O.Params, keys: O.KeySet, level: int) -> np.ndarray:
    """Oracle full-width keys [n][dnum][2][L+K][N] -> the ABI's compact layout
    [n][beta(level)][2][level+K][N]."""
    beta = prm.beta(level)
    idx = list(range(level)) + list(range(prm.L, prm.L + prm.K))
    return np.ascontiguousarray(keys.evk[:, :beta][:, :, :, idx])


def pad_cts(cts: list, stride: int, N: int) -> np.ndarray:
    """List of [2][l][N] arrays -> [n][2][stride][N] (zero padded)."""
    out = np.zeros((len(cts), 2, stride, N), np.uint64)
    for t, c in enumerate(cts):
        out[t, :, : c.shape[1]] = c
    return out
