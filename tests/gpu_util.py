"""Helpers shared by the GPU tests: device tensors from numpy words and back."""
import numpy as np
import torch


def dev(words: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(words).view(np.int64)
    return torch.from_numpy(a.copy()).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def words_for(vals, N):
    from oracle import pyint
    return pyint.encode(vals, (N + 63) // 64)
