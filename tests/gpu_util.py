"""Helpers for the GPU tests: numpy <-> torch word arrays and the oracle-side
bin check.  Holds no arithmetic of the method (the oracle does that)."""
import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    """uint32 numpy array -> int32 CUDA tensor with the same bits."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).cuda()
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).cuda()
    raise TypeError(a.dtype)


def host(t: torch.Tensor) -> np.ndarray:
    """CUDA tensor of 32/64-bit words -> unsigned numpy array."""
    a = t.cpu().numpy()
    if a.dtype in (np.int32, np.uint32):
        return a.view(np.uint32)
    return a.view(np.uint64)


def root_of_order(m: int, lognu: int, logn: int, odd: int = 1) -> int:
    """2^((nu / N) * odd) mod m (Python pow): a root of exact order N."""
    return pow(2, (1 << (lognu - logn)) * odd, m)
