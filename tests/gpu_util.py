"""Helpers shared by the GPU tests: moving numpy arrays of unsigned keys to
device tensors and back (bit patterns are preserved through signed views)."""
import numpy as np
import torch


def to_dev(a: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def to_host(t: torch.Tensor, unsigned_bits: int) -> np.ndarray:
    a = t.cpu().numpy()
    return a.view(np.uint64 if unsigned_bits == 64 else np.uint32)


def rows_host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)
