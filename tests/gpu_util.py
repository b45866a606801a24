"""Helpers of the GPU tests: host <-> device copies of key arrays."""
import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_keys(rng, n, dtype, hi=None):
    if dtype == np.uint32:
        return rng.integers(0, (1 << 32) if hi is None else hi, n, dtype=np.uint64).astype(np.uint32)
    if hi is None:
        return rng.integers(0, 1 << 63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    return rng.integers(0, hi, n, dtype=np.uint64)
