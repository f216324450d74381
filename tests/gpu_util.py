"""Helpers shared by the GPU tests: host <-> device copies of numpy arrays."""
import numpy as np
import torch

NP_TO_TORCH = {np.dtype(np.uint32): torch.uint32, np.dtype(np.int32): torch.int32,
               np.dtype(np.uint64): torch.uint64, np.dtype(np.float32): torch.float32,
               np.dtype(np.int64): torch.int64}


def dev(x: np.ndarray) -> torch.Tensor:
    x = np.ascontiguousarray(x)
    if x.size == 0:
        return torch.empty(0, dtype=NP_TO_TORCH[x.dtype], device="cuda")
    return torch.from_numpy(x).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def same_bits(x: np.ndarray, y: np.ndarray) -> bool:
    return x.dtype == y.dtype and x.shape == y.shape and x.tobytes() == y.tobytes()


def first_mismatch(x: np.ndarray, y: np.ndarray):
    """None if x and y hold the same bits, else a description of the first difference."""
    if x.dtype != y.dtype:
        return f"dtype {x.dtype} != {y.dtype}"
    if len(x) != len(y):
        return f"length {len(x)} != {len(y)}"
    if len(x) == 0:
        return None
    xb = np.ascontiguousarray(x).view(np.uint8).reshape(len(x), -1)
    yb = np.ascontiguousarray(y).view(np.uint8).reshape(len(y), -1)
    bad = np.nonzero(np.any(xb != yb, axis=1))[0]
    if len(bad) == 0:
        return None
    i = int(bad[0])
    return f"{len(bad)} mismatches, first at {i}: got {x[i]!r} want {y[i]!r}"
