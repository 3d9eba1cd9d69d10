"""Helpers shared by the GPU parity tests (device transfers only)."""
import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(x_np, dtype=torch.float32):
    """numpy (n_1..n_d) array -> device tensor with Kolda strides, same values."""
    x = np.asfortranarray(x_np)
    rev = list(reversed(range(x.ndim)))
    t = torch.from_numpy(np.ascontiguousarray(x.transpose(rev))).to(dtype).cuda()
    return t.permute(*rev)


def to_host(t):
    """Device tensor (any strides) -> float64 numpy array with the same logical shape."""
    return t.detach().to(torch.float64).cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def banner(msg):
    print(f"\n[gpu-test] {msg}", flush=True)
