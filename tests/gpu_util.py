"""Helpers shared by the GPU tests (device buffers, host copies)."""
import numpy as np
import pytest


def cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a: np.ndarray):
    torch = cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t) -> np.ndarray:
    cuda().cuda.synchronize()
    return t.cpu().numpy()


def first_mismatch(a: np.ndarray, b: np.ndarray):
    d = np.nonzero(a != b)[0]
    return None if d.size == 0 else int(d[0])
