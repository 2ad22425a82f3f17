"""Helpers for the GPU tests: torch device buffers and oracle counterparts.

Only device memory and streams come from torch; every step of the solver runs
in libcurldiv through the C ABI.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def gpu_ok():
    return torch.cuda.is_available()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def empty(n, dtype=torch.float64):
    return torch.zeros(n, dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def stream():
    return torch.cuda.current_stream().cuda_stream


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
