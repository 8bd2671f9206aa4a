"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import numpy as np
import pytest


def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
