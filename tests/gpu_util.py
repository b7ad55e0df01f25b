"""Device-buffer helpers for the GPU tests (torch supplies memory only)."""
from __future__ import annotations

import sys

import numpy as np


def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        import pytest

        pytest.skip("no GPU")
    return torch


def to_dev(a: np.ndarray):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def zeros_dev(n: int, fill: int = 0):
    torch = torch_cuda()
    t = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
    t.fill_(fill)
    return t


def to_host(t) -> np.ndarray:
    torch = torch_cuda()
    torch.cuda.synchronize()
    return t.cpu().numpy()


def note(msg: str):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(msg, file=sys.stderr, flush=True)


def first_diff(a: np.ndarray, b: np.ndarray):
    if a.shape != b.shape:
        return f"shape {a.shape} vs {b.shape}"
    d = np.nonzero(a != b)[0]
    if d.size == 0:
        return None
    return f"{d.size} bytes differ, first at {d[0]}: {a[d[0]]} vs {b[d[0]]}"
