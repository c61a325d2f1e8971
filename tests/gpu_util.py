"""Helpers for the GPU tests: move seeded inputs to the device, build a
handle, and compare against the oracle."""
from __future__ import annotations

import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a GPU test ran without a visible GPU")
    return torch


def dev(a):
    torch = torch_cuda()
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def make(ms, shape, cuts, faces):
    """Device faces + handle.  Returns (handle, device faces)."""
    df = [dev(f) for f in faces]
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=df)
    return h, df


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*args):
    """Name the case before a GPU step, flushed, so a fault names it."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()
