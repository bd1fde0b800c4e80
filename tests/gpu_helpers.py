"""Shared helpers of the GPU parity tests (no method arithmetic here)."""

import numpy as np
import torch


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def f32(z):
    """Round complex128 -> complex64 -> complex128 (the FP32 input the GPU sees)."""
    return z.astype(np.complex64).astype(np.complex128)
