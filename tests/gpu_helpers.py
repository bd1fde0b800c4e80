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


class DeviceGather:
    """Read-only array view of a device tensor: fancy-index reads gather on
    the device and return host numpy arrays, so per-site oracle routines can
    sample lattices too large to copy to the host."""

    def __init__(self, t):
        self.t = t
        self.shape = tuple(t.shape)

    def __getitem__(self, idx):
        if not isinstance(idx, tuple):
            idx = (idx,)
        idx = tuple(torch.as_tensor(np.asarray(i), device=self.t.device)
                    if isinstance(i, np.ndarray) else i for i in idx)
        return self.t[idx].cpu().numpy()


def site_rel(a, b, per=12):
    """Largest per-site error relative to that site's largest reference
    entry: max over sites of max_k |a_k - b_k| / max_k |b_k|, the complex
    entries grouped `per` to a site (12 for spinors, 9 for links).  Sites
    whose reference is zero (the other parity of a half field) must come out
    zero.  Complements the norm-wise error, which one bad entry among many
    could pass."""
    a = np.asarray(a).reshape(-1, per).astype(np.complex128)
    b = np.asarray(b).reshape(-1, per).astype(np.complex128)
    scale = np.abs(b).max(axis=1)
    err = np.abs(a - b).max(axis=1)
    zero = scale == 0
    if np.any(err[zero] != 0):
        return float("inf")
    if np.all(zero):
        return 0.0
    return float((err[~zero] / scale[~zero]).max())
