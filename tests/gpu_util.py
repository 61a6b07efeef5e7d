"""Helpers shared by the GPU parity tests (no solver arithmetic here)."""
import sys

import numpy as np


def note(msg):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def a_err(A, mu, x, xref):
    """relative A_mu-norm difference, FP64 on the host"""
    e = np.asarray(x, dtype=np.float64) - np.asarray(xref, dtype=np.float64)
    num = e @ (A @ e) + mu * (e @ e)
    den = xref @ (A @ xref) + mu * (xref @ xref)
    return float(np.sqrt(max(num, 0.0) / den))
