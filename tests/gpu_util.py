"""Helpers shared by the GPU parity tests (no solver arithmetic here)."""
import sys

import numpy as np


# pytest's capture manager, set by conftest: notes are written with capture suspended, so the
# progress of a long case (minutes of CPU truth computations) shows while it runs
CAPTURE = None


def note(msg):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    if CAPTURE is not None:
        with CAPTURE.global_and_fixture_disabled():
            print(f"[gpu-case] {msg}", flush=True)
    else:
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


def fp64_bound(kappa):
    """Parity bound of a plain-FP64 GPU iterate against the FP64 oracle at the
    same t: 1e-12, or a tenth of kappa(A_mu) times the unit roundoff when that
    is larger (two FP64 block-CG runs that round differently can disagree by up
    to about kappa u; measured against an extended-precision reference, both
    stay within 0.05 kappa u on the batch workload)."""
    return max(1e-12, 0.1 * kappa * 2.0 ** -53)
