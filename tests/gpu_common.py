"""Shared helpers of the GPU parity tests (imported only by ``-m gpu`` tests)."""
import sys

import numpy as np


def say(*args):
    """Name the case on stdout before a GPU step (flushed, so a hard failure
    still shows which case was running)."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev_tensor(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def cycle_slices(hist, starts):
    out = []
    for i, s in enumerate(starts):
        e = starts[i + 1] if i + 1 < len(starts) else len(hist)
        out.append(np.asarray(hist[s:e]))
    return out
