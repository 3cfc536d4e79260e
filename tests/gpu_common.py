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


# bf16-stored basis: the GPU and the oracle round different fp32 sums to bf16,
# so their bases differ by bf16 rounding steps (unit roundoff 2^-9) and their
# cycle histories by a relative amount of that order (measured 8.8e-4 on the
# 64^2 parity system, 1.3e-3 on the 27-point 128^3 system); below ~1e-5 the
# fp32 arithmetic of the Hessenberg matrix sets an absolute floor
BF16_REL = 2.0 ** -7
BF16_FLOOR = 2e-6


def bf16_hist_ok(h, ref):
    """|h_j - ref_j| <= BF16_REL ref_j + BF16_FLOOR on every step; returns
    (ok, (max abs gap, max relative gap, first offending steps))."""
    h = np.asarray(h, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    gap = np.abs(h - ref)
    bad = gap > BF16_REL * ref + BF16_FLOOR
    return not np.any(bad), (float(gap.max()), float((gap / np.maximum(ref, 1e-300)).max()),
                             [(int(i), float(ref[i]), float(gap[i])) for i in np.flatnonzero(bad)[:5]])
