"""Helpers shared by the GPU tests (host side only)."""
import sys

import numpy as np


def announce(msg: str):
    sys.stderr.write("[gpu-step] %s\n" % msg)
    sys.stderr.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_max_err(u, ref):
    """max |u - ref| / max |ref| (the paper's E, used as the parity metric)."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def sample_points(n, rng, extra=(), count=48, distinct_j3=6):
    """Grid indices for sampled parity checks: corners, centre, the given
    extra points and random ones, drawn over a few distinct i3 values so the
    FFT-free oracle evaluation stays cheap."""
    j3s = list(rng.choice(n, size=distinct_j3, replace=False))
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, n // 2, n // 2), (0, n - 1, 0)]
    pts += [tuple(int(v) for v in e) for e in extra]
    j3s += [p[2] for p in pts]
    for _ in range(count):
        pts.append((int(rng.integers(n)), int(rng.integers(n)), int(rng.choice(j3s))))
    return np.array(pts, dtype=np.int64)
