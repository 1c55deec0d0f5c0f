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


TILES = [8, 14, 21, 14, 8]       # tile choices of passes H1..H5


def radix_plans(n):
    """Radix plans the library has for padded length 2n."""
    N = 2 * n
    return [0] + ([1] if N in (128, 256, 384, 512, 768) else []) + ([2] if N in (128, 192, 256, 384, 512, 768) else [])


def shape_rounds(n):
    """The autotuner's rounds: round r gives pass i its candidate r mod count,
    so the rounds together cover every (radix plan, tile) of every pass."""
    cands = [[(pl, tl) for pl in radix_plans(n) for tl in range(TILES[i])] for i in range(5)]
    for r in range(max(len(c) for c in cands)):
        yield [c[r % len(c)][0] for c in cands], [c[r % len(c)][1] for c in cands]
