"""Z-order (Morton order) of the Gaussians, the layout step of Sec. 3.3
"Locality-preserving Densification": the parameter buffers are re-sorted so
that Gaussians close in 3D are close in memory.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper names the technique (z-ordering of the point set) but not its
parameters; this reading is used on both sides:
  * bounding cube: lo = per-axis minimum of the means, side e = the largest
    per-axis extent (max - min), so the three axes share one scale;
  * quantisation to 10 bits per axis, in FP32 (the decision is an integer, so
    both sides take it in the same precision): s = 1024 / e (one correctly
    rounded FP32 division), t = (x - lo) * s (two FP32 operations),
    q = min(1023, floor(t)); e == 0 gives q = 0;
  * code = bit interleave, x in bit 0: bit 3k of the code is bit k of q_x,
    bit 3k+1 of q_y, bit 3k+2 of q_z (30-bit code);
  * order: ascending code, ties by index (a stable sort).
The permutation perm lists, for each position k, the index of the Gaussian
placed there: new_plane[k] = old_plane[perm[k]].
"""
from __future__ import annotations

import numpy as np

BITS = 10


def quantize32(means: np.ndarray) -> np.ndarray:
    """means float32 [3, n] -> uint32 [3, n] cell coordinates in 0..1023."""
    m = np.asarray(means, dtype=np.float32)
    n = m.shape[1]
    if n == 0:
        return np.zeros((3, 0), np.uint32)
    lo = m.min(axis=1)
    hi = m.max(axis=1)
    e = np.float32((hi - lo).max())
    if e == 0:
        return np.zeros((3, n), np.uint32)
    s = np.float32(1024.0) / e
    with np.errstate(over="ignore"):
        t = (m - lo[:, None]).astype(np.float32) * s
    t = t.astype(np.float32)
    q = np.floor(t).astype(np.int64)
    return np.minimum(q, 1023).astype(np.uint32)


def interleave(qx: np.ndarray, qy: np.ndarray, qz: np.ndarray) -> np.ndarray:
    """30-bit Morton code from three 10-bit coordinates, x in the lowest bit:
    written out one bit at a time."""
    code = np.zeros(np.shape(qx), np.uint64)
    for k in range(BITS):
        for a, q in enumerate((qx, qy, qz)):
            bit = (np.asarray(q, np.uint64) >> np.uint64(k)) & np.uint64(1)
            code |= bit << np.uint64(3 * k + a)
    return code.astype(np.uint32)


def deinterleave(code: np.ndarray):
    """Inverse of interleave: (qx, qy, qz)."""
    c = np.asarray(code, np.uint64)
    out = []
    for a in range(3):
        q = np.zeros(c.shape, np.uint64)
        for k in range(BITS):
            q |= ((c >> np.uint64(3 * k + a)) & np.uint64(1)) << np.uint64(k)
        out.append(q.astype(np.uint32))
    return tuple(out)


def morton_codes(means: np.ndarray) -> np.ndarray:
    q = quantize32(means)
    return interleave(q[0], q[1], q[2])


def zorder_permutation(means: np.ndarray) -> np.ndarray:
    """perm[k] = index of the Gaussian at position k (stable in the index)."""
    codes = morton_codes(means)
    return np.argsort(codes, kind="stable").astype(np.uint32)
