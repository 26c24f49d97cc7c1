"""Independent geometric checks used to pin the oracle.

These are textbook, type-free definitions written in numpy (not the
oracle's typed closed forms): the distance between closed primitives as a
minimum over a plane/line projection and clamped point-segment distances,
plus dense parameter sampling.  They exist only to catch mistakes in the
oracle; they are never used as a parity reference for the HIP library.
"""
from __future__ import annotations

import numpy as np


def point_segment(p, a, b):
    e = b - a
    ee = e @ e
    t = 0.0 if ee == 0 else np.clip((p - a) @ e / ee, 0.0, 1.0)
    return np.linalg.norm(p - (a + t * e))


def point_triangle(p, t0, t1, t2):
    e0, e1 = t1 - t0, t2 - t0
    M = np.array([[e0 @ e0, e0 @ e1], [e0 @ e1, e1 @ e1]])
    rhs = np.array([e0 @ (p - t0), e1 @ (p - t0)])
    cands = [point_segment(p, t0, t1), point_segment(p, t1, t2), point_segment(p, t2, t0)]
    if abs(np.linalg.det(M)) > 0:
        u, v = np.linalg.solve(M, rhs)
        if u >= 0 and v >= 0 and u + v <= 1:
            cands.append(np.linalg.norm(p - (t0 + u * e0 + v * e1)))
    return min(cands)


def segment_segment(a0, a1, b0, b1):
    u, v, w = a1 - a0, b1 - b0, a0 - b0
    cands = [point_segment(a0, b0, b1), point_segment(a1, b0, b1),
             point_segment(b0, a0, a1), point_segment(b1, a0, a1)]
    M = np.array([[u @ u, -(u @ v)], [u @ v, -(v @ v)]])
    if abs(np.linalg.det(M)) > 1e-300:
        s, t = np.linalg.solve(M, [-(u @ w), -(v @ w)])
        if 0 <= s <= 1 and 0 <= t <= 1:
            cands.append(np.linalg.norm(w + s * u - t * v))
    return min(cands)


def pair_distance(kind, x12):
    x = np.asarray(x12, dtype=np.float64).reshape(4, 3)
    if kind == 0:
        return point_triangle(x[0], x[1], x[2], x[3])
    return segment_segment(x[0], x[1], x[2], x[3])


def sampled_distance(kind, x12, n=120):
    """Minimum over a dense parameter grid (an upper bound converging to the
    exact distance as n grows)."""
    x = np.asarray(x12, dtype=np.float64).reshape(4, 3)
    s = np.linspace(0.0, 1.0, n + 1)
    if kind == 0:
        U, V = np.meshgrid(s, s, indexing="ij")
        m = (U + V) <= 1.0
        pts = x[1] + U[m][:, None] * (x[2] - x[1]) + V[m][:, None] * (x[3] - x[1])
        return np.linalg.norm(pts - x[0], axis=1).min()
    A = x[0] + s[:, None] * (x[1] - x[0])
    B = x[2] + s[:, None] * (x[3] - x[2])
    return np.linalg.norm(A[:, None, :] - B[None, :, :], axis=2).min()


def random_rotation(rng):
    qv = rng.normal(size=4)
    qv /= np.linalg.norm(qv)
    w, x, y, z = qv
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
